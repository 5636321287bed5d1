"""tlib_ttt_noalloc (the TTT entry point that allocates nothing) against
tlib_ttt, through the C ABI, on two calls in a row (the second smaller), each
checked to the normwise bar of its dtype (FP64 1e-12, FP32 accumulation
1e-5): Sec. 5.2 Eq. ttt and ttt_indices."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1711_10912_amd as T  # noqa: E402
from paper_1711_10912_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu


def _rel(got, ref):
    g = got.double().cpu().numpy().ravel()
    r = ref.double().cpu().numpy().ravel()
    assert np.isfinite(g).all()
    return float(np.linalg.norm(g - r) / np.linalg.norm(r))


def _case(na, nb, layout, dtype, gen, dev):
    A = T.empty(na, layout, dtype, dev)
    A.copy_(torch.randn(na, generator=gen, device=dev, dtype=torch.float32).to(dtype))
    B = T.empty(nb, None, dtype, dev)
    B.copy_(torch.randn(nb, generator=gen, device=dev, dtype=torch.float32).to(dtype))
    return A, B


@pytest.mark.parametrize("dtype,bar", [(torch.float32, 1e-5), (torch.bfloat16, 1e-5), (torch.float64, 1e-12)])
def test_ttt_noalloc_matches_ttt_on_two_calls(dtype, bar):
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(171110912 + 3)
    phi, psi = (1, 2, 3, 4), (3, 1, 2)
    acc = torch.float64 if dtype == torch.float64 else torch.float32
    # first the full (96,80,64,48) x (64,48,120) contraction (split over K),
    # then a smaller one with a ragged tail, both A layouts interleaved
    cases = [((96, 80, 64, 48), (64, 48, 120), (3, 1, 4, 2)),
             ((40, 24, 40, 36), (40, 36, 56), (1, 2, 3, 4))]
    side = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(side):
        T.workspace_release()  # torch hands out pooled streams: start without a buffer
    for na, nb, lay in cases:
        A, B = _case(na, nb, lay, dtype, gen, dev)
        nc = (na[0], na[1], nb[2])
        ref = T.ttt(A, B, 2, phi, psi)
        got = torch.full(nc, float("nan"), dtype=acc, device=dev)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(dev)
        with torch.cuda.stream(side):
            T.ttt_noalloc(A, B, 2, phi, psi, out=got)
        side.synchronize()
        assert torch.cuda.memory_allocated(dev) == before
        # no workspace was created for the stream the call ran on
        assert _lib.lib().tlib_workspace_size(ctypes.c_void_p(side.cuda_stream)) == 0
        torch.cuda.synchronize()
        e = _rel(got, ref)
        print("ttt_noalloc %s %s vs ttt: %.2e" % (dtype, na, e), flush=True)
        assert e <= bar, (na, e)


def test_ttt_noalloc_rejects_what_ttt_rejects():
    dev = torch.device("cuda:0")
    A = torch.zeros((3, 4, 2, 6), dtype=torch.float32, device=dev)
    B = torch.zeros((2, 3, 4), dtype=torch.float32, device=dev)
    C = torch.zeros((3, 6, 3), dtype=torch.float32, device=dev)
    with pytest.raises(_lib.TlibError):
        T.ttt_noalloc(A, B, 2, (1, 4, 3, 2), (2, 3, 1), out=C)
