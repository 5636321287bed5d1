"""Outer product (Sec. 5.2 Table 3 outer_product: the q = 0 case of Eq. ttt
and ttt_indices) on its write-streaming kernel, against the FP64 oracle.

Every element of C is one product of two inputs.  The oracle forms it in
FP64, where the product of two FP32 (or 16-bit) values is exact, so the
kernel's product rounded once to FP32 must equal the oracle's value rounded to
FP32 bit for bit; FP64 products are the same single rounding on both sides.
Each case asserts the plan names the outer kernel, writes into NaN-filled
outputs, and checks that the gaps of a strided output view stay untouched."""
import numpy as np
import pytest

import oracle
import synth
from _util import to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu

DTYPES = ["f64", "f32", "bf16", "f16"]


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _acc(d):
    return "f64" if d == "f64" else "f32"


def _expect(A, B, phi, psi, d):
    """The oracle's outer product of the values the GPU holds, rounded once to
    the output dtype."""
    ref = np.asarray(oracle.ttt(oracle.materialize(A), oracle.materialize(B), 0, phi, psi))
    return ref if d == "f64" else ref.astype(np.float32).astype(np.float64)


CASES = [
    # (A shape, B shape, phi, psi, C layout)
    ((30, 7), (5, 8, 9), (1, 2), (1, 2, 3), None),
    ((30, 7), (5, 8, 9), (2, 1), (3, 2, 1), "last"),
    ((13,), (11,), (1,), (1,), None),
    ((6, 5, 4), (3, 7), (3, 1, 2), (2, 1), "rand"),
    ((257, 3), (129,), (1, 2), (1,), None),         # ragged: columns past a 256-lane chunk
    ((1, 64), (4, 1, 2), (1, 2), (1, 2, 3), None),  # extent-1 modes
    ((2, 3), (1000,), (1, 2), (1,), "last"),        # C's unit stride in B's group
]


@pytest.mark.parametrize("d", DTYPES)
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_outer_bitwise(T, d, ci):
    import torch
    na, nb, phi, psi, clay = CASES[ci]
    g = synth.rng(3, 700 + ci)
    A = synth.uniform(na, g)
    B = synth.uniform(nb, g)
    la = synth.random_layout(len(na), g)
    lb = list(range(len(nb), 0, -1))
    At, Bt = to_gpu(A, la, d), to_gpu(B, lb, d)
    nc = oracle.ttt_shape(na, nb, 0, phi, psi)
    p = len(nc)
    lay = None if clay is None else (list(range(p, 0, -1)) if clay == "last" else synth.random_layout(p, g))
    C = T.empty(nc, lay, torch_dtype(_acc(d)), "cuda").fill_(float("nan"))
    plan = T.plan(T.ttt, At, Bt, 0, phi, psi, out=C)
    assert "ttt outer" in plan, plan
    T.ttt(At, Bt, 0, phi, psi, out=C)
    torch.cuda.synchronize()
    exp = _expect(to_np(At), to_np(Bt), phi, psi, d)
    got = to_np(C)
    assert np.array_equal(got, exp), (d, ci, float(np.nanmax(np.abs(got - exp))))


@pytest.mark.parametrize("d", ["f64", "f32", "bf16"])
def test_outer_into_strided_view(T, d):
    """C a step-2 view of a larger buffer: the gaps keep their sentinel."""
    import torch
    g = synth.rng(3, 720)
    na, nb = (40, 6), (33,)
    A, B = synth.uniform(na, g), synth.uniform(nb, g)
    At, Bt = to_gpu(A, None, d), to_gpu(B, None, d)
    buf = torch.full((80, 6, 33), 7.0, dtype=torch_dtype(_acc(d)), device="cuda")
    C = buf[::2]
    T.ttt(At, Bt, 0, (1, 2), (1,), out=C)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), _expect(to_np(At), to_np(Bt), (1, 2), (1,), d))
    assert bool((buf[1::2] == 7.0).all())


@pytest.mark.parametrize("d", ["f32", "bf16", "f64"])
def test_outer_full_size_sampled(T, d):
    """A (512, 128) x B (64, 40) -> 167.8M outputs (670 MB FP32), the size the
    bench times: a seeded sub-grid of rows and columns against the oracle,
    bit for bit, and the rest checked to be finite (no output left unwritten)."""
    import torch
    g = synth.rng(3, 730)
    na, nb = (512, 128), (64, 40)
    A, B = synth.uniform(na, g), synth.uniform(nb, g)
    At, Bt = to_gpu(A, None, d), to_gpu(B, (2, 1), d)
    C = T.empty(na + nb, None, torch_dtype(_acc(d)), "cuda").fill_(float("nan"))
    assert "ttt outer" in T.plan(T.ttt, At, Bt, 0, (1, 2), (1, 2), out=C)
    T.ttt(At, Bt, 0, (1, 2), (1, 2), out=C)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(C).any())
    sel = [np.sort(g.choice(n, size=min(n, 9), replace=False)) for n in na + nb]
    Ah, Bh = to_np(At), to_np(Bt)
    Asub = Ah[np.ix_(sel[0], sel[1])]
    Bsub = Bh[np.ix_(sel[2], sel[3])]
    exp = _expect(Asub, Bsub, (1, 2), (1, 2), d)
    Ct = C
    for k, idx in enumerate(sel):
        Ct = Ct.index_select(k, torch.as_tensor(idx, device="cuda"))
    assert np.array_equal(to_np(Ct), exp)
    del C
    torch.cuda.empty_cache()


def test_outer_noalloc_entry_point(T):
    """tlib_ttt_noalloc takes the same outer kernel for q = 0."""
    import torch
    g = synth.rng(3, 740)
    A, B = synth.uniform((30, 7), g), synth.uniform((5, 8), g)
    At, Bt = to_gpu(A, None, "f32"), to_gpu(B, None, "f32")
    C = torch.full((30, 7, 5, 8), float("nan"), dtype=torch.float32, device="cuda")
    T.ttt_noalloc(At, Bt, 0, (1, 2), (1, 2), out=C)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(C), _expect(to_np(At), to_np(Bt), (1, 2), (1, 2), "f32"))
