"""GPU parity of the all-rows GEMM (every row of a small M in one tile, the
large operand streamed straight into the MFMAs) for TTT (Sec. 5.2 Eq. ttt,
ttt_indices), against the oracle on the same rounded inputs (FP64 1e-12,
FP32 1e-5, 16-bit with FP32 accumulation 1e-5).  Every case asserts from its
plan that the kernel ran, with the expected number of row blocks; the kernel
variant and split target are forced through a one-entry kernel table.  The
cases cover M from 7 to 120 (1 to 8 row blocks, ragged), ragged N, K of
several chunks with and without a split, and A as a strided view."""
import numpy as np
import pytest

import oracle
import synth
from _util import TOL, TOL_KERNEL16, assert_close, round_to, to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu

ROWS0 = 21  # first all-rows pick: 3 x 7 tiled-GEMM picks before it


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _ten_key(t):
    from paper_1711_10912_amd import _lib
    code = {"torch.float64": _lib.F64, "torch.float32": _lib.F32, "torch.bfloat16": _lib.BF16,
            "torch.float16": _lib.F16}[str(t.dtype)]
    return "|%d:%d" % (code, t.dim()) + "".join(",%d/%d" % (n, w) for n, w in zip(t.shape, t.stride()))


def _force(T, tmp_path, A, B, C, q, phi, psi, pick):
    key = "ttt|%d" % q + "".join("|%d" % v for v in phi) + "".join("|%d" % v for v in psi)
    key += _ten_key(A) + _ten_key(B) + _ten_key(C)
    f = tmp_path / "pick.txt"
    f.write_text("%d %s\n" % (pick, key))
    T.autotune_clear()
    T.autotune_load(str(f))


# (free A extents, contracted extents, free B extents, A a view with the first mode padded)
CASES = [((96, 80), (64, 48), (120,), 0),     # the (96,80,64,48) x (64,48,120) shape class, M = 120
         ((50, 7), (24, 40), (7,), 0),        # M = 7: one row block, ragged N
         ((300,), (16, 8), (33,), 0),         # M = 33: three row blocks, K of two chunks
         ((130,), (8, 8, 8), (2, 31), 64)]    # M = 62, three contracted pairs, A a strided view


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32", "f64"])
@pytest.mark.parametrize("r", range(6), ids=["fn1-s1024", "fn2-s1024", "fn1-s512", "fn2-s512", "fn1-s256",
                                            "fn2-s256"])
def test_ttt_rows_kernel(T, tmp_path, dtype, r):
    import torch
    g = synth.rng(74, r * 4 + ["bf16", "f16", "f32", "f64"].index(dtype))
    for fa, ka, fb, pad in CASES:
        q, ra, sb = len(ka), len(fa), len(fb)
        na, nb = fa + ka, ka + fb
        # A's contracted modes are its fastest (unit-stride K for the 16-bit loads);
        # B stored with its contracted modes first
        lay_a = list(range(ra + 1, ra + q + 1)) + list(range(1, ra + 1))
        phi = tuple(range(1, ra + q + 1))
        psi = tuple(range(q + 1, q + sb + 1)) + tuple(range(1, q + 1))
        X, Y = synth.uniform(na, g), synth.uniform(nb, g)
        if pad:
            big = np.zeros(na[:-1] + (na[-1] + pad,))
            big[..., : na[-1]] = X
            Ad = to_gpu(big, lay_a, dtype)[..., : na[-1]]
        else:
            Ad = to_gpu(X, lay_a, dtype)
        Bd = to_gpu(Y, None, dtype)
        ref = np.asarray(oracle.ttt(oracle.materialize(round_to(X, dtype)), oracle.materialize(round_to(Y, dtype)),
                                    q, phi, psi))
        acc = "f64" if dtype == "f64" else "f32"
        C = T.empty(fa + fb, None, torch_dtype(acc), "cuda")
        prev = T.set_autotune("frozen")
        try:
            _force(T, tmp_path, Ad, Bd, C, q, phi, psi, ROWS0 + r)
            plan = T.plan(T.ttt, Ad, Bd, q, phi, psi, out=C)
            C.fill_(float("nan"))
            T.ttt(Ad, Bd, q, phi, psi, out=C)
        finally:
            T.autotune_clear()
            T.set_autotune(prev)
        M = int(np.prod(fb))
        fm = 1
        while 16 * fm < M:
            fm *= 2
        assert "gemm-rows" in plan and "fm=%d fn=%d" % (fm, 1 + r % 2) in plan, plan
        tol = TOL_KERNEL16 if dtype in ("bf16", "f16") else TOL[dtype]
        assert_close(to_np(C), ref, tol, "%s %s %s" % (plan, dtype, na))
