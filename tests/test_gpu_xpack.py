"""GPU parity of TTT with the small operand packed first (Sec. 5.2 Eq. ttt,
ttt_indices).  When the large operand's contracted modes run along memory in
an order in which the small operand's do not (A last-order, B first-order;
or A first-order, B last-order), the planner copies the small operand into the
workspace as a matrix with its contracted index fastest, in the large
operand's order, and the GEMM then loads groups of consecutive k of it (and
K's modes merge wherever the large operand's do).  Every tiled pick (seven tiles, three
split targets) and every all-rows pick is forced through a one-entry kernel
table and compared with the oracle on the same rounded inputs (FP64 1e-12,
FP32 1e-5, 16-bit 1e-5); the plan must name the packing.  Cases: ragged free
extents, three contracted modes, and the small operand as a strided view."""
import numpy as np
import pytest

import oracle
import synth
from _util import TOL, TOL_KERNEL16, assert_close, round_to, to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu

GT_COUNT = 7
PICKS = list(range(3 * GT_COUNT)) + [3 * GT_COUNT + r for r in range(6)]


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


# (A extents, number of contracted modes q (A's last q), B's free extents, B a
# view padded along its last mode, A layout, B layout); A is at least 4 MB in
# every dtype, as packing requires
CASES = [((64, 64, 32, 16), 2, (5,), 0, "last", "first"),       # M = 5, K = 512
         ((67, 31, 48, 24), 2, (7,), 0, "last", "first"),       # ragged N = 2077, M = 7
         ((1024, 8, 24, 16), 3, (3,), 0, "last", "first"),      # three contracted modes, K = 3072
         ((64, 64, 32, 16), 2, (2, 3), 5, "last", "first"),     # B a strided view, two free B modes
         ((96, 64, 32, 16), 2, (6,), 0, "first", "last")]       # K merges after packing: A loads vectors along N


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32", "f64"])
def test_ttt_packed_small_operand(T, tmp_path, dtype):
    import torch
    g = synth.rng(76, ["bf16", "f16", "f32", "f64"].index(dtype))
    for na, q, fb, pad, la, lb in CASES:
        p = len(na)
        ka = na[p - q:]
        nb = ka + fb
        X, Y = synth.uniform(na, g), synth.uniform(nb, g)
        Ad = to_gpu(X, list(range(p, 0, -1)) if la == "last" else None, dtype)
        blay = list(range(len(nb), 0, -1)) if lb == "last" else None
        if pad:
            big = np.zeros(nb[:-1] + (nb[-1] + pad,))
            big[..., : nb[-1]] = Y
            Bd = to_gpu(big, blay, dtype)[..., : nb[-1]]
        else:
            Bd = to_gpu(Y, blay, dtype)
        phi = tuple(range(1, p + 1))
        psi = tuple(range(q + 1, len(nb) + 1)) + tuple(range(1, q + 1))
        ref = np.asarray(oracle.ttt(oracle.materialize(round_to(X, dtype)), oracle.materialize(round_to(Y, dtype)),
                                    q, phi, psi))
        acc = "f64" if dtype == "f64" else "f32"
        C = T.empty(na[: p - q] + fb, None, torch_dtype(acc), "cuda")
        tol = TOL_KERNEL16 if dtype in ("bf16", "f16") else TOL[dtype]
        prev = T.set_autotune("frozen")
        try:
            ran = 0
            for pick in PICKS:
                _force(T, tmp_path, Ad, Bd, C, q, phi, psi, pick)
                plan = T.plan(T.ttt, Ad, Bd, q, phi, psi, out=C)
                if "autotuned" not in plan:
                    continue  # pick not applicable to this shape: the rule ran instead
                assert "xpack" in plan, plan
                C.fill_(float("nan"))
                T.ttt(Ad, Bd, q, phi, psi, out=C)
                torch.cuda.synchronize()
                assert_close(to_np(C), ref, tol, "%s %s pick %d %s" % (dtype, na, pick, plan))
                ran += 1
            assert ran >= GT_COUNT, (na, ran)
        finally:
            T.autotune_clear()
            T.set_autotune(prev)
