"""GPU parity of every TTM kernel regime (Sec. 5.2 Eq. ttm) and of the
autotuned kernel choice, against the FP64 oracle.

The planner sends a TTM to one of: the streaming kernel for C contiguous
along j, the row-streaming kernel (band, band1, aligned or plain windows) for
C strided along j, or the tiled GEMM.  Each case below asserts which regime
its plan names, so that every regime stays covered as the rules change, and
covers ragged row counts (m not a multiple of 16), runs shorter and longer
than one window, and a strided output view."""
import zlib

import numpy as np
import pytest

import oracle
import synth
from _util import TOL, assert_close, round_to, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


# (shape, layout, mode, m, expected plan fragment)
REGIMES = [
    ((13, 13, 13, 13), [1, 2, 3, 4], 2, 64, "mode=band1"),       # n_lo = 13
    ((13, 13, 13, 13), [1, 2, 3, 4], 2, 7, "mode=band1"),        # m < 16
    ((20, 20, 20), [1, 2, 3], 2, 256, "mode=band "),             # n_lo = 20, two blocks
    ((29, 11, 9), [1, 2, 3], 2, 17, "mode=band "),               # n_lo = 29, ragged m
    ((200, 13, 5), [1, 2, 3], 2, 100, "mode=aligned"),           # n_lo = 200: four windows
    ((169, 13, 5), [1, 2, 3], 2, 100, "mode=bandw"),             # n_lo = 169, rows adjacent in C
    ((130, 16, 7), [1, 2, 3], 2, 33, "mode=bandw"),              # k = 16: deepest band-wide depth
    ((5, 13, 176), [3, 2, 1], 2, 40, "mode=bandw"),              # last-order, n_lo = 176
    ((7, 5, 190), [3, 2, 1], 2, 33, "mode=aligned"),             # last-order: n_lo = 190
    ((70, 40, 9), [1, 2, 3], 2, 64, "mode=plain"),               # k = 40: no aligned depth
    ((24, 9, 11), [1, 2, 3], 1, 256, "ttm stream"),              # C contiguous along j
    ((5, 9, 11), [3, 2, 1], 3, 16, "ttm stream"),                # last-order, mode p
    ((36, 9, 11), [1, 2, 3], 1, 256, "ttm stream"),              # B in LDS: 83 KB for FP64
    ((60, 7, 9), [1, 2, 3], 1, 200, "ttm stream"),               # 133 KB for FP64, ragged m
    ((33, 29, 6), [1, 2, 3], 2, 300, "ttm gemm"),                # m > 256
    ((30, 200, 4), [1, 2, 3], 2, 64, "ttm gemm"),                # k = 200 > 64
]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", REGIMES, ids=lambda c: "%s-q%d-m%d" % ("x".join(map(str, c[0])), c[2], c[3]))
def test_ttm_regime(T, dtype, case):
    import torch
    shape, lay, q, m, expect = case
    g = synth.rng(21, zlib.crc32(repr((shape, q, m)).encode()) % 997)
    X = synth.uniform(shape, g)
    B = synth.uniform((m, shape[q - 1]), g)
    Ad = to_gpu(X, lay, dtype)
    Bd = to_gpu(B, None, dtype)
    sc = list(shape)
    sc[q - 1] = m
    C = T.empty(sc, lay, T.acc_dtype(Ad.dtype), Ad.device)
    plan = T.plan(T.ttm, Ad, Bd, q, out=C)
    # 16-bit inputs reach deeper k in the row kernel's aligned mode: check the
    # family only
    want = expect if dtype != "bf16" else ("ttm rows" if "mode=" in expect else expect)
    assert want in plan + " ", plan
    C.fill_(float("nan"))
    T.ttm(Ad, Bd, q, out=C)
    torch.cuda.synchronize()
    ref = oracle.ttm(oracle.materialize(round_to(X, dtype)), round_to(B, dtype), q)
    tol = 1e-5 if dtype == "bf16" else TOL[dtype]
    assert_close(to_np(C), ref, tol, "%s %s" % (plan, dtype))


def test_ttm_strided_output_view(T):
    """C is a step-2 view of a larger buffer: C's innermost column stride is
    2, so the row kernel writes unshifted windows (plain)."""
    import torch
    g = synth.rng(22, 0)
    shape, q, m = (37, 20, 6), 2, 48
    X = synth.uniform(shape, g)
    B = synth.uniform((m, shape[q - 1]), g)
    Ad = to_gpu(X, None, "f64")
    Bd = to_gpu(B, None, "f64")
    big = T.empty((2 * 37, m, 6), None, torch.float64, Ad.device).fill_(float("nan"))
    C = big[::2]
    plan = T.plan(T.ttm, Ad, Bd, q, out=C)
    assert "mode=plain" in plan, plan
    T.ttm(Ad, Bd, q, out=C)
    ref = oracle.ttm(oracle.materialize(X), B, q)
    assert_close(to_np(C), ref, TOL["f64"], plan)
    assert torch.isnan(big[1::2]).all(), "the kernel wrote outside the view"


def test_autotune_ttm_ttt(T):
    """With autotuning on, the first call of each shape times the candidates
    and keeps one; results match the oracle, later (frozen) calls reuse the
    stored choice and reproduce the tuned call's result bit for bit."""
    import torch
    T.autotune_clear()
    prev = T.set_autotune("on")
    try:
        g = synth.rng(23, 0)
        cases = [((13, 13, 13, 13), [1, 2, 3, 4], 3, 64, "f64"), ((20, 20, 20), [3, 2, 1], 2, 16, "f32"),
                 ((40, 9, 11), [1, 2, 3], 1, 256, "f64"), ((30, 200, 4), [1, 2, 3], 2, 64, "f32")]
        outs = []
        for shape, lay, q, m, dt in cases:
            X = synth.uniform(shape, g)
            B = synth.uniform((m, shape[q - 1]), g)
            Ad, Bd = to_gpu(X, lay, dt), to_gpu(B, None, dt)
            C = T.ttm(Ad, Bd, q)
            torch.cuda.synchronize()
            ref = oracle.ttm(oracle.materialize(round_to(X, dt)), round_to(B, dt), q)
            assert_close(to_np(C), ref, TOL[dt], "autotuned ttm %s" % (shape,))
            outs.append((Ad, Bd, q, to_np(C)))
        A3, B3 = synth.ttt_case(shrink=4)
        Ad3, Bd3 = to_gpu(A3, [3, 1, 4, 2], "f32"), to_gpu(B3, None, "f32")
        C3 = T.ttt(Ad3, Bd3, 2, synth.TTT_PHI, synth.TTT_PSI)
        torch.cuda.synchronize()
        ref3 = oracle.ttt(oracle.materialize(round_to(A3, "f32")), oracle.materialize(round_to(B3, "f32")), 2,
                          synth.TTT_PHI, synth.TTT_PSI)
        assert_close(to_np(C3), ref3, TOL["f32"], "autotuned ttt")
        # one entry per tuned call shape, plus one per shape class (these five
        # calls fall in five classes)
        assert T.autotune_entries() == 2 * (len(cases) + 1)
        T.set_autotune("frozen")
        for Ad, Bd, q, first in outs:
            again = T.ttm(Ad, Bd, q)
            assert "autotuned" in T.plan(T.ttm, Ad, Bd, q, out=again)
            assert np.array_equal(to_np(again), first)
        assert T.autotune_entries() == 2 * (len(cases) + 1)
        # a new shape of an already tuned class (13^4 -> 14^4, mode 3, m = 64):
        # frozen, it takes the class's choice; on, it is tuned for itself and
        # adds its own entry only
        X = synth.uniform((14, 14, 14, 14), g)
        B = synth.uniform((64, 14), g)
        Ad, Bd = to_gpu(X, [1, 2, 3, 4], "f64"), to_gpu(B, None, "f64")
        C = T.empty((14, 14, 64, 14), None, torch.float64, "cuda")
        assert "autotuned(class)" in T.plan(T.ttm, Ad, Bd, 3, out=C)
        T.set_autotune("on")
        T.ttm(Ad, Bd, 3, out=C)
        torch.cuda.synchronize()
        assert T.autotune_entries() == 2 * (len(cases) + 1) + 1
        ref = oracle.ttm(oracle.materialize(X), B, 3)
        assert_close(to_np(C), ref, TOL["f64"], "tuned within a known class")
    finally:
        T.set_autotune(prev)
        T.autotune_clear()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ttm_single_row_stays_inside_output(T, dtype):
    """m = 1: the stride of j is free, so the row kernel must drop the rows of
    its 16-row blocks past the first by predicate; C sits at the start of a
    larger buffer whose tail must stay untouched."""
    import torch
    g = synth.rng(24, 0)
    shape, q = (33, 29, 17), 1
    X = synth.uniform(shape, g)
    B = synth.uniform((1, shape[0]), g)
    Ad, Bd = to_gpu(X, None, dtype), to_gpu(B, None, dtype)
    n = 29 * 17
    big = torch.full((n + 4096,), float("nan"), dtype=T.acc_dtype(Ad.dtype), device="cuda")
    C = torch.as_strided(big, (1, 29, 17), (1, 1, 29))
    plan = T.plan(T.ttm, Ad, Bd, q, out=C)
    assert "ttm rows" in plan, plan
    T.ttm(Ad, Bd, q, out=C)
    torch.cuda.synchronize()
    ref = oracle.ttm(oracle.materialize(round_to(X, dtype)), round_to(B, dtype), q)
    assert_close(to_np(C), ref, TOL[dtype], plan)
    assert torch.isnan(big[n:]).all(), "the kernel wrote past the output"


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m", [256, 200])
def test_ttm_row_groups(T, dtype, m):
    """k = 36 with m = 200..256: B's slice does not fit in one workgroup's
    LDS, so the row kernel splits the rows of B and C into groups served by
    different workgroups (ragged last group for m = 200)."""
    import torch
    g = synth.rng(25, m)
    shape, q = (37, 36, 11), 2
    X = synth.uniform(shape, g)
    B = synth.uniform((m, shape[q - 1]), g)
    Ad, Bd = to_gpu(X, None, dtype), to_gpu(B, None, dtype)
    sc = list(shape)
    sc[q - 1] = m
    C = T.empty(sc, None, T.acc_dtype(Ad.dtype), Ad.device)
    plan = T.plan(T.ttm, Ad, Bd, q, out=C)
    assert "ttm rows" in plan, plan
    if dtype == "f64":
        assert "rowgroups=1x" not in plan, plan
    C.fill_(float("nan"))
    T.ttm(Ad, Bd, q, out=C)
    torch.cuda.synchronize()
    ref = oracle.ttm(oracle.materialize(round_to(X, dtype)), round_to(B, dtype), q)
    assert_close(to_np(C), ref, TOL[dtype], plan)
