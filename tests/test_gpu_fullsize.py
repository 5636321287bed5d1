"""Parity at the benchmark's full sizes, in the same launch configuration the
benchmark times: the order-p sweep (406^3, 90^4, 36^5, 20^6, 13^7; TTV and
TTM with m = 16, 64, 256 in every mode, outputs in the benchmark's layouts)
and the (96,80,64,48) x (64,48,120) TTT, with the shipped kernel table loaded
as the benchmark loads it, so every TTM/TTT call runs the kernel and tile the
benchmark times.

Complete comparisons: every TTV output and every TTM (m = 16) output of the
sweep, for every p, mode, layout and both dtypes, written into outputs
filled with NaN beforehand (an output the kernel skips fails), and every
output of the full TTT in FP32, BF16 and FP16 for the N(0,1) case and its
x1e3 variant.  Sampled comparisons: TTM with m = 64 and 256, where the oracle
computes sampled output fibers one by one, each from a view of the inputs
that keeps a single index in every free mode.  Tolerances: 1e-12 FP64, 1e-5
FP32 and 16-bit kernel-only (same rounded inputs), 2e-2 normwise end to end
for 16-bit inputs."""
import functools
import os

import numpy as np
import pytest

import oracle
import synth
from _util import TOL, assert_close, assert_close16, round_to, to_gpu, to_np

pytestmark = pytest.mark.gpu

SAMPLES = 48


TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1711_10912_amd", "tuning",
                     "mi355x_sweep.txt")


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    prev = T.set_autotune("frozen")
    T.autotune_clear()
    T.autotune_load(TABLE)
    yield T
    T.autotune_clear()
    T.set_autotune(prev)


def _one(X, idx, keep):
    """View of X with a single index in every mode except those in `keep`."""
    sl = tuple(slice(None) if r in keep else slice(i, i + 1) for r, i in enumerate(idx))
    return X[sl]


def _nan_out(T, shape, layout, dtype):
    import torch
    C = T.empty(shape, layout, torch.float64 if dtype == "f64" else torch.float32, "cuda")
    C.fill_(float("nan"))
    return C


@functools.lru_cache(maxsize=2)
def _sweep_rounded(p, dtype):
    return round_to(synth.sweep_tensor(p), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("p", [3, 4, 5, 6, 7])
def test_sweep_ttv_ttm16_complete(T, p, dtype):
    """Every output of TTV and of TTM with m = 16, every mode, both layouts."""
    print("fullsize complete p=%d %s" % (p, dtype), flush=True)
    X = synth.sweep_tensor(p)
    n = X.shape[0]
    Xr = _sweep_rounded(p, dtype)
    Xo = oracle.materialize(Xr)
    tol = TOL[dtype]
    b, B = synth.sweep_operands(n, 16)
    br, Br = round_to(b, dtype), round_to(B, dtype)
    bd, Bd = to_gpu(b, None, dtype), to_gpu(B, [2, 1], dtype)
    ref_v = {q: np.asarray(oracle.ttv(Xo, br, q)) for q in range(1, p + 1)}
    ref_m = {}
    for lname, lay in (("first", list(range(1, p + 1))), ("last", list(range(p, 0, -1)))):
        A = to_gpu(X, lay, dtype)
        for q in range(1, p + 1):
            clay = [r if r < q else r - 1 for r in lay if r != q]
            Cv = _nan_out(T, (n,) * (p - 1), clay, dtype)
            plan = T.plan(T.ttv, A, bd, q, out=Cv)
            T.ttv(A, bd, q, out=Cv)
            assert_close(to_np(Cv), ref_v[q], tol, "ttv p=%d %s q=%d %s (%s)" % (p, lname, q, dtype, plan))
            del Cv
            if q not in ref_m:
                ref_m[q] = np.asarray(oracle.ttm(Xo, Br, q))
            shape = [n] * p
            shape[q - 1] = 16
            Cm = _nan_out(T, shape, lay, dtype)
            plan = T.plan(T.ttm, A, Bd, q, out=Cm)
            assert "autotuned" in plan, plan
            T.ttm(A, Bd, q, out=Cm)
            assert_close(to_np(Cm), ref_m[q], tol, "ttm p=%d %s q=%d m=16 %s (%s)" % (p, lname, q, dtype, plan))
            del Cm
        del A


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7])
def test_sweep_ttm_sampled(T, p):
    """TTM with m = 64 and 256: sampled output fibers."""
    print("fullsize sweep p=%d" % p, flush=True)
    X = synth.sweep_tensor(p)
    n = X.shape[0]
    g = synth.rng(40, p)
    for dtype in ("f64", "f32"):
        Xr = round_to(X, dtype)
        tol = 1e-12 if dtype == "f64" else 1e-5
        for lname, lay in (("first", list(range(1, p + 1))), ("last", list(range(p, 0, -1)))):
            A = to_gpu(X, lay, dtype)
            for q in range(1, p + 1):
                for m in (64, 256):
                    _, B = synth.sweep_operands(n, m)
                    Br = round_to(B, dtype)
                    Bd = to_gpu(B, [2, 1], dtype)  # row-major, as the benchmark allocates it
                    Cm = T.ttm(A, Bd, q)
                    plan = T.plan(T.ttm, A, Bd, q, out=Cm)
                    assert "autotuned" in plan, plan
                    got_m, ref_m = [], []
                    for _ in range(SAMPLES // 2):
                        idx = [int(v) for v in g.integers(0, n, p)]
                        view = oracle.materialize(_one(Xr, idx, {q - 1}))
                        ref_m.append(np.asarray(oracle.ttm(view, Br, q)).reshape(-1))
                        sl = tuple(slice(None) if r == q - 1 else i for r, i in enumerate(idx))
                        got_m.append(to_np(Cm[sl]))
                    assert_close(np.array(got_m), np.array(ref_m), tol,
                                 "ttm p=%d %s q=%d m=%d %s (%s)" % (p, lname, q, m, dtype, plan))
                    del Cm
            del A


@functools.lru_cache(maxsize=8)
def _ttt_ref(scale, dtype):
    """Oracle on the inputs rounded to dtype ('orig': unrounded, 'abs': the
    contraction over absolute values)."""
    X, Y = synth.ttt_case(scale=scale)
    if dtype == "abs":
        X, Y = np.abs(X), np.abs(Y)
    elif dtype != "orig":
        X, Y = round_to(X, dtype), round_to(Y, dtype)
    return np.asarray(oracle.ttt(oracle.materialize(X), oracle.materialize(Y), 2, synth.TTT_PHI, synth.TTT_PSI))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("scale", [1.0, 1e3], ids=["n01", "x1e3"])
def test_ttt_fullsize_complete(T, scale, dtype):
    """Every output of the full TTT in the three A layouts, into NaN-filled C."""
    print("fullsize ttt scale=%g %s" % (scale, dtype), flush=True)
    X, Y = synth.ttt_case(scale=scale)
    ref = _ttt_ref(scale, dtype)
    Bd = to_gpu(Y, None, dtype)
    for alay in ("first", "last", "perm3142"):
        Ad = to_gpu(X, synth.TTT_A_LAYOUTS[alay], dtype)
        C = _nan_out(T, (96, 80, 120), None, dtype)
        plan = T.plan(T.ttt, Ad, Bd, 2, synth.TTT_PHI, synth.TTT_PSI, out=C)
        T.ttt(Ad, Bd, 2, synth.TTT_PHI, synth.TTT_PSI, out=C)
        got = to_np(C)
        what = "ttt full size scale=%g A=%s %s (%s)" % (scale, alay, dtype, plan)
        assert_close(got, ref, TOL["f32"], what + " (kernel)")
        if dtype != "f32":
            assert_close16(got, _ttt_ref(scale, "orig"), _ttt_ref(scale, "abs"), TOL[dtype], what)
