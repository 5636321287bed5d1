"""Parity at the benchmark's full sizes, in the same launch configuration the
benchmark times: the order-p sweep (406^3, 90^4, 36^5, 20^6, 13^7; TTV and
TTM with m = 16, 64, 256 in every mode, outputs in the benchmark's layouts)
and the (96,80,64,48) x (64,48,120) TTT, with the shipped kernel table loaded
as the benchmark loads it, so every TTM/TTT call runs the kernel and tile the
benchmark times.  The oracle computes sampled outputs one by one, each from a
view of the inputs that keeps a single index in every free mode.  The
tolerance (1e-12 FP64, 1e-5 FP32) is applied to the sampled set."""
import os

import numpy as np
import pytest

import oracle
import synth
from _util import assert_close, round_to, to_gpu, to_np

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


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7])
def test_sweep_ttv_ttm_sampled(T, p):
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
                b, _ = synth.sweep_operands(n, 16)
                br = round_to(b, dtype)
                Cv = to_np(T.ttv(A, to_gpu(b, None, dtype), q))
                got_v, ref_v = [], []
                for _ in range(SAMPLES):
                    idx = [int(v) for v in g.integers(0, n, p)]
                    view = oracle.materialize(_one(Xr, idx, {q - 1}))
                    ref_v.append(float(np.asarray(oracle.ttv(view, br, q)).reshape(-1)[0]))
                    got_v.append(Cv[tuple(i for r, i in enumerate(idx) if r != q - 1)])
                assert_close(np.array(got_v), np.array(ref_v), tol, "ttv p=%d %s q=%d %s" % (p, lname, q, dtype))
                for m in (16, 64, 256):
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


@pytest.mark.parametrize("alay", ["first", "last", "perm3142"])
def test_ttt_fullsize_sampled(T, alay):
    X, Y = synth.ttt_case()
    g = synth.rng(41, 0)
    for dtype in ("f32", "bf16"):
        Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
        C = to_np(T.ttt(to_gpu(X, synth.TTT_A_LAYOUTS[alay], dtype), to_gpu(Y, None, dtype), 2,
                        synth.TTT_PHI, synth.TTT_PSI))
        got, ref = [], []
        for _ in range(SAMPLES):
            i1, i2, j = int(g.integers(96)), int(g.integers(80)), int(g.integers(120))
            a = oracle.materialize(Xr[i1:i1 + 1, i2:i2 + 1, :, :])
            bb = oracle.materialize(Yr[:, :, j:j + 1])
            ref.append(float(np.asarray(oracle.ttt(a, bb, 2, synth.TTT_PHI, synth.TTT_PSI)).reshape(-1)[0]))
            got.append(C[i1, i2, j])
        assert_close(np.array(got), np.array(ref), 1e-5, "ttt full size A=%s %s (kernel)" % (alay, dtype))
