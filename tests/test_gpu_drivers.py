"""GPU parity of the composite drivers (HOPM, Tucker chain), of the fused
conversion in scale, against the oracle's drivers on the same inputs."""
import math
import zlib

import numpy as np
import pytest

import oracle
import synth
from _util import TOL, assert_close, assert_close16, correctly_rounded, round_to, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _start(shape, dtype):
    return [to_gpu(np.full(n, 1.0 / math.sqrt(n)), None, dtype) for n in shape]


def test_hopm_rank_one_f64(T):
    g = synth.rng(30, 0)
    fac = [synth.orthonormal_columns(n, 1, g)[:, 0] for n in (9, 7, 11, 5)]
    X = 3.25 * np.einsum("i,j,k,l->ijkl", *fac)
    A = to_gpu(X, [2, 4, 1, 3], "f64")
    lam, us = T.hopm(A, _start(X.shape, "f64"), 2)
    assert abs(lam[-1] - 3.25) < 1e-12 * 3.25
    for k in range(4):
        assert abs(abs(float(np.dot(to_np(us[k]), fac[k]))) - 1.0) < 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hopm_vs_oracle_low_rank(T, dtype):
    A0, Us, F, sig = synth.tucker_case(n=24, rank=4, rows=8, sigma0=1e3, noise=1.0, g=synth.rng(30, 1))
    Ar = round_to(A0, dtype)
    A = to_gpu(A0, None, dtype)
    lam, us = T.hopm(A, _start(A0.shape, dtype), 5)
    lam_o, us_o = oracle.hopm(oracle.materialize(Ar), [np.full(n, 1.0 / math.sqrt(n)) for n in A0.shape], 5)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for r in range(4):
        assert abs(lam[r] - lam_o[r]) <= tol * abs(lam_o[r]), (r, lam[r], lam_o[r])
        assert_close(to_np(us[r]), us_o[r], tol, "hopm u_%d" % (r + 1))
    # HOPM converges to one of the orthogonal rank-one components (which one
    # depends on the start vectors); noise / sigma ~ 1e-3
    assert min(abs(lam[-1] - s) for s in sig) < 1e-2 * sig[0]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tucker_vs_oracle(T, dtype):
    A0, Us, F, sig = synth.tucker_case(n=40, rank=4, rows=8, sigma0=1e3, noise=1.0, g=synth.rng(31, 0))
    Ar = round_to(A0, dtype)
    A = to_gpu(A0, [4, 3, 2, 1], dtype)
    Ud = [to_gpu(U, None, dtype) for U in Us]
    core = T.tucker(A, Ud)
    ref = oracle.tucker(oracle.materialize(Ar), [round_to(U, dtype) for U in Us])
    assert_close(to_np(core), ref, 1e-12 if dtype == "f64" else 1e-5, "tucker %s" % dtype)
    # orthonormal factor rows: the core cannot be larger than the tensor
    assert np.linalg.norm(to_np(core)) <= np.linalg.norm(Ar) * (1 + 1e-6)


def test_tucker_bf16_staged(T):
    import torch
    A0, Us, F, sig = synth.tucker_case(n=40, rank=4, rows=8, sigma0=1e3, noise=1.0, g=synth.rng(31, 1))
    A = to_gpu(A0, None, "bf16")
    Ud = [to_gpu(U, None, "bf16") for U in Us]
    core = T.tucker(A, Ud, stage_dtype=torch.bfloat16)
    # the same chain in the oracle on the same rounded values, rounding every
    # intermediate to bf16 as the device does
    X = oracle.materialize(round_to(A0, "bf16"))
    for k, U in enumerate(Us, start=1):
        if k > 1:
            X = oracle.materialize(correctly_rounded(np.asarray(X), "bf16"))
        X = oracle.ttm(X, round_to(U, "bf16"), k)
    assert_close(to_np(core), np.asarray(X), 1e-5, "tucker bf16 (kernel)")
    # end to end against the FP64 chain on the unrounded values: 2e-2 normwise
    exact = oracle.tucker(oracle.materialize(A0), Us)
    absref = oracle.tucker(oracle.materialize(np.abs(A0)), [np.abs(U) for U in Us])
    assert_close16(to_np(core), exact, absref, TOL["bf16"], "tucker bf16 staged")


@pytest.mark.parametrize("src,dst", [("f32", "bf16"), ("f32", "f16"), ("f64", "f32"), ("bf16", "f32"),
                                     ("f64", "bf16")])
def test_scale_converts_with_one_rounding(T, src, dst):
    import torch
    from _util import torch_dtype
    g = synth.rng(32, 0)
    X = synth.normal((37, 29, 5), g, 3.0)
    A = to_gpu(X, [3, 1, 2], src)
    C = T.scale(1.5, A, layout=[1, 2, 3], dtype=torch_dtype(dst))
    want = correctly_rounded(1.5 * round_to(X, src), dst)
    assert np.array_equal(to_np(C), want)


@pytest.mark.parametrize("din,dout", [("f64", "f64"), ("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"),
                                      ("f16", "f32")])
def test_normalize_vs_oracle(T, din, dout):
    """tlib_normalize (the HOPM normalisation, Sec. 5.2): the FP64 norm
    against the oracle's Neumaier-summed inner product, and every quotient
    equal to the FP64 quotient by that norm rounded once to C's dtype, for a
    vector, a strided vector, a 3-way tensor in another layout and in place."""
    import torch
    from _util import correctly_rounded, round_to, torch_dtype
    g = synth.rng(60, zlib.crc32((din + dout).encode()) % 1000)
    for shape, lay, step in [((160,), None, 1), ((300,), None, 3), ((7, 11, 13), [3, 1, 2], 1)]:
        X = synth.uniform(shape, g) * 10
        if step > 1:
            big = T.empty((shape[0] * step,), None, torch_dtype(din), "cuda")
            big.copy_(torch.from_numpy(np.repeat(X, step)).to(torch_dtype(din)).cuda())
            A = big[::step]
        else:
            A = to_gpu(X, lay, din)
        Xr = to_np(A)
        out = T.empty(shape, None, torch_dtype(dout), "cuda").fill_(float("nan"))
        _, nrm = T.normalize(A, out=out)
        torch.cuda.synchronize()
        nref = math.sqrt(oracle.inner(oracle.materialize(Xr), oracle.materialize(Xr)))
        n = float(nrm.item())
        assert abs(n - nref) <= 1e-13 * nref, (n, nref)
        assert np.array_equal(to_np(out), correctly_rounded(Xr / n, dout))
        if din == dout and step == 1:
            B = A.clone()
            T.normalize(B, out=B)
            torch.cuda.synchronize()
            assert np.array_equal(to_np(B), correctly_rounded(Xr / n, dout))
