"""GPU parity: every entry point of the C ABI (through the thin binding)
against the FP64 oracle on the same seeded inputs.

Bars: FP64 1e-12, FP32 1e-5 normwise relative error; 16-bit inputs with FP32
accumulation 2e-2 normwise against the oracle on the original (unrounded)
values and 1e-5 against the oracle on the rounded inputs; integer-valued inputs
must match bit for bit (every partial sum is exact)."""
import itertools
import zlib

import numpy as np
import pytest

import oracle
import synth
from _util import TOL, TOL_KERNEL16, assert_close, assert_close16, correctly_rounded, rel_err, round_to, to_gpu, to_np

pytestmark = pytest.mark.gpu

DTYPES = ["f64", "f32", "bf16", "f16"]


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _layouts(p, g):
    outs = [list(range(1, p + 1)), list(range(p, 0, -1))]
    if p >= 3:
        outs.append(synth.random_layout(p, g))
    return outs


def _seed(*key):
    return zlib.crc32(repr(key).encode()) % 1000


def _check(got_t, ref_fn, X_inputs_rounded, X_inputs_orig, dtype, what):
    """ref_fn(*inputs) -> oracle result (numpy array).

    16-bit inputs: the kernel is held to 1e-5 against the oracle on the same
    rounded inputs, and end to end to 2e-2 normwise against the oracle on the
    unrounded inputs (relative to the contraction over absolute values only
    for a result that cancels by more than a factor 100, see assert_close16)."""
    got = to_np(got_t)
    ref = np.asarray(ref_fn(*X_inputs_rounded))
    if dtype in ("bf16", "f16"):
        assert_close(got, ref, TOL_KERNEL16, what + " (kernel)")
        ref0 = np.asarray(ref_fn(*X_inputs_orig))
        absref = np.asarray(ref_fn(*[np.abs(x) for x in X_inputs_orig]))
        assert_close16(got, ref0, absref, TOL[dtype], what)
    else:
        assert_close(got, ref, TOL[dtype], what)


# ------------------------------------------------------------------ config 1

def test_tiny_config_ttv_ttm_f64(T):
    A, b, B = synth.tiny_case()
    Ad, bd, Bd = to_gpu(A, None, "f64"), to_gpu(b, None, "f64"), to_gpu(B, None, "f64")
    Cv = T.ttv(Ad, bd, 2)
    assert_close(to_np(Cv), oracle.ttv(oracle.materialize(A), b, 2), 1e-12, "ttv 32^3 mode 2")
    Cm = T.ttm(Ad, Bd, 2)
    assert_close(to_np(Cm), oracle.ttm(oracle.materialize(A), B, 2), 1e-12, "ttm 32^3 mode 2")


# ------------------------------------------------------------------ TTV

TTV_SHAPES = [(37, 29), (70, 3, 41), (5, 67, 9), (13, 11, 9, 7), (3, 5, 2, 4, 6), (33, 1, 40), (1, 50)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", TTV_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_ttv_all_modes_layouts(T, dtype, shape):
    g = synth.rng(10, _seed(dtype, shape))
    X = synth.uniform(shape, g)
    Xr = round_to(X, dtype)
    p = len(shape)
    for lay in _layouts(p, g):
        Ad = to_gpu(X, lay, dtype)
        for m in range(1, p + 1):
            b = synth.uniform((shape[m - 1],), g)
            bd = to_gpu(b, None, dtype)
            br = round_to(b, dtype)
            for out_lay in (None, "first"):
                if out_lay is None:
                    C = T.ttv(Ad, bd, m)  # A's layout minus mode m
                else:
                    C = T.ttv(Ad, bd, m, layout=list(range(1, p)))
                _check(C, lambda Xa, bv: oracle.ttv(oracle.materialize(Xa), bv, m), (Xr, br), (X, b),
                       dtype, "ttv %s %s lay=%s m=%d out=%s" % (dtype, shape, lay, m, out_lay))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_ttv_integer_exact(T, dtype):
    g = synth.rng(11, 0)
    for shape in [(40, 33, 5), (7, 300), (9, 8, 7, 6)]:
        X = synth.integers(shape, g)
        for lay in _layouts(len(shape), g):
            Ad = to_gpu(X, lay, dtype)
            for m in range(1, len(shape) + 1):
                b = synth.integers((shape[m - 1],), g)
                C = T.ttv(Ad, to_gpu(b, None, dtype), m)
                ref = oracle.ttv(oracle.materialize(X), b, m)
                assert np.array_equal(to_np(C), np.asarray(ref)), (shape, lay, m)


def test_ttv_views_and_strided_vector(T):
    import torch
    g = synth.rng(12, 0)
    X = synth.uniform((20, 18, 16), g)
    Ad = to_gpu(X, [2, 3, 1], "f64")
    V = Ad[1:19:3, 2:17:2, 5:6]                  # a view with steps (Sec. 3.3)
    Xv = X[1:19:3, 2:17:2, 5:6]
    bbig = torch.from_numpy(synth.uniform((40,), g)).cuda()
    for m in (1, 2, 3):
        b = bbig[: 2 * V.shape[m - 1]: 2]       # strided vector
        C = T.ttv(V, b, m)
        ref = oracle.ttv(oracle.materialize(Xv), to_np(b), m)
        assert_close(to_np(C), ref, 1e-12, "view ttv m=%d" % m)


# ------------------------------------------------------------------ TTM

TTM_CASES = [((33, 29, 17), (1, 5, 16, 17, 64)), ((13, 11, 9, 7), (16, 64, 100)), ((70, 41), (256, 3)),
             ((5, 3, 4, 6, 2), (7,))]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("case", TTM_CASES, ids=lambda c: "x".join(map(str, c[0])))
def test_ttm_all_modes_layouts(T, dtype, case):
    shape, ms = case
    g = synth.rng(13, _seed(dtype, shape))
    X = synth.uniform(shape, g)
    Xr = round_to(X, dtype)
    p = len(shape)
    for lay in _layouts(p, g):
        Ad = to_gpu(X, lay, dtype)
        for m in range(1, p + 1):
            for mm in ms:
                B = synth.uniform((mm, shape[m - 1]), g)
                blay = [2, 1] if mm % 2 else None
                Bd = to_gpu(B, blay, dtype)
                C = T.ttm(Ad, Bd, m)
                _check(C, lambda Xa, Ba: oracle.ttm(oracle.materialize(Xa), Ba, m), (Xr, round_to(B, dtype)),
                       (X, B), dtype, "ttm %s %s lay=%s m=%d n'=%d" % (dtype, shape, lay, m, mm))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_ttm_integer_exact(T, dtype):
    g = synth.rng(14, 0)
    for shape, mm in [((40, 33, 5), 16), ((7, 300), 64), ((9, 8, 7, 6), 20)]:
        X = synth.integers(shape, g)
        for lay in _layouts(len(shape), g):
            Ad = to_gpu(X, lay, dtype)
            for m in range(1, len(shape) + 1):
                B = synth.integers((mm, shape[m - 1]), g)
                C = T.ttm(Ad, to_gpu(B, None, dtype), m)
                ref = oracle.ttm(oracle.materialize(X), B, m)
                assert np.array_equal(to_np(C), np.asarray(ref)), (shape, lay, m)


# ------------------------------------------------------------------ TTT

@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "f64"])
@pytest.mark.parametrize("alay", ["first", "last", "perm3142"])
@pytest.mark.parametrize("scale", [1.0, 1e3], ids=["n01", "x1e3"])
def test_ttt_config3_shrunk(T, dtype, alay, scale):
    """The (96,80,64,48) x (64,48,120) contraction with every extent divided
    by 4, N(0,1) entries and the variant scaled by 1e3 (range: the FP32
    outputs of the scaled FP16 case reach ~1e7, beyond the FP16 range)."""
    X, Y = synth.ttt_case(scale=scale, shrink=4)
    Ad = to_gpu(X, synth.TTT_A_LAYOUTS[alay], dtype)
    Bd = to_gpu(Y, None, dtype)
    C = T.ttt(Ad, Bd, 2, synth.TTT_PHI, synth.TTT_PSI)
    f = lambda Xa, Ya: oracle.ttt(oracle.materialize(Xa), oracle.materialize(Ya), 2, synth.TTT_PHI, synth.TTT_PSI)
    _check(C, f, (round_to(X, dtype), round_to(Y, dtype)), (X, Y), dtype, "ttt %s A=%s scale=%g" % (dtype, alay, scale))


def _ttt_random(g, pa, pb, q):
    na = [int(v) for v in g.integers(1, 9, pa)]
    phi = [int(v) + 1 for v in g.permutation(pa)]
    psi = [int(v) + 1 for v in g.permutation(pb)]
    nb = [int(v) for v in g.integers(1, 9, pb)]
    r, s = pa - q, pb - q
    for k in range(q):
        nb[psi[s + k] - 1] = na[phi[r + k] - 1]
    return tuple(na), tuple(nb), phi, psi


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_ttt_random_cases(T, dtype):
    g = synth.rng(15, 0)
    for trial in range(24):
        pa = int(g.integers(1, 6))
        pb = int(g.integers(1, 6))
        q = int(g.integers(0, min(pa, pb) + 1))
        if q == 0 and (pa == 0 or pb == 0):
            continue
        na, nb, phi, psi = _ttt_random(g, pa, pb, q)
        X, Y = synth.uniform(na, g), synth.uniform(nb, g)
        Ad = to_gpu(X, synth.random_layout(pa, g), dtype)
        Bd = to_gpu(Y, synth.random_layout(pb, g), dtype)
        pc = pa + pb - 2 * q
        C = T.ttt(Ad, Bd, q, phi, psi, layout=synth.random_layout(pc, g) if pc else None)
        f = lambda Xa, Ya: oracle.ttt(oracle.materialize(Xa), oracle.materialize(Ya), q, phi, psi)
        _check(C, f, (round_to(X, dtype), round_to(Y, dtype)), (X, Y), dtype,
               "ttt trial %d na=%s nb=%s q=%d phi=%s psi=%s" % (trial, na, nb, q, phi, psi))


def test_ttt_reductions_outer_inner(T):
    g = synth.rng(16, 0)
    u, v = synth.uniform((37,), g), synth.uniform((45,), g)
    C = T.ttt(to_gpu(u, None, "f64"), to_gpu(v, None, "f64"), 0, (1,), (1,))
    assert_close(to_np(C), np.outer(u, v), 1e-15, "outer")
    X = synth.uniform((7, 6, 5), g)
    Y = synth.uniform((7, 6, 5), g)
    C = T.ttt(to_gpu(X, [3, 1, 2], "f64"), to_gpu(Y, None, "f64"), 3, (1, 2, 3), (1, 2, 3))
    ref = oracle.inner(oracle.materialize(X), oracle.materialize(Y))
    assert abs(float(to_np(C)) - ref) <= 1e-12 * abs(ref)


# ------------------------------------------------------------------ inner / norm

@pytest.mark.parametrize("dtype", DTYPES)
def test_inner_norm(T, dtype):
    g = synth.rng(17, DTYPES.index(dtype))
    for shape in [(1000,), (33, 17, 9), (5, 4, 3, 2, 6), (300, 301)]:
        X, Y = synth.uniform(shape, g), synth.uniform(shape, g)
        p = len(shape)
        for la, lb in [(None, None), (None, list(range(p, 0, -1))), (synth.random_layout(p, g), None)]:
            Ad, Bd = to_gpu(X, la, dtype), to_gpu(Y, lb, dtype)
            Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
            ip = float(to_np(T.inner(Ad, Bd)))
            ref = oracle.inner(oracle.materialize(Xr), oracle.materialize(Yr))
            scale = oracle.norm(oracle.materialize(Xr)) * oracle.norm(oracle.materialize(Yr))
            assert abs(ip - ref) <= 1e-13 * scale, (shape, la, lb)
            nr = float(to_np(T.norm(Ad)))
            assert abs(nr - oracle.norm(oracle.materialize(Xr))) <= 1e-13 * nr


def test_inner_integer_exact(T):
    g = synth.rng(18, 0)
    X, Y = synth.integers((64, 64, 64), g), synth.integers((64, 64, 64), g)
    for dtype in ("f64", "f32", "bf16"):
        ip = float(to_np(T.inner(to_gpu(X, None, dtype), to_gpu(Y, [3, 1, 2], dtype))))
        assert ip == oracle.inner(oracle.materialize(X), oracle.materialize(Y))


# ------------------------------------------------------------------ add / scale / transpose

@pytest.mark.parametrize("dtype", DTYPES)
def test_add_scale_transpose(T, dtype):
    g = synth.rng(19, DTYPES.index(dtype))
    for shape in [(1000,), (33, 17, 9), (5, 4, 3, 2, 6)]:
        p = len(shape)
        X, Y = synth.uniform(shape, g), synth.uniform(shape, g)
        Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
        for la, lb, lc in [(None, None, None), (None, list(range(p, 0, -1)), synth.random_layout(p, g)),
                           (synth.random_layout(p, g), None, list(range(p, 0, -1)))]:
            Ad, Bd = to_gpu(X, la, dtype), to_gpu(Y, lb, dtype)
            C = T.add(0.75, Ad, -1.25, Bd, layout=lc)
            ref = oracle.axpby(0.75, oracle.materialize(Xr), -1.25, oracle.materialize(Yr))
            assert np.array_equal(to_np(C), correctly_rounded(np.asarray(ref), dtype)), (shape, la, lb, lc)
            S = T.scale(-3.0, Ad, layout=lc)
            ref = oracle.scale(-3.0, oracle.materialize(Xr))
            assert np.array_equal(to_np(S), correctly_rounded(np.asarray(ref), dtype))
            tau = synth.random_layout(p, g)
            Tt = T.transpose(Ad, tau, layout=lc if lc is not None else None)
            assert np.array_equal(to_np(Tt), np.transpose(Xr, [t - 1 for t in tau]))


@pytest.mark.parametrize("din,dout", [("f64", "f64"), ("f32", "f32"), ("bf16", "bf16"), ("f16", "f16"),
                                      ("f32", "bf16"), ("f64", "f32"), ("bf16", "f32")])
def test_add_scale_flat_vectors(T, din, dout):
    """Sec. 5.1 Eq. transform / scaling on one unit-stride run long enough for
    the 16-byte vector path, with a ragged tail: every element equal to the
    correctly rounded FP64 value, in place as well."""
    import torch
    from _util import torch_dtype
    g = synth.rng(19, 40 + DTYPES.index(din) * 4 + DTYPES.index(dout))
    n = (1 << 20) + 5
    X, Y = synth.uniform((n,), g), synth.uniform((n,), g)
    Xr, Yr = round_to(X, din), round_to(Y, din)
    Ad, Bd = to_gpu(X, None, din), to_gpu(Y, None, din)
    if din == dout:
        assert "flat" in T.plan(T.add, 0.75, Ad, -1.25, Bd, out=T.empty((n,), None, torch_dtype(din), "cuda"))
        C = T.add(0.75, Ad, -1.25, Bd)
        ref = oracle.axpby(0.75, oracle.materialize(Xr), -1.25, oracle.materialize(Yr))
        assert np.array_equal(to_np(C), correctly_rounded(np.asarray(ref), dout))
        T.add(0.75, Ad, -1.25, Bd, out=Ad)
        assert np.array_equal(to_np(Ad), correctly_rounded(np.asarray(ref), dout))
        Ad = to_gpu(X, None, din)
    S = T.scale(-3.0, Ad, dtype=torch_dtype(dout))
    ref = oracle.scale(-3.0, oracle.materialize(Xr))
    assert np.array_equal(to_np(S), correctly_rounded(np.asarray(ref), dout))
    # an odd offset into the buffer: not 16-byte aligned, the element path
    S2 = T.scale(-3.0, Ad[1:], dtype=torch_dtype(dout))
    assert np.array_equal(to_np(S2), correctly_rounded(np.asarray(ref)[1:], dout))


def test_add_in_place(T):
    g = synth.rng(20, 0)
    X, Y = synth.integers((40, 30), g), synth.integers((40, 30), g)
    Ad, Bd = to_gpu(X, None, "f32"), to_gpu(Y, [2, 1], "f32")
    T.add(1.0, Ad, 2.0, Bd, out=Ad)
    assert np.array_equal(to_np(Ad), X + 2.0 * Y)
    T.scale(0.5, Ad, out=Ad)
    assert np.array_equal(to_np(Ad), 0.5 * (X + 2.0 * Y))


# ------------------------------------------------------------------ errors (validated before launch)

def test_error_codes(T):
    import torch
    from paper_1711_10912_amd import TlibError
    A = T.empty((4, 5, 6), None, torch.float32, "cuda")
    with pytest.raises(TlibError) as e:
        T.ttv(A, torch.zeros(7, device="cuda"), 2)
    assert e.value.code == 2  # ESHAPE
    with pytest.raises(TlibError) as e:
        T.ttv(A, torch.zeros(5, device="cuda"), 4)
    assert e.value.code == 3  # EMODE
    with pytest.raises(TlibError) as e:
        T.ttv(A, torch.zeros(5, device="cuda", dtype=torch.float64), 2)
    assert e.value.code == 4  # EDTYPE
    with pytest.raises(TlibError) as e:
        T.ttv(A, torch.zeros(5, device="cuda"), 2, out=A[:, 0, :])
    assert e.value.code == 5  # EALIAS
    C = torch.empty(4, 6, device="cuda").as_strided((4, 6), (1, 2))
    with pytest.raises(TlibError) as e:
        T.ttv(A, torch.zeros(5, device="cuda"), 2, out=C)
    assert e.value.code == 6  # ESTRIDE
