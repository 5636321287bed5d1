"""GPU parity of the GEMM path with operands loaded as groups of consecutive
k (16-bit: 16-byte groups of eight; FP32/FP64: groups of two) for TTT (Sec.
5.2 Eq. ttt) and TTM (Eq. ttm), against the oracle on the same rounded inputs
(16-bit with FP32 accumulation and FP32: 1e-5 normwise; FP64: 1e-12).  The
cases put K's unit-stride dim in X, in Y, in both and in neither, with ragged
M and N, several tile shapes and split-K; the full-size TTT runs with the
shipped kernel table, i.e. the tiles the benchmark times."""
import os
import zlib

import numpy as np
import pytest

import oracle
import synth
from _util import TOL, TOL_KERNEL16, assert_close, round_to, to_gpu, to_np

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _kvec(plan):
    """The k-group mode of a tiled-GEMM plan; -1 for the all-rows kernel (a
    kernel table may pick it where X and Y both have unit-stride K groups)."""
    if "gemm-rows" in plan:
        return -1
    return int(plan.split("kvec=")[1].split()[0])


# A (M1, K1, K2) x B (K1, K2, N1): A{2,3} <-> B{1,2}
SHAPES = [(40, 8, 24, 33), (7, 16, 8, 300), (300, 24, 16, 20), (130, 5, 16, 70), (64, 32, 96, 48)]
A_LAYOUTS = [[1, 2, 3], [3, 2, 1], [2, 3, 1]]
B_LAYOUTS = [[1, 2, 3], [3, 1, 2], [2, 1, 3]]


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32", "f64"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_ttt_k_groups(T, dtype, shape):
    import torch
    M1, K1, K2, N1 = shape
    g = synth.rng(70, zlib.crc32(repr((shape, dtype)).encode()) % 997)
    X = synth.uniform((M1, K1, K2), g)
    Y = synth.uniform((K1, K2, N1), g)
    Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
    ref = np.asarray(oracle.ttt(oracle.materialize(Xr), oracle.materialize(Yr), 2, (1, 2, 3), (3, 1, 2)))
    seen = set()
    for la in A_LAYOUTS:
        for lb in B_LAYOUTS:
            Ad, Bd = to_gpu(X, la, dtype), to_gpu(Y, lb, dtype)
            C = T.empty((M1, N1), None, torch.float64 if dtype == "f64" else torch.float32, "cuda")
            plan = T.plan(T.ttt, Ad, Bd, 2, (1, 2, 3), (3, 1, 2), out=C)
            seen.add(_kvec(plan))
            C.fill_(float("nan"))
            T.ttt(Ad, Bd, 2, (1, 2, 3), (3, 1, 2), out=C)
            tol = TOL[dtype] if dtype in ("f32", "f64") else TOL_KERNEL16
            assert_close(to_np(C), ref, tol, "%s %s A%s B%s" % (plan, dtype, la, lb))
    if dtype in ("bf16", "f16") and K2 % 8 == 0:
        assert {1, 2} <= seen and (3 in seen or -1 in seen), seen
    if dtype in ("f32", "f64"):
        assert seen - {0}, seen


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_ttm_k_groups(T, dtype):
    """TTM through the GEMM with 16-bit operands whose k runs are contiguous."""
    g = synth.rng(71, 0 if dtype == "bf16" else 1)
    for shape, q, m in [((30, 64, 20), 2, 300), ((64, 50, 7), 1, 270), ((9, 11, 40), 3, 333)]:
        X = synth.uniform(shape, g)
        B = synth.uniform((m, shape[q - 1]), g)
        # B stored k-fastest: its rows are the contiguous k runs
        Ad, Bd = to_gpu(X, None, dtype), to_gpu(B, [2, 1], dtype)
        plan = T.plan(T.ttm, Ad, Bd, q, out=T.ttm(Ad, Bd, q))
        assert "gemm" in plan and _kvec(plan) != 0, plan
        C = T.ttm(Ad, Bd, q)
        ref = oracle.ttm(oracle.materialize(round_to(X, dtype)), round_to(B, dtype), q)
        assert_close(to_np(C), ref, TOL_KERNEL16, "%s %s" % (plan, dtype))


@pytest.mark.parametrize("alay", ["first", "last", "perm3142"])
def test_ttt_fullsize_with_table(T, alay):
    """The (96,80,64,48) x (64,48,120) TTT in BF16 and FP16 with the shipped
    kernel table loaded (frozen): sampled outputs against the oracle."""
    import torch
    X, Y = synth.ttt_case()
    g = synth.rng(72, 0)
    prev = T.set_autotune("frozen")
    try:
        T.autotune_clear()
        T.autotune_load(os.path.join(ROOT, "paper_1711_10912_amd", "tuning", "mi355x_sweep.txt"))
        for dtype in ("bf16", "f16"):
            Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
            Ad = to_gpu(X, synth.TTT_A_LAYOUTS[alay], dtype)
            Bd = to_gpu(Y, None, dtype)
            C = T.empty((96, 80, 120), None, torch.float32, "cuda")
            plan = T.plan(T.ttt, Ad, Bd, 2, synth.TTT_PHI, synth.TTT_PSI, out=C)
            T.ttt(Ad, Bd, 2, synth.TTT_PHI, synth.TTT_PSI, out=C)
            Cn = to_np(C)
            got, ref = [], []
            for _ in range(64):
                i1, i2, j = int(g.integers(96)), int(g.integers(80)), int(g.integers(120))
                a = oracle.materialize(Xr[i1:i1 + 1, i2:i2 + 1, :, :])
                bb = oracle.materialize(Yr[:, :, j:j + 1])
                ref.append(float(np.asarray(oracle.ttt(a, bb, 2, synth.TTT_PHI, synth.TTT_PSI)).reshape(-1)[0]))
                got.append(Cn[i1, i2, j])
            assert_close(np.array(got), np.array(ref), TOL_KERNEL16, "%s %s A=%s" % (plan, dtype, alay))
    finally:
        T.autotune_clear()
        T.set_autotune(prev)



def _yvec(plan):
    return int(plan.split("yvec=")[1].split()[0])


def _ten_key(t):
    from paper_1711_10912_amd import _lib
    code = {"torch.float64": _lib.F64, "torch.float32": _lib.F32, "torch.bfloat16": _lib.BF16,
            "torch.float16": _lib.F16}[str(t.dtype)]
    return "|%d:%d" % (code, t.dim()) + "".join(",%d/%d" % (n, w) for n, w in zip(t.shape, t.stride()))


def _force_ttt_tile(T, tmp_path, A, B, C, q, phi, psi, tile):
    """A one-entry kernel table that picks `tile` for this exact call shape."""
    key = "ttt|%d" % q + "".join("|%d" % v for v in phi) + "".join("|%d" % v for v in psi)
    key += _ten_key(A) + _ten_key(B) + _ten_key(C)
    f = tmp_path / "tile.txt"
    f.write_text("%d %s\n" % (tile, key))
    T.autotune_clear()
    T.autotune_load(str(f))


TILES = ["16x256", "64x128", "128x128", "256x64", "64x64", "128x64", "256x32"]


# (free A extents, contracted extents, free B extents, vectors expected)
# A's first mode may be a view of a longer one (pad): columns then run in
# pieces of that extent, spaced by the padded length.
VEC_CASES = [((40,), (24, 48), (3,), 0, True),          # N = 40 ragged against every tile
             ((12, 6), (64, 48), (5,), 16, True),       # runs of 12 columns 16 apart: some waves load singly
             ((37,), (24, 48), (2, 3), 0, False),       # K stride 37: no 16-byte alignment
             ((40,), (16, 40), (3,), 0, False)]         # K = 640 < 1024: element by element, one k-step slices


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("tile", range(len(TILES)), ids=TILES)
def test_ttt_16bit_vectors_along_n(T, tmp_path, dtype, tile):
    """16-bit operand whose GEMM N dim has unit stride (A first-order, C
    first-order): loaded as 16-byte vectors of eight columns and stored
    transposed into the LDS slice, for every tile shape (forced through a
    one-entry kernel table), with ragged N, column runs that end inside a
    wave (such waves load column by column), a K stride that rules vectors
    out, a K too short for them (below 1024), and K long enough for several
    slices and a split (Sec. 5.2 Eq. ttt)."""
    import torch
    g = synth.rng(72, tile + (0 if dtype == "bf16" else 7))
    for fa, ka, fb, pad, vec in VEC_CASES:
        na, nb = fa + ka, ka + fb
        q, r, s_ = len(ka), len(fa), len(fb)
        phi = tuple(range(1, len(na) + 1))
        psi = tuple(range(q + 1, q + s_ + 1)) + tuple(range(1, q + 1))
        X, Y = synth.uniform(na, g), synth.uniform(nb, g)
        Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
        ref = np.asarray(oracle.ttt(oracle.materialize(Xr), oracle.materialize(Yr), q, phi, psi))
        if pad:
            Xp = np.zeros((pad,) + na[1:])
            Xp[: na[0]] = X
            Ad = to_gpu(Xp, None, dtype)[: na[0]]
        else:
            Ad = to_gpu(X, None, dtype)
        Bd = to_gpu(Y, None, dtype)
        C = T.empty(fa + fb, None, torch.float32, "cuda")
        prev = T.set_autotune("frozen")
        try:
            _force_ttt_tile(T, tmp_path, Ad, Bd, C, q, phi, psi, tile)
            plan = T.plan(T.ttt, Ad, Bd, q, phi, psi, out=C)
            C.fill_(float("nan"))
            T.ttt(Ad, Bd, q, phi, psi, out=C)
        finally:
            T.autotune_clear()
            T.set_autotune(prev)
        assert "tile=%s" % TILES[tile] in plan and "autotuned" in plan, plan
        assert (_yvec(plan) == 8) == vec, plan
        assert_close(to_np(C), ref, TOL_KERNEL16, "%s %s %s" % (plan, dtype, na))
