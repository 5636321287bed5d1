"""GPU parity of entrywise ops whose output's fastest dimension differs from
the input's (transpose and add/scale into another layout, Sec. 5.1 and the
transposition of Table 3), which run through LDS tiles.  Bit for bit against
the oracle: each output is one correctly rounded FP64 expression of its
inputs."""
import zlib

import numpy as np
import pytest

import oracle
import synth
from _util import correctly_rounded, round_to, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _seed(*key):
    return zlib.crc32(repr(key).encode()) % 1000


def _rev(p):
    return list(range(p, 0, -1))


CASES = [((40, 33, 17), [3, 1, 2]), ((16, 16), [2, 1]), ((31, 5, 47), [3, 2, 1]), ((90, 7, 3, 41), [4, 3, 2, 1]),
         ((17, 2, 3, 5, 65), [5, 1, 2, 3, 4]), ((100, 1, 3, 33), [4, 2, 3, 1])]


@pytest.mark.parametrize("shape,la", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_add_into_other_layout(T, shape, la, dtype):
    """C first-order, A in layout la; B like A (read through LDS), like C (read
    directly) and in a third layout."""
    g = synth.rng(60, _seed(shape, la, dtype))
    p = len(shape)
    X, Y = synth.uniform(shape, g), synth.uniform(shape, g)
    Xr, Yr = round_to(X, dtype), round_to(Y, dtype)
    ref = correctly_rounded(np.asarray(oracle.axpby(0.75, oracle.materialize(Xr), -1.25, oracle.materialize(Yr))),
                            dtype)
    Ad = to_gpu(X, la, dtype)
    for lb, bm in ((la, "b=2"), (None, "b=1"), (synth.random_layout(p, g), None)):
        Bd = to_gpu(Y, lb, dtype)
        C = T.empty(shape, None, Ad.dtype, "cuda")
        plan = T.plan(T.add, 0.75, Ad, -1.25, Bd, out=C)
        assert "ewise tile" in plan, plan
        if bm:
            assert bm in plan, plan
        T.add(0.75, Ad, -1.25, Bd, out=C)
        assert np.array_equal(to_np(C), ref), (shape, la, lb, dtype)


@pytest.mark.parametrize("shape,la", CASES[:4])
def test_scale_convert_into_other_layout(T, shape, la):
    g = synth.rng(61, _seed(shape, la))
    X = synth.uniform(shape, g) * 1e3
    Ad = to_gpu(X, la, "f64")
    import torch
    for dt, name in ((torch.float64, "f64"), (torch.float32, "f32"), (torch.bfloat16, "bf16"),
                     (torch.float16, "f16")):
        C = T.empty(shape, None, dt, "cuda")
        assert "ewise tile" in T.plan(T.scale, -0.3, Ad, out=C)
        T.scale(-0.3, Ad, out=C)
        ref = correctly_rounded(np.asarray(oracle.scale(-0.3, oracle.materialize(X))), name)
        assert np.array_equal(to_np(C), ref), (shape, la, name)


@pytest.mark.parametrize("shape", [(40, 33, 17), (90, 7, 3, 41), (64, 64)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_transpose_tiled(T, shape, dtype):
    """Every tau whose C (first-order) puts A's first mode away from the front."""
    import itertools
    g = synth.rng(62, _seed(shape, dtype))
    p = len(shape)
    X = synth.uniform(shape, g)
    Xr = round_to(X, dtype)
    Ad = to_gpu(X, None, dtype)
    seen = 0
    for tau in itertools.permutations(range(1, p + 1)):
        tau = list(tau)
        Ct = T.empty(tuple(shape[t - 1] for t in tau), None, Ad.dtype, "cuda")
        if "ewise tile" not in T.plan(T.transpose, Ad, tau, out=Ct):
            continue
        seen += 1
        T.transpose(Ad, tau, out=Ct)
        assert np.array_equal(to_np(Ct), np.transpose(Xr, [t - 1 for t in tau])), (shape, tau)
    assert seen > 0


def test_relayout_of_stepped_view(T):
    """A is a view whose fastest mode steps by 2; C dense in another order."""
    import torch
    g = synth.rng(63, 0)
    shape = (50, 20, 37)
    X = synth.uniform(shape, g)
    big = T.empty((50, 20, 74), [3, 1, 2], torch.float32, "cuda")
    A = big[:, :, ::2]
    A.copy_(torch.from_numpy(X).float().cuda())
    C = T.empty(shape, None, torch.float32, "cuda")
    assert "ewise tile" in T.plan(T.scale, 2.0, A, out=C)
    T.scale(2.0, A, out=C)
    assert np.array_equal(to_np(C), 2.0 * round_to(X, "f32"))


def test_relayout_fullsize_views_workload(T):
    """The 90^4 FP32 views case: A = a [:, ::3] view of a reversed-layout
    tensor, C = A + A dense first-order; every element checked."""
    import torch
    n = 90
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9090)
    A = T.empty((n, 3 * n, n, n), [4, 3, 2, 1], torch.float32, "cuda")[:, ::3]
    A.copy_(torch.rand(A.shape, generator=gen, device="cuda"))
    C = T.empty(A.shape, None, torch.float32, "cuda")
    assert "ewise tile" in T.plan(T.add, 1.0, A, 1.0, A, out=C)
    T.add(1.0, A, 1.0, A, out=C)
    Xa = to_np(A)
    assert np.array_equal(to_np(C), (Xa + Xa).astype(np.float32).astype(np.float64))
