"""GPU parity of the TTV kernel regimes (Sec. 5.2 Eq. ttv) against the FP64
oracle; each case asserts the regime its plan names: the col kernel with one
wave per (lo tile, hi) unit and all k rows in flight (kr = 8..64, ragged lo,
vector widths 1/2/4), the col kernel with k split over the waves, with a grid
split over k, the fiber kernel for contiguous k-fibers and the slab kernel
(n_lo up to 63, b staged in LDS with whole slabs)."""
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


# (shape, layout, mode, expected plan fragments)
REGIMES = [
    ((64, 13, 5000), None, 2, ["ttv col", "kr=16"]),
    ((70, 13, 5000), None, 2, ["ttv col", "kr=16"]),          # ragged lo tile
    ((65, 7, 9000), None, 2, ["ttv col", "kr=8"]),            # odd lo: scalar loads
    ((129, 60, 1000), [1, 2, 3], 2, ["ttv col", "kr=0"]),     # too few units: k split over waves
    ((72, 30, 3000), None, 2, ["ttv col"]),
    ((40, 30, 1500), None, 2, ["ttv col"]),                  # n_lo 32..63, too few slabs
    ((36, 36, 3000), None, 2, ["ttv slab"]),                 # n_lo 32..63, whole slabs
    ((63, 17, 2500), [1, 2, 3], 2, ["ttv slab"]),
    ((100, 3, 20000), [1, 2, 3], 2, ["ttv col", "kr=8"]),
    ((5000, 33, 70), [3, 2, 1], 2, ["ttv col"]),              # last-order
    ((3000, 33, 40), [3, 2, 1], 2, ["ttv slab"]),             # last-order, C strided along lo
    ((37, 600, 3), None, 2, ["ttv col", "ksplit="]),
    ((8, 50, 9000), None, 2, ["ttv slab"]),
    ((300, 4000), None, 1, ["ttv fiber"]),                   # contiguous fibers of 300
    ((45, 70, 90), [3, 1, 2], 3, ["ttv fiber"]),            # last mode stored first
    ((20, 9000), None, 1, ["ttv slab"]),                     # short fibers stay on slabs
    ((13, 40000), None, 1, ["ttv slab"]),                    # slab count rounded to whole 16-byte units
]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", REGIMES, ids=lambda c: "%s-q%d" % ("x".join(map(str, c[0])), c[2]))
def test_ttv_regime(T, dtype, case):
    import torch
    shape, lay, q, expect = case
    g = synth.rng(80, zlib.crc32(repr((shape, q)).encode()) % 997)
    X = synth.uniform(shape, g)
    b = synth.uniform((shape[q - 1],), g)
    Ad, bd = to_gpu(X, lay, dtype), to_gpu(b, None, dtype)
    cs = shape[:q - 1] + shape[q:]
    C = T.empty(cs, None, T.acc_dtype(Ad.dtype), Ad.device)
    plan = T.plan(T.ttv, Ad, bd, q, out=C)
    for frag in expect:
        if dtype == "bf16" and frag.startswith("kr="):
            continue  # wider vectors for 16-bit change the row budget
        assert frag in plan, plan
    C.fill_(float("nan"))
    T.ttv(Ad, bd, q, out=C)
    torch.cuda.synchronize()
    ref = oracle.ttv(oracle.materialize(round_to(X, dtype)), round_to(b, dtype), q)
    tol = 1e-5 if dtype == "bf16" else TOL[dtype]
    assert_close(to_np(C), ref, tol, "%s %s" % (plan, dtype))
