"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers and shapes; it contains none of the
contraction arithmetic.  Every tensor is produced as a *logical* numpy array
(shape = shape tuple, float64) whose values are a function of the multi-index:
the draws are taken in first-order index order (first index fastest), so all
memory layouts of one case hold the same mathematical tensor.  Callers place
the values into whatever layout they test.

Seeds: base 171110912 + workload index; per-case generators come from
``numpy.random.SeedSequence(base).spawn`` in a fixed case order (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 171110912

# Order-p sweep at about 2^26 elements: extents equal per mode.
SWEEP_EXTENTS = {3: 406, 4: 90, 5: 36, 6: 20, 7: 13}
SWEEP_TTM_M = (16, 64, 256)


def rng(workload: int, case: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence(BASE_SEED + workload)
    child = ss.spawn(case + 1)[case]
    return np.random.Generator(np.random.PCG64(child))


def _logical(flat: np.ndarray, shape: Sequence[int]) -> np.ndarray:
    # flat[j] is the value of the multi-index whose first-order counter is j
    return flat.reshape(tuple(shape), order="F")


def uniform(shape: Sequence[int], g: np.random.Generator, lo: float = -1.0,
            hi: float = 1.0) -> np.ndarray:
    n = int(np.prod(shape, dtype=np.int64)) if len(shape) else 1
    return _logical(g.uniform(lo, hi, n), shape)


def normal(shape: Sequence[int], g: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    n = int(np.prod(shape, dtype=np.int64)) if len(shape) else 1
    return _logical(g.standard_normal(n) * scale, shape)


def integers(shape: Sequence[int], g: np.random.Generator, lo: int = -4, hi: int = 4) -> np.ndarray:
    """Small integer values stored as float64: every partial sum of products is
    exact in FP32/FP64 for the sizes used, so results must match bit for bit."""
    n = int(np.prod(shape, dtype=np.int64)) if len(shape) else 1
    return _logical(g.integers(lo, hi + 1, n).astype(np.float64), shape)


def random_layout(p: int, g: np.random.Generator) -> List[int]:
    return [int(v) + 1 for v in g.permutation(p)]


# ------------------------------------------------------------------ workloads

def tiny_case():
    """Order 3, 32^3, first-order, U[-1,1]; mode-2 TTV with a 32-vector and
    mode-2 TTM with a 16x32 matrix."""
    g = rng(0, 1)
    A = uniform((32, 32, 32), g)
    b = uniform((32,), g)
    B = uniform((16, 32), g)
    return A, b, B


@dataclass
class SweepCase:
    p: int
    n: int
    q: int          # 1-based contraction mode
    layout: str     # "first" | "last"
    m: Optional[int]  # None for TTV, else TTM rows

    @property
    def shape(self):
        return (self.n,) * self.p

    @property
    def pi(self):
        return list(range(1, self.p + 1)) if self.layout == "first" else list(range(self.p, 0, -1))


def sweep_cases(ops=("ttv", "ttm")) -> List[SweepCase]:
    out = []
    for p, n in SWEEP_EXTENTS.items():
        for layout in ("first", "last"):
            for q in range(1, p + 1):
                if "ttv" in ops:
                    out.append(SweepCase(p, n, q, layout, None))
                if "ttm" in ops:
                    for m in SWEEP_TTM_M:
                        out.append(SweepCase(p, n, q, layout, m))
    return out


def sweep_tensor(p: int, scale_down: int = 1) -> np.ndarray:
    """The order-p sweep tensor (U[-1,1]); scale_down>1 shrinks extents for tests."""
    n = max(2, SWEEP_EXTENTS[p] // scale_down)
    return uniform((n,) * p, rng(1, p))


def sweep_operands(n_q: int, m: int):
    g = rng(1, 100 + n_q * 1000 + m)
    return uniform((n_q,), g), uniform((m, n_q), g)


TTT_A_SHAPE = (96, 80, 64, 48)
TTT_B_SHAPE = (64, 48, 120)
TTT_PHI = (1, 2, 3, 4)   # free A modes 1,2; contracted A modes 3,4
TTT_PSI = (3, 1, 2)      # free B mode 3; contracted B modes 1,2 (paired by position)
TTT_A_LAYOUTS = {"first": (1, 2, 3, 4), "last": (4, 3, 2, 1), "perm3142": (3, 1, 4, 2)}


def ttt_case(scale: float = 1.0, shrink: int = 1):
    g = rng(2, 0 if scale == 1.0 else 1)
    sa = tuple(max(2, s // shrink) for s in TTT_A_SHAPE)
    sb = (sa[2], sa[3], max(2, TTT_B_SHAPE[2] // shrink))
    return normal(sa, g, scale), normal(sb, g, scale)


def orthonormal_columns(n: int, k: int, g: np.random.Generator) -> np.ndarray:
    qm, _ = np.linalg.qr(g.standard_normal((n, k)))
    return qm[:, :k]


def tucker_case(n: int = 160, rank: int = 16, rows: int = 32, sigma0: float = 1e5,
                noise: float = 1.0, g: Optional[np.random.Generator] = None):
    """Order-4 tensor N(0,1)*noise + sum_r sigma_r a_r o b_r o c_r o d_r with
    orthonormal factor columns, sigma_r = sigma0 * 0.8^(r-1); factor matrices
    U_k (rows x n) with orthonormal rows whose first `rank` rows are the true
    factors.  Returns (A, [U_1..U_4], factors, sigmas)."""
    g = g or rng(3, 0)
    facs = [orthonormal_columns(n, rows, g) for _ in range(4)]
    sig = sigma0 * 0.8 ** np.arange(rank)
    A = normal((n,) * 4, g, noise)
    F = [f[:, :rank] for f in facs]
    A = A + np.einsum("r,ir,jr,kr,lr->ijkl", sig, *F, optimize=True)
    Us = [f.T.copy() for f in facs]
    return A, Us, F, sig


@dataclass
class Request:
    rid: int
    arrival: float
    op: str               # "ttv" | "ttm" | "ttt"
    dtype: str            # "f32" | "bf16"
    a_id: int
    mode: int = 0         # ttv/ttm
    mat_id: int = -1      # ttm: resident factor matrix
    q: int = 0            # ttt
    phi: tuple = ()
    psi: tuple = ()
    b_shape: tuple = ()
    b_layout: tuple = ()
    out_layout: str = "first"


@dataclass
class ServedPools:
    tensors: List[tuple] = field(default_factory=list)    # (shape, layout)
    matrices: List[tuple] = field(default_factory=list)   # (m, n)


def _log_uniform_int(g, lo, hi):
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))


def served_pools(n_tensors: int = 1024, n_mats: int = 256, cap: int = 1 << 24,
                 g: Optional[np.random.Generator] = None) -> ServedPools:
    g = g or rng(4, 0)
    pools = ServedPools()
    # the smallest order-p tensor has 8^p elements: never draw an order the cap excludes
    pmax = max(2, min(6, int(math.floor(math.log(cap) / math.log(8) + 1e-9))))
    for _ in range(n_tensors):
        p = int(g.integers(2, pmax + 1))
        for _attempt in range(10000):
            shape = tuple(_log_uniform_int(g, 8, 512) for _ in range(p))
            if int(np.prod(shape, dtype=np.int64)) <= cap:
                break
        else:
            shape = (8,) * p
        u = g.uniform()
        if u < 0.4:
            lay = tuple(range(1, p + 1))
        elif u < 0.8:
            lay = tuple(range(p, 0, -1))
        else:
            lay = tuple(random_layout(p, g))
        pools.tensors.append((shape, lay))
    for _ in range(n_mats):
        pools.matrices.append((_log_uniform_int(g, 8, 256), _log_uniform_int(g, 8, 512)))
    return pools


def served_stream(pools: ServedPools, n_req: int, rate: float, cap: int = 1 << 24,
                  g: Optional[np.random.Generator] = None) -> List[Request]:
    """Poisson arrivals (rate per second); 40% TTV, 40% TTM, 20% TTT; dtype
    f32 or bf16 with equal probability; operands referenced by pool id."""
    g = g or rng(4, 1)
    t = 0.0
    reqs = []
    for rid in range(n_req):
        t += g.exponential(1.0 / rate)
        u = g.uniform()
        dtype = "f32" if g.uniform() < 0.5 else "bf16"
        a_id = int(g.integers(len(pools.tensors)))
        shape, lay = pools.tensors[a_id]
        p = len(shape)
        if u < 0.4:
            reqs.append(Request(rid, t, "ttv", dtype, a_id, mode=int(g.integers(1, p + 1))))
        elif u < 0.8:
            # pick a factor matrix whose n matches some mode of A; else fall back to TTV
            modes = [k + 1 for k in range(p)]
            g.shuffle(modes)
            picked = None
            for mode in modes:
                cands = [i for i, (mm, nn) in enumerate(pools.matrices) if nn == shape[mode - 1]]
                out_elems = 0
                if cands:
                    i = cands[int(g.integers(len(cands)))]
                    out_elems = int(np.prod(shape, dtype=np.int64)) // shape[mode - 1] * pools.matrices[i][0]
                    if out_elems <= cap:
                        picked = (mode, i)
                        break
            if picked is None:
                # resident pool has no matching factor: use the first mode and a fresh
                # matrix id that the server materialises (m drawn log-uniform in 8..256)
                mode = modes[0]
                mm = _log_uniform_int(g, 8, 256)
                while int(np.prod(shape, dtype=np.int64)) // shape[mode - 1] * mm > cap and mm > 1:
                    mm //= 2
                pools.matrices.append((mm, shape[mode - 1]))
                picked = (mode, len(pools.matrices) - 1)
            reqs.append(Request(rid, t, "ttm", dtype, a_id, mode=picked[0], mat_id=picked[1]))
        else:
            q = int(g.integers(1, 3)) if p >= 2 else 1
            q = min(q, p)
            contr = sorted(int(v) + 1 for v in g.choice(p, size=q, replace=False))
            free_a = [k for k in range(1, p + 1) if k not in contr]
            s = int(g.integers(0, 3))
            while True:
                free_b = tuple(_log_uniform_int(g, 8, 512) for _ in range(s))
                nb = tuple(shape[k - 1] for k in contr) + free_b
                nc = int(np.prod([shape[k - 1] for k in free_a] + list(free_b), dtype=np.int64))
                if int(np.prod(nb, dtype=np.int64)) <= cap and nc <= cap:
                    break
                s = max(0, s - 1)
            if len(free_a) + s == 0:
                s = 1
                free_b = (8,)
                nb = tuple(shape[k - 1] for k in contr) + free_b
            pb = q + s
            # B's modes: contracted first (in the order of `contr`), then its free modes
            phi = tuple(free_a + contr)
            psi = tuple(list(range(q + 1, pb + 1)) + list(range(1, q + 1)))
            reqs.append(Request(rid, t, "ttt", dtype, a_id, q=q, phi=phi, psi=psi, b_shape=nb,
                                b_layout=tuple(range(1, pb + 1))))
    return reqs
