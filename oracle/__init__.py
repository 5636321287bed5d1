"""Plain FP64 CPU oracle for the TTV / TTM / TTT contraction path of
Bassoy, "TLib: A Flexible C++ Tensor Framework for Numerical Tensor Calculus"
(arXiv 1711.10912).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark import this package.  It shares no code with
the HIP library and imports nothing from it.

Tensors are numpy float64 arrays of any (non-negative) strides: the array's
shape is the shape tuple n and its element strides are the stride tuple w of
the paper (Sec. 3.1), so a numpy view of a buffer is exactly a tensor or view
with base address gamma (Sec. 3.3).  Modes, layouts and permutations are
1-based as in the paper's equations.

The arithmetic lives in ``oracle.c`` (plain loops, one output element at a
time, contracted indices ascending).  The composite drivers below
(``times_vectors``, ``hopm``, ``tucker``) are host loops over those calls in
the order the paper gives (Sec. 5.2, tensor_times_vectors and the higher-order
power method).
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain C, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ora_strides.argtypes = [ctypes.c_int, _i64p, _i32p, _i64p]
        lib.ora_ttv.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _dp, ctypes.c_int64, ctypes.c_int,
                                _dp, _i64p]
        lib.ora_ttm.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, ctypes.c_int64, _dp, _i64p,
                                ctypes.c_int, _dp, _i64p]
        lib.ora_ttt.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, ctypes.c_int, _i64p, _dp, _i64p,
                                ctypes.c_int, _i32p, _i32p, _dp, _i64p]
        lib.ora_inner.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _dp, _i64p]
        lib.ora_inner.restype = ctypes.c_double
        lib.ora_axpby.argtypes = [ctypes.c_int, _i64p, ctypes.c_double, _dp, _i64p,
                                  ctypes.c_double, _dp, _i64p, _dp, _i64p]
        lib.ora_transpose.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _i32p, _dp, _i64p]
        for f in ("ora_strides", "ora_ttv", "ora_ttm", "ora_ttt", "ora_axpby", "ora_transpose"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _i64(vals) -> ctypes.Array:
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * max(1, len(vals)))(*vals)


def _i32(vals) -> ctypes.Array:
    vals = [int(v) for v in vals]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals)


def _ptr(a: np.ndarray):
    if a.dtype != np.float64:
        raise TypeError("oracle tensors are float64")
    return ctypes.cast(ctypes.c_void_p(a.ctypes.data), _dp)


def _w(a: np.ndarray):
    if any(s < 0 or s % 8 for s in a.strides):
        raise ValueError("oracle needs non-negative element strides")
    return [s // 8 for s in a.strides]


# ---------------------------------------------------------------- layouts

def strides(n: Sequence[int], pi: Sequence[int] | None = None) -> tuple:
    """Stride tuple w from shape n and 1-based layout tuple pi
    (Sec. 3.1 Eq. stride.tuple.permutation); pi=None is first-order."""
    p = len(n)
    if pi is None:
        pi = list(range(1, p + 1))
    w = (ctypes.c_int64 * max(1, p))()
    rc = _load().ora_strides(p, _i64(n), _i32(pi), w)
    if rc != 0:
        raise ValueError("layout %r is not a permutation of 1..%d" % (tuple(pi), p))
    return tuple(w[r] for r in range(p))


def empty(n: Sequence[int], pi: Sequence[int] | None = None) -> np.ndarray:
    """Dense float64 tensor of shape n whose memory follows layout pi."""
    n = tuple(int(v) for v in n)
    w = strides(n, pi) if n else ()
    size = int(np.prod(n, dtype=np.int64)) if n else 1
    buf = np.zeros(max(size, 1), dtype=np.float64)
    return np.lib.stride_tricks.as_strided(buf, shape=n, strides=tuple(8 * s for s in w))


def materialize(values: np.ndarray, pi: Sequence[int] | None = None) -> np.ndarray:
    """Copy the logical tensor ``values`` into a dense tensor with layout pi."""
    out = empty(values.shape, pi)
    out[...] = values
    return out


def last_order(p: int) -> list:
    """pi_L = (p, ..., 1) (Sec. 3.1 Eq. layout.tuple.last.order)."""
    return list(range(p, 0, -1))


# ---------------------------------------------------------------- contractions

def ttv(A: np.ndarray, b: np.ndarray, m: int, C: np.ndarray | None = None, pi=None) -> np.ndarray:
    """Mode-m tensor-times-vector, Sec. 5.2 Eq. ttv (m is 1-based)."""
    p = A.ndim
    b = np.asarray(b, dtype=np.float64)
    if b.ndim != 1 or not (1 <= m <= p) or b.shape[0] != A.shape[m - 1]:
        raise ValueError("ttv: b must be a vector of length n_m")
    nc = A.shape[: m - 1] + A.shape[m:]
    if C is None:
        C = empty(nc, pi)
    assert C.shape == nc
    rc = _load().ora_ttv(p, _i64(A.shape), _ptr(A), _i64(_w(A)), _ptr(b), _w(b)[0], m, _ptr(C),
                         _i64(_w(C)))
    if rc != 0:
        raise ValueError("ttv: invalid arguments")
    return C


def ttm(A: np.ndarray, B: np.ndarray, m: int, C: np.ndarray | None = None, pi=None) -> np.ndarray:
    """Mode-m tensor-times-matrix, Sec. 5.2 Eq. ttm; B has shape (n', n_m)."""
    p = A.ndim
    if B.ndim != 2 or not (1 <= m <= p) or B.shape[1] != A.shape[m - 1]:
        raise ValueError("ttm: B must have shape (n', n_m)")
    nc = A.shape[: m - 1] + (B.shape[0],) + A.shape[m:]
    if C is None:
        C = empty(nc, pi)
    assert C.shape == nc
    rc = _load().ora_ttm(p, _i64(A.shape), _ptr(A), _i64(_w(A)), B.shape[0], _ptr(B), _i64(_w(B)),
                         m, _ptr(C), _i64(_w(C)))
    if rc != 0:
        raise ValueError("ttm: invalid arguments")
    return C


def ttt_shape(na, nb, q, phi, psi) -> tuple:
    """Shape of C from Sec. 5.2 Eq. ttt_indices."""
    r, s = len(na) - q, len(nb) - q
    return tuple(na[phi[k] - 1] for k in range(r)) + tuple(nb[psi[k] - 1] for k in range(s))


def ttt(A: np.ndarray, B: np.ndarray, q: int, phi, psi, C: np.ndarray | None = None,
        pi=None) -> np.ndarray:
    """(q, phi, psi)-mode tensor-times-tensor, Sec. 5.2 Eq. ttt and ttt_indices."""
    pa, pb = A.ndim, B.ndim
    if len(phi) != pa or len(psi) != pb:
        raise ValueError("ttt: phi/psi must have the orders of A/B")
    nc = ttt_shape(A.shape, B.shape, q, phi, psi)
    if C is None:
        C = empty(nc, pi)
    assert C.shape == nc
    rc = _load().ora_ttt(pa, _i64(A.shape), _ptr(A), _i64(_w(A)), pb, _i64(B.shape), _ptr(B),
                         _i64(_w(B)), q, _i32(phi), _i32(psi), _ptr(C), _i64(_w(C) or [0]))
    if rc != 0:
        raise ValueError("ttt: invalid arguments (rc=%d)" % rc)
    return C


def inner(A: np.ndarray, B: np.ndarray) -> float:
    """<A, B> (Sec. 5.2 Table 3), Neumaier-compensated, first-order visit order."""
    if A.shape != B.shape:
        raise ValueError("inner: shapes differ")
    return float(_load().ora_inner(A.ndim, _i64(A.shape), _ptr(A), _i64(_w(A)), _ptr(B),
                                   _i64(_w(B))))


def norm(A: np.ndarray) -> float:
    """Frobenius norm sqrt(<A, A>) (Sec. 5.2 Table 3)."""
    return math.sqrt(inner(A, A))


def axpby(alpha: float, A: np.ndarray, beta: float, B: np.ndarray | None,
          C: np.ndarray | None = None, pi=None) -> np.ndarray:
    """C = alpha A + beta B (Sec. 5.1 Eq. transform with a scaled sum; B=None gives Eq. scaling)."""
    if B is not None and B.shape != A.shape:
        raise ValueError("axpby: shapes differ")
    if C is None:
        C = empty(A.shape, pi)
    bp = _ptr(B) if B is not None else None
    bw = _i64(_w(B)) if B is not None else None
    rc = _load().ora_axpby(A.ndim, _i64(A.shape), float(alpha), _ptr(A), _i64(_w(A)),
                           float(beta), bp, bw, _ptr(C), _i64(_w(C)))
    if rc != 0:
        raise ValueError("axpby: invalid arguments")
    return C


def scale(alpha: float, A: np.ndarray, C: np.ndarray | None = None, pi=None) -> np.ndarray:
    """C = alpha A (Sec. 5.1 Eq. scaling)."""
    return axpby(alpha, A, 0.0, None, C, pi)


def transpose(A: np.ndarray, tau, C: np.ndarray | None = None, pi=None) -> np.ndarray:
    """C = A^tau with i^c_r = i^a_{tau_r} (Sec. 5.2 Table 3, transpose)."""
    nc = tuple(A.shape[t - 1] for t in tau)
    if C is None:
        C = empty(nc, pi)
    rc = _load().ora_transpose(A.ndim, _i64(A.shape), _ptr(A), _i64(_w(A)), _i32(tau), _ptr(C),
                               _i64(_w(C)))
    if rc != 0:
        raise ValueError("transpose: invalid arguments")
    return C


# ---------------------------------------------------------------- composite drivers

def times_vectors(A: np.ndarray, us: Sequence[np.ndarray], excluded: int) -> np.ndarray:
    """Multiply A with u_k in every mode k except ``excluded`` (1-based), the
    highest mode first, each step one mode-k TTV (Sec. 5.2, tensor_times_vectors
    and its use in the higher-order power method).  Returns a vector."""
    p = A.ndim
    X = A
    for k in range(p, 0, -1):
        if k == excluded:
            continue
        X = ttv(X, us[k - 1], k)
    return np.ascontiguousarray(X).reshape(-1)


def hopm(A: np.ndarray, us: Sequence[np.ndarray], iters: int):
    """Higher-order power method (Sec. 5.2): for every sweep and every mode r,
    u_r <- A times all u_k (k != r); lambda_r <- ||u_r||; u_r <- u_r / lambda_r.
    Returns (lambdas, us) after ``iters`` sweeps."""
    us = [np.array(u, dtype=np.float64, copy=True) for u in us]
    lam = [0.0] * A.ndim
    for _ in range(iters):
        for r in range(A.ndim):
            v = times_vectors(A, us, r + 1)
            lam[r] = norm(v)
            us[r] = scale(1.0 / lam[r], v)
    return lam, us


def tucker(A: np.ndarray, Us: Sequence[np.ndarray]) -> np.ndarray:
    """Successive mode-k TTMs A x_1 U_1 x_2 U_2 ... (Sec. 5.2 Table 3,
    tensor_times_matrices)."""
    X = A
    for k, U in enumerate(Us, start=1):
        X = ttm(X, U, k)
    return X
