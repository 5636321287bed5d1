"""Composite drivers over the C ABI: the higher-order power method and the
Tucker (successive TTM) chain of Sec. 5.2.  These are host loops in the
paper's order; every contraction, norm and scaling runs in the HIP kernels."""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple


def hopm(A, us: Sequence, iters: int) -> Tuple[List[float], list]:
    """Higher-order power method (Sec. 5.2): for each of `iters` sweeps and each
    mode r, u_r <- A times every u_k (k != r, highest mode first);
    lambda_r <- ||u_r|| (FP64); u_r <- u_r / lambda_r.  `us` are device vectors
    of A's dtype.  The norms and the division stay on the device
    (tlib_normalize); the lambdas of the last sweep are read back once at the
    end.  Returns (lambdas as host floats, us)."""
    import torch

    from . import normalize, times_vectors

    us = [u.clone() for u in us]
    lam = torch.zeros(A.dim(), dtype=torch.float64, device=A.device)
    for _ in range(iters):
        for r in range(A.dim()):
            v = times_vectors(A, us, r + 1)
            normalize(v, out=us[r], norm_out=lam[r])
    return [float(x) for x in lam.cpu()], us


def tucker(A, Us: Sequence, stage_dtype=None):
    """A x_1 U_1 x_2 U_2 ... (Sec. 5.2 tensor_times_matrices): mode products
    with factor matrices U_k of shape (r_k, n_k), FP32/FP64 data two modes per
    pass (ttm2), 16-bit data one TTM per mode.  With `stage_dtype` (e.g.
    torch.bfloat16) every intermediate is rounded to that dtype before it
    enters the next TTM; results accumulate in FP32 (FP64 for FP64 data)."""
    import torch

    from . import scale, ttm, ttm2

    X = A
    p = len(Us)
    k = 1
    while k <= p:
        if stage_dtype is not None and X.dtype != stage_dtype:
            X = scale(1.0, X, dtype=stage_dtype)
        if k < p and X.dtype in (torch.float32, torch.float64):
            # modes k and k+1 in one pass (the intermediate is not written)
            X = ttm2(X, Us[k - 1], k, Us[k], k + 1)
            k += 2
        else:
            X = ttm(X, Us[k - 1], k)
            k += 1
    return X
