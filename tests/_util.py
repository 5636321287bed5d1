"""Helpers for the parity tests: placing logical numpy tensors on the GPU in a
given layout, reading them back exactly, and the error measures."""
import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 2e-2}
# kernel-only bound for 16-bit inputs: the oracle sees the same rounded inputs
# and the kernel accumulates in FP32
TOL_KERNEL16 = 1e-5
# A 16-bit end-to-end result is held to TOL (2e-2) of ||C*||.  Rounding the
# inputs to 16 bits perturbs each product by up to 2u (u = 2^-8 for BF16,
# 2^-11 for FP16), so the error of a contraction is bounded by about
# 2u * || |A|.|B| || (the same contraction over absolute values), and relative
# to ||C*|| by 2u times the condition number kappa = || |A|.|B| || / ||C*||.
# Where C* cancels so far that kappa > KAPPA16 (||C*|| below 1 % of
# || |A|.|B| ||), no 16-bit input can meet a bound relative to ||C*||; such a
# result is held to TOL of || |A|.|B| || instead.
KAPPA16 = 100.0


def torch_dtype(name):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[name]


def to_gpu(X: np.ndarray, layout, dtype: str):
    """Dense GPU tensor holding the logical values X (rounded to dtype) with the
    given 1-based layout (None = first-order)."""
    import torch
    import paper_1711_10912_amd as T
    t = T.empty(X.shape, layout, torch_dtype(dtype), "cuda")
    t.copy_(torch.from_numpy(np.ascontiguousarray(X)).to(torch_dtype(dtype)).cuda())
    return t


def to_np(t) -> np.ndarray:
    """Exact float64 copy of a GPU tensor's logical values."""
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """Normwise relative error ||got - ref||_F / ||ref||_F."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.reshape(-1))
    num = np.linalg.norm((got - ref).reshape(-1))
    if den == 0.0:
        return float(num)
    return float(num / den)


def assert_close(got, ref, tol, what=""):
    e = rel_err(got, ref)
    assert e <= tol, "%s: normwise relative error %.3e > %.1e" % (what, e, tol)
    return e


def assert_close16(got, ref, absref, tol, what=""):
    """End-to-end check of a result computed from 16-bit inputs: `ref` is the
    oracle on the original (unrounded) values, `absref` the same contraction
    over their absolute values.  Pass/fail on ||got - ref|| / ||ref|| <= tol,
    unless ref cancels beyond KAPPA16 (then relative to ||absref||).  Returns
    (normwise error, error relative to ||absref||, kappa)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = float(np.linalg.norm((got - ref).reshape(-1)))
    den = float(np.linalg.norm(ref.reshape(-1)))
    den_abs = float(np.linalg.norm(np.asarray(absref, dtype=np.float64).reshape(-1)))
    kappa = den_abs / den if den > 0 else np.inf
    e_rel = num / den if den > 0 else np.inf
    e_abs = num / den_abs if den_abs > 0 else num
    if kappa <= KAPPA16:
        assert e_rel <= tol, "%s (end to end): normwise relative error %.3e > %.1e (kappa %.1f)" % (
            what, e_rel, tol, kappa)
    else:
        assert e_abs <= tol, "%s (end to end, kappa %.3g > %g): error relative to |||A|.|B||| %.3e > %.1e" % (
            what, kappa, KAPPA16, e_abs, tol)
    return e_rel, e_abs, kappa


def round_to(X: np.ndarray, dtype: str) -> np.ndarray:
    """Values as the GPU holds them after rounding to `dtype` (torch's rounding)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to(torch_dtype(dtype)).to(torch.float64).numpy()


def correctly_rounded(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round float64 values to dtype with a single round-to-nearest-even step
    (round to odd into float32 first, which keeps a sticky bit, then RNE)."""
    import torch
    x = np.asarray(x, dtype=np.float64)
    if dtype == "f64":
        return x.copy()
    f = x.astype(np.float32)
    if dtype == "f32":
        return f.astype(np.float64)
    inexact = f.astype(np.float64) != x
    u = f.view(np.uint32).copy()
    toward_zero = np.abs(f.astype(np.float64)) > np.abs(x)
    u = np.where(inexact & toward_zero, u - 1, u)
    u = np.where(inexact, u | 1, u).astype(np.uint32)
    f_odd = u.view(np.float32)
    return torch.from_numpy(f_odd.copy()).to(torch_dtype(dtype)).to(torch.float64).numpy()
