"""MI355X tensor-contraction path of Bassoy's TLib (arXiv 1711.10912), Sec. 5.

Thin Python binding over libtlib.so: every function here only marshals
arguments (device pointers, shapes, strides, 1-based modes) and calls the C
ABI declared in include/tlib.h; all arithmetic runs in the HIP kernels.
PyTorch supplies device memory and the current stream.

Tensors are torch tensors on the GPU with any non-negative strides: the shape
is the paper's shape tuple n and ``tensor.stride()`` its stride tuple w
(Sec. 3.1), so a torch view is a TLib view (Sec. 3.3).  Modes, layouts and
permutations are 1-based as in the paper.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import _lib
from ._lib import TlibError

__all__ = [
    "ttv", "ttm", "ttt", "ttt_noalloc", "inner", "norm", "normalize", "add", "scale", "transpose", "times_tensor",
    "times_vectors", "strides", "layout_of", "empty", "TlibError", "plan", "hopm", "tucker",
    "set_autotune", "autotune_entries", "autotune_clear", "autotune_save", "autotune_load",
    "workspace_reserve", "workspace_size", "workspace_release",
]

_torch = None


def _t():
    global _torch
    if _torch is None:
        import torch
        _torch = torch
    return _torch


def _dtype_code(dt) -> int:
    torch = _t()
    m = {torch.float64: _lib.F64, torch.float32: _lib.F32, torch.bfloat16: _lib.BF16,
         torch.float16: _lib.F16}
    if dt not in m:
        raise TlibError(_lib.EDTYPE, "unsupported dtype %s" % dt)
    return m[dt]


def acc_dtype(dt):
    """Result dtype of a contraction: float64 for float64 input, float32 otherwise."""
    torch = _t()
    return torch.float64 if dt == torch.float64 else torch.float32


_plan_only = False


def _desc(x) -> _lib.TensorDesc:
    if x.device.type != "cuda" and not _plan_only:
        raise TlibError(_lib.EINVAL, "tensors must live on the GPU (got %s)" % x.device)
    return _lib.desc(x.data_ptr(), _dtype_code(x.dtype), tuple(x.shape), tuple(x.stride()))


def _stream(x) -> ctypes.c_void_p:
    if x.device.type != "cuda":
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(_t().cuda.current_stream(x.device).cuda_stream)


# ---------------------------------------------------------------- layouts

def strides(shape: Sequence[int], layout: Optional[Sequence[int]] = None) -> tuple:
    """Stride tuple from a shape and a 1-based layout tuple (Sec. 3.1
    Eq. stride.tuple.permutation), computed by the library."""
    p = len(shape)
    ext = (ctypes.c_int64 * max(1, p))(*[int(v) for v in shape])
    out = (ctypes.c_int64 * max(1, p))()
    ly = _lib.i32_array(layout) if layout is not None else None
    _lib.check(_lib.lib().tlib_strides_from_layout(p, ext, ly, out))
    return tuple(out[r] for r in range(p))


def layout_of(x) -> list:
    """1-based layout tuple of a dense tensor: modes ordered by increasing stride."""
    st = x.stride()
    return [r + 1 for r in sorted(range(x.dim()), key=lambda r: (st[r], r))]


def empty(shape: Sequence[int], layout: Optional[Sequence[int]] = None, dtype=None, device=None):
    """Uninitialised dense tensor of the given shape whose memory follows `layout`."""
    torch = _t()
    shape = tuple(int(v) for v in shape)
    return torch.empty_strided(shape, strides(shape, layout) if shape else (),
                               dtype=dtype or torch.float32, device=device or "cuda")


def _drop_mode_layout(x, m: int) -> list:
    lay = [r for r in layout_of(x) if r != m]
    return [r if r < m else r - 1 for r in lay]


# ---------------------------------------------------------------- operations

def ttv(A, b, m: int, out=None, layout=None):
    """Mode-m tensor-times-vector C = A x_m b (Sec. 5.2 Eq. ttv).  The result
    keeps A's layout minus mode m unless `layout` or `out` says otherwise."""
    shape = tuple(A.shape[: m - 1]) + tuple(A.shape[m:]) if 1 <= m <= A.dim() else ()
    if out is None:
        if layout is None and 1 <= m <= A.dim():
            layout = _drop_mode_layout(A, m)
        out = empty(shape, layout, acc_dtype(A.dtype), A.device)
    _lib.check(_lib.lib().tlib_ttv(ctypes.byref(_desc(A)), ctypes.byref(_desc(b)), int(m),
                                   ctypes.byref(_desc(out)), _stream(A)))
    return out


def ttm(A, B, m: int, out=None, layout=None):
    """Mode-m tensor-times-matrix C = A x_m B with B of shape (n', n_m)
    (Sec. 5.2 Eq. ttm).  The result keeps A's layout by default."""
    if out is None:
        shape = list(A.shape)
        if 1 <= m <= A.dim() and B.dim() == 2:
            shape[m - 1] = B.shape[0]
        out = empty(shape, layout if layout is not None else layout_of(A), acc_dtype(A.dtype), A.device)
    _lib.check(_lib.lib().tlib_ttm(ctypes.byref(_desc(A)), ctypes.byref(_desc(B)), int(m),
                                   ctypes.byref(_desc(out)), _stream(A)))
    return out


def ttt_shape(na, nb, q, phi, psi) -> tuple:
    r, s = len(na) - q, len(nb) - q
    return tuple(na[phi[k] - 1] for k in range(r)) + tuple(nb[psi[k] - 1] for k in range(s))


def ttm2(A, Ua, a: int, Ub, b: int, out=None, layout=None):
    """C = (A x_a Ua) x_b Ub in one pass (Sec. 5.2 Eq. ttm in two modes): the
    intermediate A x_a Ua is not written when the factors have at most 32
    rows.  FP32/FP64.  The result keeps A's layout by default."""
    if out is None:
        shape = list(A.shape)
        shape[a - 1] = Ua.shape[0]
        shape[b - 1] = Ub.shape[0]
        if layout is None:
            layout = layout_of(A)
        out = empty(tuple(shape), layout, A.dtype, A.device)
    _lib.check(_lib.lib().tlib_ttm2(ctypes.byref(_desc(A)), ctypes.byref(_desc(Ua)), int(a), ctypes.byref(_desc(Ub)),
                                    int(b), ctypes.byref(_desc(out)), _stream(A)))
    return out


def ttt(A, B, q: int, phi: Sequence[int], psi: Sequence[int], out=None, layout=None):
    """(q, phi, psi)-mode tensor-times-tensor (Sec. 5.2 Eq. ttt, ttt_indices)."""
    if out is None:
        shape = ttt_shape(tuple(A.shape), tuple(B.shape), q, phi, psi)
        out = empty(shape, layout, acc_dtype(A.dtype), A.device)
    _lib.check(_lib.lib().tlib_ttt(ctypes.byref(_desc(A)), ctypes.byref(_desc(B)), int(q),
                                   _lib.i32_array(phi), _lib.i32_array(psi), ctypes.byref(_desc(out)),
                                   _stream(A)))
    return out


def ttt_noalloc(A, B, q: int, phi: Sequence[int], psi: Sequence[int], out):
    """tlib_ttt_noalloc: the same contraction with its split-K scratch in the
    library's static device array (the library allocates nothing; `out` is
    required, so this call allocates nothing either)."""
    _lib.check(_lib.lib().tlib_ttt_noalloc(ctypes.byref(_desc(A)), ctypes.byref(_desc(B)), int(q),
                                           _lib.i32_array(phi), _lib.i32_array(psi), ctypes.byref(_desc(out)),
                                           _stream(A)))
    return out


def times_tensor(A, B, phi: Sequence[int], psi: Optional[Sequence[int]] = None, out=None):
    """Simple form of the paper's times_tensor (Sec. 5.2): contract A's modes
    phi with B's modes psi pairwise (psi defaults to phi); the free modes of A,
    then of B, appear in ascending order."""
    psi = list(phi) if psi is None else list(psi)
    free_a = [k for k in range(1, A.dim() + 1) if k not in phi]
    free_b = [k for k in range(1, B.dim() + 1) if k not in psi]
    return ttt(A, B, len(phi), free_a + list(phi), free_b + psi, out=out)


def inner(A, B, out=None):
    """<A, B> in FP64 (Sec. 5.2 Table 3); returns a 0-d float64 device tensor."""
    torch = _t()
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=A.device)
    _lib.check(_lib.lib().tlib_inner(ctypes.byref(_desc(A)), ctypes.byref(_desc(B)),
                                     ctypes.c_void_p(out.data_ptr()), _stream(A)))
    return out


def norm(A, out=None):
    """Frobenius norm in FP64 (Sec. 5.2 Table 3); 0-d float64 device tensor."""
    torch = _t()
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=A.device)
    _lib.check(_lib.lib().tlib_norm(ctypes.byref(_desc(A)), ctypes.c_void_p(out.data_ptr()), _stream(A)))
    return out


def normalize(A, out=None, norm_out=None, dtype=None):
    """out = A / ||A||_F with the FP64 norm written to norm_out (a 0-d float64
    device tensor), both on the device (Sec. 5.2, the normalisation of the
    higher-order power method).  out may be A itself.  Returns (out, norm_out)."""
    torch = _t()
    if norm_out is None:
        norm_out = torch.empty((), dtype=torch.float64, device=A.device)
    if out is None:
        out = empty(A.shape, layout_of(A), dtype or A.dtype, A.device)
    _lib.check(_lib.lib().tlib_normalize(ctypes.byref(_desc(A)), ctypes.c_void_p(norm_out.data_ptr()),
                                         ctypes.byref(_desc(out)), _stream(A)))
    return out, norm_out


def add(alpha: float, A, beta: float, B, out=None, layout=None):
    """C = alpha A + beta B (Sec. 5.1 Eq. transform); layouts may differ."""
    if out is None:
        out = empty(A.shape, layout if layout is not None else layout_of(A), A.dtype, A.device)
    _lib.check(_lib.lib().tlib_add(float(alpha), ctypes.byref(_desc(A)), float(beta), ctypes.byref(_desc(B)),
                                   ctypes.byref(_desc(out)), _stream(A)))
    return out


def scale(alpha: float, A, out=None, layout=None, dtype=None):
    """C = alpha A (Sec. 5.1 Eq. scaling); with another layout for C a relayout,
    with another dtype a conversion (rounded once, to nearest even)."""
    if out is None:
        out = empty(A.shape, layout if layout is not None else layout_of(A), dtype or A.dtype, A.device)
    _lib.check(_lib.lib().tlib_scale(float(alpha), ctypes.byref(_desc(A)), ctypes.byref(_desc(out)),
                                     _stream(A)))
    return out


def transpose(A, tau: Sequence[int], out=None, layout=None):
    """C = A^tau, C(i^c) = A(i^a) with i^c_r = i^a_{tau_r} (Sec. 5.2 Table 3)."""
    if out is None:
        shape = tuple(A.shape[t - 1] for t in tau)
        out = empty(shape, layout, A.dtype, A.device)
    _lib.check(_lib.lib().tlib_transpose(ctypes.byref(_desc(A)), _lib.i32_array(tau), ctypes.byref(_desc(out)),
                                         _stream(A)))
    return out


def times_vectors(A, us: Sequence, excluded: int, out=None):
    """c(i_r) = sum over every other index of A(i) * prod_{k != r} u_k(i_k),
    r = excluded (1-based): A multiplied with u_k in every mode but r (Sec. 5.2,
    tensor_times_vectors), in one pass over A with FP64 accumulation and one
    rounding to c's dtype (FP64 for FP64 A, FP32 otherwise).  us[r-1] is not
    read and may be None."""
    p = A.dim()
    if len(us) != p:
        raise TlibError(_lib.EINVAL, "times_vectors: need %d vectors (got %d)" % (p, len(us)))
    if out is None:
        out = empty((A.shape[excluded - 1],), None, acc_dtype(A.dtype), A.device)
    descs = [None if (k == excluded - 1 or us[k] is None) else _desc(us[k]) for k in range(p)]
    arr = (ctypes.POINTER(_lib.TensorDesc) * p)(
        *[ctypes.pointer(d) if d is not None else ctypes.POINTER(_lib.TensorDesc)() for d in descs])
    _lib.check(_lib.lib().tlib_times_vectors(ctypes.byref(_desc(A)), arr, int(excluded), ctypes.byref(_desc(out)),
                                             _stream(A)))
    return out


def times_vectors_chain(A, us: Sequence, excluded: int):
    """The same product as a chain of mode-k TTVs, highest mode first (the
    order the paper's tensor_times_vectors applies them), one launch per mode
    with the intermediate tensors in between."""
    X = A
    for k in range(A.dim(), 0, -1):
        if k == excluded:
            continue
        X = ttv(X, us[k - 1], k)
    return X.reshape(-1)


def plan(fn, *args, **kwargs) -> str:
    """Run `fn` (one of the operations above) in plan-only mode and return the
    library's description of the kernel it would launch.  Nothing runs on a
    device; output tensors must be supplied by the caller."""
    global _plan_only
    L = _lib.lib()
    L.tlib_set_plan_only(1)
    _plan_only = True
    try:
        fn(*args, **kwargs)
    finally:
        L.tlib_set_plan_only(0)
        _plan_only = False
    return L.tlib_last_plan().decode()


_AUTOTUNE = {"off": 0, "on": 1, "frozen": 2}


def set_autotune(mode: str) -> str:
    """Kernel-choice autotuning for ttm/ttt: "off" (planner rules), "on" (tune
    each new call shape on its first call, which then synchronises its
    stream) or "frozen" (use stored choices only).  Returns the previous mode."""
    prev = _lib.lib().tlib_set_autotune(_AUTOTUNE[mode])
    return {v: k for k, v in _AUTOTUNE.items()}[prev]


def autotune_entries() -> int:
    return int(_lib.lib().tlib_autotune_entries())


def autotune_clear() -> None:
    _lib.lib().tlib_autotune_clear()


def autotune_save(path: str) -> None:
    """Write the autotuning table (one "<choice> <call shape>" line per entry)."""
    _lib.check(_lib.lib().tlib_autotune_save(str(path).encode()))


def autotune_load(path: str) -> None:
    """Add the entries of a saved autotuning table."""
    _lib.check(_lib.lib().tlib_autotune_load(str(path).encode()))


def _cur_stream(device=None) -> ctypes.c_void_p:
    torch = _t()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_reserve(nbytes: int, device=None) -> None:
    """Make the current stream's workspace at least `nbytes` (not while the
    stream is capturing a graph)."""
    _lib.check(_lib.lib().tlib_workspace_reserve(_cur_stream(device), int(nbytes)))


def workspace_size(device=None) -> int:
    """Bytes of the current stream's workspace (0 before its first use)."""
    return int(_lib.lib().tlib_workspace_size(_cur_stream(device)))


def workspace_release(device=None) -> None:
    """Wait for the current stream and free its workspace."""
    _lib.check(_lib.lib().tlib_workspace_release(_cur_stream(device)))


from .drivers import hopm, tucker  # noqa: E402
