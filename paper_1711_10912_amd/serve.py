"""Serving interface over the native request server (tlib_server_* in the C ABI).

Requests (TTV, TTM, TTT of uneven order and shape, each in its own dtype)
are submitted as they arrive and refer to operands that stay resident on the
device.  The library's scheduler thread admits them in arrival order while a
stream slot is free and the result fits in the output arena (the HBM budget
for results), fuses consecutive small TTV/TTM/TTT requests into one grouped launch
replayed from a per-slot HIP graph, and times completions with GPU events.
This module only builds descriptors and forwards calls.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional

from . import _lib

_OPS = {"ttv": 0, "ttm": 1, "ttt": 2}


class Server:
    def __init__(self, hbm_budget: int = 8 << 30, slots: int = 4, device: int = 0, group_macs: int = 1 << 21,
                 group_max: int = 64, keep_results: bool = False):
        import torch

        self.torch = torch
        self.L = _lib.lib()
        self.keep = keep_results
        self.dev = torch.device("cuda", device)
        torch.cuda.set_device(self.dev)
        self.h = self.L.tlib_server_create(device, int(hbm_budget), slots, group_max, int(group_macs),
                                           1 if keep_results else 0)
        if not self.h:
            raise _lib.TlibError(_lib.ENOMEM, "tlib_server_create failed")
        self.outputs: Dict[int, object] = {}
        self._descs: Dict[tuple, object] = {}
        self._keep_alive = []

    def _desc(self, t):
        import paper_1711_10912_amd as T
        key = (t.data_ptr(), tuple(t.shape), tuple(t.stride()), t.dtype)
        d = self._descs.get(key)
        if d is None:
            d = T._desc(t)
            self._descs[key] = d
        return d

    def _out_desc(self, op, a, b, mode, q, phi, psi):
        import paper_1711_10912_amd as T
        acc = T.acc_dtype(a.dtype)
        if op == "ttv":
            shape = tuple(a.shape[: mode - 1]) + tuple(a.shape[mode:])
            lay = [r if r < mode else r - 1 for r in T.layout_of(a) if r != mode]
        elif op == "ttm":
            shape = list(a.shape)
            shape[mode - 1] = b.shape[0]
            lay = T.layout_of(a)
        else:
            shape = T.ttt_shape(tuple(a.shape), tuple(b.shape), q, phi, psi)
            lay = None
        if self.keep:
            out = T.empty(shape, lay, acc, self.dev)
            return out, T._desc(out)
        code = T._dtype_code(acc)
        return None, _lib.desc(0, code, shape, None, lay)

    def submit(self, op: str, a, b, mode: int = 0, q: int = 0, phi=(), psi=(), out=None) -> int:
        """Queue one request; `out` (a device tensor of the result's shape and
        dtype) makes the result caller-owned instead of placed by the server."""
        da, db = self._desc(a), self._desc(b)
        if out is not None:
            import paper_1711_10912_amd as T
            dc = T._desc(out)
        else:
            out, dc = self._out_desc(op, a, b, mode, q, phi, psi)
        rid = ctypes.c_int64(-1)
        pa = _lib.i32_array(phi) if op == "ttt" else None
        pb = _lib.i32_array(psi) if op == "ttt" else None
        rc = self.L.tlib_server_submit(self.h, _OPS[op], ctypes.byref(da), ctypes.byref(db), int(mode), int(q),
                                       pa, pb, ctypes.byref(dc), ctypes.byref(rid))
        _lib.check(rc)
        if out is not None and self.keep:
            self.outputs[rid.value] = out
        return rid.value

    def drain(self, timeout: float = 600.0):
        if self.L.tlib_server_drain(self.h, float(timeout)) != _lib.OK:
            raise TimeoutError("server did not drain")

    def result(self, rid: int):
        """Output tensor of a completed request (keep_results servers)."""
        err = ctypes.c_int32(0)
        d = _lib.TensorDesc()
        _lib.check(self.L.tlib_server_result(self.h, rid, ctypes.byref(d), ctypes.byref(err)))
        if err.value:
            raise _lib.TlibError(err.value, "request %d failed" % rid)
        return self.outputs[rid]

    def stats(self) -> dict:
        st = _lib.ServerStats()
        _lib.check(self.L.tlib_server_stats(self.h, ctypes.byref(st)))
        return {"requests": st.completed - st.errors, "errors": st.errors, "grouped": st.grouped,
                "p50_ms": st.p50_s * 1e3, "p99_ms": st.p99_s * 1e3, "mean_ms": st.mean_s * 1e3,
                "req_per_s": st.req_per_s}

    def reset_stats(self):
        self.L.tlib_server_reset_stats(self.h)

    def close(self):
        if self.h:
            self.drain()
            self.L.tlib_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
