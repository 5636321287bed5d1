"""Serving loop for contraction requests on one GPU.

Requests (TTV, TTM, TTT of uneven order and shape, tagged FP32 or BF16) are
submitted as they arrive and refer to operands kept resident on the device.
A scheduler thread admits them while the HBM budget (resident operands plus
outputs in flight) and a free slot allow, so requests that arrive while
others run join as soon as memory and slots free up (continuous batching).
Each slot is a HIP stream; work on different slots overlaps on the device.

Small TTV/TTM requests are fused: up to `group_max` of them are planned into
one work table (tlib_batch_plan) and run by one grouped launch, replayed from
a per-slot HIP graph captured once (the graph's kernel reads the table from a
fixed device buffer whose contents change per batch).  A request's kernel
depends only on the request itself (small TTV/TTM always take the grouped
kernel, everything else the regular entry point), so its result is the same
alone and in any mix.

Completion times come from GPU events referenced to the host clock, so
latency = completion - arrival is not blurred by polling.
"""
from __future__ import annotations

import collections
import ctypes
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

from . import _lib


@dataclass
class Job:
    rid: int
    op: str                      # "ttv" | "ttm" | "ttt"
    a: object                    # input tensor
    b: object                    # vector / matrix / second tensor
    mode: int = 0                # ttv / ttm
    q: int = 0                   # ttt
    phi: tuple = ()
    psi: tuple = ()
    arrival: float = 0.0
    out: object = None
    out_bytes: int = 0
    macs: int = 0
    grouped: bool = False
    t_done: float = 0.0
    error: Optional[str] = None


class Server:
    def __init__(self, hbm_budget: int = 64 << 30, slots: int = 4, device: str = "cuda:0",
                 group_macs: int = 1 << 21, group_max: int = 64, grid: int = 1024,
                 keep_results: bool = False, use_graphs: bool = True):
        import torch

        self.torch = torch
        self.dev = torch.device(device)
        self.budget = int(hbm_budget)
        self.group_macs = int(group_macs)
        self.group_max = int(group_max)
        self.grid = int(grid)
        self.keep = keep_results
        self.L = _lib.lib()
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]  # default priority
        self.busy: List[Optional[tuple]] = [None] * slots
        self.table_bytes = int(self.L.tlib_batch_table_bytes(self.group_max))
        self.tab_host = [torch.empty(self.table_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(slots)]
        self.tab_dev = [torch.zeros(self.table_bytes, dtype=torch.uint8, device=self.dev) for _ in range(slots)]
        self.graphs: List[Optional[object]] = [None] * slots
        if use_graphs:
            self._capture()
        self.operands: Dict[int, object] = {}
        self.resident = 0
        self.in_flight = 0
        self.pending: collections.deque = collections.deque()
        self.completed: List[Job] = []
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.next_id = 0
        self.stop_flag = False
        self.thread: Optional[threading.Thread] = None
        # time reference: a GPU event whose host time is known
        torch.cuda.synchronize(self.dev)
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.streams[0])
        torch.cuda.synchronize(self.dev)
        self.t_ref = time.perf_counter()

    # ------------------------------------------------------------ set-up
    def _capture(self):
        torch = self.torch
        for s, st in enumerate(self.streams):
            g = torch.cuda.CUDAGraph()
            # an empty but valid table while capturing (nothing executes during capture)
            with torch.cuda.graph(g, stream=st):
                rc = self.L.tlib_batch_run(ctypes.c_void_p(self.tab_dev[s].data_ptr()), self.grid,
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            _lib.check(rc)
            self.graphs[s] = g

    def register(self, tensor) -> int:
        """Keep an operand resident; returns its id.  Counts against the budget."""
        with self.lock:
            oid = len(self.operands)
            self.operands[oid] = tensor
            self.resident += tensor.numel() * tensor.element_size()
            return oid

    # ------------------------------------------------------------ client side
    def submit(self, op: str, a, b, mode: int = 0, q: int = 0, phi=(), psi=(), arrival: Optional[float] = None) -> int:
        import paper_1711_10912_amd as T

        a = self.operands[a] if isinstance(a, int) else a
        b = self.operands[b] if isinstance(b, int) else b
        job = Job(rid=-1, op=op, a=a, b=b, mode=mode, q=q, phi=tuple(phi), psi=tuple(psi),
                  arrival=time.perf_counter() if arrival is None else arrival)
        esz = 8 if a.dtype == self.torch.float64 else 4
        if op == "ttv":
            outs = a.numel() // a.shape[mode - 1]
            job.macs = a.numel()
        elif op == "ttm":
            outs = a.numel() // a.shape[mode - 1] * b.shape[0]
            job.macs = a.numel() * b.shape[0]
        else:
            shp = T.ttt_shape(tuple(a.shape), tuple(b.shape), q, job.phi, job.psi)
            outs = 1
            for v in shp:
                outs *= v
            k = 1
            for t in range(q):
                k *= a.shape[job.phi[a.dim() - q + t] - 1]
            job.macs = outs * k
        job.out_bytes = outs * esz
        job.grouped = op in ("ttv", "ttm") and job.macs <= self.group_macs
        with self.cv:
            job.rid = self.next_id
            self.next_id += 1
            self.pending.append(job)
            self.cv.notify()
        return job.rid

    def start(self):
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def drain(self, timeout: float = 600.0):
        t0 = time.perf_counter()
        while True:
            with self.lock:
                idle = not self.pending and all(x is None for x in self.busy)
            if idle:
                return
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(0.0005)

    def stop(self):
        self.drain()
        with self.cv:
            self.stop_flag = True
            self.cv.notify()
        if self.thread:
            self.thread.join()

    def stats(self) -> dict:
        lat = sorted(j.t_done - j.arrival for j in self.completed if not j.error)
        if not lat:
            return {}
        first = min(j.arrival for j in self.completed)
        last = max(j.t_done for j in self.completed)
        pick = lambda f: lat[min(len(lat) - 1, int(f * len(lat)))]
        return {"requests": len(lat), "p50_ms": pick(0.50) * 1e3, "p99_ms": pick(0.99) * 1e3,
                "mean_ms": sum(lat) / len(lat) * 1e3, "req_per_s": len(lat) / (last - first),
                "grouped": sum(1 for j in self.completed if j.grouped),
                "errors": sum(1 for j in self.completed if j.error)}

    # ------------------------------------------------------------ scheduler
    def _ev_time(self, ev) -> float:
        return self.t_ref + self.ref.elapsed_time(ev) * 1e-3

    def _retire(self):
        for s, unit in enumerate(self.busy):
            if unit is not None and unit[0].query():
                ev, jobs = unit
                t = self._ev_time(ev)
                for j in jobs:
                    j.t_done = t
                    self.in_flight -= j.out_bytes
                    if not self.keep:
                        j.out = None
                        j.a = j.b = None
                self.completed.extend(jobs)
                self.busy[s] = None

    def _alloc(self, job: Job):
        import paper_1711_10912_amd as T
        torch = self.torch
        acc = T.acc_dtype(job.a.dtype)
        if job.op == "ttv":
            m = job.mode
            shape = tuple(job.a.shape[: m - 1]) + tuple(job.a.shape[m:])
            lay = [r if r < m else r - 1 for r in T.layout_of(job.a) if r != m]
            job.out = T.empty(shape, lay, acc, self.dev)
        elif job.op == "ttm":
            shape = list(job.a.shape)
            shape[job.mode - 1] = job.b.shape[0]
            job.out = T.empty(shape, T.layout_of(job.a), acc, self.dev)
        else:
            job.out = T.empty(T.ttt_shape(tuple(job.a.shape), tuple(job.b.shape), job.q, job.phi, job.psi),
                              None, acc, self.dev)

    def _launch_single(self, s: int, job: Job):
        import paper_1711_10912_amd as T
        torch = self.torch
        with torch.cuda.stream(self.streams[s]):
            try:
                if job.op == "ttv":
                    T.ttv(job.a, job.b, job.mode, out=job.out)
                elif job.op == "ttm":
                    T.ttm(job.a, job.b, job.mode, out=job.out)
                else:
                    T.ttt(job.a, job.b, job.q, job.phi, job.psi, out=job.out)
            except _lib.TlibError as e:
                job.error = str(e)

    def _launch_group(self, s: int, jobs: List[Job]) -> List[Job]:
        """Plan and launch a grouped batch; returns jobs that must run singly."""
        import paper_1711_10912_amd as T
        torch = self.torch
        n = len(jobs)
        reqs = (_lib.Request * n)()
        keep = []
        for i, j in enumerate(jobs):
            da, db, dc = T._desc(j.a), T._desc(j.b), T._desc(j.out)
            keep.append((da, db, dc))
            reqs[i].op = 0 if j.op == "ttv" else 1
            reqs[i].mode = j.mode
            reqs[i].A = ctypes.pointer(da)
            reqs[i].B = ctypes.pointer(db)
            reqs[i].C = ctypes.pointer(dc)
        units = ctypes.c_int64(0)
        bad = ctypes.c_int32(-1)
        rc = self.L.tlib_batch_plan(reqs, n, ctypes.c_void_p(self.tab_host[s].data_ptr()), self.table_bytes,
                                    ctypes.byref(units), ctypes.byref(bad))
        if rc != _lib.OK:
            if bad.value >= 0:
                # split off the request the grouped kernel cannot take
                rest = jobs[: bad.value] + jobs[bad.value + 1:]
                single = [jobs[bad.value]]
                return single + (self._launch_group(s, rest) if rest else [])
            raise _lib.TlibError(rc, self.L.tlib_last_error().decode())
        nbytes = int(self.L.tlib_batch_table_bytes(n))
        with torch.cuda.stream(self.streams[s]):
            self.tab_dev[s][:nbytes].copy_(self.tab_host[s][:nbytes], non_blocking=True)
            if self.graphs[s] is not None:
                self.graphs[s].replay()
            else:
                _lib.check(self.L.tlib_batch_run(ctypes.c_void_p(self.tab_dev[s].data_ptr()), self.grid,
                                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return []

    def _admit(self) -> bool:
        """Admit one unit of work onto a free slot; False if nothing could start."""
        torch = self.torch
        free = [s for s, u in enumerate(self.busy) if u is None]
        if not free or not self.pending:
            return False
        s = free[0]
        head = self.pending[0]
        room = self.budget - self.resident - self.in_flight
        if head.out_bytes > room:
            return False  # wait for outputs in flight to retire (FIFO admission)
        jobs = [self.pending.popleft()]
        room -= head.out_bytes
        if head.grouped:
            while (self.pending and len(jobs) < self.group_max and self.pending[0].grouped
                   and self.pending[0].out_bytes <= room):
                j = self.pending.popleft()
                room -= j.out_bytes
                jobs.append(j)
        for j in jobs:
            self._alloc(j)
            self.in_flight += j.out_bytes
        if head.grouped:
            singles = self._launch_group(s, jobs)
            for j in singles:
                self._launch_single(s, j)
        else:
            self._launch_single(s, jobs[0])
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.streams[s])
        self.busy[s] = (ev, jobs)
        return True

    def _loop(self):
        torch = self.torch
        torch.cuda.set_device(self.dev)
        while True:
            with self.cv:
                if self.stop_flag:
                    return
                self._retire()
                started = False
                while self._admit():
                    started = True
                if not started and not self.pending and all(u is None for u in self.busy):
                    self.cv.wait(timeout=0.01)
                    continue
            if not started:
                time.sleep(0.00005)
