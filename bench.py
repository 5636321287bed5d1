#!/usr/bin/env python3
"""Throughput of the TTV / TTM / TTT contraction path on one MI355X.

One step = one pass of the whole path over the order-p sweep (p = 3..7 at
about 2^26 elements: 406^3, 90^4, 36^5, 20^6, 13^7), in first- and last-order
layout, FP64 and FP32:
  * TTV in every mode q (a dense n_q vector),
  * TTM in every mode q with m x n_q matrices, m in {16, 64, 256},
  * inner product and Frobenius norm (FP64 accumulation) and C = A + B on
    every sweep tensor,
plus the general TTT case: A (96,80,64,48) in first-order, last-order and
(3,1,4,2) layout times B (64,48,120), contracting A{3,4} with B{1,2}, in FP32,
BF16 and FP16 (FP32 accumulation), and the outer product (TTT with no
contracted pair) of A (512,128) and B (64,40) in FP64 and FP32.

After the timed steps the served mixed request stream is measured (closed
loop, open loop at 0.5 / 0.8 / 0.95 of capacity, the plain per-call FP64 path
on the same requests) and every served result is checked against the FP64
oracle; then the oracle itself is timed on a sample of the sweep.

Inputs are resident in HBM before timing starts; each call alternates between
two copies of its input tensor (several for the TTT operands) so that the
256 MB Infinity Cache cannot serve a tensor the previous call just read.
`value` is whole-step algorithmic throughput: the sum over all calls of the
bytes the definitions require (every input read once, every output written
once) divided by the step time.  Per-launch durations come from HIP events on
the launch stream; the roofline object describes the kernel with the largest
share of the step time.
"""
import argparse
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TTM/TTT TFLOP/s & TTV GB/s vs roofline; served p50/p99 latency, req/s"
HERE = os.path.dirname(os.path.abspath(__file__))
# kernel choices of the sweep's call shapes, tuned on MI355X (tlib_autotune_save format)
TUNING_TABLE = os.path.join(HERE, "paper_1711_10912_amd", "tuning", "mi355x_sweep.txt")
PEAK_HBM = 8.0e12
PEAK_FLOPS = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2516.6e12, "f16": 2516.6e12}
ESZ = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
SWEEP = {3: 406, 4: 90, 5: 36, 6: 20, 7: 13}
TTM_M = (16, 64, 256)


class Case:
    __slots__ = ("name", "family", "kernel", "bytes", "flops", "dtype", "fn", "ms", "planfn")

    def __init__(self, name, family, bytes_, flops, dtype, fn):
        self.name, self.family, self.bytes, self.flops, self.dtype, self.fn = name, family, bytes_, flops, dtype, fn
        self.kernel = None
        self.planfn = None
        self.ms = []

    def ideal_s(self):
        return max(self.bytes / PEAK_HBM, self.flops / PEAK_FLOPS[self.dtype])


def _kernel_label(plan: str) -> str:
    """Short kernel name from the library's plan string (op, kernel, dtype, tile/vec)."""
    w = plan.split()
    kv = dict(t.split("=", 1) for t in w[2:] if "=" in t)
    lab = "%s %s %s" % (w[0], w[1], kv.get("dtype", "?"))
    if "tile" in kv:
        lab += " tile=" + kv["tile"]
    if "vec" in kv:
        lab += " vec=" + kv["vec"]
    if "mode" in kv:
        lab += " mode=" + kv["mode"]
    return lab


def _plan_later(T, fn, *args, **kw):
    """The library's plan for a call, taken when the kernel label is needed
    (after autotuning has settled the choice)."""
    return lambda: T.plan(fn, *args, **kw)


def build_cases(T, torch, dev, quick=False):
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    gen = torch.Generator(device=dev)
    gen.manual_seed(171110912 + 1)
    cases = []
    keep = []  # tensors referenced by the closures
    dtypes = ("f64", "f32")
    ps = (3, 7) if quick else tuple(SWEEP)
    # one output buffer per output dtype, sized for the largest TTM result
    max_out = max(SWEEP[p] ** p // SWEEP[p] * max(TTM_M) for p in ps)
    outbuf = {d: torch.empty(max_out, dtype=tdt[d], device=dev) for d in dtypes}

    def out_view(d, shape, layout):
        st = T.strides(shape, layout)
        return torch.as_strided(outbuf[d], shape, st)

    rot = 0  # running call index: consecutive calls never read the same copy of a tensor
    for d in dtypes:
        s = ESZ[d]
        for p in ps:
            n = SWEEP[p]
            shape = (n,) * p
            N = n ** p
            for lname, lay in (("first", list(range(1, p + 1))), ("last", list(range(p, 0, -1)))):
                As = []
                for c in range(2):
                    A = T.empty(shape, lay, tdt[d], dev)
                    A.copy_(torch.rand(shape, generator=gen, device=dev, dtype=tdt[d]).mul_(2).sub_(1))
                    As.append(A)
                keep.extend(As)
                b = torch.rand(n, generator=gen, device=dev, dtype=tdt[d]).mul_(2).sub_(1)
                Bm = {m: torch.rand(m, n, generator=gen, device=dev, dtype=tdt[d]).mul_(2).sub_(1) for m in TTM_M}
                keep.append(b)
                keep.extend(Bm.values())
                for q in range(1, p + 1):
                    A = As[rot % 2]
                    rot += 1
                    cshape = shape[: q - 1] + shape[q:]
                    clay = [r if r < q else r - 1 for r in lay if r != q]
                    C = out_view(d, cshape, clay)
                    cases.append(Case("ttv p=%d %s q=%d %s" % (p, lname, q, d), "ttv", s * (N + n + N // n), 2 * N, d,
                                      (lambda A=A, b=b, q=q, C=C: T.ttv(A, b, q, out=C))))
                    cases[-1].planfn = _plan_later(T, T.ttv, A, b, q, out=C)
                for q in range(1, p + 1):
                    for m in TTM_M:
                        A = As[rot % 2]
                        rot += 1
                        cshape = shape[: q - 1] + (m,) + shape[q:]
                        C = out_view(d, cshape, lay)
                        nb = s * (N + m * n) + s * (N // n * m)
                        cases.append(Case("ttm p=%d %s q=%d m=%d %s" % (p, lname, q, m, d), "ttm", nb, 2 * N * m, d,
                                          (lambda A=A, B=Bm[m], q=q, C=C: T.ttm(A, B, q, out=C))))
                        cases[-1].planfn = _plan_later(T, T.ttm, A, Bm[m], q, out=C)
                # inner / norm / add on the sweep tensor (FP64 accumulation)
                res = torch.empty((), dtype=torch.float64, device=dev)
                cases.append(Case("inner p=%d %s %s" % (p, lname, d), "inner", 2 * s * N, 2 * N, "f64",
                                  (lambda A=As[0], B=As[1], r=res: T.inner(A, B, out=r))))
                cases[-1].planfn = _plan_later(T, T.inner, As[0], As[1], out=res)
                cases.append(Case("norm p=%d %s %s" % (p, lname, d), "norm", s * N, 2 * N, "f64",
                                  (lambda A=As[1], r=res: T.norm(A, out=r))))
                cases[-1].planfn = _plan_later(T, T.norm, As[1], out=res)
                C = out_view(d, shape, lay)
                cases.append(Case("add p=%d %s %s" % (p, lname, d), "add", 3 * s * N, 2 * N, d,
                                  (lambda A=As[0], B=As[1], C=C: T.add(1.0, A, 1.0, B, out=C))))
                cases[-1].planfn = _plan_later(T, T.add, 1.0, As[0], 1.0, As[1], out=C)
                keep.append(res)

    # outer product (q = 0): A (512,128) x B (64,40) -> C (512,128,64,40), a
    # write stream of 167.8M outputs
    for d in dtypes:
        oa, ob = (512, 128), (64, 40)
        A = torch.rand(oa, generator=gen, device=dev, dtype=tdt[d]).mul_(2).sub_(1)
        B = torch.rand(ob, generator=gen, device=dev, dtype=tdt[d]).mul_(2).sub_(1)
        keep.extend((A, B))
        C = out_view(d, oa + ob, None)
        Mo, No = 512 * 128, 64 * 40
        cases.append(Case("outer (512,128)x(64,40) %s" % d, "outer", ESZ[d] * (Mo + No + Mo * No), Mo * No, d,
                          (lambda A=A, B=B, C=C: T.ttt(A, B, 0, (1, 2), (1, 2), out=C))))
        cases[-1].planfn = _plan_later(T, T.ttt, A, B, 0, (1, 2), (1, 2), out=C)

    # TTT: A (96,80,64,48) x B (64,48,120), A{3,4} <-> B{1,2}
    na, nbs = (96, 80, 64, 48), (64, 48, 120)
    phi, psi = (1, 2, 3, 4), (3, 1, 2)
    Mt, Nt, Kt = 96 * 80, 120, 64 * 48
    for d in ("f32", "bf16", "f16"):
        for lname, lay in (("first", (1, 2, 3, 4)), ("last", (4, 3, 2, 1)), ("perm3142", (3, 1, 4, 2))):
            sets = []
            nsets = 6 if not quick else 2
            for c in range(nsets):
                # the last set is the x1e3 variant that exercises range
                sc = 1e3 if c == nsets - 1 else 1.0
                A = T.empty(na, lay, tdt[d], dev)
                A.copy_(torch.randn(na, generator=gen, device=dev, dtype=torch.float32).mul_(sc).to(tdt[d]))
                B = torch.randn(nbs, generator=gen, device=dev, dtype=torch.float32).mul_(sc).to(tdt[d])
                B = T.empty(nbs, None, tdt[d], dev).copy_(B)
                C = T.empty((96, 80, 120), None, torch.float32, dev)
                sets.append((A, B, C))
            keep.extend(sets)
            nbytes = ESZ[d] * (96 * 80 * 64 * 48 + 64 * 48 * 120) + 4 * Mt * Nt
            for c, (A, B, C) in enumerate(sets):
                tag = "x1e3" if c == len(sets) - 1 else "set=%d" % c
                cases.append(Case("ttt A=%s %s %s" % (lname, d, tag), "ttt", nbytes, 2 * Mt * Nt * Kt, d,
                                  (lambda A=A, B=B, C=C: T.ttt(A, B, 2, phi, psi, out=C))))
                cases[-1].planfn = _plan_later(T, T.ttt, A, B, 2, phi, psi, out=C)
    return cases, keep, outbuf


def hbm_ceilings(nbytes=4 << 30, reps=10):
    """Plain HBM streams timed with events on 4 GiB buffers: torch's fill_
    (write only), copy_ (read + write) and sum (read only), FP32 and FP64, in
    GB/s of bytes moved.  These are practical ceilings on this GPU for the
    kernels' write-, copy- and read-dominated regimes (the published 8 TB/s
    stays the roofline peak)."""
    import torch

    out = {"bytes": nbytes, "reps": reps}
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        n = nbytes // torch.tensor([], dtype=dt).element_size()
        x = torch.ones(n, dtype=dt, device="cuda:0")
        y = torch.empty_like(x)
        for what, fn, moved in (("fill", lambda: y.fill_(2.0), nbytes), ("copy", lambda: y.copy_(x), 2 * nbytes),
                                ("sum", lambda: x.sum(), nbytes)):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            out["%s_%s_GBps" % (what, name)] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        del x, y
        torch.cuda.empty_cache()
    return out


def recorded_traffic(label):
    """HBM bytes per launch for kernel `label` from a committed rocprofv3
    summary under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by the same
    counter on a plain copy of known size), or None when no summary covers the
    kernel or the kernel sources changed since the counters were taken."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1711_10912_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("#", "-", "|", " ")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("traffic_kernel") == label and kv.get("csrc_sha256") == sha:
            return float(kv["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def served_workload(n_req, n_tensors, n_mats, cap, seed_case=0, device="cuda:0", rate=1e9):
    """Materialise the served-stream workload on the device: a resident pool of
    tensors (FP32 and BF16 copies, layouts as drawn), factor matrices, per-request
    TTT operands and the request list (synth.served_stream)."""
    import torch

    import paper_1711_10912_amd as T
    import synth

    g = synth.rng(4, 10 + seed_case)
    pools = synth.served_pools(n_tensors=n_tensors, n_mats=n_mats, cap=cap, g=g)
    reqs = synth.served_stream(pools, n_req, rate, cap=cap, g=synth.rng(4, 20 + seed_case))
    gen = torch.Generator(device=device)
    gen.manual_seed(171110912 + 4 + seed_case)

    def make(shape, layout, dt):
        t = T.empty(shape, layout, dt, device)
        t.copy_(torch.rand(tuple(shape), generator=gen, device=device, dtype=torch.float32).mul_(2).sub_(1))
        return t

    tens = {}
    used = {r.a_id for r in reqs}
    for i in sorted(used):
        shape, lay = pools.tensors[i]
        t32 = make(shape, list(lay), torch.float32)
        tens[i] = {"f32": t32, "bf16": T.scale(1.0, t32, dtype=torch.bfloat16)}
    mats = {}
    for r in reqs:
        if r.op == "ttm" and r.mat_id not in mats:
            mm, nn = pools.matrices[r.mat_id]
            m32 = make((mm, nn), None, torch.float32)
            mats[r.mat_id] = {"f32": m32, "bf16": T.scale(1.0, m32, dtype=torch.bfloat16)}
    vecs = {}
    tttb = {}
    for r in reqs:
        shape = pools.tensors[r.a_id][0]
        if r.op == "ttv":
            n = shape[r.mode - 1]
            if n not in vecs:
                v32 = make((n,), None, torch.float32)
                vecs[n] = {"f32": v32, "bf16": T.scale(1.0, v32, dtype=torch.bfloat16)}
        elif r.op == "ttt":
            b32 = make(r.b_shape, list(r.b_layout), torch.float32)
            tttb[r.rid] = {"f32": b32, "bf16": T.scale(1.0, b32, dtype=torch.bfloat16)}

    def operands(r, dt=None):
        dt = dt or r.dtype
        a = tens[r.a_id][dt]
        if r.op == "ttv":
            return a, vecs[pools.tensors[r.a_id][0][r.mode - 1]][dt]
        if r.op == "ttm":
            return a, mats[r.mat_id][dt]
        return a, tttb[r.rid][dt]

    torch.cuda.synchronize()
    return reqs, operands


SERVE_RATES = (0.5, 0.8, 0.95)  # open-loop arrival rates as fractions of the closed-loop capacity
SERVE_TIE_EVERY = 50  # in the headline open-loop run every 50th result is kept (caller-owned output)
CHECK_MACS = 1 << 19  # oracle multiply-adds per served result in the offline check
# kernel choices for the served stream's shape classes, tuned on MI355X
SERVED_TABLE = os.path.join(HERE, "paper_1711_10912_amd", "tuning", "mi355x_served.txt")


def served_measure(n_req, slots=4, budget=64 << 30, check=True, log=None, table=SERVED_TABLE, tune_save=""):
    """The served mixed stream on the native server: closed-loop capacity,
    open-loop Poisson arrivals at 0.5 / 0.8 / 0.95 x that capacity (p50/p99
    latency, arrival to completion), the plain per-call synchronous FP64 path
    on the same requests, and (after all timing) every served result checked
    against the FP64 oracle."""
    import numpy as np
    import torch

    import paper_1711_10912_amd as T
    from paper_1711_10912_amd.serve import Server

    log = log or (lambda *a: print(*a, file=sys.stderr, flush=True))
    t0 = time.perf_counter()
    reqs, operands = served_workload(n_req, 1024, 256, 1 << 24)
    log("serve: workload ready (%d requests, %.1f s)" % (len(reqs), time.perf_counter() - t0))

    def run(srv, subset, rate=None, outs=None):
        srv.reset_stats()
        t_start = time.perf_counter()
        arr = 0.0
        g = np.random.default_rng(171110912 + 5)
        for r in subset:
            a, b = operands(r)
            if rate:
                arr += g.exponential(1.0 / rate)
                while time.perf_counter() - t_start < arr:
                    pass
            out = outs.get(r.rid) if outs else None
            srv.submit(r.op, a, b, mode=r.mode, q=r.q, phi=r.phi, psi=r.psi, out=out)
        srv.drain()
        return srv.stats()

    srv = Server(hbm_budget=budget, slots=slots)
    # the served stream runs on its own kernel table only; the caller's
    # entries (the sweep's) come back for the plain per-call baseline below
    kept = None
    if T.autotune_entries():
        fd, kept = tempfile.mkstemp(suffix=".txt")
        os.close(fd)
        T.autotune_save(kept)
    T.autotune_clear()
    tuning = {"table": None, "mode": "off"}
    if tune_save:
        # one untimed pass with autotuning on: every new shape class is tuned
        # at its first request, then the table is saved and frozen
        T.set_autotune("on")
        t1 = time.perf_counter()
        run(srv, reqs)
        T.autotune_save(tune_save)
        T.set_autotune("frozen")
        tuning = {"table": os.path.relpath(tune_save, HERE), "mode": "frozen",
                  "tuned_in_s": round(time.perf_counter() - t1, 1)}
        log("serve: tuned %d entries in %.1f s" % (T.autotune_entries(), time.perf_counter() - t1))
    elif table and os.path.exists(table):
        T.autotune_load(table)
        T.set_autotune("frozen")
        tuning = {"table": os.path.relpath(table, HERE), "mode": "frozen"}
    tuning["entries"] = T.autotune_entries()
    run(srv, reqs[:300])  # warm-up: kernels, graphs, arena
    closed = run(srv, reqs)
    mu = closed["req_per_s"]
    log("serve: closed loop %.0f req/s" % mu)
    # results kept from the headline (0.8 x) run, compared bitwise with the
    # checked results below
    tie = {r.rid: _result_tensor(T, r, operands) for r in reqs if r.rid % SERVE_TIE_EVERY == 0}
    opened = {}
    for f in SERVE_RATES:
        st = run(srv, reqs, rate=f * mu, outs=tie if f == 0.8 else None)
        opened["%.2f" % f] = st
        log("serve: open loop %.2f x: p50 %.3f ms p99 %.3f ms, %.0f req/s" % (f, st["p50_ms"], st["p99_ms"],
                                                                             st["req_per_s"]))
    check_res = None
    if check:
        check_res = served_check(srv, reqs, operands, tie, log)
    srv.close()
    del tie
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    T.autotune_clear()
    if kept:
        T.autotune_load(kept)
        os.remove(kept)

    # plain per-call FP64: the same requests, one synchronous call each
    cache = {}

    def f64(t):
        key = t.data_ptr()
        if key not in cache:
            cache[key] = T.scale(1.0, t, dtype=torch.float64)
        return cache[key]

    ops64 = [(r, f64(operands(r, "f32")[0]), f64(operands(r, "f32")[1])) for r in reqs]
    torch.cuda.synchronize()
    lat = []
    t_s = time.perf_counter()
    for r, a, b in ops64:
        t1 = time.perf_counter()
        if r.op == "ttv":
            T.ttv(a, b, r.mode)
        elif r.op == "ttm":
            T.ttm(a, b, r.mode)
        else:
            T.ttt(a, b, r.q, r.phi, r.psi)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    plain_rps = len(ops64) / (time.perf_counter() - t_s)
    del ops64, cache
    torch.cuda.empty_cache()
    lat.sort()
    log("serve: plain FP64 per call %.0f req/s" % plain_rps)
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    return {
        "requests": len(reqs),
        "slots": slots,
        "output_budget_GB": budget >> 30,
        "closed_loop": rnd(closed),
        "open_loop": {k: rnd(v) for k, v in opened.items()},
        "headline_rate": "0.80",
        "kernel_choice": tuning,
        "plain_fp64_per_call": {"requests": len(reqs), "req_per_s": round(plain_rps, 1),
                                "p50_ms": round(lat[len(lat) // 2] * 1e3, 3),
                                "p99_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))] * 1e3, 3)},
        "speedup_vs_plain_fp64": round(mu / plain_rps, 2),
        "errors_vs_oracle": check_res,
    }


def _result_tensor(T, r, operands):
    """A device tensor for request r's result (the layout the server uses)."""
    import torch

    a, b = operands(r)
    acc = T.acc_dtype(a.dtype)
    if r.op == "ttv":
        shape = tuple(a.shape[: r.mode - 1]) + tuple(a.shape[r.mode:])
        lay = [k if k < r.mode else k - 1 for k in T.layout_of(a) if k != r.mode]
    elif r.op == "ttm":
        shape = list(a.shape)
        shape[r.mode - 1] = b.shape[0]
        lay = T.layout_of(a)
    else:
        shape = T.ttt_shape(tuple(a.shape), tuple(b.shape), r.q, r.phi, r.psi)
        lay = None
    return torch.full(tuple(shape), float("nan"), dtype=acc, device=a.device) if lay is None else \
        T.empty(tuple(shape), lay, acc, a.device).fill_(float("nan"))


def _subgrid(r, a_shape, b_shape, g):
    """Index subsets of the free modes of request r so that the oracle's work
    on the sub-grid stays within CHECK_MACS (every index when the whole result
    fits).  Returns ({A mode: indices}, {B mode: indices}, whole)."""
    import numpy as np

    p = len(a_shape)
    if r.op == "ttv":
        k = a_shape[r.mode - 1]
        free = {("a", d): a_shape[d] for d in range(p) if d != r.mode - 1}
    elif r.op == "ttm":
        k = a_shape[r.mode - 1]
        free = {("a", d): a_shape[d] for d in range(p) if d != r.mode - 1}
        free[("b", 0)] = b_shape[0]
    else:
        ra = p - r.q
        k = int(np.prod([a_shape[m - 1] for m in r.phi[ra:]], dtype=np.int64))
        free = {("a", m - 1): a_shape[m - 1] for m in r.phi[:ra]}
        sb = len(b_shape) - r.q
        free.update({("b", m - 1): b_shape[m - 1] for m in r.psi[:sb]})
    sizes = dict(free)
    want = max(1, CHECK_MACS // max(1, k))
    while int(np.prod(list(sizes.values()) or [1], dtype=np.int64)) > want:
        big = max(sizes, key=lambda d: sizes[d])
        if sizes[big] == 1:
            break
        sizes[big] = (sizes[big] + 1) // 2
    whole = all(sizes[d] == free[d] for d in free)
    sel_a, sel_b = {}, {}
    for d, n in free.items():
        idx = np.arange(n) if sizes[d] == n else np.sort(g.choice(n, size=sizes[d], replace=False))
        (sel_a if d[0] == "a" else sel_b)[d[1]] = idx
    return sel_a, sel_b, whole


def _gather(t, sel):
    """t restricted to the given indices per dim (on the device), as float64 numpy."""
    import torch

    for d, idx in sel.items():
        t = t.index_select(d, torch.as_tensor(idx, device=t.device))
    return t.double().cpu().numpy()


def _check_one(r, got, operands, g):
    """Normwise error of one served result against the FP64 oracle on a seeded
    sub-grid (_subgrid); for a BF16 request also the kernel-only error (oracle
    on the BF16 operands).  Returns (error, kernel-only error or None, whole)."""
    import numpy as np

    import oracle

    a32, b32 = operands(r, "f32")
    sel_a, sel_b, whole = _subgrid(r, tuple(a32.shape), tuple(b32.shape), g)
    if r.op == "ttv":
        ref = lambda A, B: oracle.ttv(A, B, r.mode)
        cs = {(d if d < r.mode - 1 else d - 1): v for d, v in sel_a.items()}
    elif r.op == "ttm":
        ref = lambda A, B: oracle.ttm(A, B, r.mode)
        cs = dict(sel_a)
        cs[r.mode - 1] = sel_b[0]
    else:
        ref = lambda A, B: oracle.ttt(A, B, r.q, r.phi, r.psi)
        ra = len(a32.shape) - r.q
        cs = {k: sel_a[m - 1] for k, m in enumerate(r.phi[:ra])}
        cs.update({ra + k: sel_b[m - 1] for k, m in enumerate(r.psi[:len(b32.shape) - r.q])})
    G = _gather(got, cs)

    def rel(R):
        R = np.asarray(R)
        nr = float(np.linalg.norm(R.ravel()))
        d = float(np.linalg.norm((G - R).ravel()))
        return d / nr if nr > 0 else d

    e = rel(ref(_gather(a32, sel_a), _gather(b32, sel_b)))
    ek = None
    if r.dtype != "f32":
        a16, b16 = operands(r)
        ek = rel(ref(_gather(a16, sel_a), _gather(b16, sel_b)))
    return e, ek, whole


def served_check(srv, reqs, operands, tie, log, chunk=256):
    """Every served request once more through the same server (closed loop,
    caller-owned outputs), each result compared with the FP64 oracle on a
    seeded sub-grid of its outputs (the whole result when its oracle work is at
    most CHECK_MACS multiply-adds); results kept from the headline open-loop
    run must equal these bit for bit (a request's kernel does not depend on
    the mix).  BF16 requests are measured end to end (oracle on the FP32 values
    the BF16 operands were rounded from) and kernel-only (oracle on the BF16
    values)."""
    import numpy as np
    import torch

    import paper_1711_10912_amd as T

    t0 = time.perf_counter()
    g = np.random.default_rng(171110912 + 6)
    errs = {"f32": [], "bf16": [], "bf16_kernel": []}
    whole = 0
    tie_equal = tie_total = 0
    over = []
    for c0 in range(0, len(reqs), chunk):
        part = reqs[c0:c0 + chunk]
        outs = {r.rid: _result_tensor(T, r, operands) for r in part}
        srv.reset_stats()
        for r in part:
            a, b = operands(r)
            srv.submit(r.op, a, b, mode=r.mode, q=r.q, phi=r.phi, psi=r.psi, out=outs[r.rid])
        srv.drain()
        st = srv.stats()
        if st["errors"]:
            raise RuntimeError("served check: %d requests failed" % st["errors"])
        for r in part:
            got = outs[r.rid]
            if r.rid in tie:
                tie_total += 1
                tie_equal += int(torch.equal(got.view(torch.int32), tie[r.rid].view(torch.int32)))
            e, ek, w = _check_one(r, got, operands, g)
            whole += int(w)
            errs["f32" if r.dtype == "f32" else "bf16"].append(e)
            if ek is not None:
                errs["bf16_kernel"].append(ek)
            bar = 1e-5 if r.dtype == "f32" else 2e-2
            if e > bar:
                over.append({"rid": r.rid, "op": r.op, "dtype": r.dtype, "err": e})
        del outs
        if (c0 // chunk) % 8 == 0:
            log("serve check: %d / %d results (%.0f s)" % (c0 + len(part), len(reqs), time.perf_counter() - t0))

    def summ(v):
        v = np.sort(np.asarray(v))
        if v.size == 0:
            return None
        return {"results": int(v.size), "max": float(v[-1]), "p99": float(v[min(v.size - 1, int(0.99 * v.size))]),
                "median": float(v[v.size // 2])}

    return {
        "measure": "normwise ||C - C*|| / ||C*|| per result against the FP64 oracle, on a seeded sub-grid "
                   "of each result's outputs (whole result when its oracle work is <= %d multiply-adds)" % CHECK_MACS,
        "results_checked": len(reqs),
        "checked_whole": whole,
        "f32": summ(errs["f32"]),
        "bf16_end_to_end": summ(errs["bf16"]),
        "bf16_kernel_only": summ(errs["bf16_kernel"]),
        "bars": {"f32": 1e-5, "bf16": 2e-2},
        "over_bar": over[:20],
        "n_over_bar": len(over),
        "headline_run_results_bitwise_equal": "%d/%d" % (tie_equal, tie_total),
        "seconds": round(time.perf_counter() - t0, 1),
    }


def serve_bench(args):
    """The served stream alone (req/s as the value)."""
    sv = served_measure(args.requests, check=not args.no_serve_check, tune_save=args.autotune_save)
    return {
        "metric": METRIC,
        "value": round(sv["closed_loop"]["req_per_s"], 1),
        "unit": "req/s (closed-loop capacity of the served mixed stream)",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(sv["requests"] / sv["closed_loop"]["req_per_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32,bf16 (per request tag), f32 accumulation",
        "data": "synthetic request stream (seeded): orders 2..6, log-uniform extents 8..512, <=2^24 "
                "elements, 40/40/20 TTV/TTM/TTT, resident operand pool of 1024 tensors",
        "config": {"workload": "served mixed stream, %d requests" % sv["requests"], "slots": sv["slots"],
                   "output_budget_GB": sv["output_budget_GB"]},
        "served": sv,
    }


def drivers_bench(args):
    """The composite drivers on the order-4 160^4 workload: the Tucker chain
    (TTM in modes 1..4 with 32x160 factors, FP32, and BF16 inputs with BF16
    staging between steps), the one-pass multi-mode TTV for every excluded
    mode (beside the chain of TTVs it replaces) and 20 HOPM sweeps built on it
    (FP32 data, FP64 accumulation and norms).
    Algorithmic bytes count every kernel's inputs and outputs once."""
    import torch

    import paper_1711_10912_amd as T

    dev = torch.device("cuda:0")
    n, rank, rows = 160, 16, 32
    g = torch.Generator(device=dev)
    g.manual_seed(171110912 + 3)
    # N(0,1) plus a rank-16 part with orthonormal factor columns and
    # sigma_r = 1e5 * 0.8^(r-1); factors U_k (32 x 160) with orthonormal rows
    # whose first 16 are the true factors
    facs = [torch.linalg.qr(torch.randn(n, rows, generator=g, device=dev, dtype=torch.float64))[0]
            for _ in range(4)]
    sig = 1e5 * 0.8 ** torch.arange(rank, device=dev, dtype=torch.float64)
    A = torch.randn((n,) * 4, generator=g, device=dev, dtype=torch.float32)
    F = [f[:, :rank] for f in facs]
    A += torch.einsum("r,ir,jr,kr,lr->ijkl", sig, *F).float()
    Us = [f.T.contiguous().float() for f in facs]
    A16 = A.to(torch.bfloat16)
    Us16 = [u.to(torch.bfloat16) for u in Us]
    torch.cuda.synchronize()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def tucker_bytes(s_in, s_stage):
        tot, shape = 0.0, [n] * 4
        for k in range(4):
            N = math.prod(shape)
            out = N // shape[k] * rows
            if k > 0 and s_stage != 4:
                tot += N * (4 + s_stage)          # FP32 -> 16-bit staging pass
            tot += N * (s_in if k == 0 else s_stage) + out * 4 + rows * n * s_in
            shape[k] = rows
        return tot

    def tucker_flops():
        tot, shape = 0.0, [n] * 4
        for k in range(4):
            tot += 2.0 * math.prod(shape) // shape[k] * rows * shape[k]
            shape[k] = rows
        return tot

    def tucker_pair_bytes(s_in):
        # FP32 Tucker as two two-mode passes: A -> (32, 32, n, n) -> 32^4,
        # each pass reading its input and factors and writing its output once
        x1 = rows * rows * n * n
        return s_in * (n ** 4 + 2 * rows * n) + 4 * x1 + 4 * (x1 + 2 * rows * n) + 4 * rows ** 4

    def unfused():
        X = A
        for k in range(4):
            X = T.ttm(X, Us[k], k + 1)
        return X

    reps = max(1, args.steps)
    t32 = timed(lambda: T.tucker(A, Us), reps)
    t32u = timed(unfused, reps)
    t16 = timed(lambda: T.tucker(A16, Us16, stage_dtype=torch.bfloat16), reps)
    u0 = [torch.full((n,), 1.0 / math.sqrt(n), device=dev, dtype=torch.float32) for _ in range(4)]
    # the one-pass multi-mode TTV per excluded mode, against the chain of
    # three TTVs it replaces; bytes: A once, three vectors and c
    tv_bytes = 4.0 * n ** 4 + 4.0 * 4 * n
    t_tv = [timed(lambda r=r: T.times_vectors(A, u0, r), reps) for r in range(1, 5)]
    t_ch = [timed(lambda r=r: T.times_vectors_chain(A, u0, r), reps) for r in range(1, 5)]
    iters = 20
    t_h = timed(lambda: T.hopm(A, u0, iters), 1)
    # per mode update: one pass over A (the multi-mode TTV), one norm and one
    # scale of an n-vector
    per_update = tv_bytes + 4.0 * 3 * n
    h_bytes = iters * 4 * per_update
    lam, _ = T.hopm(A, u0, 2)
    return {
        "metric": METRIC,
        "value": round(tucker_pair_bytes(4) / t32 / 1e9, 1),
        "unit": "GB/s (Tucker chain FP32 in two-mode passes, algorithmic bytes / time)",
        "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(t32 * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32; bf16 inputs with f32 accumulation; f64 norms",
        "data": "synthetic: 160^4 N(0,1) + rank-16 part (seeded)",
        "config": {"workload": "Tucker chain 160^4 x_1..x_4 U_k (32x160), multi-mode TTV, HOPM 20 sweeps"},
        "tucker_f32": {"ms": round(t32 * 1e3, 3), "GB/s": round(tucker_pair_bytes(4) / t32 / 1e9, 1),
                       "TFLOP/s": round(tucker_flops() / t32 / 1e12, 2),
                       "roofline_frac": round(tucker_pair_bytes(4) / PEAK_HBM / t32, 4),
                       "passes": "ttm2(1,2) fused, ttm2(3,4)",
                       "one_ttm_per_mode_ms": round(t32u * 1e3, 3)},
        "tucker_bf16": {"ms": round(t16 * 1e3, 3), "GB/s": round(tucker_bytes(2, 2) / t16 / 1e9, 1),
                        "TFLOP/s": round(tucker_flops() / t16 / 1e12, 2),
                        "roofline_frac": round(tucker_bytes(2, 2) / PEAK_HBM / t16, 4)},
        "times_vectors_f32": {"modes": [1, 2, 3, 4], "ms": [round(t * 1e3, 3) for t in t_tv],
                              "GB/s": [round(tv_bytes / t / 1e9, 1) for t in t_tv],
                              "roofline_frac": [round(tv_bytes / PEAK_HBM / t, 4) for t in t_tv],
                              "chain_of_ttv_ms": [round(t * 1e3, 3) for t in t_ch]},
        "hopm_f32_20_sweeps": {"ms": round(t_h * 1e3, 2), "GB/s": round(h_bytes / t_h / 1e9, 1),
                               "roofline_frac": round(h_bytes / PEAK_HBM / t_h, 4),
                               "lambda_after_2_sweeps": [round(v, 2) for v in lam]},
    }


def views_bench(args):
    """Operations on strided views (ranges with steps) of order-4 90^4 tensors
    against the same operations on dense tensors of the same logical shape:
    TTV in every mode, TTM (m = 64) in modes 1 and 4, norm, inner and add.
    Bytes are the useful ones (the view's elements, outputs, operands)."""
    import torch

    import paper_1711_10912_amd as T

    dev = torch.device("cuda:0")
    n, m = 90, 64
    reps = max(1, args.steps)

    def timed(fn):
        # median over 5 batches of `reps` calls: a host-side stall (the GPU
        # idles until the next launch arrives) lands in one batch only
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / reps * 1e-3)
        return sorted(ts)[2]

    out = {}
    totals = {}
    for dname_, dt in (("f32", torch.float32), ("f64", torch.float64)):
        s = 4 if dt == torch.float32 else 8
        g = torch.Generator(device=dev)
        g.manual_seed(171110912 + 5)
        views = {
            "dense": lambda: T.empty((n, n, n, n), None, dt, dev),
            "sliced": lambda: T.empty((2 * n, n + 3, n, n), None, dt, dev)[:n, :n],
            "step2_mode1": lambda: T.empty((2 * n, n, n, n), None, dt, dev)[::2],
            "trim": lambda: T.empty((n + 2, n + 2, n + 2, n + 2), None, dt, dev)[1:n + 1, 1:n + 1, 1:n + 1, 1:n + 1],
            "step3_mode2_last": lambda: T.empty((n, 3 * n, n, n), [4, 3, 2, 1], dt, dev)[:, ::3],
            "step2_mode4_perm": lambda: T.empty((n, n, n, 2 * n), [2, 4, 1, 3], dt, dev)[:, :, :, ::2],
        }
        for name, make in views.items():
            # inner and add read a second tensor of the same view kind, so
            # that every counted byte is read from its own address
            A, A2 = make(), make()
            A.copy_(torch.rand(A.shape, generator=g, device=dev, dtype=dt))
            A2.copy_(torch.rand(A2.shape, generator=g, device=dev, dtype=dt))
            N = A.numel()
            ops = []
            for q in range(1, 5):
                b = torch.rand(n, generator=g, device=dev, dtype=dt)
                C = T.ttv(A, b, q)
                ops.append(("ttv q=%d" % q, s * (N + N // n + n), (lambda A=A, b=b, q=q, C=C: T.ttv(A, b, q, out=C)),
                            T.plan(T.ttv, A, b, q, out=C).split(" ")[1]))
            for q in (1, 4):
                B = torch.rand(m, n, generator=g, device=dev, dtype=dt)
                C = T.ttm(A, B, q)
                ops.append(("ttm q=%d m=%d" % (q, m), s * (N + N // n * m + m * n),
                            (lambda A=A, B=B, q=q, C=C: T.ttm(A, B, q, out=C)),
                            T.plan(T.ttm, A, B, q, out=C).split(" ")[1]))
            r = torch.empty((), dtype=torch.float64, device=dev)
            ops.append(("norm", s * N, (lambda A=A, r=r: T.norm(A, out=r)), "dot"))
            ops.append(("inner", 2 * s * N, (lambda A=A, A2=A2, r=r: T.inner(A, A2, out=r)), "dot"))
            Cd = T.empty(A.shape, None, dt, dev)
            ops.append(("add", 3 * s * N, (lambda A=A, A2=A2, Cd=Cd: T.add(1.0, A, 1.0, A2, out=Cd)), "ewise"))
            rec = {}
            tb = tt = 0.0
            for label, nbytes, fn, kern in ops:
                t = timed(fn)
                rec[label] = {"us": round(t * 1e6, 1), "GB/s": round(nbytes / t / 1e9, 1), "kernel": kern}
                tb += nbytes
                tt += t
            out["%s %s" % (dname_, name)] = rec
            totals["%s %s" % (dname_, name)] = tb / tt / 1e9
        del views
        torch.cuda.empty_cache()
    view_keys = [k for k in totals if not k.endswith("dense")]
    value = sum(totals[k] for k in view_keys) / len(view_keys)
    return {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s (mean over views and dtypes of useful bytes / time for TTV, TTM, norm, inner, add)",
        "n_gpus": 1, "steps": reps, "warmup": 1, "timing": "median of 5 batches of `steps` calls per op",
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32, f64", "data": "synthetic: U[0,1) views of 90^4 tensors (seeded)",
        "config": {"workload": "strided views (ranges with steps) of order-4 90^4 tensors"},
        "dense_reference_GB/s": {k: round(v, 1) for k, v in totals.items() if k.endswith("dense")},
        "views_GB/s": {k: round(v, 1) for k, v in totals.items() if not k.endswith("dense")},
        "ops": out,
    }


def run_step(cases, torch, ev):
    for i, c in enumerate(cases):
        if ev is not None:
            ev[i][0].record()
        c.fn()
        if ev is not None:
            ev[i][1].record()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_both(budget_s=15.0, budget_1t_s=12.0):
    """The oracle with the host's OpenMP threads (this process), then
    single-threaded in a child process (OMP_NUM_THREADS=1), on the same
    sample plan."""
    import subprocess

    res = cpu_baseline(budget_s)
    res["cpu_model"] = cpu_model()
    res["nproc"] = os.cpu_count()
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                            "--cpu-budget", str(budget_1t_s)], env=env, capture_output=True, text=True,
                           timeout=10 * budget_1t_s + 120)
        one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    res["single_thread"] = one
    return res


def cpu_baseline(budget_s=15.0):
    """The FP64 oracle on a bounded sample of the same sweep: TTV and TTM
    (m = 16, 64) in modes 2, 1, p, 3, ... of the first-order p = 3, 5, 7, 4, 6
    tensors (406^3, 36^5, 13^7, 90^4, 20^6), in that order, until about
    `budget_s` seconds of CPU work (each case run once)."""
    import numpy as np

    import oracle
    import synth

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    plan = []
    for p in (3, 5, 7, 4, 6):
        for q in [2, 1, p] + [k for k in range(3, p)]:
            for m in (None, 16, 64):
                plan.append((p, q, m))
    total_bytes = 0.0
    spent = 0.0
    done = []
    tensors = {}
    for p, q, m in plan:
        if spent >= budget_s:
            break
        n = SWEEP[p]
        if p not in tensors:
            tensors[p] = oracle.materialize(synth.sweep_tensor(p))
        A = tensors[p]
        N = n ** p
        g = synth.rng(1, 500 + p)
        if m is None:
            b = synth.uniform((n,), g)
            t0 = time.perf_counter()
            oracle.ttv(A, b, q)
            dt = time.perf_counter() - t0
            total_bytes += 8 * (N + n + N // n)
            done.append("ttv p=%d q=%d" % (p, q))
        else:
            B = synth.uniform((m, n), g)
            t0 = time.perf_counter()
            oracle.ttm(A, B, q)
            dt = time.perf_counter() - t0
            total_bytes += 8 * (N + m * n) + 8 * (N // n * m)
            done.append("ttm p=%d q=%d m=%d" % (p, q, m))
        spent += dt
    return {"value": total_bytes / spent / 1e9 if spent > 0 else None, "unit": "GB/s", "cores": threads,
            "kind": "oracle", "seconds": round(spent, 2),
            "sample": "FP64 oracle, first-order sweep tensors: " + ", ".join(done)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--quick", action="store_true", help="p = 3 and 7 only (for profiling runs)")
    ap.add_argument("--autotune", default="on", choices=("on", "off"),
                    help="on: preload --autotune-table, then tune the TTM/TTT kernel choice of every call "
                         "shape it lacks in the first warmup step; off: the planner's fixed rules")
    ap.add_argument("--autotune-table", default=TUNING_TABLE,
                    help="kernel-choice table to preload ('' = none); default: the MI355X table shipped "
                         "with the package")
    ap.add_argument("--autotune-save", default="", help="write the table after the first warmup step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream section of the sweep run")
    ap.add_argument("--families", default="",
                    help="comma-separated case families to keep (ttv,ttm,ttt,outer,inner,norm,add; profiling runs)")
    ap.add_argument("--no-serve-check", action="store_true",
                    help="skip the offline oracle check of the served results")
    ap.add_argument("--cases-out", default="", help="write per-case timings (JSON lines) here")
    ap.add_argument("--workload", default="sweep", choices=("sweep", "serve", "drivers", "views"),
                    help="sweep: the order-p TTV/TTM sweep + TTT (default); serve: the served "
                         "mixed request stream (latency / req/s); drivers: Tucker, multi-mode TTV, HOPM; "
                         "views: operations on strided views against dense tensors")
    ap.add_argument("--requests", type=int, default=10000, help="serve: stream length")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (3 times), the reference for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale")
    ap.add_argument("--ceilings", action="store_true",
                    help="only time plain 4 GiB HBM streams (torch fill_, copy_ and sum in FP32 and FP64): "
                         "practical write, copy and read rates to set the kernels' fractions against")
    args = ap.parse_args()
    if args.ceilings:
        print(json.dumps(hbm_ceilings()))
        return
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_budget)))
        return
    if args.calibrate_copy:
        import torch

        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 << 28, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(the path would shard A along a free mode, see the design notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1711_10912_amd as T

    if args.workload == "serve":
        print(json.dumps(serve_bench(args)))
        return
    if args.workload == "drivers":
        print(json.dumps(drivers_bench(args)))
        return
    if args.workload == "views":
        print(json.dumps(views_bench(args)))
        return

    dev = torch.device("cuda:0")
    cases, keep, outbuf = build_cases(T, torch, dev, quick=args.quick)
    if args.families:
        fams = set(args.families.split(","))
        cases = [c for c in cases if c.family in fams]
    torch.cuda.synchronize()
    print("bench: %d calls per step" % len(cases), file=sys.stderr, flush=True)
    # Autotuning (kernel choice per call shape) happens in the first warmup
    # step; the timed steps only use stored choices.
    preloaded = 0
    if args.autotune == "on" and args.autotune_table and os.path.exists(args.autotune_table):
        T.autotune_load(args.autotune_table)
        preloaded = T.autotune_entries()
    # new call shapes are tuned in the first warmup step only; without warmup
    # they take the planner's rules
    tune = "off" if args.autotune == "off" else ("on" if args.warmup > 0 else "frozen")
    T.set_autotune(tune)
    t_tune = time.perf_counter()
    for w in range(args.warmup):
        run_step(cases, torch, None)
        torch.cuda.synchronize()
        if w == 0:
            t_tune = time.perf_counter() - t_tune
            if tune == "on":
                T.set_autotune("frozen")
    if args.autotune_save:
        T.autotune_save(args.autotune_save)
    torch.cuda.synchronize()
    for c in cases:
        c.kernel = _kernel_label(c.planfn())

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]
    step_ms = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_step(cases, torch, ev)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        for i, c in enumerate(cases):
            c.ms.append(ev[i][0].elapsed_time(ev[i][1]))
        print("bench: step %d %.1f ms" % (k, step_ms[-1]), file=sys.stderr, flush=True)

    ms_per_step = sum(step_ms) / len(step_ms)
    tot_bytes = sum(c.bytes for c in cases)
    tot_ideal = sum(c.ideal_s() for c in cases)

    # per-kernel aggregation
    kern = {}
    for c in cases:
        k = kern.setdefault(c.kernel, {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0, "t_hbm": 0.0,
                                       "t_mfma": 0.0, "ideal": 0.0, "dtype": c.dtype, "family": c.family})
        avg = sum(c.ms) / len(c.ms)
        k["launches"] += 1
        k["ms"] += avg
        k["bytes"] += c.bytes
        k["flops"] += c.flops
        k["t_hbm"] += c.bytes / PEAK_HBM
        k["t_mfma"] += c.flops / PEAK_FLOPS[c.dtype]
        k["ideal"] += c.ideal_s()
    dom_name = max(kern, key=lambda n: kern[n]["ms"])
    dk = kern[dom_name]
    if dk["t_hbm"] >= dk["t_mfma"]:
        achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 4)}
    else:
        achieved = dk["flops"] / (dk["ms"] * 1e-3) / 1e12
        peak = PEAK_FLOPS[dk["dtype"]] / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4)}
    tb, src = recorded_traffic(dom_name)
    roof["traffic"] = round(tb / 1e9, 4) if tb is not None else None
    roof["traffic_unit"] = "GB per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)"
    roof["traffic_source"] = src
    roof["algorithmic_GB_per_launch"] = round(dk["bytes"] / dk["launches"] / 1e9, 4)
    roof["kernel"] = dom_name
    roof["launches_per_step"] = dk["launches"]
    roof["avg_launch_us"] = round(dk["ms"] * 1e3 / dk["launches"], 2)
    # each launch priced at its own bound (HBM or MFMA, whichever takes
    # longer): a kernel whose launches differ in bound reaches more of that
    # roofline than `frac`, which prices them all at one bound
    roof["frac_per_launch_bound"] = round(dk["ideal"] / (dk["ms"] * 1e-3), 4)

    fam = {}
    for c in cases:
        f = fam.setdefault(c.family, {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "ideal_s": 0.0})
        f["ms"] += sum(c.ms) / len(c.ms)
        f["bytes"] += c.bytes
        f["flops"] += c.flops
        f["ideal_s"] += c.ideal_s()
    breakdown = {}
    for n, f in fam.items():
        breakdown[n] = {"ms": round(f["ms"], 3), "GB/s": round(f["bytes"] / (f["ms"] * 1e-3) / 1e9, 1),
                        "TFLOP/s": round(f["flops"] / (f["ms"] * 1e-3) / 1e12, 3),
                        "roofline_frac": round(f["ideal_s"] / (f["ms"] * 1e-3), 4)}
    kernels = {n: {"launches": k["launches"], "ms": round(k["ms"], 3),
                   "GB/s": round(k["bytes"] / (k["ms"] * 1e-3) / 1e9, 1),
                   "TFLOP/s": round(k["flops"] / (k["ms"] * 1e-3) / 1e12, 3),
                   "roofline_frac": round(k["ideal"] / (k["ms"] * 1e-3), 4)}
               for n, k in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])}

    if args.cases_out:
        with open(args.cases_out, "w") as f:
            for c in cases:
                avg = sum(c.ms) / len(c.ms)
                f.write(json.dumps({"case": c.name, "kernel": c.kernel, "us": round(avg * 1e3, 2),
                                    "GB/s": round(c.bytes / (avg * 1e-3) / 1e9, 1),
                                    "TFLOP/s": round(c.flops / (avg * 1e-3) / 1e12, 3),
                                    "roofline_frac": round(c.ideal_s() / (avg * 1e-3), 4)}) + "\n")

    n_calls = len(cases)
    del cases, keep, outbuf, ev
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    served = None
    if not args.no_serve:
        served = served_measure(args.requests, check=not args.no_serve_check)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_both()

    out = {
        "metric": METRIC,
        "value": round(tot_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "unit": "GB/s (algorithmic bytes of the whole step / step time)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64,f32 (sweep); f32,bf16,f16 with f32 accumulation (ttt); f64 accumulation (inner/norm)",
        "data": "synthetic (seeded uniform[-1,1] / normal(0,1) on device)",
        "config": {"workload": "order-p sweep p=3..7 (406^3,90^4,36^5,20^6,13^7), every mode, first+last order, "
                               "f64+f32: TTV, TTM m=16/64/256, inner, norm, add; plus TTT (96,80,64,48)x(64,48,120) "
                               "A{3,4}<->B{1,2}, 3 A layouts, f32/bf16/f16, one input set of six at x1e3; "
                               "outer product (512,128)x(64,40) f64+f32"
                               + (" [quick: p=3,7 only]" if args.quick else "")
                               + (" [families: %s]" % args.families if args.families else ""),
                   "served": None if args.no_serve else "mixed stream of %d requests (see the served object)"
                   % args.requests,
                   "calls_per_step": n_calls},
        "roofline_frac_step": round(tot_ideal / (ms_per_step * 1e-3), 4),
        "autotune": {"mode": tune, "preloaded": preloaded, "entries": T.autotune_entries(),
                     "table": os.path.relpath(args.autotune_table, HERE) if preloaded else None,
                     "first_warmup_step_s": round(t_tune, 2) if args.warmup > 0 else None},
        "roofline": roof,
        "breakdown": breakdown,
        "kernels": kernels,
        "served": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
