"""Grouped launch (tlib_batch_plan / tlib_batch_run) of TTV, TTM and TTT
requests (Sec. 5.2 Eq. ttv, ttm, ttt and ttt_indices): every result against
the FP64 oracle (FP64 1e-12, FP32 1e-5; 16-bit inputs 1e-5 against the oracle
on the same rounded inputs), each request bit-identical alone and in a mix,
and one captured graph replayed over two different tables."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from _util import to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5, "f16": 1e-5}


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _requests(seed, dtypes=("f64", "f32", "bf16", "f16")):
    """A mixed list of small requests: (op, A, B, mode, q, phi, psi, C layout)."""
    g = synth.rng(3, 900 + seed)
    out = []
    for i, d in enumerate(dtypes * 3):
        p = 2 + (i % 3)
        shape = tuple(int(g.integers(3, 40 if p < 4 else 14)) for _ in range(p))
        lay = synth.random_layout(p, g) if i % 2 else list(range(p, 0, -1))
        A = synth.uniform(shape, g)
        op = i % 3
        if op == 0:
            m = int(g.integers(1, p + 1))
            out.append(("ttv", d, A, lay, synth.uniform((shape[m - 1],), g), None, m, 0, None, None))
        elif op == 1:
            m = int(g.integers(1, p + 1))
            rows = int(g.integers(1, 70))
            out.append(("ttm", d, A, lay, synth.uniform((rows, shape[m - 1]), g), None, m, 0, None, None))
        else:
            q = 1 if p == 2 else int(g.integers(1, 3))
            contr = sorted(int(v) + 1 for v in g.choice(p, size=q, replace=False))
            free_a = [k for k in range(1, p + 1) if k not in contr]
            fb = tuple(int(g.integers(2, 12)) for _ in range(int(g.integers(0, 3))))
            if not free_a and not fb:
                fb = (5,)
            nb = tuple(shape[k - 1] for k in contr) + fb
            phi = tuple(free_a + contr)
            psi = tuple(range(q + 1, len(nb) + 1)) + tuple(range(1, q + 1))
            out.append(("ttt", d, A, lay, synth.uniform(nb, g), synth.random_layout(len(nb), g), 0, q, phi, psi))
    return out


def _place(T, reqs):
    """Device operands and NaN-filled outputs of each request."""
    import torch
    placed = []
    for op, d, A, lay, B, blay, m, q, phi, psi in reqs:
        At = to_gpu(A, lay, d)
        Bt = to_gpu(B, blay, d)
        acc = torch_dtype("f64" if d == "f64" else "f32")
        if op == "ttv":
            shape = A.shape[: m - 1] + A.shape[m:]
        elif op == "ttm":
            shape = A.shape[: m - 1] + (B.shape[0],) + A.shape[m:]
        else:
            shape = oracle.ttt_shape(A.shape, B.shape, q, phi, psi)
        C = torch.full(shape, float("nan"), dtype=acc, device="cuda")
        placed.append((op, d, At, Bt, m, q, phi, psi, C))
    return placed


def _table(T, placed):
    from paper_1711_10912_amd import _lib
    L = _lib.lib()
    keep = []
    arr = (_lib.Request * len(placed))()
    for i, (op, d, At, Bt, m, q, phi, psi, C) in enumerate(placed):
        da, db, dc = T._desc(At), T._desc(Bt), T._desc(C)
        pa = _lib.i32_array(phi) if op == "ttt" else None
        pb = _lib.i32_array(psi) if op == "ttt" else None
        keep += [da, db, dc, pa, pb]
        arr[i].op = {"ttv": 0, "ttm": 1, "ttt": 2}[op]
        arr[i].mode = m
        arr[i].A, arr[i].B, arr[i].C = ctypes.pointer(da), ctypes.pointer(db), ctypes.pointer(dc)
        arr[i].q = q
        if op == "ttt":
            arr[i].phi = ctypes.cast(pa, ctypes.POINTER(ctypes.c_int32))
            arr[i].psi = ctypes.cast(pb, ctypes.POINTER(ctypes.c_int32))
        assert L.tlib_request_groupable(ctypes.byref(arr[i])) == 1, i
    nbytes = L.tlib_batch_table_bytes(len(placed))
    host = (ctypes.c_char * nbytes)()
    units = ctypes.c_int64(0)
    bad = ctypes.c_int32(0)
    rc = L.tlib_batch_plan(arr, len(placed), host, nbytes, ctypes.byref(units), ctypes.byref(bad))
    assert rc == 0, (rc, bad.value, L.tlib_last_error())
    return bytes(host), units.value


def _run(T, table, dev_table):
    import torch
    from paper_1711_10912_amd import _lib
    dev_table[: len(table)].copy_(torch.frombuffer(bytearray(table), dtype=torch.uint8))
    rc = _lib.lib().tlib_batch_run(ctypes.c_void_p(dev_table.data_ptr()), 0,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0


def _ref(op, d, At, Bt, m, q, phi, psi):
    A, B = to_np(At), to_np(Bt)
    if op == "ttv":
        return np.asarray(oracle.ttv(A, B, m))
    if op == "ttm":
        return np.asarray(oracle.ttm(A, B, m))
    return np.asarray(oracle.ttt(A, B, q, phi, psi))


def _rel(got, ref):
    n = np.linalg.norm(ref.ravel())
    e = np.linalg.norm((got - ref).ravel())
    return e / n if n > 0 else e


def test_batch_mix_vs_oracle_and_alone(T):
    import torch
    reqs = _requests(0)
    placed = _place(T, reqs)
    table, units = _table(T, placed)
    dev = torch.empty(len(table) + 64, dtype=torch.uint8, device="cuda")
    _run(T, table, dev)
    torch.cuda.synchronize()
    for i, (op, d, At, Bt, m, q, phi, psi, C) in enumerate(placed):
        got = to_np(C)
        assert np.isfinite(got).all(), (i, op, d)
        e = _rel(got, _ref(op, d, At, Bt, m, q, phi, psi))
        assert e <= TOL[d], (i, op, d, e)
    # every request alone in a batch of one: the same bits
    for i, item in enumerate(placed):
        op, d, At, Bt, m, q, phi, psi, C = item
        C2 = torch.full_like(C, float("nan"))
        one = [(op, d, At, Bt, m, q, phi, psi, C2)]
        t1, _ = _table(T, one)
        _run(T, t1, dev)
        torch.cuda.synchronize()
        assert torch.equal(C2.view(torch.int32 if C.dtype == torch.float32 else torch.int64),
                           C.view(torch.int32 if C.dtype == torch.float32 else torch.int64)), (i, op, d)


def test_batch_graph_replays_new_tables(T):
    """The grouped launch captured once replays whatever table the device
    buffer holds (two different batches, eager work between replays)."""
    import torch
    from paper_1711_10912_amd import _lib
    sets = [_place(T, _requests(s, ("f32", "bf16"))) for s in (1, 2)]
    tables = [_table(T, p)[0] for p in sets]
    dev = torch.zeros(max(len(t) for t in tables) + 64, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    dev[: len(tables[0])].copy_(torch.frombuffer(bytearray(tables[0]), dtype=torch.uint8))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        rc = _lib.lib().tlib_batch_run(ctypes.c_void_p(dev.data_ptr()), 0,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    for rep in range(2):
        for p, t in zip(sets, tables):
            for item in p:
                item[-1].fill_(float("nan"))
            dev[: len(t)].copy_(torch.frombuffer(bytearray(t), dtype=torch.uint8))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for i, (op, d, At, Bt, m, q, phi, psi, C) in enumerate(p):
                e = _rel(to_np(C), _ref(op, d, At, Bt, m, q, phi, psi))
                assert e <= TOL[d], (rep, i, op, d, e)
