"""Serving loop: results through the server equal the direct per-call results,
a request gives bit-identical results alone and in a mix, the oracle agrees
on a sample, and a tight HBM budget still drains every request."""
import numpy as np
import pytest

import oracle
from _util import assert_close, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import bench
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    reqs, operands = bench.served_workload(n_req=160, n_tensors=24, n_mats=16, cap=1 << 16, seed_case=1)
    return T, reqs, operands


def _run(T, reqs, operands, **kw):
    from paper_1711_10912_amd.serve import Server
    srv = Server(keep_results=True, **kw)
    srv.start()
    rid = {}
    for r in reqs:
        a, b = operands(r)
        rid[srv.submit(r.op, a, b, mode=r.mode, q=r.q, phi=r.phi, psi=r.psi)] = r
    srv.stop()
    out = {}
    for j in srv.completed:
        assert j.error is None, j.error
        out[rid[j.rid].rid] = (to_np(j.out), j.grouped)
    return out, srv


def _direct(T, r, operands):
    a, b = operands(r)
    if r.op == "ttv":
        return to_np(T.ttv(a, b, r.mode))
    if r.op == "ttm":
        return to_np(T.ttm(a, b, r.mode))
    return to_np(T.ttt(a, b, r.q, r.phi, r.psi))


def test_server_matches_direct_calls(setup):
    T, reqs, operands = setup
    out, srv = _run(T, reqs, operands, slots=4)
    assert len(out) == len(reqs)
    st = srv.stats()
    assert st["requests"] == len(reqs) and st["grouped"] > 0
    for r in reqs:
        got, grouped = out[r.rid]
        ref = _direct(T, r, operands)
        if grouped:
            assert_close(got, ref, 1e-5, "grouped %s %d" % (r.op, r.rid))
        else:
            assert np.array_equal(got, ref), (r.op, r.rid)


def test_alone_equals_in_mix(setup):
    T, reqs, operands = setup
    mix, _ = _run(T, reqs, operands, slots=4, group_max=64)
    for r in reqs[:40]:
        alone, _ = _run(T, [r], operands, slots=1)
        assert np.array_equal(alone[r.rid][0], mix[r.rid][0]), (r.op, r.rid)


def test_sample_vs_oracle(setup):
    T, reqs, operands = setup
    out, _ = _run(T, reqs, operands, slots=2)
    for r in reqs[:30]:
        a, b = operands(r)
        A, B = oracle.materialize(to_np(a)), to_np(b)
        if r.op == "ttv":
            ref = oracle.ttv(A, B, r.mode)
        elif r.op == "ttm":
            ref = oracle.ttm(A, B, r.mode)
        else:
            ref = oracle.ttt(A, oracle.materialize(B), r.q, r.phi, r.psi)
        assert_close(out[r.rid][0], np.asarray(ref), 1e-5, "%s %d vs oracle" % (r.op, r.rid))


def test_tight_budget_drains(setup):
    T, reqs, operands = setup
    biggest = max(int(np.prod(_direct(T, r, operands).shape)) * 4 for r in reqs)
    from paper_1711_10912_amd.serve import Server
    srv = Server(hbm_budget=2 * biggest, slots=4)
    srv.start()
    for r in reqs:
        a, b = operands(r)
        srv.submit(r.op, a, b, mode=r.mode, q=r.q, phi=r.phi, psi=r.psi)
    srv.stop()
    assert srv.stats()["requests"] == len(reqs)
    assert srv.in_flight == 0
