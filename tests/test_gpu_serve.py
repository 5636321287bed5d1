"""Request server (native scheduler behind tlib_server_*): results through the
server equal the direct per-call results, a request gives bit-identical
results alone and in a mix, the oracle agrees on a sample, and a tight output
budget still drains every request."""
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


def _run(reqs, operands, **kw):
    from paper_1711_10912_amd.serve import Server
    srv = Server(keep_results=True, **kw)
    ids = {}
    for r in reqs:
        a, b = operands(r)
        ids[r.rid] = srv.submit(r.op, a, b, mode=r.mode, q=r.q, phi=r.phi, psi=r.psi)
    srv.drain()
    out = {rid: to_np(srv.result(i)) for rid, i in ids.items()}
    st = srv.stats()
    srv.close()
    return out, st


def _direct(T, r, operands):
    a, b = operands(r)
    if r.op == "ttv":
        return to_np(T.ttv(a, b, r.mode))
    if r.op == "ttm":
        return to_np(T.ttm(a, b, r.mode))
    return to_np(T.ttt(a, b, r.q, r.phi, r.psi))


def test_server_matches_direct_calls(setup):
    T, reqs, operands = setup
    out, st = _run(reqs, operands, slots=4)
    assert st["requests"] == len(reqs) and st["errors"] == 0 and st["grouped"] > 0
    for r in reqs:
        assert_close(out[r.rid], _direct(T, r, operands), 1e-5, "%s %d" % (r.op, r.rid))


def test_alone_equals_in_mix(setup):
    T, reqs, operands = setup
    mix, _ = _run(reqs, operands, slots=4, group_max=64)
    for r in reqs[:40]:
        alone, _ = _run([r], operands, slots=1)
        assert np.array_equal(alone[r.rid], mix[r.rid]), (r.op, r.rid)


def test_sample_vs_oracle(setup):
    T, reqs, operands = setup
    out, _ = _run(reqs, operands, slots=2)
    for r in reqs[:30]:
        a, b = operands(r)
        A, B = oracle.materialize(to_np(a)), to_np(b)
        if r.op == "ttv":
            ref = oracle.ttv(A, B, r.mode)
        elif r.op == "ttm":
            ref = oracle.ttm(A, B, r.mode)
        else:
            ref = oracle.ttt(A, oracle.materialize(B), r.q, r.phi, r.psi)
        assert_close(out[r.rid], np.asarray(ref), 1e-5, "%s %d vs oracle" % (r.op, r.rid))


def test_tight_budget_drains(setup):
    T, reqs, operands = setup
    from paper_1711_10912_amd.serve import Server
    biggest = max(int(np.prod(_direct(T, r, operands).shape)) * 4 for r in reqs)
    srv = Server(hbm_budget=2 * biggest + 4096, slots=4)   # results go to the server's arena
    for r in reqs:
        a, b = operands(r)
        srv.submit(r.op, a, b, mode=r.mode, q=r.q, phi=r.phi, psi=r.psi)
    srv.drain()
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs) and st["errors"] == 0


def test_oversized_request_is_rejected(setup):
    T, reqs, operands = setup
    from paper_1711_10912_amd import TlibError
    from paper_1711_10912_amd.serve import Server
    srv = Server(hbm_budget=1024, slots=1)
    r = next(r for r in reqs if r.op == "ttm")
    a, b = operands(r)
    with pytest.raises(TlibError):
        srv.submit(r.op, a, b, mode=r.mode)
    srv.close()
