"""Entry points under HIP graph capture.  A split-K TTT (Sec. 5.2 Eq. ttt), a
TTV whose contraction is split over the grid (Eq. ttv) and an inner product
(Table 3), each of a call shape not seen before, are captured on a stream
whose workspace was reserved beforehand, and the graph is replayed several
times with eager work in between: every replay against the oracle.  A larger
reserve on the same stream then replaces the workspace; the graph keeps the
buffer it was captured with (the old one stays allocated), so later replays
stay correct.  A call that needs scratch on a capturing stream without a
workspace returns TLIB_ENOMEM instead of allocating."""
import numpy as np
import pytest

import oracle
import synth
from _util import assert_close, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1711_10912_amd as T
    assert torch.cuda.is_available()
    return T


def _ksplit(plan):
    return int(plan.split("ksplit=")[1].split()[0]) if "ksplit=" in plan else 1


def test_capture_and_replay_split_calls(T):
    import torch
    g = synth.rng(75, 0)
    # TTT (56,40,48,36) x (48,36,72) in FP32: 40k outputs over K = 1728, split
    At = to_gpu(synth.uniform((56, 40, 48, 36), g), [3, 1, 4, 2], "f32")
    Bt = to_gpu(synth.uniform((48, 36, 72), g), None, "f32")
    phi, psi = (1, 2, 3, 4), (3, 1, 2)
    # TTV over a long contraction with 384 outputs: k split over the grid
    Av = to_gpu(synth.uniform((384, 40000), g), None, "f64")
    bv = to_gpu(synth.uniform((40000,), g), None, "f64")
    # inner product of two 3-way tensors in different layouts
    X = to_gpu(synth.uniform((70, 60, 50), g), None, "f32")
    Y = to_gpu(synth.uniform((70, 60, 50), g), [3, 1, 2], "f32")

    Ct = T.empty((56, 40, 72), None, torch.float32, "cuda")
    Cv = T.empty((384,), None, torch.float64, "cuda")
    ip = torch.empty((), dtype=torch.float64, device="cuda")
    assert _ksplit(T.plan(T.ttt, At, Bt, 2, phi, psi, out=Ct)) > 1
    pv = T.plan(T.ttv, Av, bv, 2, out=Cv)
    assert "col" in pv and "ksplit" in pv and _ksplit(pv) > 1, pv

    ref_t = np.asarray(oracle.ttt(oracle.materialize(to_np(At)), oracle.materialize(to_np(Bt)), 2, phi, psi))
    ref_v = np.asarray(oracle.ttv(to_np(Av), to_np(bv), 2))
    ref_i = oracle.inner(oracle.materialize(to_np(X)), oracle.materialize(to_np(Y)))

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        T.workspace_reserve(32 << 20)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        T.ttt(At, Bt, 2, phi, psi, out=Ct)
        T.ttv(Av, bv, 2, out=Cv)
        T.inner(X, Y, out=ip)

    def check(tag):
        assert_close(to_np(Ct), ref_t, 1e-5, "ttt " + tag)
        assert_close(to_np(Cv), ref_v, 1e-12, "ttv " + tag)
        assert abs(float(ip.item()) - ref_i) <= 1e-12 * abs(ref_i), tag

    for rep in range(3):
        Ct.fill_(float("nan"))
        Cv.fill_(float("nan"))
        ip.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check("replay %d" % rep)
        # eager work on the same stream between replays
        with torch.cuda.stream(s):
            T.ttt(At, Bt, 2, phi, psi, out=Ct)
        s.synchronize()

    # a larger reserve replaces the stream's buffer; the graph keeps the old one
    with torch.cuda.stream(s):
        T.workspace_reserve(96 << 20)
        assert T.workspace_size() >= 96 << 20
        big = T.ttt(to_gpu(synth.uniform((120, 64, 48, 36), g), None, "f32"), Bt, 2, phi, psi)
    s.synchronize()
    assert np.isfinite(to_np(big)).all()
    for rep in range(2):
        Ct.fill_(float("nan"))
        Cv.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check("after reserve %d" % rep)
    del graph
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        T.workspace_release()


def test_capture_without_workspace_is_refused(T):
    """Scratch on a capturing stream without a workspace: TLIB_ENOMEM, nothing
    allocated, and the capture itself can still be ended."""
    import torch
    from paper_1711_10912_amd import TlibError
    g = synth.rng(75, 1)
    X = to_gpu(synth.uniform((40, 30), g), None, "f64")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        T.workspace_release()  # torch hands out pooled streams: start without a buffer
    graph = torch.cuda.CUDAGraph()
    raised = None
    with torch.cuda.graph(graph, stream=s):
        try:
            T.norm(X, out=out)
        except TlibError as e:
            raised = e
        out.fill_(1.0)  # a node of its own, so the captured graph is not empty
    assert raised is not None and raised.code == 7  # TLIB_ENOMEM
    graph.replay()
    torch.cuda.synchronize()
    assert float(out.item()) == 1.0
    with torch.cuda.stream(s):
        assert T.workspace_size() == 0
