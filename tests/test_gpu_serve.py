"""Serving on the GPU: every request's result in the continuous-batching mix
equals the same request run alone through the library, and captured-graph
replays equal eager launches."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2506_04891_amd import tqsim as T
    from paper_2506_04891_amd.serve import GpuExecutor, Request, Server


def _alone(r):
    c = T.Circuit(r.n, r.layers, "c64")
    dev = torch.device("cuda")
    w = torch.tensor(r.weights if r.weights.size else np.zeros(1), device=dev)
    x = torch.tensor(r.features, device=dev)
    st = c.forward(w, x)
    e = c.expval_z(st).cpu().numpy()
    gw = gx = None
    if r.want_grad:
        g = torch.ones((r.batch, r.n), dtype=torch.float64, device=dev)
        gw, gx = c.adjoint_grad(w, x, st, g)
        gw, gx = gw.cpu().numpy(), gx.cpu().numpy()
    return e, gw, gx


def _reqs(k, seed, n_range=(6, 12), b_max=64, blocks=(2, 6)):
    trace = W.serving_trace(k, qps=1e4, seed=seed, n_range=n_range, b_max=b_max, blocks_range=blocks,
                            grad_frac=0.3)
    out = []
    for t in trace:
        layers, w, x = W.request_params(t, seed=seed)
        out.append(Request(t.n, layers, w, x, want_grad=t.want_grad, rid=t.rid))
    return out


@pytest.mark.parametrize("graphs", [False, True])
def test_mix_equals_alone_gpu(graphs):
    reqs = _reqs(40, seed=11)
    # repeat some structures so that requests coalesce and graphs are replayed
    reqs += [Request(r.n, r.layers, r.weights * 0.5, r.features[::-1].copy(), want_grad=r.want_grad, rid=100 + i)
             for i, r in enumerate(reqs[:20])]
    note(f"case serve mix graphs={graphs} requests={len(reqs)}")
    srv = Server(GpuExecutor(streams=4, graphs=graphs), budget_bytes=8 << 30, streams=4, paused=True)
    futs = [srv.submit(r) for r in reqs]
    srv.resume()
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.launches < len(reqs)
    for r, got in zip(reqs, res):
        e, gw, gx = _alone(r)
        np.testing.assert_allclose(got.expz, e, atol=2e-5)
        if r.want_grad:
            for a, b in ((got.grad_weights, gw), (got.grad_features, gx)):
                assert np.max(np.abs(a - b)) <= 1e-4 * max(np.max(np.abs(b)), 1e-30)


def test_graph_replays_equal_eager():
    t = W.Request(0, 0.0, 8, 16, 3, True)
    layers, w, x = W.request_params(t, seed=3)
    ex = GpuExecutor(streams=2, graphs=True)
    srv = Server(ex, budget_bytes=1 << 30, streams=2)
    outs = []
    for rep in range(4):
        f = srv.submit(Request(8, layers, w, x, want_grad=True, rid=rep))
        outs.append(f.result(timeout=60))
        # eager work between replays
        a = torch.randn(1 << 16, device="cuda")
        (a * 2).sum().item()
    srv.close()
    e, gw, gx = _alone(Request(8, layers, w, x, want_grad=True))
    for o in outs:
        np.testing.assert_allclose(o.expz, e, atol=2e-5)
        np.testing.assert_allclose(o.grad_weights, gw, rtol=1e-4, atol=1e-6)
    assert len(ex._graphs) >= 1


def test_heavy_lane_large_requests_equal_alone():
    """Large requests (up to 20 qubits) go through the heavy lane one at a time
    while small ones pass them; every result equals the request run alone."""
    reqs = _reqs(12, seed=21, n_range=(8, 20), b_max=16, blocks=(2, 3))
    note(f"case serve heavy requests={len(reqs)} n={[r.n for r in reqs]}")
    srv = Server(GpuExecutor(streams=4, graphs=True), budget_bytes=32 << 30, streams=4, paused=True,
                 heavy_bytes=64 << 20)
    futs = [srv.submit(r) for r in reqs]
    srv.resume()
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.max_heavy_inflight <= 1
    for r, got in zip(reqs, res):
        e, gw, gx = _alone(r)
        np.testing.assert_allclose(got.expz, e, atol=2e-5)
        if r.want_grad:
            for a, b in ((got.grad_weights, gw), (got.grad_features, gx)):
                assert np.max(np.abs(a - b)) <= 1e-4 * max(np.max(np.abs(b)), 1e-30)


def test_segment_sum_rows_in_order():
    """The device segment sum: each segment's rows summed in order in FP64
    (bit for bit against a sequential host sum), empty segments zero, and the
    column block respected."""
    from paper_2506_04891_amd import tqsim as T
    rng = np.random.default_rng(7)
    rows, ld = 300, 9
    x = rng.standard_normal((rows, ld))
    seg = np.array([0, 5, 5, 77, 200, 300], dtype=np.int32)
    xd = torch.tensor(x, device="cuda")
    out = T.segment_sum_rows(xd, 2, 6, torch.tensor(seg, device="cuda")).cpu().numpy()
    ref = np.zeros((len(seg) - 1, 6))
    for s in range(len(seg) - 1):
        acc = np.zeros(6)
        for r in range(seg[s], seg[s + 1]):
            acc = acc + x[r, 2:8]
        ref[s] = acc
    np.testing.assert_array_equal(out, ref)
    assert (out[1] == 0).all()
