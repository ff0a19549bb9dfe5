"""Scheduling logic of the serving loop, on the host (no GPU): results of
requests served in a mix equal the same requests served alone, the memory
budget is never exceeded, oversize requests are refused, same-structure
requests coalesce, an injected launch failure fails only its requests, and the
plain path runs one request at a time."""
import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2506_04891_amd.serve import HostExecutor, Request, Result, Server, bucket


def oracle_fn(req):
    e = sim.forward_expval(req.n, req.layers, req.weights, req.features)
    return Result(e)


def _requests(k, seed=0, grad_frac=0.0, n_range=(3, 5), b_max=8):
    trace = W.serving_trace(k, qps=1000.0, seed=seed, n_range=n_range, b_max=b_max, blocks_range=(1, 3),
                            grad_frac=grad_frac)
    out = []
    for t in trace:
        layers, w, x = W.request_params(t, seed=seed)
        out.append(Request(t.n, layers, w, x, want_grad=t.want_grad, rid=t.rid))
    return out


def test_mix_equals_alone():
    reqs = _requests(24, seed=1)
    ex = HostExecutor(oracle_fn, delay=0.002)
    srv = Server(ex, budget_bytes=64 << 20, streams=3)
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=30) for f in futs]
    srv.close()
    for r, got in zip(reqs, res):
        alone = oracle_fn(Request(r.n, r.layers, r.weights, r.features))
        np.testing.assert_array_equal(got.expz, alone.expz)
        assert got.latency is not None and got.latency >= 0
    st = srv.stats()
    assert st["requests"] == len(reqs) and st["errors"] == 0


def test_budget_is_never_exceeded():
    reqs = _requests(40, seed=2, b_max=16)
    row = 1 << 20
    budget = 24 * row
    ex = HostExecutor(oracle_fn, delay=0.003, row_bytes=row)
    srv = Server(ex, budget_bytes=budget, streams=4)
    for r in reqs:
        srv.submit(r)
    srv.drain(timeout=60)
    srv.close()
    assert 0 < srv.peak_reserved <= budget
    assert len(srv.completed) == len(reqs)


def test_oversize_request_is_refused():
    ex = HostExecutor(oracle_fn, row_bytes=1 << 20)
    srv = Server(ex, budget_bytes=4 << 20)
    big = _requests(1, seed=3, b_max=8)[0]
    big.features = np.zeros((64, big.features.shape[1]))
    f = srv.submit(big)
    with pytest.raises(MemoryError):
        f.result(timeout=5)
    srv.close()


def test_same_structure_requests_coalesce():
    layers = W.circuit_rot_ring(4, 2)
    nw, nf = W.circuit_counts(4, layers)
    rng = np.random.default_rng(0)
    reqs = [Request(4, layers, rng.standard_normal(nw), rng.uniform(-3, 3, (2, nf)), rid=i) for i in range(12)]
    ex = HostExecutor(oracle_fn, delay=0.02)
    srv = Server(ex, budget_bytes=1 << 30, streams=1, paused=True)
    futs = [srv.submit(r) for r in reqs]
    srv.resume()
    [f.result(timeout=30) for f in futs]
    srv.close()
    assert len(ex.launched) < len(reqs)            # later requests rode along
    assert sorted(sum(ex.launched, [])) == list(range(12))
    for r, f in zip(reqs, futs):
        np.testing.assert_array_equal(f.result().expz, oracle_fn(r).expz)


def test_injected_failure_fails_only_its_requests():
    reqs = _requests(10, seed=4)
    # give every request its own structure so that no launch mixes requests
    ex = HostExecutor(oracle_fn, delay=0.001, fail_on={3})
    srv = Server(ex, budget_bytes=1 << 30, streams=2, max_rows=1)
    futs = [srv.submit(r) for r in reqs]
    for r, f in zip(reqs, futs):
        if r.rid == 3:
            with pytest.raises(RuntimeError):
                f.result(timeout=30)
        else:
            f.result(timeout=30)
    srv.close()
    assert srv.stats()["errors"] == 1


def test_plain_path_is_one_request_per_launch():
    reqs = _requests(15, seed=5)
    ex = HostExecutor(oracle_fn, delay=0.001)
    srv = Server(ex, budget_bytes=1 << 30, streams=4, plain=True)
    futs = [srv.submit(r) for r in reqs]
    [f.result(timeout=30) for f in futs]
    srv.close()
    assert ex.max_concurrent == 1
    assert all(len(l) == 1 for l in ex.launched) and len(ex.launched) == len(reqs)


def test_light_launches_beside_a_heavy_one_are_capped():
    """With light_during_heavy = 1, at most one small launch runs beside a heavy
    one, small ones still overlap with it, and every result equals the request
    alone."""
    reqs = _requests(40, seed=7, b_max=32)
    row = 1 << 20
    ex = HostExecutor(oracle_fn, delay=0.004, row_bytes=row)
    srv = Server(ex, budget_bytes=1 << 40, streams=4, heavy_bytes=8 * row, light_during_heavy=1, paused=True)
    futs = [srv.submit(r) for r in reqs]
    srv.resume()
    res = [f.result(timeout=60) for f in futs]
    srv.close()
    assert srv.max_heavy_inflight == 1
    assert srv.max_light_beside_heavy == 1
    for r, got in zip(reqs, res):
        np.testing.assert_array_equal(got.expz, oracle_fn(r).expz)


def test_bucket():
    assert [bucket(b) for b in (1, 2, 3, 5, 8, 9, 512, 513)] == [1, 2, 4, 8, 8, 16, 512, 1024]


def test_one_heavy_launch_at_a_time():
    """Launches reserving more than heavy_bytes never overlap each other, small
    ones still overlap with them, and every result equals the request alone."""
    reqs = _requests(40, seed=6, b_max=32)
    row = 1 << 20
    ex = HostExecutor(oracle_fn, delay=0.004, row_bytes=row)
    srv = Server(ex, budget_bytes=1 << 40, streams=4, heavy_bytes=8 * row, paused=True)
    futs = [srv.submit(r) for r in reqs]
    srv.resume()
    res = [f.result(timeout=60) for f in futs]
    srv.close()
    assert srv.max_heavy_inflight == 1
    assert ex.max_concurrent > 1
    assert any(bucket(r.batch) > 8 for r in reqs) and any(bucket(r.batch) <= 8 for r in reqs)
    for r, got in zip(reqs, res):
        np.testing.assert_array_equal(got.expz, oracle_fn(r).expz)
