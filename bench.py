#!/usr/bin/env python3
"""Benchmark: forward + adjoint-backward circuit evaluations per second at
16 qubits, batch 128, complex64, on the IonQ-style and IBM-style native-gate
circuits (one step = both circuits, forward <Z_i> and adjoint gradients of all
weights and features, for the whole batch).

Prints one JSON line.  Besides the headline value it reports the roofline of
the dominant kernel (HIP-event durations measured inside this run), the same
figures for the 20-qubit rotation + ZZ + CNOT-ring circuit (where the state
set exceeds the on-chip caches), and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 instructions (the kernels are built
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop/FMA x 2.4 GHz.
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
BALANCE = VALU_FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)   # flop per byte


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-20q", action="store_true")
    p.add_argument("--mode", default="auto", choices=["auto", "per_layer", "fused"])
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--serve-requests", type=int, default=160)
    p.add_argument("--serve-max-qubits", type=int, default=22)
    p.add_argument("--serve-qps-fracs", default="0.5,0.8,0.95")
    p.add_argument("--no-b512", action="store_true")
    p.add_argument("--no-graph", action="store_true", help="time eager launches instead of a replayed HIP graph")
    # after the timed region, run a plain streaming kernel (float32 negation)
    # over this many MiB three times: the known-size reference that scales
    # rocprofv3's FETCH_SIZE / WRITE_SIZE readings to bytes
    p.add_argument("--calibrate-copy-mib", type=int, default=0)
    # instead of the benchmark: time forward + adjoint of small circuits under
    # each dispatch mode (tile passes per layer, fused tile passes, dense
    # matrix-core layers) and print one JSON line per case
    p.add_argument("--dense-sweep", action="store_true")
    # instead of the benchmark: time every configuration under each dispatch
    # mode and tile size, one JSON line per case
    p.add_argument("--dispatch-sweep", action="store_true")
    p.add_argument("--memory-sweep", action="store_true",
                   help="device memory of one forward + adjoint call vs qubits (QDI circuit)")
    p.add_argument("--vq-qdi-sweep", action="store_true",
                   help="forward/backward/total time vs qubits for the VQ and QDI encodings")
    return p.parse_args()


def traffic_file(kind, workload="16q_b128"):
    return os.path.join(ROOT, "profiles", f"traffic_{kind}_{workload}.txt")


def roofline(report, traffic_path=None):
    """Roofline object of the kernel kind with the largest total time.
    `traffic` is the counter-measured HBM bytes per launch of that kernel,
    from the summary at `traffic_path` when it was taken on these sources."""
    from paper_2506_04891_amd.rocprof_summary import read_traffic
    kinds = {k: v for k, v in report.items() if v["count"] > 0}
    name = max(kinds, key=lambda k: kinds[k]["ms"])
    traffic = read_traffic(traffic_path(name), name) if traffic_path else None
    r = kinds[name]
    sec = r["ms"] / 1e3
    intensity = r["flops"] / max(r["bytes"], 1.0)
    if intensity > BALANCE:
        achieved = r["flops"] / sec / 1e12
        out = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_FP32_PEAK_TFLOPS, 1),
               "unit": "TFLOP/s", "frac": round(achieved / VALU_FP32_PEAK_TFLOPS, 4)}
    else:
        achieved = r["bytes"] / sec / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4)}
    out.update({"traffic": traffic, "kernel": name, "launches": r["count"],
                "avg_launch_us": round(r["ms"] * 1e3 / r["count"], 2),
                "bytes_per_launch": r["bytes"] / r["count"], "flops_per_launch": r["flops"] / r["count"],
                "hbm_GBps": round(r["bytes"] / sec / 1e9, 1),
                "valu_TFLOPs": round(r["flops"] / sec / 1e12, 3)})
    return out


class Job:
    """One circuit at its full batch, device tensors resident in HBM."""

    def __init__(self, name, mode, batch=None):
        import torch
        import workloads as W
        from paper_2506_04891_amd import tqsim as T
        n, B, dt, layers, w, x = W.config(name)
        if batch is not None:
            cfg = W.CONFIGS[name]
            B = batch
            w, x = W.draw_params(n, layers, B, cfg["wdist"], cfg["seed"])
        self.name, self.n, self.B = name, n, B
        self.circ = T.Circuit(n, layers, dt, mode=mode)
        dev = torch.device("cuda")
        self.w = torch.tensor(w, device=dev)
        self.x = torch.tensor(x, device=dev)
        self.g = torch.tensor(W.upstream(B, n, "ones"), device=dev)
        self.state = torch.empty((B, 2 ** n), dtype=self.circ.complex_dtype, device=dev)
        self.ws = self.circ.workspace(B, True, dev)

    def step(self):
        c = self.circ
        c.forward(self.w, self.x, state=self.state, ws=self.ws)
        self.e = c.expval_z(self.state, ws=self.ws)
        self.gw, self.gx = c.adjoint_grad(self.w, self.x, self.state, self.g, ws=self.ws)


def time_jobs(jobs, steps, warmup):
    import torch
    for _ in range(warmup):
        for j in jobs:
            j.step()
    torch.cuda.synchronize()
    for j in jobs:
        j.circ.profile_report(reset=True)
        j.circ.set_profile(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        for j in jobs:
            j.step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / steps
    merged = {}
    for j in jobs:
        j.circ.set_profile(False)
        for k, v in j.circ.profile_report(reset=True).items():
            m = merged.setdefault(k, {"count": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0})
            for f in m:
                m[f] += v[f]
    return ms, wall / steps * 1e3, merged


def serving_bench(n_req, n_max, fracs, seed=0, streams=4, budget=160 << 30, heavy=256 << 20):
    """Continuous batching vs the plain per-request path on one Poisson trace of
    rotation + CNOT-ring circuits (qubits U{6..n_max}, batch log-U[1, 512],
    blocks U{2..20}, 30% forward+gradient).  Launches reserving more than
    `heavy` bytes fill the device alone and run one at a time."""
    import numpy as np
    import workloads as W
    from paper_2506_04891_amd.serve import GpuExecutor, Request, Server

    def make(qps):
        trace = W.serving_trace(n_req, qps=qps, seed=seed, n_range=(6, n_max))
        reqs = []
        for t in trace:
            layers, w, x = W.request_params(t, seed=seed)
            reqs.append((t.t_arrive, Request(t.n, layers, w, x, want_grad=t.want_grad, rid=t.rid)))
        return reqs

    def run(reqs, plain, ex):
        srv = Server(ex, budget_bytes=budget, streams=streams, plain=plain, heavy_bytes=heavy)
        t0 = time.perf_counter()
        futs = []
        for ta, r in reqs:
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            futs.append(srv.submit(r))
        for f in futs:
            f.result(timeout=600)
        st = srv.stats()
        srv.close()
        return st

    ex = GpuExecutor(streams=streams, graphs=True)
    ex_plain = GpuExecutor(streams=1, graphs=False)
    # warm-up: compile every circuit and capture graphs (untimed)
    base = make(1e6)
    run([(0.0, Request(r.n, r.layers, r.weights, r.features, r.want_grad)) for _, r in base], False, ex)
    run([(0.0, Request(r.n, r.layers, r.weights, r.features, r.want_grad)) for _, r in base], True, ex_plain)
    sat = run([(0.0, r) for _, r in make(1e6)], False, ex)
    req_per_s = sat["requests"] / max(1e-9, (sat["evals"] / max(sat["evals_per_s"], 1e-9)))
    out = {"trace": f"{n_req} requests, qubits U{{6..{n_max}}}, batch log-U[1,512], blocks U{{2..20}}, "
                    f"30% forward+gradient, seed {seed}; {streams} streams, one launch above "
                    f"{heavy >> 20} MiB at a time; warm circuits and graphs",
           "saturation": {"requests_per_s": round(req_per_s, 1), "evals_per_s": round(sat["evals_per_s"], 1)},
           "points": []}
    for frac in fracs:
        qps = frac * req_per_s
        cb = run(make(qps), False, ex)
        pl = run(make(qps), True, ex_plain)
        out["points"].append({"qps": round(qps, 1), "frac_of_saturation": frac,
                              "continuous": {k: round(cb[k], 3) for k in ("p50_ms", "p99_ms", "evals_per_s")}
                              | {"launches": cb["launches"]},
                              "plain": {k: round(pl[k], 3) for k in ("p50_ms", "p99_ms", "evals_per_s")}})
    return out


def time_graph(jobs, steps, warmup):
    """ms per step with the whole step (every job's forward, <Z_i> and adjoint)
    captured once as a HIP graph and replayed: no per-kernel launch gaps and
    no profiling events.  Before and after the timed replays, replays
    alternate with eager steps and each replay's outputs must equal the eager
    step's bit for bit (the path is deterministic)."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for j in jobs:
            j.step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for j in jobs:
            j.step()
    outs = [(j.e, j.gw, j.gx) for j in jobs]

    def check(rounds):
        for _ in range(rounds):
            graph.replay()
            torch.cuda.synchronize()
            got = [tuple(t.clone() for t in o) for o in outs]
            for j in jobs:
                j.step()
            torch.cuda.synchronize()
            for j, g in zip(jobs, got):
                for a, b in zip(g, (j.e, j.gw, j.gx)):
                    if not torch.equal(a, b):
                        raise RuntimeError(f"graph replay of {j.name} differs from the eager step")

    check(3)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        graph.replay()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    check(1)
    ms = t0.elapsed_time(t1) / steps
    del graph
    return ms, wall / steps * 1e3


def dense_sweep(iters=30):
    """Per-call time of forward + <Z> + adjoint for n = 2..6 under each mode;
    for dense mode also the rate of the dense pass kernels on the matrix cores
    (8 * 2^n flop per amplitude per dense layer)."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for n in (2, 4, 5, 6):
        circuits = [("rot_ring", W.circuit_rot_ring(n, 10, "RY", ("RY", "RZ")), "normal")]
        if n % 2 == 0:
            circuits.append(("ionq", W.circuit_ionq(n, 8), "uniform2pi"))
        for name, layers, dist in circuits:
            for dt in ("c64", "c128"):
                for B in (16, 256, 4096):
                    row = {"n": n, "circuit": name, "dtype": dt, "batch": B}
                    for mode in ("per_layer", "fused", "dense"):
                        c = T.Circuit(n, layers, dt, mode=mode)
                        w, x = W.draw_params(n, layers, B, dist, 0)
                        wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
                        g = torch.ones((B, n), dtype=torch.float64, device=dev)
                        st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
                        ws = c.workspace(B, True, dev)

                        def step():
                            c.forward(wt, xt, state=st, ws=ws)
                            c.expval_z(st, ws=ws)
                            c.adjoint_grad(wt, xt, st, g, ws=ws)
                        for _ in range(3):
                            step()
                        torch.cuda.synchronize()
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        for _ in range(iters):
                            step()
                        e1.record()
                        torch.cuda.synchronize()
                        row[mode + "_us"] = round(e0.elapsed_time(e1) / iters * 1e3, 1)
                        if mode == "dense":
                            c.profile_report(reset=True)
                            c.set_profile(True)
                            step()
                            c.set_profile(False)
                            rep = c.profile_report(reset=True)
                            ms = sum(v["ms"] for k, v in rep.items() if k.startswith("pass"))
                            fl = sum(v["flops"] for k, v in rep.items() if k.startswith("pass"))
                            row["dense_pass_us"] = round(ms * 1e3, 1)
                            row["dense_pass_TFLOPs"] = round(fl / max(ms, 1e-9) / 1e9, 2)
                    print(json.dumps(row), flush=True)


def dispatch_sweep(iters=10):
    """ms per forward + <Z> + adjoint step of each configuration under the
    per-layer, fused and dense modes and tile sizes 10..12 (0 = automatic)."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for name in ("c1_4q_b16", "c2_12q_b256", "c4a_16q_b128_ionq", "c4b_16q_b128_ibm", "c3_20q_b32"):
        n, B, dt, layers, w, x = W.config(name)
        for mode in ("auto", "per_layer", "fused", "dense"):
            for K in ((0,) if mode in ("auto", "dense") else (0, 10, 11, 12)):
                if mode == "dense" and n > 6:
                    continue
                c = T.Circuit(n, layers, dt, mode=mode, tile_bits=K)
                wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
                g = torch.ones((B, n), dtype=torch.float64, device=dev)
                st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
                ws = c.workspace(B, True, dev)

                def step():
                    c.forward(wt, xt, state=st, ws=ws)
                    c.expval_z(st, ws=ws)
                    c.adjoint_grad(wt, xt, st, g, ws=ws)
                for _ in range(3):
                    step()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(iters):
                    step()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / iters
                plan = c.plan()
                print(json.dumps({"config": name, "mode": mode, "tile_bits": K, "plan_mode": plan["mode"],
                                  "passes": len(plan["passes"]), "ms_per_step": round(ms, 4),
                                  "evals_per_s": round(B / ms * 1e3, 1)}), flush=True)


def vq_qdi_sweep(iters=20):
    """Fig. 8's measurement on the Rz-Ry-CNOT circuit of Fig. 6 (8 blocks):
    forward (+ <Z_i>), backward (adjoint) and total time per call against the
    number of qubits, at batch 1 and 64, for VQ and QDI encodings (c64)."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for enc in ("vq", "qdi"):
        for B in (1, 64):
            for n in (4, 6, 8, 10, 12, 14, 16, 18, 20, 22):
                if B * (8 << n) > (4 << 30):
                    continue
                layers = W.circuit_rz_ry_cnot(n, 8, enc)
                c = T.Circuit(n, layers, "c64")
                w, x = W.draw_params(n, layers, B, "normal", 0)
                wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
                g = torch.ones((B, n), dtype=torch.float64, device=dev)
                st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
                ws = c.workspace(B, True, dev)

                def fwd():
                    c.forward(wt, xt, state=st, ws=ws)
                    c.expval_z(st, ws=ws)

                def step():
                    fwd()
                    c.adjoint_grad(wt, xt, st, g, ws=ws)

                row = {"encoding": enc, "batch": B, "n": n, "passes": len(c.plan()["passes"])}
                for name, fn in (("fwd", fwd), ("total", step)):
                    for _ in range(3):
                        fn()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(iters):
                        fn()
                    e1.record()
                    torch.cuda.synchronize()
                    row[name + "_us"] = round(e0.elapsed_time(e1) / iters * 1e3, 1)
                row["bwd_us"] = round(row["total_us"] - row["fwd_us"], 1)
                print(json.dumps(row), flush=True)


def memory_sweep():
    """Fig. 9's measurement on the QDI circuit of Fig. 6 (8 blocks, c64): the
    device memory of one forward + <Z_i> + adjoint call against the number of
    qubits at batch 1 and 100.  Reported: the library's workspace query, the
    state, and the peak the caching allocator saw during the call (all
    buffers the call needs); beside them, the states a per-layer
    stored-state backpropagation would keep (computed, (L+1) states)."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for B in (1, 100):
        for n in range(4, 23, 2):
            layers = W.circuit_rz_ry_cnot(n, 8, "qdi")
            c = T.Circuit(n, layers, "c64")
            w, x = W.draw_params(n, layers, B, "normal", 0)
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats()
            base = torch.cuda.memory_allocated()
            wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
            g = torch.ones((B, n), dtype=torch.float64, device=dev)
            st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
            ws = c.workspace(B, True, dev)
            c.forward(wt, xt, state=st, ws=ws)
            e = c.expval_z(st, ws=ws)
            gw, gx = c.adjoint_grad(wt, xt, st, g, ws=ws)
            torch.cuda.synchronize()
            peak = torch.cuda.max_memory_allocated() - base
            state = B * (8 << n)
            print(json.dumps({"encoding": "qdi", "batch": B, "n": n, "layers": len(layers),
                              "state_bytes": state, "workspace_bytes": c.workspace_size(B, True),
                              "peak_bytes": int(peak),
                              "stored_state_backprop_bytes": (len(layers) + 1) * state}), flush=True)
            del wt, xt, g, st, ws, e, gw, gx, c


def _oracle_samples(samples, seed_offset=0, keep=None):
    """Seconds the oracle (numpy complex128, one BLAS thread) takes for forward
    <Z_i> + adjoint gradients of `samples` rows of each 16-qubit circuit.
    keep: dict that receives {circuit: (rows, expz, grad_w, grad_x)}."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import sim
    t = 0.0
    with threadpool_limits(limits=1):
        for name in ("c4a_16q_b128_ionq", "c4b_16q_b128_ibm"):
            n, B, dt, layers, w, x = W.config(name)
            rows = [(seed_offset + k) % B for k in range(samples)]
            xs = x[rows]
            g = W.upstream(samples, n, "ones")
            t0 = time.perf_counter()
            res = sim.grad_adjoint(n, layers, w, xs, g)
            t += time.perf_counter() - t0
            if keep is not None:
                keep[name] = (rows, *res)
    return t


def _pool_worker(k, per_worker):
    return _oracle_samples(per_worker, seed_offset=k * per_worker)


def cpu_baseline(sample=12, keep=None):
    """The oracle on `sample` rows of each 16-qubit circuit, one thread."""
    t = _oracle_samples(sample, keep=keep)
    evals = 2 * sample
    return {"value": round(evals / t, 3), "unit": "circuit evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample} rows of each 16-qubit circuit (IonQ and IBM gate sets), forward + adjoint "
                      f"gradients in numpy complex128 on one thread (BLAS limited to 1); {round(t, 2)} s; "
                      f"host has {os.cpu_count()} logical CPUs"}


def errors_vs_oracle(jobs, ref):
    """Max errors of the benchmarked GPU path against the oracle rows kept by
    cpu_baseline: <Z_i> (max abs), weight and feature gradients (max abs over
    max |ref|), with the upstream gradient one on those rows and zero elsewhere."""
    import numpy as np
    import torch
    out = {}
    for j in jobs:
        if j.name not in ref:
            continue
        rows, e_ref, gw_ref, gx_ref = ref[j.name]
        c = j.circ
        c.forward(j.w, j.x, state=j.state, ws=j.ws)
        e = c.expval_z(j.state, ws=j.ws).cpu().numpy()
        g = torch.zeros_like(j.g)
        g[rows] = 1.0
        gw, gx = c.adjoint_grad(j.w, j.x, j.state, g, ws=j.ws)
        gw, gx = gw.cpu().numpy(), gx.cpu().numpy()
        out[j.name] = {"rows": rows,
                       "expz_max_abs": float(np.max(np.abs(e[rows] - e_ref))),
                       "grad_weights_max_rel": float(np.max(np.abs(gw - gw_ref)) / np.max(np.abs(gw_ref))),
                       "grad_features_max_rel": float(np.max(np.abs(gx[rows] - gx_ref)) / np.max(np.abs(gx_ref)))}
    return out


def cpu_baseline_pool(per_worker=6):
    """The same oracle over a process pool (one process per core, one thread
    each; at most 16 cores), parallel over samples.  Run before the GPU is
    initialised: the pool forks this process."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.starmap(_pool_worker, [(k, per_worker) for k in range(cores)])
    wall = time.perf_counter() - t0
    evals = 2 * per_worker * cores
    return {"value": round(evals / wall, 3), "unit": "circuit evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{per_worker} rows of each 16-qubit circuit per process, {cores} processes; "
                      f"{round(wall, 2)} s wall including pool start-up"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    # the CPU baselines run first: the pooled one forks, which must happen
    # before anything initialises the GPU in this process
    oracle_rows = {}
    sweep = a.dense_sweep or a.dispatch_sweep or a.vq_qdi_sweep or a.memory_sweep
    cpu = None if (a.no_cpu_baseline or sweep) else cpu_baseline(keep=oracle_rows)
    cpu_pool = None if (a.no_cpu_baseline or sweep) else cpu_baseline_pool()
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_2506_04891_amd import tqsim as T
    T.lib()   # fails loudly when the HIP library is missing
    if a.dense_sweep:
        dense_sweep()
        return
    if a.dispatch_sweep:
        dispatch_sweep()
        return
    if a.vq_qdi_sweep:
        vq_qdi_sweep()
        return
    if a.memory_sweep:
        memory_sweep()
        return

    jobs = [Job("c4a_16q_b128_ionq", a.mode), Job("c4b_16q_b128_ibm", a.mode)]
    # per-kernel times: an eager run with the library's HIP events
    ms_eager, wall_eager, rep = time_jobs(jobs, a.steps, a.warmup)
    if a.no_graph:
        ms, wall_ms = ms_eager, wall_eager
    else:
        ms, wall_ms = time_graph(jobs, a.steps, a.warmup)
    evals = sum(j.B for j in jobs)
    value = evals / (ms / 1e3)
    out = {
        "metric": "fwd+bwd circuit evals/s @16q batch128",
        "value": round(value, 1),
        "unit": "circuit evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "wall_ms_per_step": round(wall_ms, 4),
        "execution": ("eager launches" if a.no_graph else
                      "one HIP graph per step (both circuits' forward, <Z_i> and adjoint), replayed; "
                      "replays checked bit for bit against eager steps before and after timing"),
        "eager_ms_per_step": round(ms_eager, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (f32 state, f64 reductions)",
        "data": "synthetic (seeded weights U(0,2pi), features U(-pi,pi), upstream dL/d<Z>=1)",
        "config": {"workload": "16 qubits, batch 128, complex64: IonQ GPI/GPI2/MS and IBM RZ/SX/ECR "
                               "native-gate circuits, 8 blocks each, forward <Z_i> + adjoint gradients",
                   "n_qubits": 16, "batch": 128, "circuits": [j.name for j in jobs],
                   "mode": a.mode, "passes": {j.name: len(j.circ.plan()["passes"]) for j in jobs}},
        "roofline": roofline(rep, traffic_file),
        "kernels": {k: {"count": v["count"], "ms_per_step": round(v["ms"] / a.steps, 4)} for k, v in rep.items()},
        "errors_vs_oracle": errors_vs_oracle(jobs, oracle_rows),
    }
    if a.calibrate_copy_mib > 0:
        src = torch.ones(a.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not a.no_b512:
        jb = [Job("c4a_16q_b128_ionq", a.mode, 512), Job("c4b_16q_b128_ibm", a.mode, 512)]
        msb, _, repb = time_jobs(jb, max(3, a.steps // 4), 2)
        out["q16_b512"] = {"workload": "the same two 16-qubit circuits at batch 512 (256 MiB per state set, "
                                       "larger than the last-level cache)",
                           "evals_per_s": round(1024 / (msb / 1e3), 1), "ms_per_step": round(msb, 3),
                           "roofline": roofline(repb)}
        del jb
    if not a.no_20q:
        j20 = Job("c3_20q_b32", a.mode)
        ms20, _, rep20 = time_jobs([j20], max(3, a.steps // 4), 2)
        out["q20"] = {"workload": "20 qubits, batch 32, complex64: RX embedding + 6 x [RX, RY, RZ, ZZ ring, "
                                  "CNOT ring], forward <Z_i> + adjoint gradients",
                      "evals_per_s": round(j20.B / (ms20 / 1e3), 1), "ms_per_step": round(ms20, 3),
                      "roofline": roofline(rep20, lambda k: traffic_file(k, "20q_b32")),
                      "kernels": {k: {"count": v["count"], "ms": round(v["ms"], 3)} for k, v in rep20.items()}}
        del j20
    if not a.no_serve:
        out["serving"] = serving_bench(a.serve_requests, a.serve_max_qubits,
                                       [float(f) for f in a.serve_qps_fracs.split(",")])
    out["cpu_baseline"] = cpu
    out["cpu_baseline_all_cores"] = cpu_pool
    print(json.dumps(out))


if __name__ == "__main__":
    main()
