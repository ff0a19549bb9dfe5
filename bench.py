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
import itertools
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
    p.add_argument("--serve-requests", type=int, default=300,
                   help="measured requests per arrival rate (2000 for the full protocol)")
    p.add_argument("--serve-max-qubits", type=int, default=22)
    p.add_argument("--serve-qps-fracs", default="0.5,0.8,0.95")
    p.add_argument("--no-b512", action="store_true")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the complex128 headline, the 4-qubit and the 12-qubit legs")
    p.add_argument("--serve-warmup", type=int, default=50,
                   help="warm-up requests per arrival rate, left out of the statistics (200 for the full protocol)")
    p.add_argument("--serve-light-during-heavy", type=int, default=1,
                   help="continuous path: at most this many small launches beside a heavy one (negative: no cap)")
    p.add_argument("--serve-compare-light-cap", type=int, default=None,
                   help="also run the continuous path under this cap at every point")
    p.add_argument("--serve-only", action="store_true",
                   help="run only the serving comparison and print its JSON")
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
    p.add_argument("--technique-sweep", action="store_true",
                   help="forward time of one layer of each kind under each layer technique, n = 4..20")
    p.add_argument("--tile-sweep", action="store_true",
                   help="forward + adjoint at batch 1-16, n = 14..20, for tile sizes 10..12")
    p.add_argument("--backward-sweep", action="store_true",
                   help="adjoint vs stored-state backward on the benchmark workloads")
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

    def __init__(self, name, mode, batch=None, dtype=None, grad=True):
        import torch
        import workloads as W
        from paper_2506_04891_amd import tqsim as T
        n, B, dt, layers, w, x = W.config(name)
        if batch is not None:
            cfg = W.CONFIGS[name]
            B = batch
            w, x = W.draw_params(n, layers, B, cfg["wdist"], cfg["seed"])
        self.name, self.n, self.B, self.grad = name, n, B, grad
        self.layers, self.w_host, self.x_host = layers, w, x
        # the dispatcher's backward: stored states while they fit its memory
        # cap (8 GiB), the adjoint uncompute otherwise
        self.circ = T.Circuit(n, layers, dtype or dt, mode=mode, backward="auto")
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
        if self.grad:
            self.gw, self.gx = c.adjoint_grad(self.w, self.x, self.state, self.g, ws=self.ws)

    def outputs(self):
        return (self.e, self.gw, self.gx) if self.grad else (self.e,)


def time_jobs(jobs, steps, warmup):
    import torch
    for _ in range(warmup):
        for j in jobs:
            j.step()
    torch.cuda.synchronize()
    for j in jobs:
        j.circ.profile_report(reset=True)
        j.circ.set_profile(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        for j in jobs:
            j.step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    ms = ev[0].elapsed_time(ev[steps]) / steps
    merged = {}
    for j in jobs:
        j.circ.set_profile(False)
        for k, v in j.circ.profile_report(reset=True).items():
            m = merged.setdefault(k, {"count": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0})
            for f in m:
                m[f] += v[f]
    return ms, wall / steps * 1e3, merged, step_stats(per)


def step_stats(per):
    """mean, std and median of per-step times (ms): the paper's protocol
    (mean and spread after warm-up, Sec. 2.1) and the median."""
    import numpy as np
    a = np.asarray(per, dtype=float)
    return {"steps": int(a.size), "mean_ms": round(float(a.mean()), 4), "std_ms": round(float(a.std()), 4),
            "median_ms": round(float(np.median(a)), 4), "min_ms": round(float(a.min()), 4),
            "max_ms": round(float(a.max()), 4)}


def serving_bench(n_req, n_max, fracs, seed=0, streams=4, budget=160 << 30, heavy=256 << 20, warm=200,
                  light_during_heavy=1, compare_light=None):
    """Continuous batching vs the plain per-request path on one Poisson trace of
    rotation + CNOT-ring circuits (qubits U{6..n_max}, batch log-U[1, 512],
    blocks U{2..20}, 30% forward+gradient): `warm` requests, then `n_req`
    measured ones, per arrival rate.  Launches reserving more than `heavy`
    bytes run one at a time, with at most `light_during_heavy` small launches
    beside them (None: every free stream).  With `compare_light`, each point
    also runs the continuous path under that cap instead."""
    import numpy as np
    import workloads as W
    from paper_2506_04891_amd.serve import GpuExecutor, Request, Server

    def make(qps):
        trace = W.serving_trace(warm + n_req, qps=qps, seed=seed, n_range=(6, n_max))
        reqs = []
        for t in trace:
            layers, w, x = W.request_params(t, seed=seed)
            reqs.append((t.t_arrive, Request(t.n, layers, w, x, want_grad=t.want_grad, rid=t.rid)))
        return reqs

    def run(reqs, plain, ex, light=light_during_heavy):
        print(f"serving: {len(reqs)} requests, {'plain' if plain else 'continuous'}", file=sys.stderr, flush=True)
        srv = Server(ex, budget_bytes=budget, streams=streams, plain=plain, heavy_bytes=heavy,
                     light_during_heavy=light)
        t0 = time.perf_counter()
        futs = []
        for ta, r in reqs:
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            futs.append(srv.submit(r))
        for f in futs:
            f.result(timeout=600)
        st = srv.stats(min_rid=warm)
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
    out = {"trace": f"{warm} warm-up + {n_req} measured requests per point, qubits U{{6..{n_max}}}, batch log-U[1,512], blocks U{{2..20}}, "
                    f"30% forward+gradient, seed {seed}; {streams} streams, one launch above "
                    f"{heavy >> 20} MiB at a time"
                    + (f" with at most {light_during_heavy} other launch(es) beside it" if light_during_heavy is not None else "")
                    + "; warm circuits and graphs",
           "saturation": {"requests_per_s": round(req_per_s, 1), "evals_per_s": round(sat["evals_per_s"], 1)},
           "points": []}
    for frac in fracs:
        qps = frac * req_per_s
        cb = run(make(qps), False, ex)
        pl = run(make(qps), True, ex_plain)
        point = {"qps": round(qps, 1), "frac_of_saturation": frac,
                 "continuous": {k: round(cb[k], 3) for k in ("p50_ms", "p99_ms", "evals_per_s")}
                 | {"launches": cb["launches"]},
                 "plain": {k: round(pl[k], 3) for k in ("p50_ms", "p99_ms", "evals_per_s")}}
        if compare_light is not None:
            cc = run(make(qps), False, ex, light=compare_light)
            point[f"continuous_light_cap_{compare_light}"] = (
                {k: round(cc[k], 3) for k in ("p50_ms", "p99_ms", "evals_per_s")} | {"launches": cc["launches"]})
        out["points"].append(point)
    return out


def light_cap(v):
    return None if v is None or v < 0 else v


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
    outs = [j.outputs() for j in jobs]

    def check(rounds):
        for _ in range(rounds):
            graph.replay()
            torch.cuda.synchronize()
            got = [tuple(t.clone() for t in o) for o in outs]
            for j in jobs:
                j.step()
            torch.cuda.synchronize()
            for j, g in zip(jobs, got):
                for a, b in zip(g, j.outputs()):
                    if not torch.equal(a, b):
                        raise RuntimeError(f"graph replay of {j.name} differs from the eager step")

    check(3)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        graph.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    check(1)
    ms = ev[0].elapsed_time(ev[steps]) / steps
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    del graph
    return ms, wall / steps * 1e3, step_stats(per)


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
    """Fig. 8's measurement on the Rz-Ry-CNOT circuit of Fig. 6 (8 blocks), and
    Figs. 12-13's on the IonQ and IBM native-gate circuits of App. B (8
    blocks): forward (+ <Z_i>), backward (adjoint) and total time per call
    against the number of qubits, at batch 1 and 64, for VQ and QDI encodings
    (c64); eager calls, and the same calls replayed as HIP graphs."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    circuits = (("rz_ry_cnot", W.circuit_rz_ry_cnot, "normal"), ("ionq", W.circuit_ionq, "uniform2pi"),
                ("ibm", W.circuit_ibm, "uniform2pi"))
    for (cname, build, dist), enc in itertools.product(circuits, ("vq", "qdi")):
        for B in (1, 64):
            for n in (4, 6, 8, 10, 12, 14, 16, 18, 20, 22):
                if B * (8 << n) > (4 << 30):
                    continue
                layers = build(n, 8, enc)
                c = T.Circuit(n, layers, "c64")
                w, x = W.draw_params(n, layers, B, dist, 0)
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

                row = {"circuit": cname, "encoding": enc, "batch": B, "n": n,
                       "passes": len(c.plan()["passes"])}
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
                # the same calls replayed as HIP graphs (tqsim.StepGraph): no
                # per-launch host cost
                for name, gr in (("fwd", None), ("total", g)):
                    sg = T.StepGraph(c, wt, xt, gr)
                    for _ in range(3):
                        sg.replay()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(iters):
                        sg.replay()
                    e1.record()
                    torch.cuda.synchronize()
                    row["graph_" + name + "_us"] = round(e0.elapsed_time(e1) / iters * 1e3, 1)
                    del sg
                print(json.dumps(row), flush=True)


def memory_sweep(iters=10):
    """Fig. 9's measurement on the QDI circuit of Fig. 6 (8 blocks, c64), for
    both backward modes: the device memory of one forward + <Z_i> + backward
    call against the number of qubits at batch 1 and 100 -- the peak the
    caching allocator saw during the call (state, workspace, parameters,
    outputs), measured, beside the library's workspace query -- and the time
    per call.  "adjoint" uncomputes psi; "stored" keeps every forward pass's
    output (the paper's stored-state backpropagation at pass granularity)."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for B in (1, 100):
        for n in range(4, 23, 2):
            layers = W.circuit_rz_ry_cnot(n, 8, "qdi")
            for bwd in ("adjoint", "stored"):
                c = T.Circuit(n, layers, "c64", backward=bwd)
                if bwd == "stored" and c.workspace_size(B, True) > (96 << 30):
                    continue
                w, x = W.draw_params(n, layers, B, "normal", 0)
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                torch.cuda.reset_peak_memory_stats()
                base = torch.cuda.memory_allocated()
                wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
                g = torch.ones((B, n), dtype=torch.float64, device=dev)
                st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
                ws = c.workspace(B, True, dev)

                def step():
                    c.forward(wt, xt, state=st, ws=ws)
                    c.expval_z(st, ws=ws)
                    return c.adjoint_grad(wt, xt, st, g, ws=ws)
                gw, gx = step()
                torch.cuda.synchronize()
                peak = torch.cuda.max_memory_allocated() - base
                for _ in range(2):
                    step()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(iters):
                    step()
                e1.record()
                torch.cuda.synchronize()
                state = B * (8 << n)
                passes = len([p for p in c.plan()["passes"] if not p["bwd_only"]])
                print(json.dumps({"encoding": "qdi", "backward": bwd, "batch": B, "n": n, "layers": len(layers),
                                  "forward_passes": passes, "state_bytes": state,
                                  "workspace_bytes": c.workspace_size(B, True), "peak_bytes": int(peak),
                                  "peak_states": round(peak / state, 2),
                                  "us_per_call": round(e0.elapsed_time(e1) / iters * 1e3, 1)}), flush=True)
                del wt, xt, g, st, ws, gw, gx, c


def technique_sweep(iters=20):
    """The per-layer benchmark of Secs. 2.2-2.5 (Figs. 2-5) on this GPU: the
    forward time of one layer of each kind under each technique the
    dispatcher can select, in per-layer mode, against the number of qubits,
    at batch 1 and 64 (c64).  The circuit is RY(x) embedding, CNOT ring, then
    the layer under test; the embedding-and-ring circuit alone is timed too,
    so the layer's own time is the difference."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    lead = [W.L("RY", "ALL", "INPUT"), W.L("CNOT", "RING")]
    kinds = {
        "RX": ([W.L("RX", "ALL", "WEIGHT")], ("kron", "hrz")),
        "RY": ([W.L("RY", "ALL", "WEIGHT")], ("kron", "hrz")),
        "Rot": ([W.L("ROT", "ALL", "WEIGHT")], ("kron", "hrz")),
        "GPI2": ([W.L("GPI2", "ALL", "WEIGHT")], ("kron", "hrz")),
        "H": ([W.L("H", "ALL")], ("real", "fhwt")),
        "RZ": ([W.L("RZ", "ALL", "WEIGHT")], ("tables", "einsum")),
        "ZZ": ([W.L("ZZ", "RING", "WEIGHT")], ("tables", "einsum")),
        "GPI": ([W.L("GPI", "ALL", "WEIGHT")], ("tables", "einsum")),
        "CNOT": ([W.L("CNOT", "RING")], ("gather",)),
    }
    opts = {"kron": {}, "hrz": {"hrz": True}, "real": {"fhwt": False}, "fhwt": {"fhwt": True},
            "tables": {"diag": "tables"}, "einsum": {"diag": "einsum"}, "gather": {}}

    def fwd_us(layers, n, B, **kw):
        c = T.Circuit(n, layers, "c64", mode="per_layer", **kw)
        w, x = W.draw_params(n, layers, B, "normal", 0)
        wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
        st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
        ws = c.workspace(B, False, dev)
        for _ in range(3):
            c.forward(wt, xt, state=st, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            c.forward(wt, xt, state=st, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) / iters * 1e3, 2)

    for B in (1, 64):
        for n in (4, 6, 8, 10, 12, 14, 16, 18, 20):
            base = fwd_us(lead, n, B)
            for kind, (ly, techs) in kinds.items():
                row = {"layer": kind, "n": n, "batch": B, "lead_us": base}
                for t in techs:
                    row[t + "_us"] = fwd_us(lead + ly, n, B, **opts[t])
                print(json.dumps(row), flush=True)


def tile_sweep(iters=10):
    """Forward + <Z_i> + adjoint of the QDI Fig. 6 circuit at small batch for
    tile sizes K = 10, 11, 12 (more workgroups per pass against more passes)."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for B in (1, 4, 16):
        for n in (14, 16, 18, 20):
            row = {"n": n, "B": B}
            for K in (10, 11, 12):
                layers = W.circuit_rz_ry_cnot(n, 8, "qdi")
                c = T.Circuit(n, layers, "c64", tile_bits=K)
                w, x = W.draw_params(n, layers, B, "normal", 0)
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
                row[f"K{K}_us"] = round(e0.elapsed_time(e1) / iters * 1e3, 1)
                row[f"K{K}_passes"] = len(c.plan()["passes"])
            print(json.dumps(row), flush=True)


def backward_sweep(iters=10):
    """Adjoint (uncompute) against stored-state backward on the benchmark
    workloads: ms per forward + <Z_i> + backward step, and workspace bytes."""
    import torch
    import workloads as W
    from paper_2506_04891_amd import tqsim as T
    dev = torch.device("cuda")
    for name in ("c2_12q_b256", "c4a_16q_b128_ionq", "c4b_16q_b128_ibm", "c3_20q_b32"):
        n, B, dt, layers, w, x = W.config(name)
        row = {"config": name}
        for bwd in ("adjoint", "stored"):
            c = T.Circuit(n, layers, dt, backward=bwd)
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
            row[bwd + "_ms"] = round(e0.elapsed_time(e1) / iters, 4)
            row[bwd + "_workspace_bytes"] = c.workspace_size(B, True)
            del c, ws, st
        print(json.dumps(row), flush=True)


C4 = ("c4a_16q_b128_ionq", "c4b_16q_b128_ibm")
C3_ORACLE_ROWS = (0, 10, 21, 31)


def _oracle_task(name, rows):
    """<Z_i> and adjoint gradients of `rows` of a configuration in the oracle
    (numpy complex128, one BLAS thread), upstream gradient one on those rows.
    Returns (name, rows, expz, grad_w summed over the rows, grad_x, seconds)."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import sim
    n, B, dt, layers, w, x = W.config(name)
    rows = list(rows)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        e, gw, gx = sim.grad_adjoint(n, layers, w, x[rows], W.upstream(len(rows), n, "ones"))
        return name, rows, e, gw, gx, time.perf_counter() - t0


def _merge(results):
    """Concatenate per-task oracle results per configuration (weight
    gradients summed over the tasks' rows)."""
    import numpy as np
    out = {}
    for name, rows, e, gw, gx, t in results:
        if name not in out:
            out[name] = [list(rows), [e], gw.copy(), [gx], t]
        else:
            o = out[name]
            o[0] += rows
            o[1].append(e)
            o[2] += gw
            o[3].append(gx)
            o[4] += t
    return {k: (v[0], np.concatenate(v[1]), v[2], np.concatenate(v[3]), v[4]) for k, v in out.items()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample=12):
    """The oracle on `sample` rows of each 16-qubit circuit, one thread."""
    t = sum(_oracle_task(name, range(sample))[-1] for name in C4)
    evals = 2 * sample
    return {"value": round(evals / t, 3), "unit": "circuit evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample} rows of each 16-qubit circuit (IonQ and IBM gate sets), forward + adjoint "
                      f"gradients in numpy complex128 on one thread (BLAS limited to 1); {round(t, 2)} s; "
                      f"host: {cpu_model()}, {os.cpu_count()} logical CPUs"}


def oracle_pool():
    """The oracle over a process pool (one process per core, one thread each,
    at most 16), parallel over samples.  First every row of both 16-qubit
    circuits (timed: the all-cores baseline); then four rows of the 20-qubit
    circuit, every row of the 12-qubit one and the 4-qubit forward.  The
    results are kept to check the GPU outputs on the same rows.  Run before
    the GPU is initialised: the pool forks this process."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        r16 = pool.starmap(_oracle_task, [(name, range(k, k + 8)) for name in C4 for k in range(0, 128, 8)])
        wall16 = time.perf_counter() - t0
        t1 = time.perf_counter()
        other = ([("c3_20q_b32", [r]) for r in C3_ORACLE_ROWS] +
                 [("c2_12q_b256", range(k, k + 32)) for k in range(0, 256, 32)] + [("c1_4q_b16", range(16))])
        rest = pool.starmap(_oracle_task, other)
        wall_rest = time.perf_counter() - t1
    ref = _merge(r16 + rest)
    c3_t = [r[-1] for r in rest if r[0] == "c3_20q_b32"]
    return ref, {
        "all_cores": {"value": round(256 / wall16, 3), "unit": "circuit evals/s", "cores": cores, "kind": "oracle",
                      "sample": f"all 128 rows of each 16-qubit circuit over {cores} processes (one thread each); "
                                f"{round(wall16, 2)} s wall including pool start-up"},
        "c3_20q_b32": {"rows": list(C3_ORACLE_ROWS), "seconds_per_eval": round(sum(c3_t) / len(c3_t), 2),
                       "evals_per_s_one_core": round(len(c3_t) / sum(c3_t), 4),
                       "sample": "4 of the 32 samples, forward + adjoint, one process per row, one thread each"},
        "c2_12q_b256": {"evals_per_s_one_core": round(256 / ref["c2_12q_b256"][4], 2),
                        "sample": "all 256 rows, forward + adjoint"},
        "c1_4q_b16": {"cpu_seconds": round(ref["c1_4q_b16"][4], 4),
                      "sample": "all 16 rows, forward <Z_i> (and the adjoint, which the oracle computes with it)"},
        "wall_s_other": round(wall_rest, 2)}


def errors_vs_oracle(job, ref):
    """Max errors of the GPU path against the oracle rows `ref`: <Z_i> (max
    abs), weight and feature gradients (max abs over max |ref|), with the
    upstream gradient one on those rows and zero elsewhere."""
    import numpy as np
    import torch
    rows, e_ref, gw_ref, gx_ref, _ = ref
    c = job.circ
    c.forward(job.w, job.x, state=job.state, ws=job.ws)
    e = c.expval_z(job.state, ws=job.ws).cpu().numpy()
    out = {"rows": rows if len(rows) <= 16 else f"all {len(rows)}",
           "expz_max_abs": float(np.max(np.abs(e[rows] - e_ref)))}
    if job.grad:
        g = torch.zeros_like(job.g)
        g[rows] = 1.0
        gw, gx = c.adjoint_grad(job.w, job.x, job.state, g, ws=job.ws)
        gw, gx = gw.cpu().numpy(), gx.cpu().numpy()
        out["grad_weights_max_rel"] = float(np.max(np.abs(gw - gw_ref)) / np.max(np.abs(gw_ref)))
        out["grad_features_max_rel"] = float(np.max(np.abs(gx[rows] - gx_ref)) / np.max(np.abs(gx_ref)))
    return out


def pass_bandwidth(rep):
    """HBM bytes over time of the tile-pass launches (algorithmic bytes: one
    read and one write of each state a pass streams), forward, backward and
    both, against the 8 TB/s peak."""
    out = {}
    for label, pre in (("fwd", "pass_fwd"), ("bwd", "pass_bwd"), ("all", "pass_")):
        ks = [v for k, v in rep.items() if k.startswith(pre)]
        ms = sum(v["ms"] for v in ks)
        by = sum(v["bytes"] for v in ks)
        if ms > 0:
            out[label] = {"GBps": round(by / (ms / 1e3) / 1e9, 1), "frac": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "launches": sum(v["count"] for v in ks), "ms": round(ms, 3)}
    return out


# The paper's own figures (context, not targets: other hardware, its own
# PyTorch implementation in complex128, against PennyLane default.qubit).
PAPER_CONTEXT = [
    {"claim": "forward + backward speedup over PennyLane default.qubit", "value": "about 10x for n <= 10, "
     "about 3x beyond", "hardware": "1 CPU thread and 1 GPU (model not named)", "where": "Sec. 3, Fig. 8"},
    {"claim": "IBM native-gate QDI circuit speedup", "value": "up to about 10x up to about 15 qubits, then "
     "converging", "hardware": "1 CPU thread, 1 GPU", "where": "App. B, Fig. 12"},
    {"claim": "IonQ native-gate QDI circuit speedup", "value": "about 10x; 20 qubits reached vs 17 at batch 1",
     "hardware": "1 CPU thread, 1 GPU", "where": "App. B, Fig. 13"},
    {"claim": "PyTorch steady-state speedup over PennyLane-Torch", "value": "up to 10x", "hardware":
     "48-core CPU node; 1 NVIDIA A100", "where": "Sec. 4"},
]


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    # the CPU baselines run first: the pooled one forks, which must happen
    # before anything initialises the GPU in this process
    sweep = (a.dense_sweep or a.dispatch_sweep or a.vq_qdi_sweep or a.memory_sweep or a.serve_only
             or a.backward_sweep or a.technique_sweep or a.tile_sweep)
    cpu = None if (a.no_cpu_baseline or sweep) else cpu_baseline()
    ref, cpu_pool = ({}, None) if (a.no_cpu_baseline or sweep) else oracle_pool()
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
    if a.backward_sweep:
        backward_sweep()
        return
    if a.technique_sweep:
        technique_sweep()
        return
    if a.tile_sweep:
        tile_sweep()
        return
    if a.serve_only:
        print(json.dumps(serving_bench(a.serve_requests, a.serve_max_qubits,
                                       [float(f) for f in a.serve_qps_fracs.split(",")], warm=a.serve_warmup,
                                       light_during_heavy=light_cap(a.serve_light_during_heavy),
                                       compare_light=a.serve_compare_light_cap)))
        return

    def errs(j):
        return errors_vs_oracle(j, ref[j.name]) if j.name in ref else None

    jobs = [Job(name, a.mode) for name in C4]
    # per-kernel times: an eager run with the library's HIP events
    ms_eager, wall_eager, rep, st_eager = time_jobs(jobs, a.steps, a.warmup)
    if a.no_graph:
        ms, wall_ms, st = ms_eager, wall_eager, st_eager
    else:
        ms, wall_ms, st = time_graph(jobs, a.steps, a.warmup)
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
        "step_stats": st,
        "evals_per_s_at_median": round(evals / (st["median_ms"] / 1e3), 1),
        "wall_ms_per_step": round(wall_ms, 4),
        "execution": ("eager launches" if a.no_graph else
                      "one HIP graph per step (both circuits' forward, <Z_i> and adjoint), replayed; "
                      "replays checked bit for bit against eager steps before and after timing"),
        "eager_ms_per_step": round(ms_eager, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "precision": "complex64 states; FP64 gate matrices and angles; every sum over amplitudes beyond one "
                     "thread's 16 registers (gradient partials, <Z_i>, norms) in FP64",
        "data": "synthetic (seeded weights U(0,2pi), features U(-pi,pi), upstream dL/d<Z>=1)",
        "config": {"workload": "16 qubits, batch 128, complex64: IonQ GPI/GPI2/MS and IBM RZ/SX/ECR "
                               "native-gate circuits, 8 blocks each, forward <Z_i> + adjoint gradients",
                   "n_qubits": 16, "batch": 128, "circuits": [j.name for j in jobs],
                   "mode": a.mode, "passes": {j.name: len(j.circ.plan()["passes"]) for j in jobs}},
        "roofline": roofline(rep, traffic_file),
        "kernels": {k: {"count": v["count"], "ms_per_step": round(v["ms"] / a.steps, 4)} for k, v in rep.items()},
        "errors_vs_oracle": {j.name: errs(j) for j in jobs},
    }
    del jobs
    if a.calibrate_copy_mib > 0:
        src = torch.ones(a.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    short = max(5, a.steps // 2)
    if not a.no_extra:
        # the headline workload in complex128 (the paper's precision, Sec. 2.1)
        j128 = [Job(name, a.mode, dtype="c128") for name in C4]
        ms128, _, st128 = time_graph(j128, short, 2)
        out["q16_c128"] = {"workload": "the headline workload in complex128", "evals_per_s": round(256 / (ms128 / 1e3), 1),
                           "ms_per_step": round(ms128, 4), "step_stats": st128,
                           "errors_vs_oracle": {j.name: errs(j) for j in j128}}
        del j128
        # 4 qubits, batch 16, complex128, plain forward <Z_i>
        j1 = Job("c1_4q_b16", a.mode, grad=False)
        ms1, _, st1 = time_graph([j1], a.steps, a.warmup)
        out["c1_4q_b16"] = {"workload": "4 qubits, batch 16, complex128: RY(x) + 2 x [RX, RZ, CNOT ring], forward <Z_i>",
                            "ms_per_step": round(ms1, 4), "step_stats": st1,
                            "evals_per_s": round(16 / (ms1 / 1e3), 1), "errors_vs_oracle": errs(j1)}
        del j1
        # 12 qubits, batch 256, complex64, forward + adjoint
        j2 = Job("c2_12q_b256", a.mode)
        ms2, _, st2 = time_graph([j2], a.steps, a.warmup)
        out["c2_12q_b256"] = {"workload": "12 qubits, batch 256, complex64: RY(x) + 10 x [RY, RZ, CNOT ring], "
                                          "forward <Z_i> + adjoint gradients",
                              "ms_per_step": round(ms2, 4), "step_stats": st2,
                              "evals_per_s": round(256 / (ms2 / 1e3), 1), "errors_vs_oracle": errs(j2)}
        del j2
    if not a.no_b512:
        jb = [Job(name, a.mode, 512) for name in C4]
        msb, _, repb, stb = time_jobs(jb, max(3, a.steps // 4), 2)
        out["q16_b512"] = {"workload": "the same two 16-qubit circuits at batch 512 (256 MiB per state set, "
                                       "larger than the last-level cache)",
                           "evals_per_s": round(1024 / (msb / 1e3), 1), "ms_per_step": round(msb, 3),
                           "step_stats": stb, "roofline": roofline(repb),
                           "pass_bandwidth": pass_bandwidth(repb)}
        del jb
    if not a.no_20q:
        j20 = Job("c3_20q_b32", a.mode)
        ms20e, _, rep20, st20e = time_jobs([j20], max(5, a.steps // 2), 2)
        ms20, _, st20 = time_graph([j20], max(5, a.steps // 2), 2)
        out["q20"] = {"workload": "20 qubits, batch 32, complex64: RX embedding + 6 x [RX, RY, RZ, ZZ ring, "
                                  "CNOT ring], forward <Z_i> + adjoint gradients",
                      "evals_per_s": round(j20.B / (ms20 / 1e3), 1), "ms_per_step": round(ms20, 3),
                      "step_stats": st20, "eager_ms_per_step": round(ms20e, 3),
                      "hbm": pass_bandwidth(rep20),
                      "roofline": roofline(rep20, lambda k: traffic_file(k, "20q_b32")),
                      "kernels": {k: {"count": v["count"], "ms": round(v["ms"], 3)} for k, v in rep20.items()},
                      "errors_vs_oracle": errs(j20)}
        del j20
    if not a.no_serve:
        out["serving"] = serving_bench(a.serve_requests, a.serve_max_qubits,
                                       [float(f) for f in a.serve_qps_fracs.split(",")],
                                       warm=a.serve_warmup, light_during_heavy=light_cap(a.serve_light_during_heavy))
    out["cpu_baseline"] = cpu
    if cpu_pool is not None:
        out["cpu_baseline_all_cores"] = cpu_pool.pop("all_cores")
        out["cpu_oracle_other"] = cpu_pool
    out["host"] = {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
                   "gpu": torch.cuda.get_device_name(0)}
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out))


if __name__ == "__main__":
    main()
