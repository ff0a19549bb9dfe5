"""A short, fixed run of one benchmark workload, for profilers.

    python -m paper_2506_04891_amd.profile_run --workload c4 --steps 3 [--calibrate-copy-mib 1024]

Workloads: c4 (the 16-qubit IonQ and IBM circuits at batch 128), c3 (20 qubits,
batch 32), c2 (12 qubits, batch 256), dense6 (RY(x) + 10 x [RY, RZ, CNOT ring]
on 6 qubits at batch 4096, complex64, every layer as a full 64 x 64 matrix on
the matrix cores).  One untimed warm-up step, then `steps`
steps of forward + <Z_i> + adjoint gradient.  With --calibrate-copy-mib, a
float32 negation over that many MiB runs three times afterwards: a streaming
kernel of known size against which rocprofv3's byte counters are scaled.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {"c4": ["c4a_16q_b128_ionq", "c4b_16q_b128_ibm"], "c3": ["c3_20q_b32"], "c2": ["c2_12q_b256"],
             "dense6": []}


class DenseJob:
    """The dense-mode workload: forward + <Z_i> + adjoint on full-layer matrices."""

    def __init__(self, n=6, batch=4096):
        import torch
        import workloads as W
        from paper_2506_04891_amd import tqsim as T
        layers = W.circuit_rot_ring(n, 10, "RY", ("RY", "RZ"))
        self.circ = T.Circuit(n, layers, "c64", mode="dense")
        assert self.circ.plan()["mode"] == "dense"
        dev = torch.device("cuda")
        w, x = W.draw_params(n, layers, batch, "normal", 0)
        self.w, self.x = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
        self.g = torch.ones((batch, n), dtype=torch.float64, device=dev)
        self.state = torch.empty((batch, 2 ** n), dtype=self.circ.complex_dtype, device=dev)
        self.ws = self.circ.workspace(batch, True, dev)

    def step(self):
        c = self.circ
        c.forward(self.w, self.x, state=self.state, ws=self.ws)
        c.expval_z(self.state, ws=self.ws)
        c.adjoint_grad(self.w, self.x, self.state, self.g, ws=self.ws)


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="c4")
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--calibrate-copy-mib", type=int, default=0)
    a = p.parse_args(argv)
    import torch
    from bench import Job
    jobs = [DenseJob()] if a.workload == "dense6" else [Job(name, "auto") for name in WORKLOADS[a.workload]]
    for j in jobs:
        j.step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(a.steps):
        for j in jobs:
            j.step()
    torch.cuda.synchronize()
    print(f"{a.workload}: {(time.perf_counter() - t) / a.steps * 1e3:.3f} ms/step", flush=True)
    if a.calibrate_copy_mib > 0:
        src = torch.ones(a.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 x {a.calibrate_copy_mib} MiB read + written", flush=True)


if __name__ == "__main__":
    main()
