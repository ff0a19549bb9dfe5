"""A short, fixed run of one benchmark workload, for profilers.

    python -m paper_2506_04891_amd.profile_run --workload c4 --steps 3 [--calibrate-copy-mib 1024]

Workloads: c4 (the 16-qubit IonQ and IBM circuits at batch 128), c3 (20 qubits,
batch 32), c2 (12 qubits, batch 256).  One untimed warm-up step, then `steps`
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

WORKLOADS = {"c4": ["c4a_16q_b128_ionq", "c4b_16q_b128_ibm"], "c3": ["c3_20q_b32"], "c2": ["c2_12q_b256"]}


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="c4")
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--calibrate-copy-mib", type=int, default=0)
    a = p.parse_args(argv)
    import torch
    from bench import Job
    jobs = [Job(name, "auto") for name in WORKLOADS[a.workload]]
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
