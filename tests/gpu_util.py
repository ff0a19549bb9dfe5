"""Shared helpers of the GPU parity tests: run the HIP path, run the oracle,
compare with the stated tolerances."""
import sys

import numpy as np
import torch

from oracle import sim

# tolerances (per output tensor): complex128 1e-12 relative; complex64 2e-5
# absolute on <Z_i>, 1e-4 relative on gradients; states: 1e-12 (c128) and
# 2e-5 (c64) absolute per amplitude after normalisation.
TOL = {
    "c128": dict(state=1e-12, expz=1e-12, grad=1e-12),
    "c64": dict(state=2e-5, expz=2e-5, grad=1e-4),
}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def gpu_run(circ, w, x, g=None, batch=None):
    dev = torch.device("cuda")
    wt = torch.tensor(np.asarray(w, dtype=np.float64).reshape(-1), device=dev)
    xt = torch.tensor(np.asarray(x, dtype=np.float64), device=dev)
    state = circ.forward(wt, xt, batch=batch)
    psi = state.cpu().numpy().copy()
    e, norm = circ.expval_z(state, with_norm=True)
    out = dict(psi=psi, e=e.cpu().numpy(), norm=norm.cpu().numpy())
    if g is not None:
        gt = torch.tensor(np.asarray(g, dtype=np.float64), device=dev)
        gw, gx = circ.adjoint_grad(wt, xt, state, gt)
        torch.cuda.synchronize()
        out["gw"] = gw.cpu().numpy()
        out["gx"] = gx.cpu().numpy()
    return out


def oracle_run(n, layers, w, x, g=None):
    psi = sim.run_o2(n, layers, w, x)
    out = dict(psi=psi, e=sim.expval_z(psi, n))
    if g is not None:
        _, gw, gx = sim.grad_adjoint(n, layers, w, x, g)
        out["gw"], out["gx"] = gw[: len(w)], gx[:, : x.shape[1]]
    return out


def compare(got, ref, dtype, what=("psi", "e", "gw", "gx"), label=""):
    tol = TOL[dtype]
    errs = {}
    if "psi" in what:
        errs["psi"] = float(np.max(np.abs(got["psi"] - ref["psi"])))
        assert errs["psi"] <= tol["state"], (label, errs)
    if "e" in what:
        errs["e"] = float(np.max(np.abs(got["e"] - ref["e"])))
        assert errs["e"] <= tol["expz"], (label, errs)
    for k in ("gw", "gx"):
        if k in what and k in ref and ref[k].size:
            errs[k] = rel_err(got[k], ref[k])
            assert errs[k] <= tol["grad"], (label, k, errs)
    return errs
