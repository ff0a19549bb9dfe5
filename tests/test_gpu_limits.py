"""Large states on the GPU, up to 2^30 amplitudes per sample (the largest
circuit the library accepts): 64-bit global indexing, many workgroups per
sample.  Checked against closed forms that hold at any size: after an RY(x)
embedding and a CNOT ring,
<Z_k> = prod_{i<=k} cos x_i (k >= 1) and <Z_0> = prod_{i>=1} cos x_i; diagonal
layers after the ring change no <Z_k>, so their weight gradients are zero."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2506_04891_amd import tqsim as T


def _closed_form(x):
    c, s = np.cos(x), np.sin(x)
    B, n = x.shape
    e = np.cumprod(c, axis=1)
    e[:, 0] = np.prod(c[:, 1:], axis=1)
    # d<Z_k>/dx_j = -sin x_j prod_{i in S_k, i != j} cos x_i over the wires S_k of <Z_k>
    gx = np.zeros((B, n))
    for k in range(n):
        S = range(1, n) if k == 0 else range(0, k + 1)
        for j in S:
            others = [i for i in S if i != j]
            gx[:, j] += -s[:, j] * np.prod(c[:, others], axis=1)
    return e, gx


@pytest.mark.parametrize("n,B", [(30, 1), (28, 2), (26, 2), (24, 5), (21, 3)])
def test_large_state_closed_form(n, B):
    b = W._Builder(n)
    b.add("RY", "ALL", "INPUT").add("CNOT", "RING").add("RZ", "ALL", "WEIGHT").add("ZZ", "RING", "WEIGHT")
    layers = b.layers
    nw, nf = W.circuit_counts(n, layers)
    rng = np.random.default_rng(100 + n)
    # angles near 0 keep the cosine products away from zero
    x = rng.uniform(-0.35, 0.35, (B, nf))
    w = rng.standard_normal(nw)
    note(f"case large n={n} B={B}")
    c = T.Circuit(n, layers, "c64")
    dev = torch.device("cuda")
    wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
    st = c.forward(wt, xt)
    e, norm = c.expval_z(st, with_norm=True)
    gw, gx = c.adjoint_grad(wt, xt, st, torch.ones((B, n), dtype=torch.float64, device=dev))
    e_ref, gx_ref = _closed_form(x)
    np.testing.assert_allclose(norm.cpu().numpy(), 1.0, atol=1e-5)
    assert np.max(np.abs(e.cpu().numpy() - e_ref)) <= 2e-5
    assert np.max(np.abs(gx.cpu().numpy() - gx_ref)) <= 1e-4 * np.max(np.abs(gx_ref))
    assert np.max(np.abs(gw.cpu().numpy())) <= 1e-4
