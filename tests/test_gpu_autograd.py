"""The torch.autograd.Function over the library: <Z_i> forward and adjoint
backward through torch's autograd, against the oracle's gradients, and against
torch's own finite-difference check in complex128."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import sim
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2506_04891_amd import tqsim as T


@pytest.mark.parametrize("dtype,tol,gtol", [("c64", 2e-5, 1e-4), ("c128", 1e-12, 1e-12)])
def test_autograd_matches_oracle(dtype, tol, gtol):
    n, B = 6, 5
    layers = W.circuit_rot_ring(n, 3, "RY", ("RX", "RZ"), zz=True)
    w, x = W.draw_params(n, layers, B, "normal", 4)
    g = W.upstream(B, n, "normal", 4)
    note(f"case autograd {dtype}")
    c = T.Circuit(n, layers, dtype)
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    e = T.expval(c, wt, xt)
    (e * torch.tensor(g, device="cuda")).sum().backward()
    e_ref, gw_ref, gx_ref = sim.grad_adjoint(n, layers, w, x, g)
    assert np.max(np.abs(e.detach().cpu().numpy() - e_ref)) <= tol
    for got, ref in ((wt.grad, gw_ref), (xt.grad, gx_ref)):
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= gtol * np.max(np.abs(ref))


def test_autograd_weights_only_and_second_backward():
    n, B = 5, 3
    layers = W.circuit_rot_ring(n, 2)
    w, x = W.draw_params(n, layers, B, "normal", 5)
    c = T.Circuit(n, layers, "c64")
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    xt = torch.tensor(x, device="cuda")          # features are constants here
    e = T.expval(c, wt, xt)
    loss = e.sum()
    loss.backward(retain_graph=True)
    _, gw_ref, _ = sim.grad_adjoint(n, layers, w, x, np.ones((B, n)))
    assert np.max(np.abs(wt.grad.cpu().numpy() - gw_ref)) <= 1e-4 * np.max(np.abs(gw_ref))
    assert xt.grad is None
    g1 = wt.grad.clone()
    wt.grad = None
    loss.backward()          # the saved state was uncomputed: recomputed first
    torch.testing.assert_close(wt.grad, g1, rtol=0, atol=0)


def test_autograd_gradcheck_c128():
    n, B = 4, 2
    layers = W.circuit_ionq(n, 2)
    w, x = W.draw_params(n, layers, B, "uniform2pi", 6)
    c = T.Circuit(n, layers, "c128")
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: T.QCircuitFn.apply(c, a, b), (wt, xt), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)
