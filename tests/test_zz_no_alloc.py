"""The allocation-free readout entry point, tqs_expval_z_noalloc, through the C
ABI: it must give exactly what tqs_expval_z gives with a caller workspace (the
same kernels run on the same state), and match the oracle at the stated
tolerances, on two calls in a row, the second with a smaller input (the static
scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import TOL, note, oracle_run

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2506_04891_amd import tqsim as T


def _call_noalloc(circ, state, with_norm):
    """tqs_expval_z_noalloc called directly through ctypes."""
    B = state.shape[0]
    expz = torch.full((B, circ.n), float("nan"), dtype=torch.float64, device=state.device)
    norm = torch.full((B,), float("nan"), dtype=torch.float64, device=state.device) if with_norm else None
    st = T.lib().tqs_expval_z_noalloc(circ.handle, B, ctypes.c_void_p(state.data_ptr()),
                                      ctypes.c_void_p(expz.data_ptr()),
                                      None if norm is None else ctypes.c_void_p(norm.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, T.lib().tqs_last_error().decode()
    return expz, norm


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_readout_equals_workspace_readout(dtype):
    # first call: 16 qubits, 48 samples (16 units of partials per sample);
    # second: 13 qubits, 5 samples -- smaller, over the stale first contents
    cases = [(16, 48, W.circuit_ionq(16, 2), "uniform2pi"),
             (13, 5, W.circuit_rot_ring(13, 2, "RX", ("RX", "RY", "RZ"), zz=True), "normal")]
    dev = torch.device("cuda")
    for n, B, layers, dist in cases:
        note(f"case noalloc {dtype} n={n} B={B}")
        w, x = W.draw_params(n, layers, B, dist, 17 + n)
        c = T.Circuit(n, layers, dtype)
        wt, xt = torch.tensor(w, device=dev), torch.tensor(x, device=dev)
        state = c.forward(wt, xt)
        e_ws, n_ws = c.expval_z(state, with_norm=True)
        e_na, n_na = _call_noalloc(c, state, with_norm=True)
        torch.cuda.synchronize()
        assert torch.equal(e_na, e_ws), (n, B)
        assert torch.equal(n_na, n_ws), (n, B)
        ref = oracle_run(n, layers, w, x)
        err = float(np.max(np.abs(e_na.cpu().numpy() - ref["e"])))
        assert err <= TOL[dtype]["expz"], (n, B, err)
        np.testing.assert_allclose(n_na.cpu().numpy(), 1.0, atol=1e-5 if dtype == "c64" else 1e-13)
        # without the norm output
        e2, _ = _call_noalloc(c, state, with_norm=False)
        torch.cuda.synchronize()
        assert torch.equal(e2, e_ws)


def test_noalloc_rejects_oversized_batch():
    # 20 qubits: 256 units of 13 doubles per sample, 26624 bytes; 316 samples
    # need 8.4 MB > 8 MiB.  Rejected on the host before anything is launched.
    n = 20
    c = T.Circuit(n, W.circuit_rot_ring(n, 1, "RX", ("RX",)), "c64")
    B = 316
    state = torch.zeros((1, 1), dtype=torch.complex64, device="cuda")
    expz = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    st = T.lib().tqs_expval_z_noalloc(c.handle, B, ctypes.c_void_p(state.data_ptr()),
                                      ctypes.c_void_p(expz.data_ptr()), None, None)
    assert st == 1
    assert "static scratch" in T.lib().tqs_last_error().decode()
