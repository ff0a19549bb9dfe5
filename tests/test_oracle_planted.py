"""Planted mistakes: each plausible slip in the oracle must make a pin fail.

Every case patches the oracle (on the CPU only), runs one of the pins of
test_oracle_pins.py and expects it to fail; the patch is undone afterwards.
"""
import numpy as np
import pytest

import tests.test_oracle_pins as P
from oracle import gates as G
from oracle import sim


def _expect_failure(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_transposed_ry_is_caught(monkeypatch):
    monkeypatch.setattr(G, "RY", lambda t: G.RY.__wrapped__(t).T if hasattr(G.RY, "__wrapped__")
                        else np.array([[np.cos(t / 2), np.sin(t / 2)], [-np.sin(t / 2), np.cos(t / 2)]],
                                      dtype=complex))
    _expect_failure(P.test_rotations_are_exponentials, 0.7)


def test_missing_half_angle_in_rz_is_caught(monkeypatch):
    monkeypatch.setattr(G, "RZ", lambda t: np.diag([np.exp(-1j * t), np.exp(1j * t)]))
    monkeypatch.setitem(G.PARAM, "RZ", (G.RZ, G.dRZ))
    _expect_failure(P.test_rz_layer_eigenphase, 3)


def test_flipped_wire_order_is_caught(monkeypatch):
    def counting_lsb_first(n):
        j = np.arange(2 ** n)
        return ((j[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    monkeypatch.setattr(sim, "counting_matrix", counting_lsb_first)
    _expect_failure(P.test_k_rz_worked_example_sec241)
    _expect_failure(P.test_expval_wire_order)


def test_reversed_ring_order_is_caught(monkeypatch):
    orig = sim.pattern_wires

    def reversed_ring(n, ly):
        w = orig(n, ly)
        return w[::-1] if ly.pattern == "RING" else w
    monkeypatch.setattr(sim, "pattern_wires", reversed_ring)
    _expect_failure(P.test_ry_then_cnot_ring_closed_form, 4)


def test_ring_without_wrap_pair_is_caught(monkeypatch):
    orig = sim.pattern_wires

    def open_ring(n, ly):
        w = orig(n, ly)
        return w[:-1] if ly.pattern == "RING" and n > 2 else w
    monkeypatch.setattr(sim, "pattern_wires", open_ring)
    _expect_failure(P.test_zz_ring_uses_k_rzz, 4)


def test_adjoint_missing_factor_two_is_caught(monkeypatch):
    orig = G.generators
    monkeypatch.setattr(G, "generators", lambda gate, t, ph=(0.0, 0.0): [0.5 * x for x in orig(gate, t, ph)])
    _expect_failure(P.test_gradient_routes_agree, P.GRAD_CASES[0])


def test_transposed_cnot_control_is_caught(monkeypatch):
    swapped = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=complex)
    monkeypatch.setitem(G.FIXED, "CNOT", lambda: swapped)
    _expect_failure(P.test_sigma_cnot_sec23)


def test_wrong_ecr_row_is_caught(monkeypatch):
    bad = G.ECR().copy()
    bad[2, 1] = -bad[2, 1]
    monkeypatch.setitem(G.FIXED, "ECR", lambda: bad)
    _expect_failure(P.test_all_gates_unitary)


def test_reversed_layer_order_in_o1_is_caught(monkeypatch):
    def run_o1_reversed(n, layers, weights, features):
        B = features.shape[0]
        out = np.zeros((B, 2 ** n), dtype=np.complex128)
        for b in range(B):
            psi = np.zeros(2 ** n, dtype=np.complex128)
            psi[0] = 1.0
            for li in reversed(range(len(layers))):
                psi = sim.layer_unitary(n, layers, li, weights, features[b]) @ psi
            out[b] = psi
        return out
    monkeypatch.setattr(sim, "run_o1", run_o1_reversed)
    _expect_failure(P.test_o1_equals_o2_whole_circuit, P.WHOLE_CIRCUITS[0], 4)


def test_o1_without_per_sample_features_is_caught(monkeypatch):
    def run_o1_first_row(n, layers, weights, features):
        B = features.shape[0]
        out = np.zeros((B, 2 ** n), dtype=np.complex128)
        for b in range(B):
            psi = np.zeros(2 ** n, dtype=np.complex128)
            psi[0] = 1.0
            for li in range(len(layers)):
                psi = sim.layer_unitary(n, layers, li, weights, features[0]) @ psi
            out[b] = psi
        return out
    monkeypatch.setattr(sim, "run_o1", run_o1_first_row)
    _expect_failure(P.test_o1_equals_o2_whole_circuit, P.WHOLE_CIRCUITS[2], 4)


def test_k_rzz_pairing_wrong_neighbour_is_caught(monkeypatch):
    def k_rzz_left(n):
        K = sim.k_rz(n)
        return K * K[:, (np.arange(n) - 1) % n]
    monkeypatch.setattr(sim, "k_rzz_ring", k_rzz_left)
    _expect_failure(P.test_zz_ring_uses_k_rzz, 4)
    _expect_failure(P.test_k_rzz_columns_are_neighbour_parities)


def test_shared_parameter_shift_is_not_reported():
    """A feature read by several layers has no two-term shift rule; the oracle
    must leave it as NaN rather than return a one-gate value."""
    import workloads as W
    n = 3
    layers = W.circuit_rz_ry_cnot(n, 2, "qdi")
    w, x = W.draw_params(n, layers, 2, "normal", 3)
    sw, sx = sim.grad_param_shift(n, layers, w, x, W.upstream(2, n, "normal", 1))
    assert np.all(np.isnan(sx))
    assert not np.any(np.isnan(sw))


def test_ms_entry_as_printed_is_caught(monkeypatch):
    """MS(phi0, phi1, theta) with entry (3, 0) exactly as printed (App. A)."""
    orig = G.MSP

    def printed(phi0, phi1, t):
        U = orig(phi0, phi1, t).copy()
        U[3, 0] = -1j * np.exp(-2j * np.pi * (phi0 + phi1)) * np.sin(np.pi * t)
        return U
    monkeypatch.setattr(G, "MSP", printed)
    _expect_failure(P.test_ms_with_phases, 0.13, -0.41, 0.37)


def test_rot_with_swapped_phases_is_caught(monkeypatch):
    orig = G.ROT
    monkeypatch.setattr(G, "ROT", lambda t, phi, lam: orig(t, lam, phi))
    _expect_failure(P.test_rot_appendix_a, 0.7, -1.3, 2.1)
