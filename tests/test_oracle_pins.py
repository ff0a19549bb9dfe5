"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (fixtures under tests/golden/), library special cases (scipy's
expm), closed forms, invariants, and brute force on tiny inputs.
"""
import os

import numpy as np
import pytest
from scipy.linalg import expm

import workloads as W
from oracle import gates as G
from oracle import sim

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def _rand_state(B, n, seed=0):
    return W.random_states(B, n, seed)


def _layers(*specs):
    return [W.L(*s) if isinstance(s, tuple) else s for s in specs]


# ---------------------------------------------------------------- fixtures --

def _read_rows(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line)
    return rows


def test_sigma_cnot_sec23():
    """CNOT acts as the gather phi' = phi[sigma] with sigma = (1 2 4 3) (Sec. 2.3)."""
    sigma = np.array([int(v) for v in _read_rows("sigma_cnot.txt")[0].split()]) - 1
    psi = _rand_state(3, 2)
    out = sim.run_o2(2, [W.L("CNOT", "WIRE", wire=0, wire2=1)], np.zeros(0),
                     np.zeros((3, 0)), psi0=psi)
    np.testing.assert_allclose(out, psi[:, sigma], atol=0)


def test_k_rz_worked_example_sec241():
    rows = np.array([[int(v) for v in r.split()] for r in _read_rows("k_rz_n3.txt")])
    np.testing.assert_array_equal(sim.counting_matrix(3), rows[:, :3])
    np.testing.assert_array_equal(sim.k_rz(3), rows[:, 3:])


def test_appendix_a_fixed_gates_as_printed():
    for r in _read_rows("appendix_a_fixed.txt"):
        head, body = r.split(":")
        name, pref = head.split()
        M = np.array([[complex(*map(float, e.split(","))) for e in row.split()]
                      for row in body.split(";")]) * float(pref)
        U = G.matrix(name)
        np.testing.assert_allclose(U[: M.shape[0]], M, atol=1e-15, err_msg=name)


# ------------------------------------------------ library special cases --

@pytest.mark.parametrize("t", [-2.3, -0.4, 0.0, 0.7, 3.1, 5.9])
def test_rotations_are_exponentials(t):
    np.testing.assert_allclose(G.RX(t), expm(-0.5j * t * G.X), atol=1e-14)
    np.testing.assert_allclose(G.RY(t), expm(-0.5j * t * G.Y), atol=1e-14)
    np.testing.assert_allclose(G.RZ(t), expm(-0.5j * t * G.Z), atol=1e-14)
    np.testing.assert_allclose(G.ZZ(t), expm(-0.5j * t * np.kron(G.Z, G.Z)), atol=1e-14)
    np.testing.assert_allclose(G.MS(t), expm(-1j * np.pi * t * np.kron(G.X, G.X)), atol=1e-13)


def test_fixed_gate_identities():
    I2, I4 = np.eye(2), np.eye(4)
    np.testing.assert_allclose(G.SX() @ G.SX(), G.X, atol=1e-15)
    np.testing.assert_allclose(G.H() @ G.H(), I2, atol=1e-15)
    np.testing.assert_allclose(G.ECR() @ G.ECR(), I4, atol=1e-15)
    np.testing.assert_allclose(G.ECR(), (np.kron(I2, G.X) - np.kron(G.X, G.Y)) / np.sqrt(2), atol=1e-15)
    np.testing.assert_allclose(G.S() @ G.S(), G.Z, atol=1e-15)
    # SX equals RX(pi/2) only up to the global phase e^{i pi/4}
    np.testing.assert_allclose(G.SX(), np.exp(0.25j * np.pi) * G.RX(np.pi / 2), atol=1e-15)


def test_all_gates_unitary():
    for name in G.FIXED:
        U = G.matrix(name)
        np.testing.assert_allclose(U.conj().T @ U, np.eye(len(U)), atol=1e-14, err_msg=name)
    for name in G.PARAM:
        for t in (-1.3, 0.2, 2.9):
            U = G.matrix(name, t)
            np.testing.assert_allclose(U.conj().T @ U, np.eye(len(U)), atol=1e-14, err_msg=name)


@pytest.mark.parametrize("name", sorted(G.PARAM))
def test_derivatives_match_finite_differences(name):
    for t in (-1.1, 0.3, 2.2):
        h = 1e-6
        fd = (G.matrix(name, t + h) - G.matrix(name, t - h)) / (2 * h)
        np.testing.assert_allclose(G.dmatrix(name, t), fd, atol=1e-8)
        Gm = G.generator(name, t)
        np.testing.assert_allclose(Gm, Gm.conj().T, atol=1e-13)


def test_generators_of_paper_gates():
    """Output-side generators: rotations P/2; ZZ Z(x)Z/2; MS pi X(x)X; GPI 2 pi Z."""
    for t in (0.4, -2.0):
        np.testing.assert_allclose(G.generator("RX", t), G.X / 2, atol=1e-14)
        np.testing.assert_allclose(G.generator("RY", t), G.Y / 2, atol=1e-14)
        np.testing.assert_allclose(G.generator("RZ", t), G.Z / 2, atol=1e-14)
        np.testing.assert_allclose(G.generator("ZZ", t), np.kron(G.Z, G.Z) / 2, atol=1e-14)
        np.testing.assert_allclose(G.generator("MS", t), np.pi * np.kron(G.X, G.X), atol=1e-13)
        np.testing.assert_allclose(G.generator("GPI", t), 2 * np.pi * G.Z, atol=1e-13)


# ------------------------------------------- techniques of the paper ----

@pytest.mark.parametrize("n", [1, 3, 5])
def test_rz_layer_eigenphase(n):
    """RZ layer = psi o exp(-(i/2) K_Rz theta): the eigenphase computation of
    Sec. 2.4.1 with the sign and scale of Appendix A's Rz."""
    th = RNG.standard_normal(n)
    psi = _rand_state(2, n, 1)
    out = sim.run_o2(n, [W.L("RZ", "ALL", "WEIGHT")], th, np.zeros((2, 0)), psi0=psi)
    np.testing.assert_allclose(out, psi * np.exp(-0.5j * (sim.k_rz(n) @ th))[None], atol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 6])
def test_zz_ring_uses_k_rzz(n):
    """Rzz ring (with the (n-1, 0) pair) = psi o exp(-(i/2) K_Rzz theta)
    (Sec. 2.4.1, with Appendix A's sign): the oracle's K_Rzz builder against
    the ring applied gate by gate (O2) and as its Kronecker-built layer
    matrix (O1), both of which use only Appendix A's Rzz matrix."""
    th = RNG.standard_normal(n)
    Kzz = sim.k_rzz_ring(n)
    assert Kzz.shape == (2 ** n, n) and set(np.unique(Kzz)) <= {-1, 1}
    psi = _rand_state(2, n, 2)
    ref = psi * np.exp(-0.5j * (Kzz @ th))[None]
    layers = [W.L("ZZ", "RING", "WEIGHT")]
    out = sim.run_o2(n, layers, th, np.zeros((2, 0)), psi0=psi)
    np.testing.assert_allclose(out, ref, atol=1e-14)
    U = sim.layer_unitary(n, layers, 0, th, None)
    np.testing.assert_allclose(U, np.diag(np.exp(-0.5j * (Kzz @ th))), atol=1e-14)


def test_k_rzz_columns_are_neighbour_parities():
    """Column j of K_Rzz is +1 exactly where wires j and j+1 (mod n) hold the
    same bit: checked on basis states written out bit by bit."""
    n = 4
    Kzz = sim.k_rzz_ring(n)
    for idx in range(2 ** n):
        bits = [(idx >> (n - 1 - w)) & 1 for w in range(n)]   # wire 0 = MSB
        for j in range(n):
            same = bits[j] == bits[(j + 1) % n]
            assert Kzz[idx, j] == (1 if same else -1), (idx, j)


@pytest.mark.parametrize("n", [1, 3, 5])
def test_gpi_layer_reversal(n):
    """GPI layer: psi'[2^n-1-i] = (psi o exp(i K theta))[i] with theta_q = 2 pi phi_q."""
    phi = RNG.uniform(0, 1, n)
    psi = _rand_state(2, n, 3)
    out = sim.run_o2(n, [W.L("GPI", "ALL", "WEIGHT")], phi, np.zeros((2, 0)), psi0=psi)
    ref = (psi * np.exp(1j * (sim.k_rz(n) @ (2 * np.pi * phi)))[None])[:, ::-1]
    np.testing.assert_allclose(out, ref, atol=1e-14)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_diagonal_tensor_product(n):
    """diag(U) = (x)_i diag(U^(i)) (Sec. 2.4.2); the sequential Kronecker
    product of n length-2 diagonals takes 2^{n+1} - 4 multiplications."""
    th = RNG.standard_normal(n)
    d = np.ones(1, dtype=complex)
    mults = 0
    for q in range(n):
        d = np.kron(d, np.diag(G.RZ(th[q])))
        mults += d.size if q else 0
    assert mults == 2 ** (n + 1) - 4
    U = sim.layer_unitary(n, [W.L("RZ", "ALL", "WEIGHT")], 0, th, None)
    np.testing.assert_allclose(np.diag(U), d, atol=1e-14)
    np.testing.assert_allclose(U, np.diag(d), atol=1e-14)


def test_cnot_ring_is_one_permutation():
    """A ring of CNOTs composes into a single permutation (Sec. 2.3): the layer
    matrix is 0/1 with one 1 per row and column."""
    for n in (2, 3, 5):
        U = sim.layer_unitary(n, [W.L("CNOT", "RING")], 0, np.zeros(0), None)
        assert set(np.unique(U.real)) <= {0.0, 1.0} and np.all(U.imag == 0)
        np.testing.assert_array_equal(U.sum(0), 1)
        np.testing.assert_array_equal(U.sum(1), 1)


def test_h_rz_expansion_rx_and_readings():
    """Sec. 2.5: Rx = H Rz H holds; the printed Ry identity does not (it gives
    Rx(-t) conjugated), Ry = S H Rz H S^dag does; GPI2 matches
    Rz(-t) Rx(pi/2) Rz(t) with t = -2 pi phi."""
    H, S = G.H(), G.S()
    for t in (0.3, -1.7, 2.5):
        np.testing.assert_allclose(H @ G.RZ(t) @ H, G.RX(t), atol=1e-14)
        assert np.abs(G.Z @ H @ G.RZ(t) @ H @ G.Z - G.RY(t)).max() > 1e-3
        np.testing.assert_allclose(S @ H @ G.RZ(t) @ H @ S.conj().T, G.RY(t), atol=1e-14)
    for phi in (0.1, 0.37, -0.2):
        t = -2 * np.pi * phi
        np.testing.assert_allclose(G.RZ(-t) @ G.RX(np.pi / 2) @ G.RZ(t), G.GPI2(phi), atol=1e-14)


def _phase(a):
    """diag(1, e^{ia}) from the library exponential."""
    return expm(0.5j * a * (np.eye(2) - G.Z))


@pytest.mark.parametrize("t,phi,lam", [(0.7, -1.3, 2.1), (-2.2, 0.4, -0.9), (0.0, 1.1, 0.3)])
def test_rot_appendix_a(t, phi, lam):
    """App. A Rot(theta, phi, lambda) is the phase-Ry-phase product built from
    library exponentials, reduces to RY for phi = lambda = 0 and to a phase for
    theta = 0, and is unitary."""
    U = G.ROT(t, phi, lam)
    np.testing.assert_allclose(U, _phase(phi) @ expm(-0.5j * t * G.Y) @ _phase(lam), atol=1e-14)
    np.testing.assert_allclose(G.ROT(t, 0.0, 0.0), G.RY(t), atol=1e-15)
    np.testing.assert_allclose(G.ROT(0.0, phi, lam), np.diag([1, np.exp(1j * (phi + lam))]), atol=1e-15)
    np.testing.assert_allclose(U.conj().T @ U, np.eye(2), atol=1e-14)
    h = 1e-6
    for k, d in enumerate(G.dROT(t, phi, lam)):
        a, b = [t, phi, lam], [t, phi, lam]
        a[k] += h
        b[k] -= h
        np.testing.assert_allclose(d, (G.ROT(*a) - G.ROT(*b)) / (2 * h), atol=1e-8)


@pytest.mark.parametrize("phi0,phi1,t", [(0.13, -0.41, 0.37), (0.5, 0.25, -0.8), (0.0, 0.0, 0.21)])
def test_ms_with_phases(phi0, phi1, t):
    """App. A MS(phi0, phi1, theta) as read: exp(-i pi theta P(phi1) (x) P(phi0))
    with P the GPI matrix (library exponential), unitary, MS(theta) at zero
    phases.  The printed entry (3, 0) would make the matrix non-unitary for
    phi0 + phi1 not a multiple of 1/2."""
    U = G.MSP(phi0, phi1, t)
    np.testing.assert_allclose(U, expm(-1j * np.pi * t * np.kron(G.GPI(phi1), G.GPI(phi0))), atol=1e-14)
    np.testing.assert_allclose(U.conj().T @ U, np.eye(4), atol=1e-14)
    np.testing.assert_allclose(G.MSP(0.0, 0.0, t), G.MS(t), atol=1e-15)
    printed = U.copy()
    printed[3, 0] = -1j * np.exp(-2j * np.pi * (phi0 + phi1)) * np.sin(np.pi * t)
    if abs(np.sin(2 * np.pi * (phi0 + phi1))) > 1e-3 and abs(np.sin(np.pi * t)) > 1e-3:
        assert np.abs(printed.conj().T @ printed - np.eye(4)).max() > 1e-3
    h = 1e-6
    np.testing.assert_allclose(G.dMSP(phi0, phi1, t),
                               (G.MSP(phi0, phi1, t + h) - G.MSP(phi0, phi1, t - h)) / (2 * h), atol=1e-8)


# ------------------------------------------------------------ invariants ----

ALL_LAYERS = [
    ("RX", "ALL", "WEIGHT"), ("RY", "ALL", "WEIGHT"), ("RZ", "ALL", "WEIGHT"),
    ("H", "ALL"), ("X", "ALL"), ("Z", "ALL"), ("S", "ALL"), ("SX", "ALL"),
    ("GPI", "ALL", "WEIGHT"), ("GPI2", "ALL", "WEIGHT"),
    ("CNOT", "RING"), ("CNOT", "CHAIN"), ("CZ", "RING"), ("SWAP", "CHAIN"),
    ("ZZ", "RING", "WEIGHT"), ("ZZ", "CHAIN", "WEIGHT"),
    ("MS", "PAIRS_EVEN", "WEIGHT"), ("MS", "PAIRS_ODD", "WEIGHT"),
    ("ECR", "PAIRS_EVEN"), ("ECR", "PAIRS_ODD"), ("CNOT", "PAIRS_ODD"),
    ("RY", "ALL", "INPUT"), ("RZ", "ALL", "INPUT"),
    ("ROT", "ALL", "WEIGHT"), ("ROT", "ALL", "INPUT"),
]


def _one_layer(spec, n):
    ly = W.L(*spec)
    nw, nf = sim.param_counts(n, [ly])
    w = RNG.standard_normal(max(nw, 1))
    x = RNG.uniform(-np.pi, np.pi, (3, max(nf, 1)))
    return [ly], w, x


@pytest.mark.parametrize("spec", ALL_LAYERS)
@pytest.mark.parametrize("n", [2, 4, 5])
def test_o1_equals_o2_every_layer(spec, n):
    if "PAIRS" in spec[1] and n % 2:
        pytest.skip("brick pairs need even n")
    layers, w, x = _one_layer(spec, n)
    psi = _rand_state(3, n, 5)
    o2 = sim.run_o2(n, layers, w, x, psi0=psi)
    o1 = np.stack([sim.layer_unitary(n, layers, 0, w, x[b]) @ psi[b] for b in range(3)])
    np.testing.assert_allclose(o1, o2, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(o2, axis=1), 1.0, atol=1e-13)
    U = sim.layer_unitary(n, layers, 0, w, x[0])
    np.testing.assert_allclose(U.conj().T @ U, np.eye(2 ** n), atol=1e-13)


WHOLE_CIRCUITS = [
    ("rot_ring_zz", lambda n: W.circuit_rot_ring(n, 2, "RX", ("RX", "RY", "RZ"), zz=True), "normal"),
    ("rot_ring", lambda n: W.circuit_rot_ring(n, 2, "RY", ("RY", "RZ")), "normal"),
    ("ionq", lambda n: W.circuit_ionq(n, 2), "uniform2pi"),
    ("ibm", lambda n: W.circuit_ibm(n, 2), "uniform2pi"),
    ("ionq_qdi", lambda n: W.circuit_ionq(n, 2, "qdi"), "uniform2pi"),
    ("ibm_qdi", lambda n: W.circuit_ibm(n, 2, "qdi"), "uniform2pi"),
    ("rz_ry_cnot_qdi", lambda n: W.circuit_rz_ry_cnot(n, 2, "qdi"), "normal"),
]


@pytest.mark.parametrize("case", WHOLE_CIRCUITS, ids=[c[0] for c in WHOLE_CIRCUITS])
@pytest.mark.parametrize("n", [2, 4, 6])
def test_o1_equals_o2_whole_circuit(case, n):
    """The O1 driver (per-sample products of full layer unitaries, Sec. 2.2.1)
    against O2 (gate-by-gate contraction, Sec. 2.2.2) on whole circuits with
    per-sample inputs, and the O1 readout path of forward_expval."""
    _, build, dist = case
    layers = build(n)
    w, x = W.draw_params(n, layers, 3, dist, 31)
    o1 = sim.run_o1(n, layers, w, x)
    o2 = sim.run_o2(n, layers, w, x)
    np.testing.assert_allclose(o1, o2, atol=1e-13)
    np.testing.assert_allclose(sim.forward_expval(n, layers, w, x, tier="o1"),
                               sim.forward_expval(n, layers, w, x, tier="o2"), atol=1e-13)


def test_o1_layer_order_matters():
    """Two non-commuting layers in either order give different O1 states, so
    the O1 driver's layer order is observable (a reversed product would fail
    the whole-circuit comparison above)."""
    n = 2
    a = [W.L("RY", "ALL", "INPUT"), W.L("CNOT", "RING"), W.L("RX", "ALL", "WEIGHT", offset=0)]
    b = [a[0], a[2], a[1]]
    w = np.array([0.4, -1.1])
    x = np.array([[0.3, 1.2]])
    assert np.abs(sim.run_o1(n, a, w, x) - sim.run_o1(n, b, w, x)).max() > 1e-2


def test_embed_matrix_general_path_matches_kron():
    M = G.ECR() @ np.kron(G.RX(0.3), G.RY(-1.2))
    for n in (3, 5):
        for w0 in range(n - 1):
            kron = sim.embed_matrix(n, M, (w0, w0 + 1))
            # non-ascending placement via the entry-by-entry definition
            Msw = G.SWAP() @ M @ G.SWAP()
            gen = sim.embed_matrix(n, Msw, (w0 + 1, w0))
            np.testing.assert_allclose(gen, kron, atol=1e-15)


def test_forward_then_inverse_returns_state():
    n = 4
    layers = W.circuit_ibm(n, 2) + W.circuit_ionq(n, 2)
    w, x = W.draw_params(n, layers, 3, "uniform2pi", 7)
    psi = _rand_state(3, n, 9)
    out = sim.run_o2(n, layers, w, x, psi0=psi)
    for inst in reversed(sim.expand(n, layers)):
        out = sim.apply_instance(out, n, inst, sim.instance_param(inst, w, x), adjoint=True)
    np.testing.assert_allclose(out, psi, atol=1e-13)


# ----------------------------------------------------------- closed forms ----

@pytest.mark.parametrize("n", [1, 3, 6])
def test_ry_embedding_closed_form(n):
    x = RNG.uniform(-np.pi, np.pi, (4, n))
    layers = [W.L("RY", "ALL", "INPUT")]
    e = sim.forward_expval(n, layers, np.zeros(0), x)
    np.testing.assert_allclose(e, np.cos(x), atol=1e-14)
    _, _, gx = sim.grad_adjoint(n, layers, np.zeros(0), x, np.ones((4, n)))
    np.testing.assert_allclose(gx, -np.sin(x), atol=1e-13)


@pytest.mark.parametrize("n", [3, 4, 7])
def test_ry_then_cnot_ring_closed_form(n):
    """<Z_k> = prod_{i<=k} cos x_i (k >= 1); <Z_0> = prod_{i>=1} cos x_i."""
    x = RNG.uniform(-np.pi, np.pi, (3, n))
    e = sim.forward_expval(n, [W.L("RY", "ALL", "INPUT"), W.L("CNOT", "RING")], np.zeros(0), x)
    c = np.cos(x)
    ref = np.cumprod(c, axis=1)
    ref[:, 0] = np.prod(c[:, 1:], axis=1)
    np.testing.assert_allclose(e, ref, atol=1e-14)


def test_rx_after_ry_closed_form():
    x = RNG.uniform(-np.pi, np.pi, (5, 1))
    th = np.array([0.77])
    layers = [W.L("RY", "ALL", "INPUT"), W.L("RX", "ALL", "WEIGHT")]
    e = sim.forward_expval(1, layers, th, x)
    np.testing.assert_allclose(e[:, 0], np.cos(x[:, 0]) * np.cos(th[0]), atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 6])
def test_ghz_from_h_and_cnot_chain(n):
    layers = [W.L("H", "WIRE", wire=0), W.L("CNOT", "CHAIN")]
    psi = sim.run_o2(n, layers, np.zeros(0), np.zeros((1, 0)))
    ref = np.zeros(2 ** n, dtype=complex)
    ref[0] = ref[-1] = 1 / np.sqrt(2)
    np.testing.assert_allclose(psi[0], ref, atol=1e-15)
    np.testing.assert_allclose(sim.expval_z(psi, n), 0.0, atol=1e-15)


def test_expval_wire_order():
    """X on wire 0 flips the most significant bit: <Z_0> = -1, others +1."""
    n = 4
    e = sim.forward_expval(n, [W.L("X", "WIRE", wire=0)], np.zeros(0), np.zeros((1, 0)))
    np.testing.assert_allclose(e[0], [-1, 1, 1, 1])
    psi = sim.run_o2(n, [W.L("X", "WIRE", wire=0)], np.zeros(0), np.zeros((1, 0)))
    assert abs(psi[0, 8]) == 1.0


# ------------------------------------------------------------- gradients ----

GRAD_CASES = [
    ("rot_ring", lambda: (4, W.circuit_rot_ring(4, 2, "RY", ("RX", "RZ")), "normal")),
    ("rot_ring_zz", lambda: (4, W.circuit_rot_ring(4, 1, "RX", ("RX", "RY", "RZ"), zz=True), "normal")),
    ("ionq", lambda: (4, W.circuit_ionq(4, 2), "uniform2pi")),
    ("ibm", lambda: (4, W.circuit_ibm(4, 2), "uniform2pi")),
    ("rot_gate", lambda: (3, _layers(("ROT", "ALL", "WEIGHT"), ("CNOT", "RING"), ("ROT", "ALL", "INPUT"),
                                     ("CZ", "CHAIN"), ("RX", "ALL", "WEIGHT")), "normal")),
    ("ms_phases", lambda: (4, [W.L("RY", "ALL", "INPUT"), W.L("GPI2", "ALL", "WEIGHT", offset=0),
                               W.L("MS", "PAIRS_EVEN", "WEIGHT", offset=4, fixed2=0.13, fixed3=-0.41),
                               W.L("GPI", "ALL", "WEIGHT", offset=6),
                               W.L("MS", "PAIRS_ODD", "INPUT", offset=4, fixed2=0.3, fixed3=0.05)],
                           "uniform2pi")),
]


@pytest.mark.parametrize("case", GRAD_CASES, ids=[c[0] for c in GRAD_CASES])
def test_gradient_routes_agree(case):
    n, layers, dist = case[1]()
    w, x = W.draw_params(n, layers, 3, dist, 11)
    g = W.upstream(3, n, "normal", 3)
    _, gw, gx = sim.grad_adjoint(n, layers, w, x, g)
    sw, sx = sim.grad_param_shift(n, layers, w, x, g)
    fw, fx = sim.grad_fd(n, layers, w, x, g)
    m = ~np.isnan(sw)
    np.testing.assert_allclose(gw[m], sw[m], atol=1e-12)
    m = ~np.isnan(sx)
    np.testing.assert_allclose(gx[m], sx[m], atol=1e-12)
    np.testing.assert_allclose(gw, fw, atol=1e-7)
    np.testing.assert_allclose(gx, fx, atol=1e-7)


def test_rz_before_readout_has_zero_gradient():
    n = 3
    layers = [W.L("RY", "ALL", "INPUT"), W.L("CNOT", "RING"), W.L("RZ", "ALL", "WEIGHT"),
              W.L("ZZ", "RING", "WEIGHT")]
    w = RNG.standard_normal(6)
    x = RNG.uniform(-3, 3, (2, 3))
    _, gw, _ = sim.grad_adjoint(n, layers, w, x, W.upstream(2, n, "normal", 1))
    np.testing.assert_allclose(gw, 0.0, atol=1e-14)


def _untied(n, layers):
    """The same circuit with a separate feature column block per INPUT layer."""
    out, k = [], 0
    for ly in layers:
        if ly.source == "INPUT":
            ly = ly._replace(offset=k * n)
            k += 1
        out.append(ly)
    return out, k


QDI_CIRCUITS = [
    ("rz_ry_cnot", lambda n, blocks: W.circuit_rz_ry_cnot(n, blocks, "qdi"), "normal"),
    ("ionq", lambda n, blocks: W.circuit_ionq(n, blocks, "qdi"), "uniform2pi"),
    ("ibm", lambda n, blocks: W.circuit_ibm(n, blocks, "qdi"), "uniform2pi"),
]


@pytest.mark.parametrize("case", QDI_CIRCUITS, ids=[c[0] for c in QDI_CIRCUITS])
@pytest.mark.parametrize("n", [2, 4])
def test_qdi_reuploaded_feature_gradient(case, n):
    """QDI encoding (Sec. 3 for the Fig. 6 circuit, App. B for the native-gate
    circuits): the features enter every encoding layer, so dL/dx_q is the sum
    over blocks of the gradients of a circuit whose encoding layers have their
    own copies of x (the chain rule for a shared input), and it agrees with
    central differences of the tied circuit."""
    _, build, dist = case
    blocks = 3
    layers = build(n, blocks)
    assert W.circuit_counts(n, layers)[1] == n
    w, x = W.draw_params(n, layers, 2, dist, 21)
    g = W.upstream(2, n, "normal", 4)
    e, gw, gx = sim.grad_adjoint(n, layers, w, x, g)
    untied, k = _untied(n, layers)
    assert k == blocks
    xu = np.tile(x, (1, blocks))
    eu, gwu, gxu = sim.grad_adjoint(n, untied, w, xu, g)
    np.testing.assert_allclose(e, eu, atol=1e-14)
    np.testing.assert_allclose(gw, gwu, atol=1e-13)
    np.testing.assert_allclose(gx, gxu.reshape(2, blocks, n).sum(axis=1), atol=1e-13)
    fw, fx = sim.grad_fd(n, layers, w, x, g)
    np.testing.assert_allclose(gw, fw, atol=1e-7)
    np.testing.assert_allclose(gx, fx, atol=1e-7)
    # the per-block contributions differ, so a gradient that kept only one
    # block's share would fail the sum above
    per_block = gxu.reshape(2, blocks, n)
    assert np.max(np.abs(per_block[:, 0] - gx)) > 1e-3


def test_native_qdi_reuploads_every_block():
    """App. B QDI form: each block opens with the encoding pair, so the
    native-gate circuits hold one RZ(x) layer per block, all reading the same
    n feature columns."""
    for build, lead in ((W.circuit_ionq, "GPI2"), (W.circuit_ibm, "SX")):
        layers = build(6, 4, "qdi")
        enc = [i for i, ly in enumerate(layers) if ly.source == "INPUT"]
        assert len(enc) == 4
        assert all(layers[i].gate == "RZ" and layers[i].offset == 0 for i in enc)
        assert all(layers[i - 1].gate == lead for i in enc)
        assert len([ly for ly in build(6, 4, "vq") if ly.source == "INPUT"]) == 1


def test_vq_encodes_first_rz_only():
    """Sec. 3, VQ encoding: one feature layer (the first RZ), the other RZ
    layers trained; with all weights zero the state after the trained RY and
    the CNOT ring is |0...0>, on which RZ(x) is a pure phase."""
    n, blocks = 4, 3
    layers = W.circuit_rz_ry_cnot(n, blocks, "vq")
    nw, nf = W.circuit_counts(n, layers)
    assert nf == n and nw == n * (1 + 2 * blocks - 1)
    assert [ly.source for ly in layers if ly.gate == "RZ"] == ["INPUT"] + ["WEIGHT"] * (blocks - 1)
    x = np.random.default_rng(5).uniform(-np.pi, np.pi, (2, n))
    e = sim.forward_expval(n, layers, np.zeros(nw), x)
    np.testing.assert_allclose(e, 1.0, atol=1e-14)
