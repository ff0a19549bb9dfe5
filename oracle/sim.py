"""Plain complex128 state-vector simulation (TEST INFRASTRUCTURE).

What is computed (the paper's problem statement, Sec. 1 and Sec. 2.2.1): for
sample b, psi_b = U_L ... U_1 |0...0>, where U_l is the 2^n x 2^n matrix of
layer l -- the ordered product of its gates, each embedded on its wires with
wire 0 as the most significant index bit.  The readout is <Z_i> = psi^dag Z_i
psi for every wire i (the single-qubit observables of Figs. 6 and 11), and the
gradients are those of L = sum_{b,i} g_{b,i} <Z_i>_b for an upstream g.

Two tiers:
* O1 (``run_o1``): builds each layer's full unitary from Kronecker products and
  multiplies it into the state -- the "Unitary operation" of Sec. 2.2.1.
  Feasible for n <= 10.
* O2 (``run_o2``): applies every gate as a tensor contraction on the state
  reshaped to [B, 2, ..., 2] -- the "Sequential Einsum" of Sec. 2.2.2.

Gradients (``grad_adjoint``, ``grad_param_shift``, ``grad_fd``) are three
independent routes to the same exact derivative.
"""
from __future__ import annotations

import numpy as np

from . import gates as G

PARAM_GATES = tuple(G.PARAM) + ("ROT",)
ONE_QUBIT = ("RX", "RY", "RZ", "H", "X", "Z", "S", "SX", "GPI", "GPI2", "ROT")


def n_params(gate):
    """Parameters one gate reads (Rot: theta, phi, lambda)."""
    return G.N_PARAMS.get(gate, 1) if gate in PARAM_GATES else 0


# ---------------------------------------------------------------------------
# circuit expansion
# ---------------------------------------------------------------------------

def pattern_wires(n, ly):
    """Wires of each gate of a layer, in application order.

    ALL: every wire; WIRE: the named wire(s); RING: (i, i+1 mod n) for
    i = 0..n-1 (a ring of CNOTs "to entangle all qubits", Sec. 2.3, and the
    nearest-neighbour Rzz ring with the (n-1, 0) pair, Sec. 2.4.1), read as the
    single pair (0, 1) for n = 2 and empty for n = 1; CHAIN: (i, i+1);
    PAIRS_EVEN: (2i, 2i+1); PAIRS_ODD: (2i+1, 2i+2 mod n)."""
    p = ly.pattern
    if ly.gate in ONE_QUBIT:
        if p == "ALL":
            return [(q,) for q in range(n)]
        if p == "WIRE":
            return [(ly.wire,)]
        raise ValueError(p)
    if p == "WIRE":
        return [(ly.wire, ly.wire2)]
    if p == "RING":
        return [] if n < 2 else ([(0, 1)] if n == 2 else [(i, (i + 1) % n) for i in range(n)])
    if p == "CHAIN":
        return [(i, i + 1) for i in range(n - 1)]
    if p == "PAIRS_EVEN":
        return [(2 * i, 2 * i + 1) for i in range(n // 2)]
    if p == "PAIRS_ODD":
        return [(2 * i + 1, (2 * i + 2) % n) for i in range(n // 2)]
    raise ValueError(p)


def param_counts(n, layers):
    """(n_weights, n_features) addressed by the layer offsets."""
    nw = nf = 0
    for ly in layers:
        if ly.gate in PARAM_GATES and ly.source != "FIXED":
            k = n_params(ly.gate) * len(pattern_wires(n, ly))
            if ly.source == "WEIGHT":
                nw = max(nw, ly.offset + k)
            else:
                nf = max(nf, ly.offset + k)
    return nw, nf


def expand(n, layers):
    """Gate instances in application order:
    (gate, wires, source, first parameter index, fixed, layer_id, fixed2, fixed3)."""
    out = []
    for li, ly in enumerate(layers):
        npar = max(1, n_params(ly.gate))
        for k, wires in enumerate(pattern_wires(n, ly)):
            src = ly.source if ly.gate in PARAM_GATES else "FIXED"
            out.append((ly.gate, tuple(wires), src, ly.offset + npar * k, ly.fixed, li,
                        getattr(ly, "fixed2", 0.0), getattr(ly, "fixed3", 0.0)))
    return out


def instance_param(inst, weights, features):
    """The gate's parameter: a scalar (FIXED/WEIGHT) or per-sample vector
    (INPUT); for Rot a 3-vector, or [B, 3] per sample; None without one."""
    gate, _, src, idx, fixed = inst[:5]
    if gate not in PARAM_GATES:
        return None
    if gate == "ROT":
        if src == "FIXED":
            return np.array([fixed, inst[6], inst[7]], dtype=np.float64)
        if src == "WEIGHT":
            return np.asarray(weights[idx:idx + 3], dtype=np.float64)
        return np.asarray(features[:, idx:idx + 3], dtype=np.float64)
    if src == "FIXED":
        return float(fixed)
    if src == "WEIGHT":
        return float(weights[idx])
    return np.asarray(features[:, idx], dtype=np.float64)


def _per_sample(gate, theta):
    """Whether a parameter value holds one entry per sample."""
    return np.ndim(theta) == (2 if gate == "ROT" else 1)


def _phases(inst):
    return (inst[6], inst[7]) if inst[0] == "MS" else (0.0, 0.0)


# ---------------------------------------------------------------------------
# the paper's K_Rz matrix (Sec. 2.4.1): J = binary counting matrix, K = 1 - 2J
# ---------------------------------------------------------------------------

def counting_matrix(n):
    """J: 2^n x n, row j = binary digits of j, first column most significant."""
    j = np.arange(2 ** n)
    return ((j[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.int64)


def k_rz(n):
    return 1 - 2 * counting_matrix(n)


def k_rzz_ring(n):
    """K_Rzz[i, j] = K_Rz[i, j] * K_Rz[i, (j + 1) mod n] (Sec. 2.4.1)."""
    K = k_rz(n)
    return K * K[:, (np.arange(n) + 1) % n]


def expval_z(psi, n):
    """<Z_i> for every wire: K_Rz^T applied to the probabilities |psi|^2."""
    p = np.abs(psi) ** 2
    return p @ k_rz(n).astype(np.float64)


def diag_hamiltonian(g, n):
    """Diagonal of H_b = sum_i g_{b,i} Z_i for every sample: [B, 2^n]."""
    return g @ k_rz(n).T.astype(np.float64)


# ---------------------------------------------------------------------------
# O2: per-gate tensor contraction
# ---------------------------------------------------------------------------

def _apply_local(psi, n, U, wires):
    """Contract a (possibly per-sample) 2^k x 2^k matrix into the wires of psi.

    psi: [B, 2^n]; U: [2^k, 2^k] or [B, 2^k, 2^k]; wires in matrix bit order."""
    B = psi.shape[0]
    k = len(wires)
    t = psi.reshape((B,) + (2,) * n)
    axes = [1 + w for w in wires]
    t = np.moveaxis(t, axes, list(range(1, 1 + k)))
    rest = t.shape[1 + k:]
    t = t.reshape(B, 2 ** k, -1)
    if U.ndim == 2:
        t = np.einsum("ij,bjm->bim", U, t)
    else:
        t = np.einsum("bij,bjm->bim", U, t)
    t = t.reshape((B,) + (2,) * k + rest)
    t = np.moveaxis(t, list(range(1, 1 + k)), axes)
    return t.reshape(B, 2 ** n)


def _inst_matrix(inst, theta, B):
    gate = inst[0]
    if theta is None:
        return G.matrix(gate)
    if not _per_sample(gate, theta):
        return G.matrix(gate, theta, _phases(inst))
    return np.stack([G.matrix(gate, t, _phases(inst)) for t in theta])


def apply_instance(psi, n, inst, theta, adjoint=False):
    U = _inst_matrix(inst, theta, psi.shape[0])
    if adjoint:
        U = np.conj(np.swapaxes(U, -1, -2))
    return _apply_local(psi, n, U, inst[1])


def zero_state(B, n):
    psi = np.zeros((B, 2 ** n), dtype=np.complex128)
    psi[:, 0] = 1.0
    return psi


def run_o2(n, layers, weights, features, batch=None, psi0=None):
    """Final states [B, 2^n] by sequential per-gate contraction."""
    if batch is None:
        batch = features.shape[0]
    psi = zero_state(batch, n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for inst in expand(n, layers):
        psi = apply_instance(psi, n, inst, instance_param(inst, weights, features))
    return psi


# ---------------------------------------------------------------------------
# O1: full layer unitaries from Kronecker products
# ---------------------------------------------------------------------------

def embed_matrix(n, M, wires):
    """Full 2^n x 2^n matrix of a k-qubit matrix M acting on ``wires``.

    Adjacent ascending wires use np.kron (wire 0 = most significant factor);
    other placements write the definition out entry by entry."""
    k = len(wires)
    if list(wires) == list(range(wires[0], wires[0] + k)):
        left = np.eye(2 ** wires[0], dtype=np.complex128)
        right = np.eye(2 ** (n - wires[0] - k), dtype=np.complex128)
        return np.kron(np.kron(left, M), right)
    N = 2 ** n
    F = np.zeros((N, N), dtype=np.complex128)
    bitpos = [n - 1 - w for w in wires]
    mask = sum(1 << p for p in bitpos)
    for col in range(N):
        cin = 0
        for p in bitpos:
            cin = (cin << 1) | ((col >> p) & 1)
        base = col & ~mask
        for rout in range(2 ** k):
            row = base
            for i, p in enumerate(bitpos):
                if (rout >> (k - 1 - i)) & 1:
                    row |= 1 << p
            F[row, col] += M[rout, cin]
    return F


def layer_unitary(n, layers, li, weights, x_row):
    """Full unitary of layer ``li`` for one sample (features row ``x_row``)."""
    U = np.eye(2 ** n, dtype=np.complex128)
    feats = None if x_row is None else np.asarray(x_row)[None, :]
    for inst in expand(n, [layers[li]]):
        inst = inst[:5] + (li,) + inst[6:]
        th = instance_param(inst, weights, feats)
        if th is not None and _per_sample(inst[0], th):
            th = th[0]
        U = embed_matrix(n, _inst_matrix(inst, th, 1), inst[1]) @ U
    return U


def run_o1(n, layers, weights, features):
    """Final states [B, 2^n] from per-sample products of full layer unitaries."""
    assert n <= 10, "O1 builds 2^n x 2^n matrices"
    B = features.shape[0]
    out = np.zeros((B, 2 ** n), dtype=np.complex128)
    for b in range(B):
        psi = np.zeros(2 ** n, dtype=np.complex128)
        psi[0] = 1.0
        for li in range(len(layers)):
            psi = layer_unitary(n, layers, li, weights, features[b]) @ psi
        out[b] = psi
    return out


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def forward_expval(n, layers, weights, features, tier="o2"):
    run = run_o2 if tier == "o2" else run_o1
    return expval_z(run(n, layers, weights, features), n)


def loss(n, layers, weights, features, g, tier="o2"):
    return float(np.sum(g * forward_expval(n, layers, weights, features, tier)))


def grad_adjoint(n, layers, weights, features, g):
    """Adjoint sweep gate by gate (complex128).

    lambda = H psi with H = sum_i g_i Z_i; then for each gate in reverse order:
    dL/dparam += 2 Im <lambda|G|psi> (G the output-side generator), followed by
    psi <- U^dag psi, lambda <- U^dag lambda.  Returns (expz, g_w, g_x)."""
    B = features.shape[0]
    nw, nf = param_counts(n, layers)
    psi = run_o2(n, layers, weights, features)
    e = expval_z(psi, n)
    lam = psi * diag_hamiltonian(g, n)
    gw = np.zeros(max(nw, len(weights)))
    gx = np.zeros((B, max(nf, features.shape[1])))
    for inst in reversed(expand(n, layers)):
        th = instance_param(inst, weights, features)
        gate, wires, src = inst[0], inst[1], inst[2]
        if gate in PARAM_GATES and src != "FIXED":
            if not _per_sample(gate, th):
                gens = G.generators(gate, th, _phases(inst))
            else:
                per = [G.generators(gate, t, _phases(inst)) for t in th]
                gens = [np.stack([p[k] for p in per]) for k in range(len(per[0]))]
            for k, Gm in enumerate(gens):
                Gpsi = _apply_local(psi, n, Gm, wires)
                per_b = 2.0 * np.imag(np.sum(np.conj(lam) * Gpsi, axis=1))
                if src == "WEIGHT":
                    gw[inst[3] + k] += per_b.sum()
                else:
                    gx[:, inst[3] + k] += per_b
        psi = apply_instance(psi, n, inst, th, adjoint=True)
        lam = apply_instance(lam, n, inst, th, adjoint=True)
    return e, gw, gx


# Rot = P(phi) RY(theta) P(lambda), P(a) = diag(1, e^{ia}) = e^{ia/2} RZ(a):
# each of its parameters enters as exp(-i a P / 2) up to a global phase
_SHIFT = {"RX": (np.pi / 2, 0.5), "RY": (np.pi / 2, 0.5), "RZ": (np.pi / 2, 0.5),
          "ZZ": (np.pi / 2, 0.5), "MS": (0.25, np.pi), "ROT": (np.pi / 2, 0.5)}


def _per_sample_losses(n, layers, w, x, g):
    return np.sum(g * forward_expval(n, layers, w, x), axis=1)


def grad_param_shift(n, layers, weights, features, g):
    """Two-term parameter shift, exact for gates exp(-i a P) with P^2 = I:
    rotations and ZZ: [f(t + pi/2) - f(t - pi/2)] / 2;
    MS(t) = exp(-i pi t XX): pi [f(t + 1/4) - f(t - 1/4)].
    Parameters of GPI / GPI2 layers are left as NaN (no two-term rule), and
    so is every parameter that more than one gate reads (a feature re-uploaded
    in several layers): the two-term rule is exact only for a parameter that
    enters the circuit once."""
    nw, nf = param_counts(n, layers)
    gw = np.full(len(weights), np.nan)
    gx = np.full(features.shape, np.nan)
    kind_w, kind_x = {}, {}
    for inst in expand(n, layers):
        for k in range(n_params(inst[0])):
            if inst[2] == "WEIGHT":
                kind_w.setdefault(inst[3] + k, []).append(inst[0])
            elif inst[2] == "INPUT":
                kind_x.setdefault(inst[3] + k, []).append(inst[0])
    kind_w = {i: g[0] for i, g in kind_w.items() if len(g) == 1}
    kind_x = {i: g[0] for i, g in kind_x.items() if len(g) == 1}
    for i, gate in kind_w.items():
        if gate not in _SHIFT:
            continue
        s, c = _SHIFT[gate]
        wp, wm = weights.copy(), weights.copy()
        wp[i] += s
        wm[i] -= s
        gw[i] = c * (loss(n, layers, wp, features, g) - loss(n, layers, wm, features, g))
    for i, gate in kind_x.items():
        if gate not in _SHIFT:
            continue
        s, c = _SHIFT[gate]
        xp, xm = features.copy(), features.copy()
        xp[:, i] += s
        xm[:, i] -= s
        gx[:, i] = c * (_per_sample_losses(n, layers, weights, xp, g)
                        - _per_sample_losses(n, layers, weights, xm, g))
    return gw, gx


def grad_fd(n, layers, weights, features, g, h=1e-6):
    """Central finite differences of the loss in every weight and feature."""
    gw = np.zeros(len(weights))
    for i in range(len(weights)):
        wp, wm = weights.copy(), weights.copy()
        wp[i] += h
        wm[i] -= h
        gw[i] = (loss(n, layers, wp, features, g) - loss(n, layers, wm, features, g)) / (2 * h)
    gx = np.zeros(features.shape)
    for i in range(features.shape[1]):
        xp, xm = features.copy(), features.copy()
        xp[:, i] += h
        xm[:, i] -= h
        gx[:, i] = (_per_sample_losses(n, layers, weights, xp, g)
                    - _per_sample_losses(n, layers, weights, xm, g)) / (2 * h)
    return gw, gx
