"""Seeded synthetic workloads: circuit descriptions and their input draws.

This module holds data only -- the layer-list format, the circuits of the
benchmark configurations and the seeded random draws of weights, features and
serving traces.  It contains none of the simulation arithmetic, so that both
the CPU oracle and the GPU path can take their inputs from it without sharing
any computation.

Layer format
------------
A circuit is an ordered list of uniform layers (the paper's framing of a QML
ansatz as alternating layers of uniformly applied gates, Sec. 1 and Fig. 6).
Each ``Layer`` names one gate type, a placement pattern and a parameter source:

* ``gate``     one of GATES (matrices in the paper's Appendix A).
* ``pattern``  ALL        -- the 1-qubit gate on every wire 0..n-1;
               WIRE       -- one gate on ``wire`` (and ``wire2`` for 2-qubit gates);
               RING       -- pairs (i, i+1 mod n), i = 0..n-1 in increasing i
                             (n = 2: the single pair (0, 1); n = 1: no gate);
               CHAIN      -- pairs (i, i+1), i = 0..n-2;
               PAIRS_EVEN -- disjoint pairs (2i, 2i+1), n even;
               PAIRS_ODD  -- disjoint pairs (2i+1, 2i+2 mod n), n even.
* ``source``   FIXED  -- every gate uses ``fixed``;
               WEIGHT -- gate k of the layer uses weights[offset + k];
               INPUT  -- gate k uses features[b, offset + k] for sample b.
               ROT reads three parameters per gate, (theta, phi, lambda) at
               offset + 3k .. offset + 3k + 2 (FIXED: fixed, fixed2, fixed3).
* ``fixed2``, ``fixed3``  MS: the phases (phi0, phi1) in turns of
               MS(phi0, phi1, theta) (Appendix A); ROT with FIXED source: phi
               and lambda.

Wire 0 is the most significant bit of the amplitude index (the bit order of the
paper's binary counting matrix J in Sec. 2.4.1 and of its CNOT permutation
vector in Sec. 2.3).
"""
from __future__ import annotations

import math
from collections import namedtuple

import numpy as np

GATES_1Q = ("RX", "RY", "RZ", "H", "X", "Z", "S", "SX", "GPI", "GPI2", "ROT")
GATES_2Q = ("CNOT", "CZ", "SWAP", "ZZ", "MS", "ECR")
GATES = GATES_1Q + GATES_2Q
# parametrized gates (Table 1, "Parametrized" column; GPI is read as
# parametrized, as in the caption of the paper's Fig. 4); ROT takes three
PARAM_GATES = ("RX", "RY", "RZ", "GPI", "GPI2", "ZZ", "MS", "ROT")
GATE_NPARAMS = {"ROT": 3}
PATTERNS = ("ALL", "WIRE", "RING", "CHAIN", "PAIRS_EVEN", "PAIRS_ODD")
SOURCES = ("FIXED", "WEIGHT", "INPUT")

Layer = namedtuple("Layer", "gate pattern source wire wire2 offset fixed fixed2 fixed3")
Layer.__new__.__defaults__ = (0, 1, 0, 0.0, 0.0, 0.0)


def L(gate, pattern="ALL", source="FIXED", wire=0, wire2=1, offset=0, fixed=0.0, fixed2=0.0, fixed3=0.0):
    """Convenience constructor with keyword defaults."""
    return Layer(gate, pattern, source, int(wire), int(wire2), int(offset), float(fixed), float(fixed2),
                 float(fixed3))


def gate_arity(gate: str) -> int:
    return 1 if gate in GATES_1Q else 2


def layer_wires(layer: Layer, n: int):
    """Wire tuples of the gate instances of ``layer`` in application order."""
    g, p = layer.gate, layer.pattern
    if gate_arity(g) == 1:
        if p == "ALL":
            return [(q,) for q in range(n)]
        if p == "WIRE":
            return [(layer.wire,)]
        raise ValueError(f"pattern {p} is not valid for 1-qubit gate {g}")
    if p == "WIRE":
        return [(layer.wire, layer.wire2)]
    if p == "RING":
        if n == 1:
            return []
        if n == 2:
            return [(0, 1)]
        return [(i, (i + 1) % n) for i in range(n)]
    if p == "CHAIN":
        return [(i, i + 1) for i in range(n - 1)]
    if p == "PAIRS_EVEN":
        return [(2 * i, 2 * i + 1) for i in range(n // 2)]
    if p == "PAIRS_ODD":
        return [(2 * i + 1, (2 * i + 2) % n) for i in range(n // 2)]
    raise ValueError(f"pattern {p} is not valid for 2-qubit gate {g}")


def layer_nparams(layer: Layer, n: int) -> int:
    if layer.gate not in PARAM_GATES or layer.source == "FIXED":
        return 0
    return GATE_NPARAMS.get(layer.gate, 1) * len(layer_wires(layer, n))


def circuit_counts(n: int, layers):
    """(n_weights, n_features) implied by the offsets of a layer list."""
    nw = nf = 0
    for ly in layers:
        k = layer_nparams(ly, n)
        if ly.source == "WEIGHT":
            nw = max(nw, ly.offset + k)
        elif ly.source == "INPUT":
            nf = max(nf, ly.offset + k)
    return nw, nf


class _Builder:
    """Appends layers and assigns contiguous parameter offsets in layer order,
    so that weights are laid out C-order as [block, gate slot, wire or pair]."""

    def __init__(self, n):
        self.n, self.layers, self.nw, self.nf = n, [], 0, 0

    def add(self, gate, pattern="ALL", source="FIXED", fixed=0.0, wire=0, wire2=1, fixed2=0.0, fixed3=0.0):
        ly = L(gate, pattern, source, wire, wire2, 0, fixed, fixed2, fixed3)
        k = layer_nparams(ly, self.n)
        if source == "WEIGHT":
            ly = ly._replace(offset=self.nw)
            self.nw += k
        elif source == "INPUT":
            ly = ly._replace(offset=self.nf)
            self.nf += k
        self.layers.append(ly)
        return self


# --------------------------------------------------------------------------
# Benchmark configurations (circuit shapes of the paper's Figs. 6 and 11)
# --------------------------------------------------------------------------

def circuit_rot_ring(n, blocks, embed="RY", rots=("RY", "RZ"), zz=False):
    """Angle embedding, then ``blocks`` x [rotations on every wire, optional
    IsingZZ ring, CNOT ring] -- the rotation + CNOT-ring ansatz of Fig. 6."""
    b = _Builder(n).add(embed, "ALL", "INPUT")
    for _ in range(blocks):
        for r in rots:
            b.add(r, "ALL", "WEIGHT")
        if zz:
            b.add("ZZ", "RING", "WEIGHT")
        b.add("CNOT", "RING")
    return b.layers


def circuit_rz_ry_cnot(n, blocks=8, encoding="qdi"):
    """The Rz-Ry-CNOT benchmark circuit of Sec. 3 (Fig. 6): a trained RY layer
    and a CNOT ring, then ``blocks`` x [RZ, RY, CNOT ring].

    encoding "vq" (vanilla quantum): the features enter the first RZ layer
    only; later RZ layers are trained.  encoding "qdi" (quantum depth
    infused): every RZ layer takes the same n features (feature q on wire q
    in every block), so the feature gradient sums over the blocks."""
    if encoding not in ("vq", "qdi"):
        raise ValueError(encoding)
    b = _Builder(n).add("RY", "ALL", "WEIGHT").add("CNOT", "RING")
    for k in range(blocks):
        if encoding == "qdi" or k == 0:
            b.layers.append(L("RZ", "ALL", "INPUT", 0, 1, 0, 0.0))
            b.nf = max(b.nf, n)
        else:
            b.add("RZ", "ALL", "WEIGHT")
        b.add("RY", "ALL", "WEIGHT").add("CNOT", "RING")
    return b.layers


def _encoding_blocks(b, n, blocks, encoding, lead, block):
    """Blocks of a native-gate circuit with its encoding pair [lead, RZ(x)].

    "vq": the pair once, before the blocks (the features enter one layer).
    "qdi": the pair opens every block, with the same n features (feature q on
    wire q) re-uploaded each time, so the feature gradient sums over blocks."""
    if encoding not in ("vq", "qdi"):
        raise ValueError(encoding)
    for k in range(blocks):
        if encoding == "qdi" or k == 0:
            lead(b)
            b.layers.append(L("RZ", "ALL", "INPUT", 0, 1, 0, 0.0))
            b.nf = max(b.nf, n)
        block(b, k)
    if blocks == 0:
        lead(b)
        b.add("RZ", "ALL", "INPUT")
    return b.layers


def circuit_ionq(n, blocks=8, encoding="vq"):
    """IonQ-style native gates (Appendix B, Fig. 11(b)): the encoding pair
    GPI2(0), RZ(x), and blocks of [GPI, GPI2, MS on brick pairs]; the pair
    sits before the blocks ("vq") or opens every block ("qdi")."""
    def lead(b):
        b.add("GPI2", "ALL", "FIXED", 0.0)

    def block(b, k):
        b.add("GPI", "ALL", "WEIGHT").add("GPI2", "ALL", "WEIGHT")
        b.add("MS", "PAIRS_EVEN" if k % 2 == 0 else "PAIRS_ODD", "WEIGHT")
    return _encoding_blocks(_Builder(n), n, blocks, encoding, lead, block)


def circuit_ibm(n, blocks=8, encoding="vq"):
    """IBM-style native gates (Appendix B, Fig. 11(a)): the encoding pair
    SX, RZ(x), and blocks of [RZ, SX, RZ, ECR on brick pairs]; the pair sits
    before the blocks ("vq") or opens every block ("qdi")."""
    def lead(b):
        b.add("SX", "ALL")

    def block(b, k):
        b.add("RZ", "ALL", "WEIGHT").add("SX", "ALL").add("RZ", "ALL", "WEIGHT")
        b.add("ECR", "PAIRS_EVEN" if k % 2 == 0 else "PAIRS_ODD")
    return _encoding_blocks(_Builder(n), n, blocks, encoding, lead, block)


CONFIGS = {
    # name: (n, batch, dtype, layers builder, weight dist, seed index)
    "c1_4q_b16": dict(n=4, batch=16, dtype="c128",
                      layers=lambda: circuit_rot_ring(4, 2, "RY", ("RX", "RZ")),
                      wdist="normal", seed=1, grad=False),
    "c2_12q_b256": dict(n=12, batch=256, dtype="c64",
                        layers=lambda: circuit_rot_ring(12, 10, "RY", ("RY", "RZ")),
                        wdist="normal", seed=2, grad=True),
    "c3_20q_b32": dict(n=20, batch=32, dtype="c64",
                       layers=lambda: circuit_rot_ring(20, 6, "RX", ("RX", "RY", "RZ"), zz=True),
                       wdist="normal", seed=3, grad=True),
    "c4a_16q_b128_ionq": dict(n=16, batch=128, dtype="c64", layers=lambda: circuit_ionq(16),
                              wdist="uniform2pi", seed=4, grad=True),
    "c4b_16q_b128_ibm": dict(n=16, batch=128, dtype="c64", layers=lambda: circuit_ibm(16),
                             wdist="uniform2pi", seed=4, grad=True),
}


def draw_params(n, layers, batch, wdist="normal", seed=0):
    """Weights ~ N(0,1) (or U(0, 2*pi)) from default_rng(1000+seed) and features
    ~ U(-pi, pi) from default_rng(2000+seed), in float64, C order."""
    nw, nf = circuit_counts(n, layers)
    rw = np.random.default_rng(1000 + seed)
    if wdist == "normal":
        w = rw.standard_normal(nw)
    elif wdist == "uniform2pi":
        w = rw.uniform(0.0, 2.0 * math.pi, nw)
    else:
        raise ValueError(wdist)
    rf = np.random.default_rng(2000 + seed)
    x = rf.uniform(-math.pi, math.pi, (batch, nf))
    return w.astype(np.float64), x.astype(np.float64)


def config(name):
    """(n, batch, dtype, layers, weights, features) of a named configuration."""
    c = CONFIGS[name]
    layers = c["layers"]()
    w, x = draw_params(c["n"], layers, c["batch"], c["wdist"], c["seed"])
    return c["n"], c["batch"], c["dtype"], layers, w, x


def upstream(batch, n, kind="ones", seed=0):
    """Upstream gradient g = dLoss/d<Z_i>: ones (the summed readout of the
    paper's Fig. 6) or N(0,1) draws from default_rng(5000+seed)."""
    if kind == "ones":
        return np.ones((batch, n), dtype=np.float64)
    return np.random.default_rng(5000 + seed).standard_normal((batch, n))


def random_states(batch, n, seed=0, dtype=np.complex128):
    """Normalised random complex states [batch, 2**n] from default_rng(4000+seed)."""
    r = np.random.default_rng(4000 + seed)
    s = r.standard_normal((batch, 2 ** n)) + 1j * r.standard_normal((batch, 2 ** n))
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    return s.astype(dtype)


# --------------------------------------------------------------------------
# Serving trace: Poisson arrivals of rotation + CNOT-ring circuits
# --------------------------------------------------------------------------

Request = namedtuple("Request", "rid t_arrive n batch blocks want_grad")


def serving_trace(n_requests, qps, seed=0, n_range=(6, 22), b_max=512,
                  blocks_range=(2, 20), grad_frac=0.3):
    """Arrival times ~ Poisson(qps) from default_rng(3000+seed); shapes from
    default_rng(3001+seed): n ~ U{6..22}, batch = round(exp(U(0, ln 512))),
    blocks ~ U{2..20}, 30% forward+gradient."""
    ra = np.random.default_rng(3000 + seed)
    rs = np.random.default_rng(3001 + seed)
    gaps = ra.exponential(1.0 / qps, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        n = int(rs.integers(n_range[0], n_range[1] + 1))
        b = int(round(math.exp(rs.uniform(0.0, math.log(b_max)))))
        blocks = int(rs.integers(blocks_range[0], blocks_range[1] + 1))
        g = bool(rs.uniform() < grad_frac)
        out.append(Request(i, float(t[i]), n, max(1, b), blocks, g))
    return out


def request_params(req, seed=0):
    """Layers, weights and features of one serving request (default_rng(3002+id))."""
    layers = circuit_rot_ring(req.n, req.blocks, "RY", ("RY", "RZ"))
    nw, nf = circuit_counts(req.n, layers)
    r = np.random.default_rng(3002 + seed * 100003 + req.rid)
    w = r.standard_normal(nw)
    x = r.uniform(-math.pi, math.pi, (req.batch, nf))
    return layers, w, x
