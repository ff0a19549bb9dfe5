"""Parity of the HIP path with the CPU oracle, element by element.

Every case builds a circuit through the C ABI (via the thin binding), runs
forward, <Z_i> and the adjoint gradient on the GPU, and compares with the
oracle's complex128 results at the tolerances in tests/gpu_util.py.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import sim
from tests.gpu_util import compare, gpu_run, note, oracle_run

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2506_04891_amd import tqsim as T


def _circuit(n, layers, dtype, mode="auto", tile_bits=0):
    return T.Circuit(n, layers, dtype, mode=mode, tile_bits=tile_bits)


def _params(n, layers, B, seed, dist="normal"):
    w, x = W.draw_params(n, layers, B, dist, seed)
    g = W.upstream(B, n, "normal", seed)
    return w, x, g


LAYER_KINDS = [
    ("RX", "ALL", "WEIGHT"), ("RY", "ALL", "WEIGHT"), ("RZ", "ALL", "WEIGHT"),
    ("H", "ALL"), ("X", "ALL"), ("Z", "ALL"), ("S", "ALL"), ("SX", "ALL"),
    ("GPI", "ALL", "WEIGHT"), ("GPI2", "ALL", "WEIGHT"), ("RZ", "ALL", "INPUT"),
    ("CNOT", "RING"), ("CNOT", "CHAIN"), ("CZ", "RING"), ("SWAP", "CHAIN"),
    ("ZZ", "RING", "WEIGHT"), ("ZZ", "CHAIN", "WEIGHT"), ("ZZ", "RING", "INPUT"),
    ("MS", "PAIRS_EVEN", "WEIGHT"), ("MS", "PAIRS_ODD", "WEIGHT"),
    ("ECR", "PAIRS_EVEN"), ("ECR", "PAIRS_ODD"), ("CNOT", "PAIRS_ODD"),
]


def _sandwich(n, spec):
    """Embedding, an entangler (so the layer under test is not folded into the
    product state), the layer under test, then a rotation layer so that its
    parameters reach the <Z> readout."""
    b = W._Builder(n)
    b.add("RY", "ALL", "INPUT").add("RX", "ALL", "WEIGHT").add("CNOT", "CHAIN")
    b.add(*spec[:3]) if len(spec) == 3 else b.add(*spec)
    b.add("RX", "ALL", "WEIGHT").add("CZ", "CHAIN").add("RY", "ALL", "WEIGHT")
    return b.layers


@pytest.mark.parametrize("mode", ["per_layer", "fused"])
@pytest.mark.parametrize("n", [2, 5, 6, 13, 14])
@pytest.mark.parametrize("spec", LAYER_KINDS, ids=["-".join(s) for s in LAYER_KINDS])
def test_layer_kind_c64(spec, n, mode):
    if "PAIRS" in spec[1] and n % 2:
        pytest.skip("brick pairs need even n")
    layers = _sandwich(n, spec)
    B = 3
    w, x, g = _params(n, layers, B, seed=n)
    note(f"case layer={spec} n={n} mode={mode} c64")
    got = gpu_run(_circuit(n, layers, "c64", mode), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c64", label=f"{spec} n={n} {mode}")


@pytest.mark.parametrize("mode", ["per_layer", "fused"])
@pytest.mark.parametrize("n", [3, 6, 12])
@pytest.mark.parametrize("spec", LAYER_KINDS, ids=["-".join(s) for s in LAYER_KINDS])
def test_layer_kind_c128(spec, n, mode):
    if "PAIRS" in spec[1] and n % 2:
        pytest.skip("brick pairs need even n")
    layers = _sandwich(n, spec)
    B = 2
    w, x, g = _params(n, layers, B, seed=100 + n)
    note(f"case layer={spec} n={n} mode={mode} c128")
    got = gpu_run(_circuit(n, layers, "c128", mode), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c128", label=f"{spec} n={n} {mode}")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("spec", LAYER_KINDS, ids=["-".join(s) for s in LAYER_KINDS])
def test_layer_kind_dense_c64(spec, n):
    """Full-unitary layers on the matrix cores (n <= 6), single precision."""
    if "PAIRS" in spec[1] and n % 2:
        pytest.skip("brick pairs need even n")
    layers = _sandwich(n, spec)
    B = 5
    w, x, g = _params(n, layers, B, seed=200 + n)
    note(f"case layer={spec} n={n} mode=dense c64")
    c = _circuit(n, layers, "c64", "dense")
    assert c.plan()["mode"] == "dense"
    got = gpu_run(c, w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c64", label=f"{spec} n={n} dense")


@pytest.mark.parametrize("n", [2, 4, 6])
@pytest.mark.parametrize("spec", LAYER_KINDS, ids=["-".join(s) for s in LAYER_KINDS])
def test_layer_kind_dense_c128(spec, n):
    """Full-unitary layers on the FP64 matrix cores, double precision."""
    layers = _sandwich(n, spec)
    B = 3
    w, x, g = _params(n, layers, B, seed=300 + n)
    note(f"case layer={spec} n={n} mode=dense c128")
    got = gpu_run(_circuit(n, layers, "c128", "dense"), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c128", label=f"{spec} n={n} dense")


@pytest.mark.parametrize("B", [1, 17, 65])
@pytest.mark.parametrize("name,n,builder,dist", [
    ("ionq", 6, lambda n: W.circuit_ionq(n, 4), "uniform2pi"),
    ("ibm", 6, lambda n: W.circuit_ibm(n, 4), "uniform2pi"),
    ("rot_ring_zz", 5, lambda n: W.circuit_rot_ring(n, 3, "RX", ("RX", "RY", "RZ"), zz=True), "normal"),
])
def test_dense_circuits(name, n, builder, dist, B):
    """Whole native-gate circuits in dense mode, ragged sample groups."""
    layers = builder(n)
    w, x, g = _params(n, layers, B, seed=B, dist=dist)
    note(f"case dense {name} n={n} B={B}")
    got = gpu_run(_circuit(n, layers, "c64", "dense"), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c64", label=f"dense {name} n={n} B={B}")


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [4, 5, 6])
def test_dense_multi_tile(n, dt):
    """Dense mode over many sample tiles with a ragged last one (129 samples:
    16, 32 or 64 per tile), in both precisions: every wave's output block, the
    layer rows fetched one op ahead, and the gradient-only stages shared out
    among the waves, against the oracle on every row."""
    layers = W.circuit_rot_ring(n, 3, "RY", ("RY", "RZ"))
    B = 129
    w, x, g = _params(n, layers, B, seed=400 + n, dist="normal")
    note(f"case dense multi-tile n={n} B={B} {dt}")
    c = _circuit(n, layers, dt, "dense")
    assert c.plan()["mode"] == "dense"
    got = gpu_run(c, w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, dt, label=f"dense multi-tile n={n} {dt}")


def test_config1_dense_exact():
    n, B, dt, layers, w, x = W.config("c1_4q_b16")
    g = W.upstream(B, n, "normal", 1)
    note("case c1 mode=dense")
    got = gpu_run(_circuit(n, layers, dt, "dense"), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c128", label="c1 dense")


@pytest.mark.parametrize("tile_bits", [10, 11, 12])
@pytest.mark.parametrize("name,builder,dist", [
    ("rot_ring_zz", lambda n: W.circuit_rot_ring(n, 3, "RX", ("RX", "RY", "RZ"), zz=True), "normal"),
    ("ionq", lambda n: W.circuit_ionq(n, 4), "uniform2pi"),
    ("ibm", lambda n: W.circuit_ibm(n, 4), "uniform2pi"),
])
@pytest.mark.parametrize("n", [11, 12, 14])
@pytest.mark.parametrize("mode", ["per_layer", "fused"])
def test_config_shapes_multipass(name, builder, dist, n, tile_bits, mode):
    if name in ("ionq", "ibm") and n % 2:
        pytest.skip("brick pairs need even n")
    layers = builder(n)
    B = 3
    w, x, g = _params(n, layers, B, seed=7, dist=dist)
    note(f"case {name} n={n} K={tile_bits} mode={mode}")
    got = gpu_run(_circuit(n, layers, "c64", mode, tile_bits), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c64", label=f"{name} n={n} K={tile_bits} {mode}")


def test_config1_exact():
    """4 qubits, batch 16, complex128: every output against the oracle at 1e-12."""
    n, B, dt, layers, w, x = W.config("c1_4q_b16")
    g = W.upstream(B, n, "normal", 1)
    for mode in ("per_layer", "fused"):
        note(f"case c1 mode={mode}")
        got = gpu_run(_circuit(n, layers, dt, mode), w, x, g)
        ref = oracle_run(n, layers, w, x, g)
        compare(got, ref, "c128", label=f"c1 {mode}")
        np.testing.assert_allclose(got["norm"], 1.0, atol=1e-13)


@pytest.mark.parametrize("B", [1, 5, 17, 64, 65])
@pytest.mark.parametrize("n", [1, 2, 4, 7, 9])
def test_small_n_batches(n, B):
    """Several samples per workgroup, ragged last workgroup, virtual padding for n < 4."""
    layers = W.circuit_rot_ring(n, 2, "RY", ("RY", "RZ"))
    w, x, g = _params(n, layers, B, seed=B + 10 * n)
    note(f"case small n={n} B={B}")
    got = gpu_run(_circuit(n, layers, "c64"), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, "c64", label=f"small n={n} B={B}")


def test_ghz_and_bell():
    for n in (2, 3, 6, 13):
        layers = [W.L("H", "WIRE", wire=0), W.L("CNOT", "CHAIN")]
        c = _circuit(n, layers, "c128")
        note(f"case ghz n={n}")
        got = gpu_run(c, np.zeros(0), np.zeros((1, 0)), batch=1)
        ref = np.zeros(2 ** n, dtype=complex)
        ref[0] = ref[-1] = 1 / np.sqrt(2)
        np.testing.assert_allclose(got["psi"][0], ref, atol=1e-15)
        np.testing.assert_allclose(got["e"][0], 0.0, atol=1e-15)


def test_ry_embedding_closed_form():
    for n in (1, 4, 12, 14):
        layers = [W.L("RY", "ALL", "INPUT")]
        x = np.random.default_rng(n).uniform(-np.pi, np.pi, (4, n))
        c = _circuit(n, layers, "c128")
        note(f"case ry-embed n={n}")
        got = gpu_run(c, np.zeros(0), x, np.ones((4, n)))
        np.testing.assert_allclose(got["e"], np.cos(x), atol=1e-13)
        np.testing.assert_allclose(got["gx"], -np.sin(x), atol=1e-12)


def test_deterministic_repeat():
    n, B, dt, layers, w, x = W.config("c4a_16q_b128_ionq")
    n = 14
    layers = W.circuit_ionq(n, 8)
    w, x = W.draw_params(n, layers, 8, "uniform2pi", 4)
    g = W.upstream(8, n, "normal", 2)
    c = _circuit(n, layers, "c64")
    a = gpu_run(c, w, x, g)
    b = gpu_run(c, w, x, g)
    for k in ("psi", "e", "gw", "gx"):
        np.testing.assert_array_equal(a[k], b[k])


# ---------------------------------------------------------------- full size --

def _sampled_full(name, samples, spec=None):
    n, B, dt, layers, w, x = spec if spec is not None else W.config(name)
    g = np.zeros((B, n))
    g[samples] = W.upstream(len(samples), n, "normal", 9)
    note(f"case full {name} samples={samples}")
    got = gpu_run(_circuit(n, layers, dt), w, x, g)
    # the oracle computes only the sampled rows; weight gradients only receive
    # contributions from samples with a nonzero upstream gradient
    ref = oracle_run(n, layers, w, x[samples], g[samples])
    np.testing.assert_allclose(got["e"][samples], ref["e"], atol=2e-5)
    np.testing.assert_allclose(got["norm"], 1.0, atol=1e-5)
    e1 = np.max(np.abs(got["gw"] - ref["gw"])) / np.max(np.abs(ref["gw"]))
    e2 = np.max(np.abs(got["gx"][samples] - ref["gx"])) / np.max(np.abs(ref["gx"]))
    assert e1 <= 1e-4 and e2 <= 1e-4, (e1, e2)
    others = [b for b in range(B) if b not in samples]
    np.testing.assert_array_equal(got["gx"][others], 0.0)
    return got


def test_full_c2_sampled():
    _sampled_full("c2_12q_b256", [0, 97, 255])


def test_full_c4a_sampled():
    _sampled_full("c4a_16q_b128_ionq", [0, 37, 90, 127])


def test_full_c4b_sampled():
    _sampled_full("c4b_16q_b128_ibm", [5, 64, 101, 126])


def test_full_c3_sampled():
    """20 qubits, batch 32 (the full workload): first, last and two interior
    rows against the oracle; and one row's final state element by element."""
    got = _sampled_full("c3_20q_b32", [0, 13, 22, 31])
    n, B, dt, layers, w, x = W.config("c3_20q_b32")
    psi = sim.run_o2(n, layers, w, x[[22]])
    assert np.max(np.abs(got["psi"][22] - psi[0])) <= 2e-5


# ------------------------------------------- Fig. 6 circuit, VQ and QDI --

@pytest.mark.parametrize("encoding", ["vq", "qdi"])
@pytest.mark.parametrize("n,dtype,mode,B", [
    (4, "c128", "auto", 5), (4, "c128", "dense", 5), (6, "c64", "dense", 3),
    (9, "c64", "per_layer", 3), (9, "c64", "fused", 3), (12, "c64", "fused", 3),
    (13, "c128", "fused", 2), (14, "c64", "per_layer", 2), (16, "c64", "fused", 2),
])
def test_rz_ry_cnot_vq_qdi(encoding, n, dtype, mode, B):
    """The Rz-Ry-CNOT circuit of Sec. 3 with features in the first RZ layer
    (VQ) or in all eight (QDI, one shared feature column per wire)."""
    layers = W.circuit_rz_ry_cnot(n, 8, encoding)
    w, x, g = _params(n, layers, B, seed=30 + n)
    note(f"case fig6 {encoding} n={n} {dtype} mode={mode} B={B}")
    got = gpu_run(_circuit(n, layers, dtype, mode), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, dtype, label=f"fig6 {encoding} n={n} {mode}")


@pytest.mark.parametrize("encoding", ["vq", "qdi"])
@pytest.mark.parametrize("circuit", ["ionq", "ibm"])
@pytest.mark.parametrize("n,dtype,mode,B", [
    (4, "c128", "auto", 5), (4, "c64", "dense", 3), (6, "c128", "per_layer", 3), (8, "c64", "fused", 4),
    (10, "c128", "fused", 2), (12, "c64", "per_layer", 3), (14, "c64", "fused", 3), (16, "c64", "fused", 2),
    (16, "c128", "fused", 1),
])
def test_native_vq_qdi(circuit, encoding, n, dtype, mode, B):
    """The IonQ and IBM native-gate circuits of App. B with the encoding pair
    once (VQ) or opening every block (QDI, the same features re-uploaded)."""
    build = W.circuit_ionq if circuit == "ionq" else W.circuit_ibm
    layers = build(n, 8, encoding)
    w, x, g = _params(n, layers, B, seed=40 + n, dist="uniform2pi")
    note(f"case native {circuit} {encoding} n={n} {dtype} mode={mode} B={B}")
    got = gpu_run(_circuit(n, layers, dtype, mode), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, dtype, label=f"native {circuit} {encoding} n={n} {mode}")


@pytest.mark.parametrize("encoding", ["vq", "qdi"])
def test_rz_ry_cnot_16q_b64_sampled(encoding):
    """Fig. 8's batch-64 shape at 16 qubits, whole batch on the GPU, sampled
    rows against the oracle."""
    n, B = 16, 64
    layers = W.circuit_rz_ry_cnot(n, 8, encoding)
    w, x = W.draw_params(n, layers, B, "normal", 6)
    _sampled_full(f"fig6 {encoding}", [0, 63], spec=(n, B, "c64", layers, w, x))


# ------------------------------------------------------- captured graphs --

@pytest.mark.parametrize("name", ["c4a_16q_b128_ionq", "c4b_16q_b128_ibm", "c3_20q_b32"])
def test_step_graph_replays_equal_eager(name):
    """Forward, <Z_i> and adjoint captured as one HIP graph (the timed mode of
    the benchmark): replays alternate with eager steps and program work, each
    replay equals the eager step bit for bit, and sampled rows match the oracle."""
    n, B, dt, layers, w, x = W.config(name)
    B = 8
    w, x = W.draw_params(n, layers, B, W.CONFIGS[name]["wdist"], W.CONFIGS[name]["seed"])
    g = W.upstream(B, n, "normal", 3)
    note(f"case graph {name} B={B}")
    dev = torch.device("cuda")
    c = _circuit(n, layers, dt)
    wt, xt, gt = (torch.tensor(v, device=dev) for v in (w, x, g))
    st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
    ws = c.workspace(B, True, dev)

    def step():
        c.forward(wt, xt, state=st, ws=ws)
        e = c.expval_z(st, ws=ws)
        gw, gx = c.adjoint_grad(wt, xt, st, gt, ws=ws)
        return e, gw, gx

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in outs]
        _ = torch.randn(1000, device=dev).sum().item()   # program work between replays
        ref = step()
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), (name, r)
    rows = [0, B - 1] if n < 20 else [B - 1]
    o = oracle_run(n, layers, w, x[rows], g[rows])
    np.testing.assert_allclose(got[0].cpu().numpy()[rows], o["e"], atol=2e-5)
    gx = got[2].cpu().numpy()[rows]
    assert np.max(np.abs(gx - o["gx"])) / np.max(np.abs(o["gx"])) <= 1e-4


@pytest.mark.parametrize("n,B,with_grad,backward", [(4, 1, True, "adjoint"), (6, 3, False, "adjoint"),
                                                    (14, 1, True, "adjoint"), (16, 5, True, "adjoint"),
                                                    (16, 5, True, "stored")])
def test_step_graph_helper(n, B, with_grad, backward):
    """tqsim.StepGraph: replays alternate with eager steps and program work;
    each replay equals the eager step bit for bit, also after the weights and
    features are changed in place between replays; one replay is checked
    against the oracle.  The stored-state backward reads the pass outputs the
    captured forward kept in the graph's own workspace."""
    layers = W.circuit_rz_ry_cnot(n, 3, "qdi")
    w, x = W.draw_params(n, layers, B, "normal", 7)
    g = W.upstream(B, n, "normal", 7)
    note(f"case step graph n={n} B={B} grad={with_grad} backward={backward}")
    dev = torch.device("cuda")
    c = T.Circuit(n, layers, "c64", backward=backward)
    wt, xt, gt = (torch.tensor(v, device=dev) for v in (w, x, g))
    sg = T.StepGraph(c, wt, xt, gt if with_grad else None)
    st = torch.empty((B, 2 ** n), dtype=c.complex_dtype, device=dev)
    ws = c.new_workspace(B, True, dev)
    for r in range(4):
        if r == 2:
            wt.mul_(0.5).add_(0.25)
            xt.mul_(-1.0)
        out = sg.replay()
        torch.cuda.synchronize()
        got = [None if t is None else t.clone() for t in out]
        _ = torch.randn(1000, device=dev).sum().item()   # program work between replays
        c.forward(wt, xt, state=st, ws=ws)
        ref = [c.expval_z(st, ws=ws)]
        ref += list(c.adjoint_grad(wt, xt, st, gt, ws=ws)) if with_grad else [None, None]
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert (a is None) == (b is None)
            if a is not None:
                assert torch.equal(a, b), (n, B, r)
    o = oracle_run(n, layers, wt.cpu().numpy(), xt.cpu().numpy(), g)
    np.testing.assert_allclose(got[0].cpu().numpy(), o["e"], atol=2e-5)
    if with_grad:
        gw = got[1].cpu().numpy()
        assert np.max(np.abs(gw - o["gw"])) <= 1e-4 * max(np.max(np.abs(o["gw"])), 1e-30)


# ------------------------------------------- stored-state backpropagation --

@pytest.mark.parametrize("name,builder,dist", [
    ("rot_ring_zz", lambda n: W.circuit_rot_ring(n, 3, "RX", ("RX", "RY", "RZ"), zz=True), "normal"),
    ("ionq_qdi", lambda n: W.circuit_ionq(n, 4, "qdi"), "uniform2pi"),
    ("ibm", lambda n: W.circuit_ibm(n, 4), "uniform2pi"),
    ("fig6_qdi", lambda n: W.circuit_rz_ry_cnot(n, 4, "qdi"), "normal"),
])
@pytest.mark.parametrize("n,dtype,mode,B", [
    (2, "c64", "auto", 5), (4, "c128", "dense", 3), (6, "c64", "per_layer", 17), (8, "c128", "fused", 2),
    (12, "c64", "per_layer", 3), (14, "c64", "fused", 3), (16, "c128", "fused", 2), (18, "c64", "fused", 2),
])
def test_stored_state_backward(name, builder, dist, n, dtype, mode, B):
    """The stored-state backward (the backpropagation of the paper's training:
    forward pass outputs kept, psi read back instead of uncomputed) against
    the oracle, in every dispatch mode."""
    layers = builder(n)
    w, x, g = _params(n, layers, B, seed=60 + n, dist=dist)
    note(f"case stored {name} n={n} {dtype} mode={mode} B={B}")
    c = T.Circuit(n, layers, dtype, mode=mode, backward="stored")
    got = gpu_run(c, w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, dtype, label=f"stored {name} n={n} {mode}")


def test_stored_state_full_c3_rows():
    """The 20-qubit workload (32 samples) with the stored-state backward: four
    rows against the oracle, and the remaining rows' feature gradients zero."""
    n, B, dt, layers, w, x = W.config("c3_20q_b32")
    rows = [0, 31]
    g = np.zeros((B, n))
    g[rows] = W.upstream(len(rows), n, "normal", 8)
    note("case stored full c3")
    c = T.Circuit(n, layers, dt, backward="stored")
    got = gpu_run(c, w, x, g)
    ref = oracle_run(n, layers, w, x[rows], g[rows])
    np.testing.assert_allclose(got["e"][rows], ref["e"], atol=2e-5)
    e1 = np.max(np.abs(got["gw"] - ref["gw"])) / np.max(np.abs(ref["gw"]))
    e2 = np.max(np.abs(got["gx"][rows] - ref["gx"])) / np.max(np.abs(ref["gx"]))
    assert e1 <= 1e-4 and e2 <= 1e-4, (e1, e2)


def test_auto_backward_follows_the_cap():
    """backward="auto": stored states while they fit the cap (per batch size),
    the adjoint beyond; both give the oracle's gradients.  (The state-set
    threshold is set to zero here so that the cap alone decides.)"""
    n = 12
    layers = W.circuit_rot_ring(n, 3, "RY", ("RY", "RZ"))
    state = (8 << n)
    c = T.Circuit(n, layers, "c64", tile_bits=10, backward="auto", stored_cap=8 * state, stored_min=0)
    adj = T.Circuit(n, layers, "c64", tile_bits=10)
    passes = len([p for p in c.plan()["passes"] if not p["bwd_only"]])
    assert passes >= 2
    for B in (1, 64):
        stored = (passes - 1) * B * state <= 8 * state
        extra = c.workspace_size(B, True) - adj.workspace_size(B, True)
        assert (extra >= (passes - 1) * B * state) == stored, (B, extra)
        w, x, g = _params(n, layers, B, seed=B)
        note(f"case auto backward B={B} stored={stored}")
        got = gpu_run(c, w, x, g)
        compare(got, oracle_run(n, layers, w, x, g), "c64", label=f"auto B={B}")


# --------------------------------- remaining gates and layer techniques --

ROT_MS_CIRCUITS = [
    ("rot", lambda n: [W.L("ROT", "ALL", "INPUT", offset=0), W.L("CNOT", "RING"), W.L("ROT", "ALL", "WEIGHT"),
                       W.L("CZ", "CHAIN"), W.L("ROT", "WIRE", "WEIGHT", wire=n - 1, offset=3 * n),
                       W.L("ROT", "ALL", "FIXED", fixed=0.4, fixed2=-1.1, fixed3=0.7), W.L("RX", "ALL", "WEIGHT",
                                                                                   offset=3 * n + 3)], "normal"),
    ("ms_phases", lambda n: [W.L("RY", "ALL", "INPUT"), W.L("GPI2", "ALL", "WEIGHT"),
                             W.L("MS", "PAIRS_EVEN", "WEIGHT", offset=n, fixed2=0.13, fixed3=-0.41),
                             W.L("GPI", "ALL", "WEIGHT", offset=n + n // 2),
                             W.L("MS", "PAIRS_ODD", "INPUT", offset=n, fixed2=0.3, fixed3=0.05),
                             W.L("MS", "PAIRS_EVEN", "FIXED", fixed=0.2, fixed2=-0.25, fixed3=0.6),
                             W.L("RX", "ALL", "WEIGHT", offset=2 * n + n // 2)], "uniform2pi"),
]


@pytest.mark.parametrize("case", ROT_MS_CIRCUITS, ids=[c[0] for c in ROT_MS_CIRCUITS])
@pytest.mark.parametrize("n,dtype,mode,B", [
    (2, "c128", "auto", 3), (4, "c64", "dense", 5), (6, "c128", "per_layer", 3), (8, "c64", "fused", 17),
    (12, "c64", "per_layer", 2), (14, "c64", "fused", 3), (14, "c128", "per_layer", 2), (16, "c64", "fused", 2),
])
def test_rot_and_phased_ms(case, n, dtype, mode, B):
    """Appendix A's Rot(theta, phi, lambda) (three parameters per gate, from
    weights, features or fixed values) and MS(phi0, phi1, theta) with phases,
    against the oracle in every dispatch mode."""
    name, build, dist = case
    layers = build(n)
    w, x, g = _params(n, layers, B, seed=70 + n, dist=dist)
    note(f"case {name} n={n} {dtype} mode={mode} B={B}")
    got = gpu_run(_circuit(n, layers, dtype, mode), w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, dtype, label=f"{name} n={n} {mode}")


TECHNIQUE_CIRCUITS = [
    ("rx_ry_gpi2_rot", lambda n: [W.L("RY", "ALL", "INPUT"), W.L("RX", "ALL", "WEIGHT"), W.L("CNOT", "RING"),
                                  W.L("RY", "ALL", "WEIGHT", offset=n), W.L("GPI2", "ALL", "WEIGHT", offset=2 * n),
                                  W.L("CZ", "CHAIN"), W.L("ROT", "ALL", "WEIGHT", offset=3 * n),
                                  W.L("H", "ALL"), W.L("ZZ", "RING", "WEIGHT", offset=6 * n),
                                  W.L("RZ", "ALL", "INPUT", offset=n), W.L("H", "ALL"),
                                  W.L("GPI", "ALL", "WEIGHT", offset=7 * n), W.L("RX", "ALL", "WEIGHT", offset=8 * n)],
     "normal"),
    ("fig6_qdi", lambda n: W.circuit_rz_ry_cnot(n, 3, "qdi"), "normal"),
    ("rot_ring_zz", lambda n: W.circuit_rot_ring(n, 2, "RX", ("RX", "RY", "RZ"), zz=True), "normal"),
]


@pytest.mark.parametrize("case", TECHNIQUE_CIRCUITS, ids=[c[0] for c in TECHNIQUE_CIRCUITS])
@pytest.mark.parametrize("hrz,fhwt,diag", [(True, True, "tables"), (False, False, "tables"),
                                           (False, True, "einsum"), (True, True, "einsum")])
@pytest.mark.parametrize("n,dtype,mode,B", [
    (3, "c128", "per_layer", 3), (6, "c64", "dense", 5), (9, "c64", "per_layer", 3), (13, "c64", "per_layer", 2),
    (13, "c64", "fused", 2), (14, "c128", "per_layer", 1),
])
def test_layer_techniques(case, hrz, fhwt, diag, n, dtype, mode, B):
    """The layer techniques the dispatcher can select -- H-Rz expansion of
    rotation layers (Sec. 2.5), Hadamard layers by the fast Walsh-Hadamard
    transform (Sec. 2.5), diagonal layers by split eigenphase tables (Secs.
    2.4.1-2.4.2) or gate by gate (diagonal Einsum, Sec. 2.4.3) -- all give the
    oracle's states, readouts and gradients."""
    name, build, dist = case
    layers = build(n)
    w, x, g = _params(n, layers, B, seed=80 + n, dist=dist)
    note(f"case technique {name} hrz={hrz} fhwt={fhwt} diag={diag} n={n} {dtype} mode={mode} B={B}")
    c = T.Circuit(n, layers, dtype, mode=mode, hrz=hrz, fhwt=fhwt, diag=diag)
    got = gpu_run(c, w, x, g)
    ref = oracle_run(n, layers, w, x, g)
    compare(got, ref, dtype, label=f"technique {name} hrz={hrz} fhwt={fhwt} diag={diag} n={n} {mode}")


# -------------------------------------------------- out-of-bounds writes --

@pytest.mark.parametrize("n,B,dtype,backward", [(3, 5, "c64", "adjoint"), (7, 17, "c64", "stored"),
                                                (13, 3, "c128", "adjoint"), (14, 2, "c64", "stored")])
def test_buffers_untouched_outside_their_extent(n, B, dtype, backward):
    """State, workspace and output buffers sit inside larger allocations whose
    padding holds a canary pattern; after forward, <Z_i> and the adjoint at a
    ragged batch the padding is unchanged (no kernel writes past a buffer)."""
    layers = W.circuit_rot_ring(n, 2, "RX", ("RX", "RY", "RZ"), zz=True)
    w, x, g = _params(n, layers, B, seed=90 + n)
    note(f"case canary n={n} B={B} {dtype} {backward}")
    dev = torch.device("cuda")
    c = T.Circuit(n, layers, dtype, backward=backward)
    PAD = 4096

    def padded(nbytes):
        buf = torch.empty(nbytes + 2 * PAD, dtype=torch.uint8, device=dev)
        buf.fill_(0xA5)
        return buf

    def inner(buf, nbytes, dt, shape):
        return buf[PAD:PAD + nbytes].view(dt).view(shape)

    es = 8 if dtype == "c64" else 16
    st_b = padded(B * es << n)
    ws_n = c.workspace_size(B, True)
    ws_b = padded(ws_n)
    ez_b, gw_b, gx_b = padded(B * n * 8), padded(max(1, c.n_weights) * 8), padded(B * max(1, c.n_features) * 8)
    state = inner(st_b, B * es << n, c.complex_dtype, (B, 2 ** n))
    ws = ws_b[PAD:PAD + ws_n]
    wt, xt, gt = (torch.tensor(v, device=dev) for v in (w, x, g))
    c.forward(wt, xt, state=state, ws=ws)
    ez = inner(ez_b, B * n * 8, torch.float64, (B, n))
    L = T.lib()
    import ctypes
    T._check(L.tqs_expval_z(c.handle, B, ctypes.c_void_p(state.data_ptr()), ctypes.c_void_p(ez.data_ptr()), None,
                            ctypes.c_void_p(ws.data_ptr()), ws_n, T._stream(None)))
    gw = inner(gw_b, max(1, c.n_weights) * 8, torch.float64, (-1,))
    gx = inner(gx_b, B * max(1, c.n_features) * 8, torch.float64, (B, -1))
    T._check(L.tqs_adjoint_grad(c.handle, B, ctypes.c_void_p(wt.data_ptr()), ctypes.c_void_p(xt.data_ptr()),
                                ctypes.c_void_p(state.data_ptr()), ctypes.c_void_p(gt.data_ptr()),
                                ctypes.c_void_p(gw.data_ptr()), ctypes.c_void_p(gx.data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), ws_n, T._stream(None)))
    torch.cuda.synchronize()
    for name, buf, nb in (("state", st_b, B * es << n), ("workspace", ws_b, ws_n), ("expz", ez_b, B * n * 8),
                          ("grad_w", gw_b, max(1, c.n_weights) * 8), ("grad_x", gx_b, B * max(1, c.n_features) * 8)):
        head, tail = buf[:PAD].cpu().numpy(), buf[PAD + nb:].cpu().numpy()
        assert (head == 0xA5).all() and (tail == 0xA5).all(), name
    ref = oracle_run(n, layers, w, x, g)
    compare(dict(e=ez.cpu().numpy(), gw=gw.cpu().numpy()[: c.n_weights], gx=gx.cpu().numpy()[:, : c.n_features]),
            ref, dtype, what=("e", "gw", "gx"), label=f"canary n={n}")


def test_prepared_cold_circuit_captures_into_a_graph():
    """A circuit never run before, prepared with tqs_circuit_prepare, can have
    its first forward / readout / adjoint calls captured into a HIP graph;
    replays equal an eager step of an identical circuit bit for bit."""
    n, B = 10, 6
    layers = W.circuit_ibm(n, 3)
    w, x, g = _params(n, layers, B, seed=5, dist="uniform2pi")
    dev = torch.device("cuda")
    wt, xt, gt = (torch.tensor(v, device=dev) for v in (w, x, g))
    note("case prepared capture")
    cold = _circuit(n, layers, "c64").prepare()
    st = torch.empty((B, 2 ** n), dtype=cold.complex_dtype, device=dev)
    ws = cold.workspace(B, True, dev)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=side):
        cold.forward(wt, xt, state=st, ws=ws)
        e = cold.expval_z(st, ws=ws)
        gw, gx = cold.adjoint_grad(wt, xt, st, gt, ws=ws)
    warm = _circuit(n, layers, "c64")
    ref = gpu_run(warm, w, x, g)
    for _ in range(2):
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(e.cpu().numpy(), ref["e"])
        np.testing.assert_array_equal(gw.cpu().numpy(), ref["gw"])
        np.testing.assert_array_equal(gx.cpu().numpy(), ref["gx"])
