"""Python binding of libtqsim (argument marshalling only).

Every step of the simulation runs in the HIP library; this module converts
layer lists to the C struct, hands torch device pointers and the current HIP
stream to the C ABI and turns status codes into exceptions.  The library must
have been built (``paper_2506_04891_amd._build.build()``); without it the
import fails loudly -- there is no other execution path.
"""
from __future__ import annotations

import atexit
import ctypes
import threading
import json
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtqsim.so")

GATES = {"RX": 0, "RY": 1, "RZ": 2, "H": 3, "X": 4, "Z": 5, "S": 6, "SX": 7, "GPI": 8, "GPI2": 9,
         "CNOT": 10, "CZ": 11, "SWAP": 12, "ZZ": 13, "MS": 14, "ECR": 15, "ROT": 16}
PATTERNS = {"ALL": 0, "WIRE": 1, "RING": 2, "CHAIN": 3, "PAIRS_EVEN": 4, "PAIRS_ODD": 5}
SOURCES = {"FIXED": 0, "WEIGHT": 1, "INPUT": 2}
DTYPES = {"c64": 0, "c128": 1}
MODES = {"auto": 0, "per_layer": 1, "fused": 2, "dense": 3}
BACKWARDS = {"adjoint": 0, "stored": 1, "auto": 2}
STATUS = {0: "TQS_OK", 1: "TQS_EINVAL", 2: "TQS_ENOMEM", 3: "TQS_EDEVICE", 4: "TQS_EUNSUPPORTED"}


class TqsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class tqs_layer(ctypes.Structure):
    _fields_ = [("gate", ctypes.c_int32), ("pattern", ctypes.c_int32), ("source", ctypes.c_int32),
                ("wire", ctypes.c_int32), ("wire2", ctypes.c_int32), ("offset", ctypes.c_int32),
                ("fixed_param", ctypes.c_double), ("fixed_param2", ctypes.c_double),
                ("fixed_param3", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_04891_amd._build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.tqs_circuit_create.argtypes = [i32, ctypes.POINTER(tqs_layer), i32, i32, ctypes.POINTER(vp)]
    L.tqs_circuit_destroy.argtypes = [vp]
    L.tqs_circuit_prepare.argtypes = [vp]
    L.tqs_circuit_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.tqs_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
    L.tqs_forward.argtypes = [vp, i32, vp, vp, vp, vp, sz, vp]
    L.tqs_expval_z.argtypes = [vp, i32, vp, vp, vp, vp, sz, vp]
    L.tqs_expval_z_noalloc.argtypes = [vp, i32, vp, vp, vp, vp]
    L.tqs_adjoint_grad.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.tqs_set_option.argtypes = [vp, ctypes.c_char_p, i64]
    L.tqs_segment_sum_rows.argtypes = [vp, i32, i32, i32, i32, vp, i32, vp, vp]
    L.tqs_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
    L.tqs_profile_report.argtypes = [vp, i32, ctypes.c_char_p, sz]
    L.tqs_status_string.argtypes = [i32]
    L.tqs_status_string.restype = ctypes.c_char_p
    L.tqs_last_error.restype = ctypes.c_char_p
    for f in ("tqs_circuit_create", "tqs_circuit_destroy", "tqs_circuit_prepare", "tqs_circuit_info",
              "tqs_workspace_size", "tqs_forward", "tqs_expval_z", "tqs_expval_z_noalloc", "tqs_adjoint_grad",
              "tqs_set_option", "tqs_plan_describe", "tqs_segment_sum_rows", "tqs_profile_report"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise TqsError(st, lib().tqs_last_error().decode())


def _enum(table, v):
    return table[v] if isinstance(v, str) else int(v)


def to_c_layers(layers):
    arr = (tqs_layer * max(1, len(layers)))()
    for i, ly in enumerate(layers):
        arr[i].gate = _enum(GATES, ly.gate)
        arr[i].pattern = _enum(PATTERNS, ly.pattern)
        arr[i].source = _enum(SOURCES, ly.source)
        arr[i].wire = int(ly.wire)
        arr[i].wire2 = int(ly.wire2)
        arr[i].offset = int(ly.offset)
        arr[i].fixed_param = float(ly.fixed)
        arr[i].fixed_param2 = float(getattr(ly, "fixed2", 0.0))
        arr[i].fixed_param3 = float(getattr(ly, "fixed3", 0.0))
    return arr


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# Circuits dropped by Python are destroyed later, at a safe point: destroying one
# frees device memory, which would invalidate a HIP graph capture that happens
# to be running when the garbage collector finalises the circuit.
_released = []
_released_lock = threading.Lock()


def release_pending():
    """Destroy the circuits dropped since the last call.  Called when a circuit
    is created and before the serving executor captures a graph; call it at any
    other point where no graph capture is in progress."""
    with _released_lock:
        hs = list(_released)
        _released.clear()
    for h in hs:
        if _lib is not None:
            _lib.tqs_circuit_destroy(h)


atexit.register(release_pending)


class Circuit:
    """A compiled circuit: ``Circuit(n, layers, dtype="c64")``.

    ``layers`` is a list of objects with fields gate, pattern, source, wire,
    wire2, offset, fixed (e.g. ``workloads.Layer``); enum fields may be names
    or integers.  ``mode`` and ``tile_bits`` override the dispatcher; ``hrz``
    (H-Rz expansion of rotation layers), ``fhwt`` (Hadamard layers by the fast
    Walsh-Hadamard transform) and ``diag`` ("tables": split eigenphase tables,
    "einsum": one diagonal factor per gate) choose layer techniques.
    ``backward``: "adjoint" (uncompute psi with the inverse layers; two state
    sets of memory at any depth), "stored" (every forward pass keeps its
    output in the workspace and the backward reads psi from there; the
    adjoint_grad call must get the workspace of the forward call, untouched
    in between), or "auto" (stored when the adjoint's state set outgrows the
    last-level cache, ``stored_min`` bytes, and the stored states fit
    ``stored_cap`` bytes)."""

    def __init__(self, n, layers, dtype="c64", mode="auto", tile_bits=0, backward="adjoint", stored_cap=None,
                 hrz=False, fhwt=True, diag="tables", stored_min=None):
        L = lib()
        release_pending()
        self.n = int(n)
        self.dtype = dtype
        self.layers = list(layers)
        arr = to_c_layers(self.layers)
        h = ctypes.c_void_p()
        _check(L.tqs_circuit_create(self.n, arr, len(self.layers), DTYPES[dtype], ctypes.byref(h)))
        self._h = h
        if mode != "auto":
            _check(L.tqs_set_option(h, b"mode", _enum(MODES, mode)))
        if tile_bits:
            _check(L.tqs_set_option(h, b"tile_bits", int(tile_bits)))
        if hrz:
            _check(L.tqs_set_option(h, b"hrz", 1))
        if not fhwt:
            _check(L.tqs_set_option(h, b"fhwt", 0))
        if diag != "tables":
            _check(L.tqs_set_option(h, b"diag", {"einsum": 1}[diag]))
        self.backward = backward
        if backward != "adjoint":
            _check(L.tqs_set_option(h, b"backward", _enum(BACKWARDS, backward)))
        if stored_cap is not None:
            _check(L.tqs_set_option(h, b"stored_cap", int(stored_cap)))
        if stored_min is not None:
            _check(L.tqs_set_option(h, b"stored_min", int(stored_min)))
        nw, nf, sb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(L.tqs_circuit_info(h, ctypes.byref(nw), ctypes.byref(nf), ctypes.byref(sb)))
        self.n_weights, self.n_features, self.state_bytes = nw.value, nf.value, sb.value
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        lock = _released_lock
        if h is not None and lock is not None:   # None at interpreter shutdown
            with lock:
                _released.append(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def complex_dtype(self):
        return torch.complex64 if self.dtype == "c64" else torch.complex128

    def prepare(self):
        """Upload the plan now (before capturing calls into a HIP graph)."""
        _check(lib().tqs_circuit_prepare(self._h))
        return self

    def plan(self):
        buf = ctypes.create_string_buffer(1 << 20)
        _check(lib().tqs_plan_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def set_profile(self, on=True):
        _check(lib().tqs_set_option(self._h, b"profile", int(bool(on))))

    def profile_report(self, reset=True):
        """Per kernel kind: {count, ms, bytes, flops} of the launches timed so far."""
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().tqs_profile_report(self._h, int(bool(reset)), buf, len(buf)))
        return json.loads(buf.value.decode())

    def workspace_size(self, batch, with_grad=True):
        sz = ctypes.c_size_t()
        _check(lib().tqs_workspace_size(self._h, int(batch), int(bool(with_grad)), ctypes.byref(sz)))
        return sz.value

    def new_workspace(self, batch, with_grad=True, device=None):
        """A fresh (uncached) device workspace for ``batch`` samples."""
        device = torch.device(device or "cuda")
        return torch.empty(max(1, self.workspace_size(batch, with_grad)), dtype=torch.uint8, device=device)

    def workspace(self, batch, with_grad=True, device=None):
        """A cached device workspace (uint8 tensor) for ``batch`` samples."""
        device = torch.device(device or "cuda")
        key = (int(batch), bool(with_grad), str(device))
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(max(1, self.workspace_size(batch, with_grad)), dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws

    def _params(self, weights, features, batch, device):
        if weights is None or weights.numel() == 0:
            weights = torch.zeros(max(1, self.n_weights), dtype=torch.float64, device=device)
        if features is None or features.numel() == 0:
            features = torch.zeros((batch, max(1, self.n_features)), dtype=torch.float64, device=device)
        for t, name in ((weights, "weights"), (features, "features")):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        if weights.numel() < self.n_weights:
            raise ValueError("too few weights")
        if features.dim() != 2 or features.shape[0] != batch or features.shape[1] < self.n_features:
            raise ValueError("features must be [batch, n_features]")
        if features.shape[1] != self.n_features and self.n_features > 0:
            raise ValueError("features must have exactly n_features columns")
        return weights, features

    def forward(self, weights, features, batch=None, state=None, ws=None, stream=None):
        """Final states [batch, 2^n] (complex tensor on the device)."""
        if batch is None:
            batch = features.shape[0]
        device = (features if features is not None else weights).device
        weights, features = self._params(weights, features, batch, device)
        if state is None:
            state = torch.empty((batch, 2 ** self.n), dtype=self.complex_dtype, device=device)
        if ws is None:
            ws = self.workspace(batch, True, device)
        _check(lib().tqs_forward(self._h, batch, _ptr(weights), _ptr(features), _ptr(state), _ptr(ws),
                                 ws.numel(), _stream(stream)))
        return state

    def expval_z(self, state, ws=None, stream=None, with_norm=False):
        batch = state.shape[0]
        if ws is None:
            ws = self.workspace(batch, True, state.device)
        expz = torch.empty((batch, self.n), dtype=torch.float64, device=state.device)
        norm = torch.empty(batch, dtype=torch.float64, device=state.device) if with_norm else None
        _check(lib().tqs_expval_z(self._h, batch, _ptr(state), _ptr(expz), _ptr(norm), _ptr(ws),
                                  ws.numel(), _stream(stream)))
        return (expz, norm) if with_norm else expz

    def expval_z_noalloc(self, state, stream=None, with_norm=False):
        """expval_z through the entry point that takes no workspace (the library's
        static scratch).  The output tensors are the caller's allocations."""
        batch = state.shape[0]
        expz = torch.empty((batch, self.n), dtype=torch.float64, device=state.device)
        norm = torch.empty(batch, dtype=torch.float64, device=state.device) if with_norm else None
        _check(lib().tqs_expval_z_noalloc(self._h, batch, _ptr(state), _ptr(expz), _ptr(norm), _stream(stream)))
        return (expz, norm) if with_norm else expz

    def adjoint_grad(self, weights, features, state, grad_expz, ws=None, stream=None, want_features=True):
        """(grad_weights [n_weights], grad_features [batch, n_features]); clobbers ``state``."""
        batch = state.shape[0]
        weights, features = self._params(weights, features, batch, state.device)
        if ws is None:
            ws = self.workspace(batch, True, state.device)
        g = grad_expz.to(torch.float64).contiguous()
        gw = torch.empty(max(1, self.n_weights), dtype=torch.float64, device=state.device)
        gx = torch.empty((batch, max(1, self.n_features)), dtype=torch.float64, device=state.device)
        _check(lib().tqs_adjoint_grad(self._h, batch, _ptr(weights), _ptr(features), _ptr(state), _ptr(g),
                                      _ptr(gw), _ptr(gx) if want_features else None, _ptr(ws), ws.numel(),
                                      _stream(stream)))
        return gw[: self.n_weights], gx[:, : self.n_features]


class StepGraph:
    """One step of a circuit on fixed device tensors -- forward, <Z_i> and, when
    ``grad_expz`` is given, the adjoint gradient -- captured once as a HIP
    graph.  ``replay()`` reruns the step: it reads the current contents of
    ``weights``, ``features`` and ``grad_expz`` (update them in place between
    replays) and refreshes ``expz``, ``grad_weights`` and ``grad_features``.
    Small calls (few qubits, batch 1) are bound by the host's per-launch cost,
    which a replay does not pay.  The graph holds its own state and
    workspace; the circuit must outlive it."""

    def __init__(self, circ, weights, features, grad_expz=None):
        batch = features.shape[0]
        dev = features.device
        self.circ = circ.prepare()
        self.weights, self.features, self.grad_expz = weights, features, grad_expz
        self.state = torch.empty((batch, 2 ** circ.n), dtype=circ.complex_dtype, device=dev)
        self.ws = circ.new_workspace(batch, True, dev)
        self.grad_weights = self.grad_features = None
        release_pending()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step()

    def _step(self):
        c = self.circ
        c.forward(self.weights, self.features, state=self.state, ws=self.ws)
        self.expz = c.expval_z(self.state, ws=self.ws)
        if self.grad_expz is not None:
            self.grad_weights, self.grad_features = c.adjoint_grad(self.weights, self.features, self.state,
                                                                   self.grad_expz, ws=self.ws)

    def replay(self):
        """Run the captured step on the current stream; returns (expz,
        grad_weights, grad_features), the graph's own output tensors."""
        self.graph.replay()
        return self.expz, self.grad_weights, self.grad_features


class QCircuitFn(torch.autograd.Function):
    """<Z_i> of a circuit, differentiable in weights and features by the adjoint
    method.  Only the final state is kept for backward (no intermediate
    states); the adjoint sweep uncomputes it, so a second backward through the
    same graph (retain_graph, gradcheck) recomputes the forward state first."""

    @staticmethod
    def forward(ctx, circ, weights, features):
        # a stored-state backward reads the forward's workspace: each forward
        # keeps its own until its backward has run
        ws = circ.new_workspace(features.shape[0], True, features.device) if circ.backward != "adjoint" else None
        state = circ.forward(weights, features, ws=ws)
        expz = circ.expval_z(state, ws=ws)
        ctx.circ = circ
        ctx.save_for_backward(weights, features)
        ctx.state = state
        ctx.ws = ws
        return expz

    @staticmethod
    def backward(ctx, g):
        weights, features = ctx.saved_tensors
        ws = ctx.ws
        if ctx.state is not None:
            state = ctx.state
        else:
            state = ctx.circ.forward(weights, features, ws=ws)
        ctx.state = None
        want_x = ctx.needs_input_grad[2]
        gw, gx = ctx.circ.adjoint_grad(weights, features, state, g.contiguous(), ws=ws, want_features=want_x)
        gw = gw.to(weights.dtype) if ctx.needs_input_grad[1] else None
        gx = gx.to(features.dtype) if want_x else None
        return None, gw, gx


def segment_sum_rows(x, col_begin, n_cols, seg, out=None, stream=None):
    """out[s] = x[seg[s]:seg[s+1], col_begin:col_begin+n_cols].sum(0) on the device
    (FP64, rows in order).  x: [rows, ld] float64; seg: int32 [n_seg + 1]."""
    if x.dtype != torch.float64 or x.dim() != 2 or not x.is_contiguous():
        raise ValueError("x must be a contiguous [rows, ld] float64 tensor")
    if seg.dtype != torch.int32 or seg.dim() != 1 or not seg.is_contiguous():
        raise ValueError("seg must be a contiguous int32 vector")
    n_seg = seg.numel() - 1
    if out is None:
        out = torch.empty((max(0, n_seg), n_cols), dtype=torch.float64, device=x.device)
    _check(lib().tqs_segment_sum_rows(_ptr(x), x.shape[0], x.shape[1], int(col_begin), int(n_cols), _ptr(seg),
                                      n_seg, _ptr(out), _stream(stream)))
    return out


def expval(circ, weights, features):
    return QCircuitFn.apply(circ, weights, features)
