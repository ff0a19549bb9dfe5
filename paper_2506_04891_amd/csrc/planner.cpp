// Host-side circuit compiler of libtqsim.
//
// 1. Validation and gate expansion of the layer list (placement patterns of
//    tqsim.h).
// 2. Embedding: for every wire the 1-qubit gates that act before any 2-qubit
//    gate touches it are multiplied into one 2x2 matrix per wire; the state
//    after them is a product state, written analytically by the first pass.
// 3. IR: the remaining gates become ops.  Two dispatcher modes:
//    - per-layer: each layer is applied with its own technique, as in the
//      paper's layer study (Sec. 2): Kronecker layers as 2x2 ops per wire
//      (Einsum / unitary-real structure, Sec. 2.2), diagonal layers as one
//      split-table phase multiply (diagonal tensor product, Sec. 2.4.2),
//      permutation layers as one GF(2) index map (Sec. 2.3), GPI as phase then
//      index reversal (Sec. 2.4.1), MS / ECR as 4x4 pair ops;
//    - fused: consecutive 1-qubit gates on a wire are multiplied into one 2x2;
//      CNOT chains stay index maps; a ring's closing CNOT (which maps the
//      least to the most significant bit) becomes an in-tile 4x4 permutation
//      so that the chain map keeps low tiles contiguous.
// 4. Scheduling: ops are placed greedily into passes, each pass choosing the
//    tile bit set that lets it apply the most ops while respecting the order
//    of non-commuting ops; inside a pass ops are list-scheduled into stages of
//    RB register bits.
// 5. Device tables, parameter-preparation items and gradient bookkeeping.
#include "planner.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <sstream>

namespace tqs {

// Dense (full layer unitary) dispatch: allowed up to this many qubits; chosen
// automatically up to DENSE_AUTO_MAX_QUBITS.
constexpr int DENSE_MAX_QUBITS = 6;
constexpr int DENSE_AUTO_MAX_QUBITS = 0;

// gate ids (tqs_gate)
// gates a layer may name (tqs_gate), then factors the planner makes of them:
// GPI_DIAG diag(e^{2 pi i p}, e^{-2 pi i p}); PHASE diag(1, e^{ip}); RZT = RZ(2 pi p);
// RZNT = RZ(-2 pi p)
enum { RX = 0, RY, RZ, H, X, Z, S, SX, GPI, GPI2, CNOT, CZ, SWAP, ZZ, MS, ECR, ROT,
       GPI_DIAG = 100, PHASE = 101, RZT = 102, RZNT = 103 };
enum { PAT_ALL = 0, PAT_WIRE, PAT_RING, PAT_CHAIN, PAT_PEVEN, PAT_PODD };
enum { SRC_FIXED = 0, SRC_WEIGHT, SRC_INPUT };

static bool is_1q(int g) { return (g >= RX && g <= GPI2) || g == ROT || g == PHASE || g == RZT || g == RZNT; }
static bool is_param(int g) {
  return g == RX || g == RY || g == RZ || g == GPI || g == GPI2 || g == ZZ || g == MS || g == ROT || g == GPI_DIAG ||
         g == PHASE || g == RZT || g == RZNT;
}
static bool is_diag1(int g) { return g == RZ || g == Z || g == S || g == GPI_DIAG || g == PHASE || g == RZT || g == RZNT; }
static int gate_params(int g) { return g == ROT ? 3 : (is_param(g) ? 1 : 0); }
static bool is_diag2(int g) { return g == ZZ || g == CZ; }
static bool is_real_gate(int g) { return g == RY || g == H || g == X || g == Z || g == CNOT || g == SWAP || g == CZ; }
static int popc(uint32_t x) { return __builtin_popcount(x); }

// ---------------------------------------------------------------- GF(2) --
GF2 GF2::identity(int n) {
  GF2 g;
  g.n = n;
  for (int i = 0; i < n; ++i) g.cols[i] = 1u << i;
  return g;
}
uint32_t GF2::apply(uint32_t x) const {
  uint32_t y = c;
  for (int i = 0; i < n; ++i)
    if ((x >> i) & 1) y ^= cols[i];
  return y;
}
GF2 GF2::after(const GF2 &f) const {
  GF2 r;
  r.n = n;
  for (int i = 0; i < n; ++i) r.cols[i] = apply(f.cols[i]) ^ c;
  r.c = apply(f.c);
  return r;
}
GF2 GF2::inverse() const {
  // Gauss-Jordan on [A | I] with A's columns as bit vectors: work on rows.
  uint32_t rows[NQMAX], inv[NQMAX];
  for (int r = 0; r < n; ++r) {
    rows[r] = 0;
    for (int i = 0; i < n; ++i)
      if ((cols[i] >> r) & 1) rows[r] |= 1u << i;
    inv[r] = 1u << r;
  }
  for (int col = 0; col < n; ++col) {
    int piv = -1;
    for (int r = col; r < n; ++r)
      if ((rows[r] >> col) & 1) {
        piv = r;
        break;
      }
    if (piv < 0) return GF2::identity(n);  // singular: cannot happen for permutations
    std::swap(rows[col], rows[piv]);
    std::swap(inv[col], inv[piv]);
    for (int r = 0; r < n; ++r)
      if (r != col && ((rows[r] >> col) & 1)) {
        rows[r] ^= rows[col];
        inv[r] ^= inv[col];
      }
  }
  GF2 g;
  g.n = n;
  for (int i = 0; i < n; ++i) {
    g.cols[i] = 0;
    for (int r = 0; r < n; ++r)
      if ((inv[r] >> i) & 1) g.cols[i] |= 1u << r;
  }
  // x = A^-1 (y ^ c)
  uint32_t ci = 0;
  for (int i = 0; i < n; ++i)
    if ((c >> i) & 1) ci ^= g.cols[i];
  g.c = ci;
  return g;
}
bool GF2::is_identity() const {
  if (c) return false;
  for (int i = 0; i < n; ++i)
    if (cols[i] != (1u << i)) return false;
  return true;
}

// ----------------------------------------------------------- validation --
struct Inst {
  int gate, w0, w1, src, pidx, layer;
  double fixed;
};

static std::vector<std::pair<int, int>> pattern_pairs(int n, const LayerSpec &L) {
  std::vector<std::pair<int, int>> v;
  switch (L.pattern) {
    case PAT_WIRE: v.push_back({L.wire, L.wire2}); break;
    case PAT_RING:
      if (n == 2) v.push_back({0, 1});
      else if (n > 2)
        for (int i = 0; i < n; ++i) v.push_back({i, (i + 1) % n});
      break;
    case PAT_CHAIN:
      for (int i = 0; i + 1 < n; ++i) v.push_back({i, i + 1});
      break;
    case PAT_PEVEN:
      for (int i = 0; i < n / 2; ++i) v.push_back({2 * i, 2 * i + 1});
      break;
    case PAT_PODD:
      for (int i = 0; i < n / 2; ++i) v.push_back({2 * i + 1, (2 * i + 2) % n});
      break;
  }
  return v;
}

std::string validate_layers(int n, const LayerSpec *layers, int n_layers, int *nw, int *nf) {
  char buf[256];
  if (n < 1 || n > NQMAX) {
    snprintf(buf, sizeof buf, "EINVAL: n_qubits=%d outside [1, %d]", n, NQMAX);
    return buf;
  }
  if (n_layers < 0 || (n_layers > 0 && !layers)) return "EINVAL: bad layer array";
  int w = 0, f = 0;
  for (int li = 0; li < n_layers; ++li) {
    const LayerSpec &L = layers[li];
    if (L.gate < RX || L.gate > ROT) {
      snprintf(buf, sizeof buf, "EINVAL: layer %d: unknown gate %d", li, L.gate);
      return buf;
    }
    if (L.pattern < PAT_ALL || L.pattern > PAT_PODD) {
      snprintf(buf, sizeof buf, "EINVAL: layer %d: unknown pattern %d", li, L.pattern);
      return buf;
    }
    if (L.source < SRC_FIXED || L.source > SRC_INPUT) {
      snprintf(buf, sizeof buf, "EINVAL: layer %d: unknown source %d", li, L.source);
      return buf;
    }
    int count = 0;
    if (is_1q(L.gate)) {
      if (L.pattern == PAT_ALL) count = n;
      else if (L.pattern == PAT_WIRE) {
        if (L.wire < 0 || L.wire >= n) {
          snprintf(buf, sizeof buf, "EINVAL: layer %d: wire %d out of range", li, L.wire);
          return buf;
        }
        count = 1;
      } else {
        snprintf(buf, sizeof buf, "EINVAL: layer %d: pattern %d invalid for a 1-qubit gate", li, L.pattern);
        return buf;
      }
    } else {
      if (L.pattern == PAT_ALL) {
        snprintf(buf, sizeof buf, "EINVAL: layer %d: pattern ALL invalid for a 2-qubit gate", li);
        return buf;
      }
      if (L.pattern == PAT_WIRE) {
        if (L.wire < 0 || L.wire >= n || L.wire2 < 0 || L.wire2 >= n || L.wire == L.wire2) {
          snprintf(buf, sizeof buf, "EINVAL: layer %d: wires (%d, %d) invalid", li, L.wire, L.wire2);
          return buf;
        }
      }
      if ((L.pattern == PAT_PEVEN || L.pattern == PAT_PODD) && (n % 2 != 0)) {
        snprintf(buf, sizeof buf, "EINVAL: layer %d: brick pairs need an even qubit count (n=%d)", li, n);
        return buf;
      }
      count = (int)pattern_pairs(n, L).size();
    }
    if (is_param(L.gate) && L.source != SRC_FIXED) {
      if (L.offset < 0) {
        snprintf(buf, sizeof buf, "EINVAL: layer %d: negative offset", li);
        return buf;
      }
      // int64: an offset near INT32_MAX must not wrap the parameter count
      const long long end = (long long)L.offset + (long long)gate_params(L.gate) * count;
      if (end > INT32_MAX) {
        snprintf(buf, sizeof buf, "EINVAL: layer %d: offset + parameter count exceeds INT32_MAX", li);
        return buf;
      }
      if (L.source == SRC_WEIGHT) w = std::max(w, (int)end);
      else f = std::max(f, (int)end);
    }
  }
  if (nw) *nw = w;
  if (nf) *nf = f;
  return "";
}

// One gate of a sub-layer, before placement on wires: gate, source, parameter
// offset relative to the gate's first parameter, fixed value.
struct SubGate {
  int gate, src, poff;
  double fixed;
};

// The sub-layers one 1-qubit gate becomes (application order).  Rot(theta,
// phi, lambda) = P(phi) RY(theta) P(lambda) (Appendix A, P = diag(1, e^{ia})).
// With the H-Rz expansion (Sec. 2.5): RX = H RZ H; RY = S H RZ H S^dag;
// GPI2(phi) = RZ(2 pi phi) RX(pi/2) RZ(-2 pi phi), RX(pi/2) = H RZ(pi/2) H.
static std::vector<SubGate> sub_gates_1q(int g, int src, double fixed, double f2, double f3, bool hrz) {
  const double hp = 1.5707963267948966;
  auto ry = [&](int s, int off, double fx) -> std::vector<SubGate> {
    if (!hrz) return {{RY, s, off, fx}};
    return {{PHASE, SRC_FIXED, 0, -hp}, {H, SRC_FIXED, 0, 0.0}, {RZ, s, off, fx}, {H, SRC_FIXED, 0, 0.0},
            {PHASE, SRC_FIXED, 0, hp}};
  };
  if (g == ROT) {
    std::vector<SubGate> v = {{PHASE, src, 2, f3}};
    for (const SubGate &x : ry(src, 0, fixed)) v.push_back(x);
    v.push_back({PHASE, src, 1, f2});
    return v;
  }
  if (hrz && g == RX) return {{H, SRC_FIXED, 0, 0.0}, {RZ, src, 0, fixed}, {H, SRC_FIXED, 0, 0.0}};
  if (hrz && g == RY) return ry(src, 0, fixed);
  if (hrz && g == GPI2)
    return {{RZNT, src, 0, fixed}, {H, SRC_FIXED, 0, 0.0}, {RZ, SRC_FIXED, 0, hp}, {H, SRC_FIXED, 0, 0.0},
            {RZT, src, 0, fixed}};
  return {{g, src, 0, fixed}};
}

// Gate instances in application order.  A layer whose gates become several
// factors is emitted as consecutive sub-layers (all wires' first factors,
// then all second factors, ...): factors on different wires commute, so this
// is the same product, and the per-layer dispatcher sees uniform layers.
static std::vector<Inst> expand(int n, const LayerSpec *layers, int n_layers, bool hrz) {
  constexpr int SUBS = 16;   // sub-layer slots per layer
  std::vector<Inst> out;
  for (int li = 0; li < n_layers; ++li) {
    const LayerSpec &L = layers[li];
    const int src = is_param(L.gate) ? L.source : SRC_FIXED;
    const int np = std::max(1, gate_params(L.gate));
    if (is_1q(L.gate)) {
      const std::vector<SubGate> sg = sub_gates_1q(L.gate, src, L.fixed, L.fixed2, L.fixed3, hrz);
      std::vector<int> wires;
      if (L.pattern == PAT_ALL)
        for (int q = 0; q < n; ++q) wires.push_back(q);
      else
        wires.push_back(L.wire);
      for (size_t k = 0; k < sg.size(); ++k)
        for (size_t i = 0; i < wires.size(); ++i) {
          const int first = L.offset + np * (L.pattern == PAT_ALL ? wires[i] : 0);
          const SubGate &x = sg[k];
          out.push_back({x.gate, wires[i], -1, x.src, x.src == SRC_FIXED ? 0 : first + x.poff,
                         li * SUBS + (int)k, x.fixed});
        }
    } else {
      const auto pr = pattern_pairs(n, L);
      // MS(phi0, phi1, theta) = (D1 (x) D0) MS(theta) (D1 (x) D0)^dag with
      // D = RZ(2 pi phi) (P(phi) = D X D^dag, Appendix A as read)
      const bool phased = L.gate == MS && (L.fixed2 != 0.0 || L.fixed3 != 0.0);
      const double tp = 6.283185307179586;
      if (phased)
        for (size_t k = 0; k < pr.size(); ++k) {
          out.push_back({RZ, pr[k].first, -1, SRC_FIXED, 0, li * SUBS, -tp * L.fixed3});
          out.push_back({RZ, pr[k].second, -1, SRC_FIXED, 0, li * SUBS, -tp * L.fixed2});
        }
      for (size_t k = 0; k < pr.size(); ++k)
        out.push_back({L.gate, pr[k].first, pr[k].second, src, L.offset + (int)k, li * SUBS + 1, L.fixed});
      if (phased)
        for (size_t k = 0; k < pr.size(); ++k) {
          out.push_back({RZ, pr[k].first, -1, SRC_FIXED, 0, li * SUBS + 2, tp * L.fixed3});
          out.push_back({RZ, pr[k].second, -1, SRC_FIXED, 0, li * SUBS + 2, tp * L.fixed2});
        }
    }
  }
  return out;
}

// --------------------------------------------------------------- IR build --
namespace {

struct Builder {
  Plan &P;
  int n;
  explicit Builder(Plan &p) : P(p), n(p.n) {}

  int add_factor(const Inst &in, int gate_override = -1) {
    Factor f;
    f.gate = gate_override >= 0 ? gate_override : in.gate;
    f.src = in.src;
    f.pidx = in.pidx;
    f.wires = 0;
    f.fixed = in.fixed;
    P.factors.push_back(f);
    return (int)P.factors.size() - 1;
  }
  int bit(int w) const { return n - 1 - w; }

  int new_op(int kind) {
    IrOp op;
    op.kind = kind;
    if (kind == IR_PERM) op.F = GF2::identity(n);
    P.ops.push_back(op);
    return (int)P.ops.size() - 1;
  }

  // CNOT / SWAP / X as a forward basis map
  GF2 perm_of(int gate, int w0, int w1) const {
    GF2 g = GF2::identity(n);
    if (gate == X) {
      g.c = 1u << bit(w0);
    } else if (gate == CNOT) {
      g.cols[bit(w0)] |= 1u << bit(w1);   // target flips when control is set
    } else if (gate == SWAP) {
      g.cols[bit(w0)] = 1u << bit(w1);
      g.cols[bit(w1)] = 1u << bit(w0);
    }
    return g;
  }
};

}  // namespace

static void finish_op(Plan &P, IrOp &op) {
  const int n = P.n;
  (void)n;
  op.mask = 0;
  if (op.kind == IR_U1) op.mask = 1u << op.bits[0];
  if (op.kind == IR_U2) op.mask = (1u << op.bits[0]) | (1u << op.bits[1]);
  if (op.kind == IR_PERM || op.kind == IR_DENSE) op.mask = (P.n >= 32) ? 0xffffffffu : ((1u << P.n) - 1u);
  if (op.kind == IR_GRAD1) op.mask = 1u << op.bits[0];
  if (op.kind == IR_GRAD2) op.mask = (1u << op.bits[0]) | (1u << op.bits[1]);
  std::vector<int> fs = op.factors;
  for (const IrTerm &t : op.terms) {
    fs.push_back(t.factor);
    op.mask |= 1u << t.bits[0];
    if (t.nbits == 2) op.mask |= 1u << t.bits[1];
  }
  op.per_sample = false;
  op.has_grad = false;
  op.real = true;
  op.diagonal = true;
  for (int fi : fs) {
    const Factor &f = P.factors[fi];
    if (f.src == SRC_INPUT) op.per_sample = true;
    if (is_param(f.gate) && f.src != SRC_FIXED) op.has_grad = true;
    if (!is_real_gate(f.gate)) op.real = false;
    if (!(is_diag1(f.gate) || is_diag2(f.gate))) op.diagonal = false;
  }
  if (op.kind == IR_U2 && !op.factors.empty()) {
    const int g = P.factors[op.factors[0]].gate;
    op.real = is_real_gate(g);
    op.diagonal = is_diag2(g);
  }
  if (op.kind == IR_DENSE) op.has_grad = false;
}

static std::string build_ir(Plan &P, const std::vector<Inst> &insts) {
  Builder B(P);
  const int n = P.n;
  const bool fused = (P.mode == 2);
  const bool multi = P.resident && P.nv < std::max(P.nv, KMIN);  // several samples per workgroup
  // embedding: leading 1q gates per wire
  P.embed.assign(n, {});
  std::vector<char> touched(n, 0), consumed(insts.size(), 0);
  for (size_t i = 0; i < insts.size(); ++i) {
    const Inst &in = insts[i];
    if (is_1q(in.gate)) {
      if (!touched[in.w0]) {
        P.embed[in.w0].push_back(B.add_factor(in));
        consumed[i] = 1;
      }
    } else {
      touched[in.w0] = touched[in.w1] = 1;
    }
  }
  P.embed_per_sample = false;
  for (int w = 0; w < n; ++w)
    for (int fi : P.embed[w])
      if (P.factors[fi].src == SRC_INPUT) P.embed_per_sample = true;

  std::vector<int> open_u1(n, -1);
  int cur_layer = -1, layer_diag = -1, layer_perm = -1, gpi_diag = -1, gpi_perm = -1;
  // CNOT / SWAP gates after the last other gate of the circuit: they only
  // permute the final state, so they all become one index map, which the last
  // pass applies as it stores (no pass of their own)
  size_t trailing_from = 0;
  for (size_t i = 0; i < insts.size(); ++i)
    if (!consumed[i] && insts[i].gate != CNOT && insts[i].gate != SWAP) trailing_from = i + 1;
  for (size_t i = 0; i < insts.size(); ++i) {
    if (consumed[i]) continue;
    if (P.dense) {
      // a layer without per-sample parameters becomes one full-unitary op
      // (the paper's unitary operation, Sec. 2.2.1) plus gradient-only sums
      std::vector<size_t> mem;
      bool input = false;
      for (size_t j = i; j < insts.size() && insts[j].layer == insts[i].layer; ++j)
        if (!consumed[j]) {
          mem.push_back(j);
          if (insts[j].src == SRC_INPUT) input = true;
        }
      if (!input) {
        const int od = B.new_op(IR_DENSE);
        std::vector<IrOp> grads;
        for (size_t j : mem) {
          const Inst &q = insts[j];
          const int f = B.add_factor(q);
          P.factors[f].wires = B.bit(q.w0) | ((q.w1 >= 0 ? B.bit(q.w1) + 1 : 0) << 8);
          P.ops[od].factors.push_back(f);
          if (is_param(q.gate) && q.src != SRC_FIXED) {
            IrOp g;
            g.kind = is_1q(q.gate) ? IR_GRAD1 : IR_GRAD2;
            g.bits[0] = B.bit(q.w0);
            g.bits[1] = q.w1 >= 0 ? B.bit(q.w1) : -1;
            g.factors.push_back(f);
            grads.push_back(g);
          }
          consumed[j] = 1;
        }
        for (auto &g : grads) P.ops.push_back(g);
        for (int w = 0; w < n; ++w) open_u1[w] = -1;
        layer_diag = layer_perm = gpi_diag = gpi_perm = -1;
        cur_layer = insts[i].layer;
        continue;
      }
    }
    const Inst &in = insts[i];
    if (in.layer != cur_layer) {
      cur_layer = in.layer;
      layer_diag = layer_perm = gpi_diag = gpi_perm = -1;
    }
    const int g = in.gate;
    if (is_1q(g)) {
      if (fused) {
        const int w = in.w0;
        if (open_u1[w] >= 0 && open_u1[w] == open_u1[w]) {
          P.ops[open_u1[w]].factors.push_back(B.add_factor(in));
        } else {
          const int o = B.new_op(IR_U1);
          P.ops[o].bits[0] = B.bit(w);
          P.ops[o].factors.push_back(B.add_factor(in));
          open_u1[w] = o;
        }
        layer_diag = layer_perm = -1;
        continue;
      }
      // per-layer techniques
      if (is_diag1(g)) {
        if (!(layer_diag >= 0 && layer_diag == (int)P.ops.size() - 1)) layer_diag = B.new_op(IR_DIAG);
        IrTerm t;
        t.factor = B.add_factor(in);
        t.nbits = 1;
        t.bits[0] = B.bit(in.w0);
        t.bits[1] = -1;
        P.ops[layer_diag].terms.push_back(t);
      } else if (g == X) {
        if (!(layer_perm >= 0 && layer_perm == (int)P.ops.size() - 1)) layer_perm = B.new_op(IR_PERM);
        P.ops[layer_perm].F = B.perm_of(X, in.w0, -1).after(P.ops[layer_perm].F);
      } else if (g == GPI) {
        // GPI(phi) = X diag(e^{2 pi i phi}, e^{-2 pi i phi}): phase then index
        // reversal.  All GPI gates of a layer share one diagonal op and one map
        // (a phase on one wire commutes with X on another).
        IrTerm t;
        t.factor = B.add_factor(in, GPI_DIAG);
        t.nbits = 1;
        t.bits[0] = B.bit(in.w0);
        t.bits[1] = -1;
        if (gpi_diag >= 0 && gpi_perm == (int)P.ops.size() - 1) {
          P.ops[gpi_diag].terms.push_back(t);
          P.ops[gpi_perm].F = B.perm_of(X, in.w0, -1).after(P.ops[gpi_perm].F);
        } else {
          gpi_diag = B.new_op(IR_DIAG);
          P.ops[gpi_diag].terms.push_back(t);
          gpi_perm = B.new_op(IR_PERM);
          P.ops[gpi_perm].F = B.perm_of(X, in.w0, -1);
        }
        layer_diag = layer_perm = -1;
      } else {
        const int o = B.new_op(IR_U1);
        P.ops[o].bits[0] = B.bit(in.w0);
        P.ops[o].factors.push_back(B.add_factor(in));
        layer_diag = layer_perm = -1;
      }
      continue;
    }
    // two-qubit gates
    open_u1[in.w0] = open_u1[in.w1] = -1;
    if (is_diag2(g) && !(multi && in.src == SRC_INPUT)) {
      if (!(layer_diag >= 0 && layer_diag == (int)P.ops.size() - 1)) layer_diag = B.new_op(IR_DIAG);
      IrTerm t;
      t.factor = B.add_factor(in);
      t.nbits = 2;
      t.bits[0] = B.bit(in.w0);
      t.bits[1] = B.bit(in.w1);
      P.ops[layer_diag].terms.push_back(t);
      layer_perm = -1;
    } else if ((g == CNOT || g == SWAP) && !P.resident) {
      const bool down = (g == CNOT) && (B.bit(in.w0) > B.bit(in.w1));
      if (!fused || down || i >= trailing_from) {
        if (!(layer_perm >= 0 && layer_perm == (int)P.ops.size() - 1)) layer_perm = B.new_op(IR_PERM);
        P.ops[layer_perm].F = B.perm_of(g, in.w0, in.w1).after(P.ops[layer_perm].F);
      } else {
        const int o = B.new_op(IR_U2);
        P.ops[o].bits[0] = B.bit(in.w0);
        P.ops[o].bits[1] = B.bit(in.w1);
        P.ops[o].factors.push_back(B.add_factor(in));
        layer_perm = -1;
      }
      layer_diag = -1;
    } else if ((g == CNOT || g == SWAP) && P.resident) {
      // resident tiles permute in LDS: one map per layer
      if (!(layer_perm >= 0 && layer_perm == (int)P.ops.size() - 1)) layer_perm = B.new_op(IR_PERM);
      P.ops[layer_perm].F = B.perm_of(g, in.w0, in.w1).after(P.ops[layer_perm].F);
      layer_diag = -1;
    } else {
      const int o = B.new_op(IR_U2);
      P.ops[o].bits[0] = B.bit(in.w0);
      P.ops[o].bits[1] = B.bit(in.w1);
      P.ops[o].factors.push_back(B.add_factor(in));
      layer_diag = layer_perm = -1;
    }
  }
  // merge consecutive permutations
  std::vector<IrOp> merged;
  for (auto &op : P.ops) {
    if (op.kind == IR_PERM && !merged.empty() && merged.back().kind == IR_PERM) {
      merged.back().F = op.F.after(merged.back().F);
      continue;
    }
    merged.push_back(op);
  }
  P.ops.swap(merged);
  // drop identity permutations and empty diagonals
  std::vector<IrOp> kept;
  for (auto &op : P.ops) {
    if (op.kind == IR_PERM && op.F.is_identity()) continue;
    kept.push_back(op);
  }
  P.ops.swap(kept);
  for (auto &op : P.ops) finish_op(P, op);
  // single-sample-per-workgroup tiles cannot hold per-sample diagonal tables when
  // several samples share a workgroup: turn such terms into 1q / 2q ops
  // and with the diagonal-Einsum technique every diagonal layer is applied
  // gate by gate, one diagonal factor per gate (Sec. 2.4.3)
  if (multi || P.opts.diag == 1) {
    std::vector<IrOp> out;
    for (auto &op : P.ops) {
      if (op.kind == IR_DIAG && (op.per_sample || P.opts.diag == 1)) {
        for (const IrTerm &t : op.terms) {
          IrOp o;
          o.kind = t.nbits == 1 ? IR_U1 : IR_U2;
          o.bits[0] = t.bits[0];
          o.bits[1] = t.bits[1];
          o.factors.push_back(t.factor);
          finish_op(P, o);
          out.push_back(o);
        }
      } else {
        out.push_back(op);
      }
    }
    P.ops.swap(out);
  }
  return "";
}

// ------------------------------------------------------------ scheduling --
namespace {

struct Sched {
  Plan &P;
  int n, K;
  std::vector<char> placed;
  explicit Sched(Plan &p, int k) : P(p), n(p.n), K(k), placed(p.ops.size(), 0) {}

  static uint32_t tile_mask(const std::vector<int> &T) {
    uint32_t m = 0;
    for (int b : T) m |= 1u << b;
    return m;
  }

  // extra TL index bits a diagonal op needs on tile T (split at h = K/2)
  int diag_extras(const IrOp &op, const std::vector<int> &T) const {
    std::map<int, int> tix;
    for (size_t i = 0; i < T.size(); ++i) tix[T[i]] = (int)i;
    const int h = K / 2;
    std::vector<int> extra;
    for (const IrTerm &t : op.terms) {
      int tb[2] = {-1, -1};
      for (int q = 0; q < t.nbits; ++q)
        if (tix.count(t.bits[q])) tb[q] = tix[t.bits[q]];
      bool lowside = false;
      for (int q = 0; q < t.nbits; ++q)
        if (tb[q] >= 0 && tb[q] < h) lowside = true;
      if (!lowside) continue;
      for (int q = 0; q < t.nbits; ++q)
        if (tb[q] >= h && std::find(extra.begin(), extra.end(), tb[q]) == extra.end()) extra.push_back(tb[q]);
    }
    return (int)extra.size();
  }

  bool preserving(const GF2 &M, const std::vector<int> &T) const {
    const uint32_t tm = tile_mask(T);
    for (int b : T)
      if ((M.cols[b] & ~tm) != 0) return false;
    return true;
  }

  struct Sim {
    std::vector<int> ops;
    int perm = -1;          // IR op attached at the end
    bool perm_store = false;
    int score = 0;
  };

  Sim simulate(const std::vector<int> &T, bool has_load) const {
    Sim s;
    const uint32_t tm = tile_mask(T);
    uint32_t blocked_all = 0, blocked_nd = 0;
    int ndiag = 0;
    (void)has_load;
    for (size_t i = 0; i < P.ops.size(); ++i) {
      if (placed[i]) continue;
      const IrOp &op = P.ops[i];
      if (op.kind == IR_PERM) {
        if ((blocked_all | blocked_nd) == 0) {
          s.perm = (int)i;
          bool last = true;
          for (size_t j = i + 1; j < P.ops.size(); ++j)
            if (!placed[j]) last = false;
          s.perm_store = last || preserving(op.F, T);
        }
        break;
      }
      bool ok;
      if (op.kind == IR_DIAG)
        ok = !(op.mask & blocked_all) && ndiag < MAX_DIAG_OPS && diag_extras(op, T) <= MAX_DIAG_EXTRA;
      else
        ok = ((op.mask & ~tm) == 0) && !(op.mask & (blocked_all | blocked_nd));
      if (ok && (int)s.ops.size() >= MAX_OPS / 2) ok = false;
      if (ok) {
        s.ops.push_back((int)i);
        if (op.kind == IR_DIAG) ++ndiag;
      } else if (op.kind == IR_DIAG) {
        blocked_nd |= op.mask;
      } else {
        blocked_all |= op.mask;
      }
    }
    s.score = (int)s.ops.size();
    return s;
  }

  std::vector<int> t_low() const {
    std::vector<int> T;
    for (int b = 0; b < K; ++b) T.push_back(b);
    return T;
  }

  std::vector<int> t_need(int c) const {
    uint32_t T = 0;
    for (int b = 0; b < c; ++b) T |= 1u << b;
    for (size_t i = 0; i < P.ops.size(); ++i) {
      if (placed[i]) continue;
      const IrOp &op = P.ops[i];
      if (op.kind == IR_PERM) break;
      if (op.kind == IR_DIAG) continue;
      const uint32_t need = op.mask & ~T;
      if (popc(T) + popc(need) <= K) T |= need;
    }
    for (int b = 0; b < n && popc(T) < K; ++b) T |= 1u << b;
    std::vector<int> v;
    for (int b = 0; b < n; ++b)
      if ((T >> b) & 1) v.push_back(b);
    return v;
  }
};

}  // namespace

// Runs of consecutive Hadamard ops on distinct register bits of one stage
// become one OP_WHT op (the fast Walsh-Hadamard transform over those bits).
static void group_wht(Plan &P, int begin) {
  std::vector<DevOp> out;
  size_t i = begin;
  while (i < P.dop.size()) {
    if (!(P.dop[i].kind == OP_U1 && (P.dop[i].flags & F_HADAMARD))) {
      out.push_back(P.dop[i++]);
      continue;
    }
    int mask = 0;
    size_t j = i;
    while (j < P.dop.size() && P.dop[j].kind == OP_U1 && (P.dop[j].flags & F_HADAMARD) &&
           !(mask & (1 << P.dop[j].r0)))
      mask |= 1 << P.dop[j++].r0;
    DevOp o;
    std::memset(&o, 0, sizeof o);
    o.kind = OP_WHT;
    o.r0 = mask;
    o.acc = -1;
    out.push_back(o);
    i = j;
  }
  P.dop.resize(begin);
  P.dop.insert(P.dop.end(), out.begin(), out.end());
}

// Runs of consecutive complex single-qubit ops (shared matrices) on distinct
// register bits of one stage become one OP_U1G op: they commute, so the kernel
// applies them back to back and takes their gradients at the group's output.
static void group_u1(Plan &P, int begin) {
  // members share one table: all shared matrices or all per-sample ones
  auto eligible = [](const DevOp &o) { return o.kind == OP_U1 && !(o.flags & (F_REAL | F_DIAGONAL)); };
  std::vector<DevOp> out;
  size_t i = begin;
  while (i < P.dop.size()) {
    if (!eligible(P.dop[i])) {
      out.push_back(P.dop[i++]);
      continue;
    }
    const int ps = P.dop[i].flags & F_PERSAMPLE;
    size_t j = i;
    int mask = 0;
    while (j < P.dop.size() && eligible(P.dop[j]) && (P.dop[j].flags & F_PERSAMPLE) == ps &&
           !(mask & (1 << P.dop[j].r0)))
      mask |= 1 << P.dop[j++].r0;
    if (j - i < 2) {
      out.push_back(P.dop[i++]);
      continue;
    }
    DevGroup g;
    DevOp o;
    std::memset(&o, 0, sizeof o);
    for (int r = 0; r < RB; ++r) g.mat[r] = g.acc[r] = -1;
    for (size_t k = i; k < j; ++k) {
      const DevOp &u = P.dop[k];
      g.mat[u.r0] = u.mat;
      if (u.flags & F_GRAD) {
        g.acc[u.r0] = u.acc;
        o.flags |= F_GRAD;
      }
    }
    o.kind = OP_U1G;
    o.flags |= ps;
    o.r0 = mask;
    o.acc = -1;
    o.aux = (int)P.dgroup.size();
    P.dgroup.push_back(g);
    out.push_back(o);
    i = j;
  }
  P.dop.resize(begin);
  P.dop.insert(P.dop.end(), out.begin(), out.end());
}

// Pairs of consecutive structured MS or ECR ops of one stage on disjoint
// register-bit pairs become one OP_U2G op (they commute).
static void group_u2(Plan &P, int begin) {
  auto eligible = [](const DevOp &o) {
    return o.kind == OP_U2 && !(o.flags & F_PERSAMPLE) && (o.sub == U2_MS || o.sub == U2_ECR);
  };
  std::vector<DevOp> out;
  size_t i = begin;
  while (i < P.dop.size()) {
    const DevOp &x = P.dop[i];
    if (i + 1 < P.dop.size() && eligible(x) && eligible(P.dop[i + 1]) && P.dop[i + 1].sub == x.sub) {
      DevOp y = P.dop[i + 1];
      DevOp f = x;
      const int mx = (1 << x.r0) | (1 << x.r1), my = (1 << y.r0) | (1 << y.r1);
      if (!(mx & my)) {
        // the pair holding register bit 0 goes first
        if (!(my & 1) && !(mx & 1)) {
          out.push_back(P.dop[i++]);
          continue;
        }
        if (my & 1) std::swap(f, y);
        DevGroup g;
        for (int r = 0; r < RB; ++r) g.mat[r] = g.acc[r] = -1;
        g.mat[0] = f.mat;
        g.mat[1] = y.mat;
        DevOp o;
        std::memset(&o, 0, sizeof o);
        o.kind = OP_U2G;
        o.sub = x.sub;
        o.r0 = f.r0 << 6 | f.r1 << 4 | y.r0 << 2 | y.r1;
        o.acc = -1;
        if (f.flags & F_GRAD) g.acc[0] = f.acc;
        if (y.flags & F_GRAD) g.acc[1] = y.acc;
        if ((f.flags | y.flags) & F_GRAD) o.flags |= F_GRAD;
        o.aux = (int)P.dgroup.size();
        P.dgroup.push_back(g);
        out.push_back(o);
        i += 2;
        continue;
      }
    }
    out.push_back(P.dop[i++]);
  }
  P.dop.resize(begin);
  P.dop.insert(P.dop.end(), out.begin(), out.end());
}

// The stage program of brick-layer circuits -- pair gates on (0,1),(2,3), 2x2
// gates on all four register bits, a pair gate on (1,2), 2x2 gates on bits 1
// and 2 (or a prefix of at least the first two steps) -- becomes one OP_SEQ op:
// straight-line code for the whole run, with no op-loop merge between steps.
static void group_seq(Plan &P, int begin) {
  std::vector<DevOp> out;
  size_t i = begin;
  const size_t end = P.dop.size();
  while (i < end) {
    const DevOp &a = P.dop[i];
    // the stage program reads shared matrices only
    const bool head = a.kind == OP_U2G && a.r0 == (0 << 6 | 1 << 4 | 2 << 2 | 3) &&
                      i + 1 < end && P.dop[i + 1].kind == OP_U1G && P.dop[i + 1].r0 == 15 &&
                      !(P.dop[i + 1].flags & F_PERSAMPLE);
    if (!head) {
      out.push_back(P.dop[i++]);
      continue;
    }
    int len = 2;
    if (i + 2 < end) {
      const DevOp &u = P.dop[i + 2];
      if (u.kind == OP_U2 && u.r0 == 1 && u.r1 == 2 && u.sub == a.sub && !(u.flags & F_PERSAMPLE)) {
        len = 3;
        if (i + 3 < end && P.dop[i + 3].kind == OP_U1G && P.dop[i + 3].r0 == 6 &&
            !(P.dop[i + 3].flags & F_PERSAMPLE))
          len = 4;
      }
    }
    DevSeq q;
    for (int k = 0; k < SEQ_SLOTS; ++k) q.mat[k] = q.acc[k] = -1;
    const DevGroup &g2 = P.dgroup[a.aux];
    q.mat[0] = g2.mat[0];
    q.mat[1] = g2.mat[1];
    q.acc[0] = g2.acc[0];
    q.acc[1] = g2.acc[1];
    const DevGroup &g1 = P.dgroup[P.dop[i + 1].aux];
    for (int r = 0; r < RB; ++r) {
      q.mat[2 + r] = g1.mat[r];
      q.acc[2 + r] = g1.acc[r];
    }
    if (len >= 3) {
      const DevOp &u = P.dop[i + 2];
      q.mat[6] = u.mat;
      q.acc[6] = (u.flags & F_GRAD) ? u.acc : -1;
    }
    if (len == 4) {
      const DevGroup &g3 = P.dgroup[P.dop[i + 3].aux];
      q.mat[7] = g3.mat[1];
      q.acc[7] = g3.acc[1];
      q.mat[8] = g3.mat[2];
      q.acc[8] = g3.acc[2];
    }
    DevOp o;
    std::memset(&o, 0, sizeof o);
    o.kind = OP_SEQ;
    o.sub = a.sub;
    o.r0 = len;
    o.acc = -1;
    for (int k = 0; k < SEQ_SLOTS; ++k)
      if (q.acc[k] >= 0) o.flags |= F_GRAD;
    o.aux = (int)P.dseq.size();
    P.dseq.push_back(q);
    out.push_back(o);
    i += len;
  }
  P.dop.resize(begin);
  P.dop.insert(P.dop.end(), out.begin(), out.end());
}

static std::string schedule(Plan &P, int K) {
  const int n = P.n;
  P.passes.clear();
  if (P.resident) {
    // the whole state of a sample is one tile: one pass holds every op
    PlanPass pp;
    pp.K = K;
    for (int b = 0; b < P.nv; ++b) pp.tile.push_back(b);
    pp.load_mode = LOAD_EMBED;
    for (size_t i = 0; i < P.ops.size(); ++i) pp.ops.push_back((int)i);
    P.passes.push_back(pp);
    return "";
  }
  Sched S(P, K);
  bool first = true;
  bool pending = false;
  GF2 pending_map;
  for (int guard = 0; guard < 100000; ++guard) {
    bool any = pending;
    for (size_t i = 0; i < P.ops.size(); ++i)
      if (!S.placed[i]) any = true;
    if (!any && !first) break;
    PlanPass pp;
    pp.K = K;
    pp.load_mode = first ? LOAD_EMBED : LOAD_GLOBAL;
    if (pending) {
      pp.has_load = true;
      pp.load_map = pending_map.inverse();
      pending = false;
    }
    // a permutation waiting at the front becomes this pass's gather
    if (!first && !pp.has_load) {
      for (size_t i = 0; i < P.ops.size(); ++i) {
        if (S.placed[i]) continue;
        if (P.ops[i].kind == IR_PERM) {
          bool last = true;
          for (size_t j = i + 1; j < P.ops.size(); ++j)
            if (!S.placed[j]) last = false;
          if (!last) {
            pp.has_load = true;
            pp.load_map = P.ops[i].F.inverse();
            S.placed[i] = 1;
          }
        }
        break;
      }
    }
    std::vector<std::vector<int>> cands = {S.t_low(), S.t_need(6), S.t_need(4)};
    int best = -1;
    Sched::Sim bs;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      Sched::Sim s = S.simulate(cands[ci], pp.has_load);
      int sc = s.score * 2 + (s.perm >= 0 ? 1 : 0);
      int bsc = best < 0 ? -1 : bs.score * 2 + (bs.perm >= 0 ? 1 : 0);
      if (sc > bsc) {
        best = (int)ci;
        bs = s;
      }
    }
    pp.tile = cands[best];
    pp.ops = bs.ops;
    for (int i : bs.ops) S.placed[i] = 1;
    if (bs.perm >= 0) {
      S.placed[bs.perm] = 1;
      if (bs.perm_store) {
        pp.has_store = true;
        pp.store_map = P.ops[bs.perm].F;
      } else {
        pending = true;
        pending_map = P.ops[bs.perm].F;
      }
    }
    if (pp.ops.empty() && !pp.has_store && !pp.has_load && !first) {
      return "internal: scheduler made no progress";
    }
    P.passes.push_back(pp);
    first = false;
  }
  (void)n;
  return "";
}

// --------------------------------------------------------- device tables --
namespace {

struct Emit {
  Plan &P;
  int n, K;
  std::vector<Factor> pf;          // factors, contiguous per prep item
  std::map<std::pair<int, int>, std::vector<Contrib>> by_param;   // (src, pidx) -> contribs
  long long acc_prefix = 0;

  Emit(Plan &p) : P(p), n(p.n), K(0) {}

  int factors_slice(const std::vector<int> &fs) {
    const int b = (int)pf.size();
    for (int f : fs) pf.push_back(P.factors[f]);
    return b;
  }
  bool any_input(const std::vector<int> &fs, size_t from = 0) const {
    for (size_t k = from; k < fs.size(); ++k)
      if (P.factors[fs[k]].src == SRC_INPUT) return true;
    return false;
  }
  int alloc_mat(bool ps, int count) {
    int &ctr = ps ? P.n_mats_ps : P.n_mats;
    const int o = ctr;
    ctr += count;
    return o;
  }
  int alloc_dbl(bool ps, int count) {
    int &ctr = ps ? P.n_dbl_ps : P.n_dbl;
    const int o = ctr;
    ctr += count;
    return o;
  }
  void prep(int kind, bool ps, int out, int fb, int fe, int k) {
    PrepItem it;
    it.kind = kind;
    it.per_sample = ps ? 1 : 0;
    it.out = out;
    it.f_begin = fb;
    it.f_end = fe;
    it.k = k;
    it.pad[0] = it.pad[1] = 0;
    P.prep.push_back(it);
  }
  void contrib(const Factor &f, int acc_global, int nacc, int coef, bool coef_ps) {
    Contrib c;
    c.acc = acc_global;
    c.n = nacc;
    c.coef = coef;
    c.coef_ps = coef_ps ? 1 : 0;
    by_param[{f.src, f.pidx}].push_back(c);
  }
  // gradient bookkeeping for a chain of 1q factors measured by Pauli sums
  void u1_contribs(const std::vector<int> &fs, int acc_global) {
    const int sl = factors_slice(fs);
    for (size_t k = 0; k < fs.size(); ++k) {
      const Factor &f = P.factors[fs[k]];
      if (!is_param(f.gate) || f.src == SRC_FIXED) continue;
      const bool ps = any_input(fs, k);
      const int co = alloc_dbl(ps, 3);
      prep(PREP_COEF1, ps, co, sl, sl + (int)fs.size(), sl + (int)k);
      contrib(f, acc_global, 3, co, ps);
    }
  }
};

}  // namespace

static std::string emit(Plan &P) {
  Emit E(P);
  const int n = P.n;
  P.dpass.clear();
  P.dstage.clear();
  P.dop.clear();
  P.ddiag.clear();
  P.diag_jobs.clear();
  P.n_diag_tab = 0;
  P.dterm.clear();
  P.dtgrad.clear();
  P.dperm.clear();
  P.dgroup.clear();
  P.dseq.clear();
  P.prep.clear();
  P.contribs.clear();
  P.n_mats = P.n_mats_ps = P.n_dbl = P.n_dbl_ps = 0;
  P.acc_static.clear();
  P.acc_units.clear();
  P.pass_prefix.clear();
  P.pass_units.clear();
  P.n_acc = 0;

  // embed matrices: one 2x2 per wire
  int embed_mat = E.alloc_mat(P.embed_per_sample, 4 * n);
  for (int w = 0; w < n; ++w) {
    const int sl = E.factors_slice(P.embed[w]);
    E.prep(PREP_MAT1, P.embed_per_sample, embed_mat + 4 * w, sl, sl + (int)P.embed[w].size(), 0);
  }
  std::vector<char> embed_grad(n, 0);
  for (int w = 0; w < n; ++w)
    for (int fi : P.embed[w])
      if (is_param(P.factors[fi].gate) && P.factors[fi].src != SRC_FIXED) embed_grad[w] = 1;

  // op matrices / angles
  std::vector<int> op_mat(P.ops.size(), -1), op_ps(P.ops.size(), 0);
  std::vector<std::vector<int>> term_ang(P.ops.size());
  for (size_t i = 0; i < P.ops.size(); ++i) {
    IrOp &op = P.ops[i];
    if (op.kind == IR_U1) {
      const int sl = E.factors_slice(op.factors);
      op_mat[i] = E.alloc_mat(op.per_sample, 4);
      op_ps[i] = op.per_sample;
      E.prep(PREP_MAT1, op.per_sample, op_mat[i], sl, sl + (int)op.factors.size(), 0);
    } else if (op.kind == IR_U2) {
      const int sl = E.factors_slice(op.factors);
      op_mat[i] = E.alloc_mat(op.per_sample, 16);
      op_ps[i] = op.per_sample;
      E.prep(PREP_MAT2, op.per_sample, op_mat[i], sl, sl + 1, 0);
    } else if (op.kind == IR_DENSE) {
      const int dim = 1 << P.nv;
      const int sl = E.factors_slice(op.factors);
      op_mat[i] = E.alloc_mat(false, dim * dim);
      E.prep(PREP_DENSE, false, op_mat[i], sl, sl + (int)op.factors.size(), 0);
    } else if (op.kind == IR_DIAG) {
      for (const IrTerm &t : op.terms) {
        const bool ps = P.factors[t.factor].src == SRC_INPUT;
        const int sl = E.factors_slice({t.factor});
        const int a = E.alloc_dbl(ps, 1 << t.nbits);
        E.prep(PREP_ANG, ps, a, sl, sl + 1, 0);
        term_ang[i].push_back(a);
      }
    }
  }

  // embed-gradient wires: first pass touching the wire's bit, if the bit is in its tile
  std::vector<int> first_touch(n, -1);
  for (size_t p = 0; p < P.passes.size(); ++p) {
    uint32_t m = 0;
    for (int oi : P.passes[p].ops) m |= P.ops[oi].mask;
    for (int b = 0; b < n; ++b)
      if (((m >> b) & 1) && first_touch[b] < 0) first_touch[b] = (int)p;
    if (P.passes[p].has_store || P.passes[p].has_load) {
      // a map touches every bit; bits not yet touched are first touched here
      for (int b = 0; b < n; ++b)
        if (first_touch[b] < 0) first_touch[b] = (int)p;
    }
  }
  // a pass with a load map cannot host gradients of bits first touched by its own map
  std::vector<int> leftovers;
  for (int w = 0; w < n; ++w) {
    if (!embed_grad[w]) continue;
    const int b = n - 1 - w;
    int p = first_touch[b];
    if (p < 0) p = 0;   // untouched wire: any point of the backward sweep will do
    bool ok = p < (int)P.passes.size() && std::find(P.passes[p].tile.begin(), P.passes[p].tile.end(), b) != P.passes[p].tile.end();
    if (ok && P.passes[p].has_load) ok = false;   // state at its start is not the embed frame
    if (ok) P.passes[p].grad_wires.push_back(w);
    else leftovers.push_back(w);
  }
  // the rest: at the end of the embedding pass's backward, from the product-state
  // environment (the embedding output is a product state, so the sums over pairs
  // that straddle the tile factor into an in-tile overlap times outside factors)
  int embed_pass = -1;
  for (size_t p = 0; p < P.passes.size(); ++p)
    if (P.passes[p].load_mode == LOAD_EMBED && !P.passes[p].bwd_only) {
      embed_pass = (int)p;
      break;
    }
  if (!leftovers.empty() && embed_pass >= 0 && P.nv > P.passes[embed_pass].K) {
    for (int w : leftovers) {
      const int b = n - 1 - w;
      const auto &tl = P.passes[embed_pass].tile;
      if (std::find(tl.begin(), tl.end(), b) != tl.end())
        P.passes[embed_pass].grad_wires.push_back(w);
      else
        P.passes[embed_pass].outside_wires.push_back(w);
    }
    leftovers.clear();
  }
  // gradient-only passes for whatever is left, prepended (they run last in the backward sweep)
  if (!leftovers.empty()) {
    const int K = P.passes.empty() ? std::min(P.nv, KMAX) : P.passes[0].K;
    std::vector<PlanPass> extra;
    std::vector<int> bits;
    for (int w : leftovers) bits.push_back(n - 1 - w);
    std::sort(bits.begin(), bits.end());
    size_t k = 0;
    while (k < bits.size()) {
      PlanPass pp;
      pp.K = K;
      pp.bwd_only = true;
      uint32_t T = 0;
      std::vector<int> ws;
      // keep low coalescing bits, then as many leftover bits as fit
      const int c = std::min(4, K);
      for (int b = 0; b < c && b < n; ++b) T |= 1u << b;
      while (k < bits.size() && (popc(T | (1u << bits[k])) <= K)) {
        T |= 1u << bits[k];
        ws.push_back(n - 1 - bits[k]);
        ++k;
      }
      for (int b = 0; b < n && popc(T) < K; ++b) T |= 1u << b;
      for (int b = 0; b < n; ++b)
        if ((T >> b) & 1) pp.tile.push_back(b);
      pp.grad_wires = ws;
      extra.push_back(pp);
    }
    P.passes.insert(P.passes.begin(), extra.begin(), extra.end());
  }

  // ---- per pass ----
  for (size_t p = 0; p < P.passes.size(); ++p) {
    PlanPass &pp = P.passes[p];
    const int K = pp.K;
    E.K = K;
    DevPass d;
    std::memset(&d, 0, sizeof d);
    d.K = K;
    d.n = n;
    d.nv = P.nv;
    const bool multi = P.nv < K;
    d.spw_log = multi ? K - P.nv : 0;
    d.tiles_log = multi ? 0 : P.nv - K;
    std::map<int, int> tix;
    for (int t = 0; t < K; ++t) {
      const int b = t < (int)pp.tile.size() ? pp.tile[t] : t;   // multi: sample bits above nv
      d.tpos[t] = b;
      tix[b] = t;
    }
    int nr = 0;
    if (!multi)
      for (int b = 0; b < n; ++b)
        if (!tix.count(b)) d.rest[nr++] = b;
    d.has_load_map = pp.has_load;
    d.has_store_map = pp.has_store;
    if (pp.has_load) {
      for (int t = 0; t < K; ++t) d.load_tcol[t] = pp.load_map.cols[d.tpos[t]];
      for (int r = 0; r < nr; ++r) d.load_rcol[r] = pp.load_map.cols[d.rest[r]];
      d.load_c = pp.load_map.c;
    }
    if (pp.has_store) {
      for (int t = 0; t < K; ++t) d.store_tcol[t] = pp.store_map.cols[d.tpos[t]];
      for (int r = 0; r < nr; ++r) d.store_rcol[r] = pp.store_map.cols[d.rest[r]];
      d.store_c = pp.store_map.c;
    }
    d.load_mode = pp.load_mode;
    d.has_dense = 0;
    d.embed_mat = embed_mat;
    d.embed_per_sample = P.embed_per_sample;
    d.diag_begin = (int)P.ddiag.size();
    d.stage_begin = (int)P.dstage.size();

    // -------- stage list scheduling --------
    const std::vector<int> &po = pp.ops;
    const size_t m = po.size();
    std::vector<char> done(m, 0);
    std::vector<std::vector<int>> deps(m);
    for (size_t j = 0; j < m; ++j)
      for (size_t i = 0; i < j; ++i) {
        const IrOp &a = P.ops[po[i]], &b = P.ops[po[j]];
        if ((a.mask & b.mask) && !(a.kind == IR_DIAG && b.kind == IR_DIAG)) deps[j].push_back((int)i);
      }
    int n_acc = 0;
    std::vector<int> diag_index(P.ops.size(), -1);
    auto tile_bits_of = [&](const IrOp &op) {
      std::vector<int> v;
      if (op.kind == IR_U1 || op.kind == IR_GRAD1) v.push_back(tix.at(op.bits[0]));
      if (op.kind == IR_U2 || op.kind == IR_GRAD2) {
        v.push_back(tix.at(op.bits[0]));
        v.push_back(tix.at(op.bits[1]));
      }
      return v;
    };
    const int reg_limit = multi ? P.nv : K;   // register bits must be state bits
    auto pad_regs = [&](std::vector<int> &S, const std::vector<int> &prefer) {
      for (int b : prefer)
        if ((int)S.size() < RB && std::find(S.begin(), S.end(), b) == S.end()) S.push_back(b);
      for (int b = 0; b < reg_limit && (int)S.size() < RB; ++b)
        if (std::find(S.begin(), S.end(), b) == S.end()) S.push_back(b);
    };
    std::vector<int> prev_regs;
    std::string emit_error;
    size_t n_done = 0;
    auto emit_op = [&](const IrOp &op, int oi_ir, const std::vector<int> &S) {
      DevOp o;
      std::memset(&o, 0, sizeof o);
      o.acc = -1;
      auto ridx = [&](int tb) {
        for (int k = 0; k < RB; ++k)
          if (S[k] == tb) return k;
        return -1;
      };
      if (op.kind == IR_U1) {
        o.kind = OP_U1;
        o.r0 = ridx(tix.at(op.bits[0]));
        o.mat = op_mat[oi_ir];
        o.flags = (op.real ? F_REAL : 0) | (op.per_sample ? F_PERSAMPLE : 0) | (op.diagonal ? F_DIAGONAL : 0);
        if (P.opts.fhwt && op.factors.size() == 1 && P.factors[op.factors[0]].gate == H) o.flags |= F_HADAMARD;
        if (op.has_grad) {
          o.flags |= F_GRAD;
          o.acc = n_acc;
          E.u1_contribs(op.factors, P.n_acc + n_acc);
          n_acc += 3;
        }
      } else if (op.kind == IR_U2) {
        o.kind = OP_U2;
        o.r0 = ridx(tix.at(op.bits[0]));
        o.r1 = ridx(tix.at(op.bits[1]));
        o.mat = op_mat[oi_ir];
        o.flags = (op.per_sample ? F_PERSAMPLE : 0);
        {
          const int g = P.factors[op.factors[0]].gate;
          o.sub = g == CNOT ? U2_CNOT : g == SWAP ? U2_SWAP : g == CZ ? U2_CZ : g == MS ? U2_MS
                : g == ECR ? U2_ECR : g == ZZ ? U2_DIAG : U2_GEN;
        }
        if (op.has_grad) {
          const Factor &f = P.factors[op.factors[0]];
          o.flags |= F_GRAD;
          o.acc = n_acc;
          o.aux = (f.gate == MS) ? (1 | (1 << 2)) : (3 | (3 << 2));   // XX or ZZ
          const bool ps = f.src == SRC_INPUT;
          const int co = E.alloc_dbl(ps, 1);
          const int sl = E.factors_slice(op.factors);
          E.prep(PREP_COEF2, ps, co, sl, sl + 1, sl);
          E.contrib(f, P.n_acc + n_acc, 1, co, ps);
          n_acc += 1;
        }
      } else if (op.kind == IR_DIAG) {
        o.kind = OP_DIAG;
        if (diag_index[oi_ir] < 0) {
          DevDiag dg;
          std::memset(&dg, 0, sizeof dg);
          dg.h = K / 2;
          dg.term_begin = (int)P.dterm.size();
          std::vector<int> extra;
          for (size_t ti = 0; ti < op.terms.size(); ++ti) {
            const IrTerm &t = op.terms[ti];
            DevTerm dt;
            std::memset(&dt, 0, sizeof dt);
            dt.nbits = t.nbits;
            dt.acc = -1;
            bool low = false, high = false;
            for (int q = 0; q < 2; ++q) {
              dt.tb[q] = -1;
              dt.gb[q] = -1;
            }
            for (int q = 0; q < t.nbits; ++q) {
              dt.gb[q] = t.bits[q];
              if (tix.count(t.bits[q])) {
                dt.tb[q] = tix.at(t.bits[q]);
                if (dt.tb[q] < dg.h) low = true;
                else high = true;
              }
            }
            dt.tab = low ? 0 : (high ? 1 : 2);
            if (low)
              for (int q = 0; q < t.nbits; ++q)
                if (dt.tb[q] >= dg.h && std::find(extra.begin(), extra.end(), dt.tb[q]) == extra.end())
                  extra.push_back(dt.tb[q]);
            const Factor &f = P.factors[t.factor];
            dt.per_sample = f.src == SRC_INPUT;
            dt.ang = term_ang[oi_ir][ti];
            if (is_param(f.gate) && f.src != SRC_FIXED) {
              dt.acc = n_acc;
              const bool ps = f.src == SRC_INPUT;
              const int co = E.alloc_dbl(ps, 1);
              const int sl = E.factors_slice({t.factor});
              E.prep(PREP_COEFD, ps, co, sl, sl + 1, sl);
              E.contrib(f, P.n_acc + n_acc, 1, co, ps);
              ++n_acc;
            }
            P.dterm.push_back(dt);
          }
          dg.term_end = (int)P.dterm.size();
          if ((int)extra.size() > MAX_DIAG_EXTRA) {
            emit_error = "EUNSUPPORTED: diagonal layer couples too many tile halves";
            return;
          }
          dg.n_extra = (int)extra.size();
          for (size_t k = 0; k < extra.size() && k < (size_t)MAX_DIAG_EXTRA; ++k) dg.extra[k] = extra[k];
          dg.lds_off = d.diag_lds;
          const int entries = (1 << (dg.h + dg.n_extra)) + (1 << (K - dg.h));
          d.diag_lds += entries;
          dg.gtab = -1;
          if (!op.per_sample) {
            // angles shared by every sample: tables built once per call for
            // each tile position of the pass
            const int tiles_log = P.nv > K ? P.nv - K : 0;
            dg.gtab = (int)P.n_diag_tab;
            P.n_diag_tab += (long long)entries << tiles_log;
            DiagJob j;
            j.pass = (int)P.dpass.size();
            j.diag = (int)P.ddiag.size();
            j.tiles_log = tiles_log;
            j.entries = entries;
            P.diag_jobs.push_back(j);
          }
          diag_index[oi_ir] = (int)P.ddiag.size() - d.diag_begin;
          P.ddiag.push_back(dg);
          d.n_diag++;
        }
        o.aux = diag_index[oi_ir];
        o.flags = op.has_grad ? F_GRAD : 0;
        // per-stage gradient entries of the terms that have parameters
        o.mat = (int)P.dtgrad.size();
        o.r1 = 0;
        {
          const DevDiag &dg = P.ddiag[d.diag_begin + o.aux];
          for (int ti = dg.term_begin; ti < dg.term_end; ++ti) {
            const DevTerm &dt = P.dterm[ti];
            if (dt.acc < 0) continue;
            DevTermGrad g;
            g.acc = dt.acc;
            g.m = 0;
            g.tmask = g.gmask = 0;
            for (int q = 0; q < dt.nbits; ++q) {
              if (dt.tb[q] < 0) {
                g.gmask |= 1u << dt.gb[q];
              } else {
                const int rk = ridx(dt.tb[q]);
                if (rk >= 0)
                  g.m |= 1 << rk;
                else
                  g.tmask |= 1u << dt.tb[q];
              }
            }
            P.dtgrad.push_back(g);
            ++o.r1;
          }
        }
      } else if (op.kind == IR_DENSE) {
        o.kind = OP_DENSE;
        o.mat = op_mat[oi_ir];
        d.has_dense = 1;
      } else if (op.kind == IR_GRAD1) {
        o.kind = OP_GRAD1;
        o.r0 = ridx(tix.at(op.bits[0]));
        o.flags = F_GRAD;
        o.mat = 0;
        o.acc = n_acc;
        E.u1_contribs(op.factors, P.n_acc + n_acc);
        n_acc += 3;
      } else if (op.kind == IR_GRAD2) {
        const Factor &f = P.factors[op.factors[0]];
        o.kind = OP_GRAD2;
        o.r0 = ridx(tix.at(op.bits[0]));
        o.r1 = ridx(tix.at(op.bits[1]));
        o.flags = F_GRAD;
        o.acc = n_acc;
        o.aux = (f.gate == MS) ? (1 | (1 << 2)) : (3 | (3 << 2));
        const int co = E.alloc_dbl(false, 1);
        const int sl = E.factors_slice(op.factors);
        E.prep(PREP_COEF2, false, co, sl, sl + 1, sl);
        E.contrib(f, P.n_acc + n_acc, 1, co, false);
        n_acc += 1;
      } else if (op.kind == IR_PERM) {
        o.kind = OP_PERM;
        DevPerm pm;
        std::memset(&pm, 0, sizeof pm);
        const GF2 G = op.F.inverse();   // gather: new[t] = old[G(t)]
        for (int t = 0; t < K; ++t) pm.cols[t] = (t < n) ? G.cols[t] : (1u << t);
        pm.cxor = G.c;
        o.aux = (int)P.dperm.size();
        P.dperm.push_back(pm);
      }
      P.dop.push_back(o);
    };

    while (n_done < m) {
      std::vector<int> S;
      DevStage st;
      std::memset(&st, 0, sizeof st);
      st.op_begin = (int)P.dop.size();
      std::vector<int> stage_ops;
      bool perm_stage = false;
      bool progress = true;
      while (progress && !perm_stage) {
        progress = false;
        for (size_t j = 0; j < m; ++j) {
          if (done[j]) continue;
          bool ready = true;
          for (int i : deps[j])
            if (!done[i]) ready = false;
          if (!ready) continue;
          const IrOp &op = P.ops[po[j]];
          if (op.kind == IR_PERM || op.kind == IR_DENSE) {
            if (stage_ops.empty()) {
              stage_ops.push_back((int)j);
              done[j] = 1;
              perm_stage = true;
              progress = true;
            }
            break;
          }
          if (op.kind == IR_DIAG) {
            stage_ops.push_back((int)j);
            done[j] = 1;
            progress = true;
            continue;
          }
          std::vector<int> tb = tile_bits_of(op);
          std::vector<int> U = S;
          for (int b : tb)
            if (std::find(U.begin(), U.end(), b) == U.end()) U.push_back(b);
          if ((int)U.size() <= RB) {
            S = U;
            stage_ops.push_back((int)j);
            done[j] = 1;
            progress = true;
          }
        }
      }
      if (stage_ops.empty()) return "internal: stage scheduler stalled";
      if (perm_stage) {
        S = prev_regs.empty() ? std::vector<int>() : prev_regs;
      }
      pad_regs(S, prev_regs);
      for (int k = 0; k < RB; ++k) st.rbits[k] = S[k];
      for (int j : stage_ops) emit_op(P.ops[po[j]], po[j], S);
      if (!emit_error.empty()) return emit_error;
      group_wht(P, st.op_begin);
      group_u1(P, st.op_begin);
      group_u2(P, st.op_begin);
      group_seq(P, st.op_begin);
      st.op_end = (int)P.dop.size();
      P.dstage.push_back(st);
      prev_regs = S;
      n_done += stage_ops.size();
    }
    d.n_stages = (int)P.dstage.size() - d.stage_begin;
    if ((int)m > MAX_OPS || d.n_stages > MAX_STAGES * 4) return "EUNSUPPORTED: pass too large";

    // -------- embed-gradient tail stages --------
    d.grad_stage_begin = (int)P.dstage.size();
    {
      std::vector<int> gb;
      for (int w : pp.grad_wires) gb.push_back(tix.at(n - 1 - w));
      size_t k = 0;
      while (k < gb.size()) {
        std::vector<int> S;
        std::vector<int> ws;
        while (k < gb.size() && (int)S.size() < RB) {
          S.push_back(gb[k]);
          ws.push_back(pp.grad_wires[k]);
          ++k;
        }
        pad_regs(S, {});
        DevStage st;
        std::memset(&st, 0, sizeof st);
        for (int q = 0; q < RB; ++q) st.rbits[q] = S[q];
        st.op_begin = (int)P.dop.size();
        for (size_t q = 0; q < ws.size(); ++q) {
          DevOp o;
          std::memset(&o, 0, sizeof o);
          o.kind = OP_GRAD1;
          o.r0 = (int)q;
          o.flags = F_GRAD | (P.embed_per_sample ? F_PERSAMPLE : 0);
          o.mat = embed_mat + 4 * ws[q];
          o.acc = n_acc;
          E.u1_contribs(P.embed[ws[q]], P.n_acc + n_acc);
          n_acc += 3;
          P.dop.push_back(o);
        }
        st.op_end = (int)P.dop.size();
        P.dstage.push_back(st);
      }
    }
    d.n_grad_stages = (int)P.dstage.size() - d.grad_stage_begin;
    // environment embed gradients (X, Y, Z sums per outside bit, ascending bit order)
    d.outside_mask = 0;
    d.outside_acc = -1;
    if (!pp.outside_wires.empty()) {
      std::vector<int> ob;
      for (int w : pp.outside_wires) ob.push_back(n - 1 - w);
      std::sort(ob.begin(), ob.end());
      d.outside_acc = n_acc;
      for (int b : ob) {
        d.outside_mask |= 1u << b;
        E.u1_contribs(P.embed[n - 1 - b], P.n_acc + n_acc);
        n_acc += 3;
      }
    }
    d.n_acc = n_acc;
    // units per sample of this pass's partials
    int units;
    if (!multi) {
      units = (1 << (P.nv - K)) * (1 << (K - RB - 6));
    } else {
      const int tps = P.nv - RB;
      const int sl = tps < 6 ? tps : 6;
      units = 1 << (tps - sl);
    }
    P.pass_units.push_back(units);
    P.pass_prefix.push_back(E.acc_prefix);
    for (int a = 0; a < n_acc; ++a) {
      P.acc_static.push_back(E.acc_prefix + (long long)a * units);
      P.acc_units.push_back(units);
    }
    E.acc_prefix += (long long)n_acc * units;
    P.n_acc += n_acc;
    P.dpass.push_back(d);
  }
  P.units_total = E.acc_prefix;
  // eight inert entries after the diagonal-term gradients: a pass reads term
  // descriptors eight at a time without bounds tests
  for (int q = 0; q < 8; ++q) {
    DevTermGrad g;
    std::memset(&g, 0, sizeof g);
    g.acc = -1;
    P.dtgrad.push_back(g);
  }
  for (DevStage &st : P.dstage) {
    for (int k = 0; k < RB; ++k) st.rsorted[k] = st.rbits[k];
    std::sort(st.rsorted, st.rsorted + RB);
    bool grad_only = st.op_end > st.op_begin;
    for (int o = st.op_begin; o < st.op_end; ++o)
      grad_only = grad_only && (P.dop[o].kind == OP_GRAD1 || P.dop[o].kind == OP_GRAD2);
    st.flags = grad_only ? STAGE_GRAD_ONLY : 0;
  }
  // forward: distance to the next stage that changes the state
  for (const DevPass &d : P.dpass)
    for (int si = d.stage_begin; si < d.stage_begin + d.n_stages; ++si) {
      int k = si + 1;
      while (k < d.stage_begin + d.n_stages && (P.dstage[k].flags & STAGE_GRAD_ONLY)) ++k;
      P.dstage[si].fwd_next = k - si;
    }
  // full-layer matrix ops name the matrix of the pass's next one in either
  // direction, so that a pass fetches it while the current one runs
  for (DevPass &d : P.dpass) {
    d.dense_first_mat[0] = d.dense_first_mat[1] = -1;
    std::vector<int> dops;
    for (int si = d.stage_begin; si < d.stage_begin + d.n_stages; ++si)
      for (int o = P.dstage[si].op_begin; o < P.dstage[si].op_end; ++o)
        if (P.dop[o].kind == OP_DENSE) dops.push_back(o);
    for (size_t k = 0; k < dops.size(); ++k) {
      DevStage *st = nullptr;
      for (int si = d.stage_begin; si < d.stage_begin + d.n_stages; ++si)
        if (P.dstage[si].op_begin == dops[k]) st = &P.dstage[si];
      if (!st) return "internal: a full-layer matrix op must open its stage";
      st->flags |= STAGE_DENSE;
      st->dense_next[0] = k + 1 < dops.size() ? P.dop[dops[k + 1]].mat : -1;
      st->dense_next[1] = k > 0 ? P.dop[dops[k - 1]].mat : -1;
    }
    if (!dops.empty()) {
      d.dense_first_mat[0] = P.dop[dops.front()].mat;
      d.dense_first_mat[1] = P.dop[dops.back()].mat;
    }
  }

  // backward of the first forward pass need not store unless gradient-only passes follow
  {
    int first_fwd = -1;
    bool bwd_only_exist = false;
    for (size_t p = 0; p < P.passes.size(); ++p) {
      if (P.passes[p].bwd_only) bwd_only_exist = true;
      else if (first_fwd < 0) first_fwd = (int)p;
    }
    if (first_fwd >= 0 && !bwd_only_exist) P.dpass[first_fwd].skip_bwd_store = 1;
  }
  // ping-pong requirements
  P.any_oop = false;
  for (auto &pp : P.passes)
    if (pp.has_load || pp.has_store) P.any_oop = true;

  // prep factors table
  P.factors = E.pf;   // prep items index this contiguous table from now on
  // gradient CSR: weights then features
  P.cptr.assign(P.n_weights + P.n_features + 1, 0);
  std::vector<std::vector<Contrib>> lists(P.n_weights + P.n_features);
  for (auto &kv : E.by_param) {
    const int src = kv.first.first, idx = kv.first.second;
    const int pid = src == SRC_WEIGHT ? idx : P.n_weights + idx;
    if (pid < 0 || pid >= (int)lists.size()) continue;
    for (auto &c : kv.second) lists[pid].push_back(c);
  }
  for (size_t i = 0; i < lists.size(); ++i) {
    P.cptr[i + 1] = P.cptr[i] + (int)lists[i].size();
    for (auto &c : lists[i]) P.contribs.push_back(c);
  }
  return "";
}

std::string build_plan(Plan &P, int n, const LayerSpec *layers, int n_layers, int dtype,
                       const PlanOptions &opts) {
  std::string err = validate_layers(n, layers, n_layers, &P.n_weights, &P.n_features);
  if (!err.empty()) return err;
  P.opts = opts;
  const int mode = opts.mode, tile_bits = opts.tile_bits;
  P.n = n;
  P.nv = std::max(n, RB);
  P.dtype = dtype;
  P.mode = mode == 0 ? 2 : mode;
  const bool want_dense = (P.mode == 3) || (mode == 0 && n <= DENSE_AUTO_MAX_QUBITS);
  if (P.mode == 3) P.mode = 2;
  P.tile_bits = tile_bits;
  const int kdef = dtype == 0 ? 12 : 11;
  int K = tile_bits ? tile_bits : kdef;
  if (dtype == 1 && K > 11) K = 11;
  P.resident = P.nv <= K;
  if (P.resident) K = std::max(P.nv, KMIN);
  // full layer unitaries need the whole state of a sample in the tile and at
  // least 16 samples per workgroup (one MFMA column block)
  P.dense = want_dense && P.resident && P.nv <= DENSE_MAX_QUBITS && K - P.nv >= 4;
  P.factors.clear();
  P.ops.clear();
  std::vector<Inst> insts = expand(n, layers, n_layers, opts.hrz != 0);
  err = build_ir(P, insts);
  if (!err.empty()) return err;
  err = schedule(P, K);
  if (!err.empty()) return err;
  if (P.passes.empty()) {
    PlanPass pp;
    pp.K = K;
    for (int b = 0; b < std::min(P.nv, K); ++b) pp.tile.push_back(b);
    pp.load_mode = LOAD_EMBED;
    P.passes.push_back(pp);
  }
  return emit(P);
}

// Parameters read by an IR op (weights or features; fixed gates have none).
static int op_params(const Plan &P, const IrOp &op) {
  int k = 0;
  for (int fi : op.factors)
    if (is_param(P.factors[fi].gate) && P.factors[fi].src != SRC_FIXED) ++k;
  for (const IrTerm &t : op.terms)
    if (is_param(P.factors[t.factor].gate) && P.factors[t.factor].src != SRC_FIXED) ++k;
  return k;
}

void pass_flops(const Plan &P, int pass, double *fwd, double *bwd) {
  const PlanPass &pp = P.passes[pass];
  double f = 0.0, g = 0.0;
  for (int oi : pp.ops) {
    const IrOp &op = P.ops[oi];
    double of = 0.0;
    switch (op.kind) {
      case IR_U1:
        if (P.opts.fhwt && op.factors.size() == 1 && P.factors[op.factors[0]].gate == H)
          of = 2.0;   // a complex add or subtract per amplitude (the scale is shared)
        else
          of = op.diagonal ? 6.0 : (op.real ? 8.0 : 16.0);
        break;
      case IR_U2: {
        const int gt = op.factors.empty() ? -1 : P.factors[op.factors[0]].gate;
        if (gt == CNOT || gt == SWAP) of = 0.0;
        else if (gt == CZ) of = 0.5;
        else if (gt == ZZ) of = 6.0;
        else if (gt == MS || gt == ECR) of = 6.0;
        else of = 32.0;
        break;
      }
      case IR_DIAG: of = 6.0; break;
      case IR_DENSE: of = 8.0 * (double)(1 << P.nv); break;
      default: of = 0.0; break;   // permutations, gradient-only sums
    }
    f += of;
    g += 2.0 * of + 2.0 * op_params(P, op);
  }
  // embedding gradients taken at the end of this pass's backward
  for (const std::vector<int> *ws : {&pp.grad_wires, &pp.outside_wires})
    for (int w : *ws)
      for (int fi : P.embed[w])
        if (is_param(P.factors[fi].gate) && P.factors[fi].src != SRC_FIXED) g += 2.0;
  if (fwd) *fwd = f;
  if (bwd) *bwd = g;
}

std::string describe_plan(const Plan &P) {
  std::ostringstream o;
  o << "{\"n\":" << P.n << ",\"dtype\":\"" << (P.dtype ? "c128" : "c64") << "\",\"mode\":\""
    << (P.dense ? "dense" : (P.mode == 1 ? "per_layer" : "fused")) << "\",\"resident\":" << (P.resident ? "true" : "false")
    << ",\"n_weights\":" << P.n_weights << ",\"n_features\":" << P.n_features << ",\"n_ops\":" << P.ops.size()
    << ",\"n_acc\":" << P.n_acc << ",\"hrz\":" << P.opts.hrz << ",\"fhwt\":" << P.opts.fhwt
    << ",\"diag\":\"" << (P.opts.diag ? "einsum" : "tables") << "\",\"passes\":[";
  for (size_t p = 0; p < P.passes.size(); ++p) {
    const PlanPass &pp = P.passes[p];
    const DevPass &d = P.dpass[p];
    int nu1 = 0, nu2 = 0, ndg = 0, npm = 0, ndense = 0, ngrp = 0, nwht = 0;
    for (int s = d.stage_begin; s < d.stage_begin + d.n_stages; ++s)
      for (int oi = P.dstage[s].op_begin; oi < P.dstage[s].op_end; ++oi) {
        const int k = P.dop[oi].kind;
        nu1 += k == OP_U1;
        if (k == OP_U1G) {
          nu1 += __builtin_popcount((unsigned)P.dop[oi].r0);
          ++ngrp;
        }
        if (k == OP_SEQ) {
          const int len = P.dop[oi].r0;
          nu1 += 4 + (len == 4 ? 2 : 0);
          nu2 += 2 + (len >= 3 ? 1 : 0);
          ++ngrp;
        }
        nu2 += (k == OP_U2) + 2 * (k == OP_U2G);
        if (k == OP_WHT) nwht += __builtin_popcount((unsigned)P.dop[oi].r0);
        ndg += k == OP_DIAG;
        npm += k == OP_PERM;
        ndense += k == OP_DENSE;
      }
    o << (p ? "," : "") << "{\"K\":" << pp.K << ",\"tile\":[";
    for (size_t t = 0; t < pp.tile.size(); ++t) o << (t ? "," : "") << pp.tile[t];
    o << "],\"load\":\"" << (pp.load_mode == LOAD_EMBED ? "embed" : (pp.has_load ? "gather" : "tile"))
      << "\",\"store\":\"" << (pp.has_store ? "scatter" : "tile") << "\",\"bwd_only\":"
      << (pp.bwd_only ? "true" : "false") << ",\"stages\":" << d.n_stages << ",\"u1\":" << nu1
      << ",\"u1_groups\":" << ngrp << ",\"u2\":" << nu2 << ",\"diag\":" << ndg << ",\"perm\":" << npm
      << ",\"dense\":" << ndense << ",\"wht\":" << nwht
      << ",\"grad_wires\":"
      << pp.grad_wires.size() << ",\"outside_wires\":" << pp.outside_wires.size() << ",\"n_acc\":" << d.n_acc;
    double ff = 0, fb = 0;
    pass_flops(P, (int)p, &ff, &fb);
    o << ",\"flops_per_amp_fwd\":" << ff << ",\"flops_per_amp_bwd\":" << fb << "}";
  }
  o << "]}";
  return o.str();
}

}  // namespace tqs
