// Host-side circuit compiler: layer list -> ops -> passes -> device tables.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"

namespace tqs {

// GF(2)-affine map on n-bit state indices: y = A x ^ c, cols[i] = A e_i.
struct GF2 {
  int n = 0;
  uint32_t cols[NQMAX] = {};
  uint32_t c = 0;
  static GF2 identity(int n);
  uint32_t apply(uint32_t x) const;
  GF2 after(const GF2 &first) const;   // (*this) o first
  GF2 inverse() const;
  bool is_identity() const;
};

enum IrKind { IR_U1 = 1, IR_U2 = 2, IR_DIAG = 3, IR_PERM = 4, IR_DENSE = 5, IR_GRAD1 = 6, IR_GRAD2 = 7 };

struct IrTerm {
  int factor;
  int nbits;
  int bits[2];   // state bits, first = more significant matrix bit
};

struct IrOp {
  int kind = 0;
  int bits[2] = {-1, -1};          // U1: bits[0]; U2: (first wire's bit, second wire's bit)
  std::vector<int> factors;        // U1: factors in application order; U2: one factor
  std::vector<IrTerm> terms;       // DIAG
  GF2 F;                           // PERM: forward basis map (amplitude at j moves to F(j))
  uint32_t mask = 0;               // state bits touched
  bool per_sample = false;
  bool real = false, diagonal = false;
  bool has_grad = false;
};

struct LayerSpec {
  int gate, pattern, source, wire, wire2, offset;
  double fixed, fixed2, fixed3;   // fixed2/3: MS phases (phi0, phi1); FIXED Rot's phi, lambda
};

// Dispatcher choices that change the plan.
struct PlanOptions {
  int mode = 0;          // 0 auto, 1 per-layer passes, 2 fused passes, 3 dense
  int tile_bits = 0;     // 0 auto, else K
  int hrz = 0;           // 1: H-Rz expansion of RX, RY, GPI2 and Rot layers (Sec. 2.5)
  int fhwt = 1;          // 1: Hadamard layers as add/subtract butterflies (fast Walsh-Hadamard)
  int diag = 0;          // 0: diagonal layers by split eigenphase tables (Secs. 2.4.1-2.4.2);
                         // 1: gate by gate, one diagonal factor per gate (diagonal Einsum, Sec. 2.4.3)
};

struct PlanPass {
  int K = 12;
  std::vector<int> tile;           // tile bits -> state bits (ascending)
  std::vector<int> ops;            // IR op indices placed in this pass, in placement order
  int load_mode = LOAD_GLOBAL;
  bool has_load = false, has_store = false;
  GF2 load_map, store_map;         // gather (src = load_map(k)), scatter (dst = store_map(k))
  bool bwd_only = false;           // gradient-only pass (embed gradients)
  std::vector<int> grad_wires;     // embed gradient wires handled at the end of this pass's backward
  std::vector<int> outside_wires;  // embedding pass: embed gradients of wires outside its tile
};

struct Plan {
  // configuration
  int n = 0, nv = 0, dtype = 0, mode = 0, tile_bits = 0;
  PlanOptions opts;
  bool dense = false;                    // weight-only layers applied as full unitaries (MFMA)
  int n_weights = 0, n_features = 0;
  bool resident = false;
  // IR
  std::vector<Factor> factors;
  std::vector<std::vector<int>> embed;   // per wire: factor ids of the embedded 1q chain
  bool embed_per_sample = false;
  std::vector<IrOp> ops;
  std::vector<PlanPass> passes;
  // device tables
  std::vector<DevPass> dpass;
  std::vector<DevStage> dstage;
  std::vector<DevOp> dop;
  std::vector<DevDiag> ddiag;
  std::vector<DiagJob> diag_jobs;        // shared diagonal ops whose tables are prebuilt per call
  long long n_diag_tab = 0;              // complex elements of the prebuilt tables
  std::vector<DevTerm> dterm;
  std::vector<DevTermGrad> dtgrad;
  std::vector<DevPerm> dperm;
  std::vector<DevGroup> dgroup;
  std::vector<DevSeq> dseq;
  std::vector<PrepItem> prep;
  std::vector<Contrib> contribs;
  std::vector<int> cptr;                 // CSR over params: weights then features
  std::vector<long long> acc_static;     // per global accumulator: region/B
  std::vector<int> acc_units;            // per global accumulator
  std::vector<long long> pass_prefix;    // per pass: accumulator prefix (units, times B at run time)
  std::vector<int> pass_units;
  int n_acc = 0;
  int n_mats = 0, n_mats_ps = 0, n_dbl = 0, n_dbl_ps = 0;
  long long units_total = 0;             // sum over accumulators of units per sample
  bool any_oop = false;                  // some pass needs a ping-pong buffer
  std::vector<int> fwd_oop, bwd_oop;     // per pass
  int first_fwd_writes_x = 0;            // first forward pass writes the workspace buffer
};

// Validates the layer list (returns a message starting with "EINVAL:" or
// "EUNSUPPORTED:" on failure) and fills n_weights / n_features.
std::string validate_layers(int n, const LayerSpec *layers, int n_layers, int *n_weights,
                            int *n_features);

// Builds the plan; returns an empty string on success or an error message.
std::string build_plan(Plan &P, int n, const LayerSpec *layers, int n_layers, int dtype,
                       const PlanOptions &opts);

std::string describe_plan(const Plan &P);

// Algorithmic flops per amplitude of pass `pass`, forward and backward: a
// complex 2x2 16, a real 2x2 8, a diagonal layer (one phase multiply) 6, MS and
// ECR 6 (their structured form), CZ 0.5, CNOT / SWAP / permutations 0, a general
// 4x4 32, a full-layer unitary 8 * 2^nv; the backward is twice the forward
// (psi and lambda are both uncomputed) plus one multiply-add (2 flops) per
// parameter, embedding gradients included.  This is the arithmetic the
// method needs, not the instructions issued.
void pass_flops(const Plan &P, int pass, double *fwd, double *bwd);

}  // namespace tqs
