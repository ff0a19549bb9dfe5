// Execution-plan structures shared by the host planner and the gfx950 kernels.
//
// A circuit (ordered list of uniform gate layers, Sec. 1 / Fig. 6 of the paper)
// is compiled into a list of *passes*.  A pass streams the batched state once
// through HBM: every workgroup loads one tile of 2^K amplitudes whose index
// bits are a chosen set of K bit positions (the other bits -- and the batch
// index -- select the tile), applies a sequence of *stages* to it in LDS and
// registers, and stores it back.  Within a stage every thread holds 2^RB
// amplitudes that differ in RB chosen tile bits ("register bits"), so gates on
// those bits are applied in registers (the Kronecker / Einsum structure of
// Sec. 2.2.2); diagonal layers are applied through split phase tables (the
// diagonal tensor product of Sec. 2.4.2); permutation layers (Sec. 2.3) become
// GF(2)-affine index maps folded into a pass's load or store.
#pragma once
#include <stdint.h>

namespace tqs {

constexpr int RB = 4;                 // register bits per stage
constexpr int NREG = 1 << RB;         // amplitudes per thread per stage
constexpr int KMIN = 10;              // smallest tile (64 threads)
constexpr int KMAX = 12;              // largest tile (256 threads)
constexpr int DENSE_SUBS = 4;         // waves per tile (each with a copy of the tile) in passes with full-layer matrix ops
constexpr int NQMAX = 30;             // largest qubit count
constexpr int MAX_STAGES = 48;        // per pass
constexpr int MAX_OPS = 512;          // per pass
constexpr int MAX_DIAG_EXTRA = 3;     // extra index bits of a split diagonal table
constexpr int MAX_DIAG_OPS = 4;       // diagonal ops with tables per pass

constexpr int32_t STAGE_GRAD_ONLY = 1;
constexpr int32_t STAGE_DENSE = 2;

enum OpKind : int32_t {
  OP_U1 = 1,     // 2x2 on register bit r0
  OP_U2 = 2,     // 4x4 on register bits (r0 = more significant matrix bit, r1)
  OP_DIAG = 3,   // diagonal phase from split tables (any tile / base bits)
  OP_GRAD1 = 4,  // gradient-only Pauli sums on register bit r0 (no gate)
  OP_PERM = 5,   // in-tile GF(2)-affine permutation (resident passes only)
  OP_DENSE = 6,  // full 2^nv x 2^nv layer unitary on every sample of the tile (MFMA)
  OP_GRAD2 = 7,  // gradient-only Pauli-pair sum on register bits (r0, r1) (no gate)
  OP_U1G = 8,    // complex 2x2 gates on several register bits at once: r0 = bit mask,
                 // aux = DevGroup index (the gates act on distinct bits, so they commute)
  OP_U2G = 9,    // two structured 4x4 gates of one kind (sub) on disjoint register-bit
                 // pairs: r0 = a<<6 | b<<4 | c<<2 | d for pairs (a,b), (c,d); aux = DevGroup
  OP_WHT = 11,   // Hadamard gates on the register bits of mask r0, applied as the
                 // fast Walsh-Hadamard transform: add / subtract butterflies, one scale
  OP_SEQ = 10,   // the brick-layer stage program, one op: pair gates of kind `sub` on
                 // register pairs (0,1),(2,3); 2x2 gates on bits 0-3; then (r0 >= 3) a pair
                 // gate on (1,2); then (r0 == 4) 2x2 gates on bits 1, 2.  r0 = program
                 // length (2..4), aux = DevSeq index
};

enum OpFlag : int32_t {
  F_REAL = 1,        // matrix is real
  F_PERSAMPLE = 2,   // matrix / angles differ per sample
  F_GRAD = 4,        // op carries gradient accumulators
  F_DIAGONAL = 8,    // U1/U2 matrix is diagonal
  F_HADAMARD = 16,   // U1 matrix is the Hadamard gate (no parameter)
};

// Structure of a 4x4 op, chosen by the planner from the gate.
enum U2Kind : int32_t {
  U2_GEN = 0,    // dense complex 4x4
  U2_CNOT = 1,   // swap |10> <-> |11>
  U2_SWAP = 2,   // swap |01> <-> |10>
  U2_CZ = 3,     // negate |11>
  U2_MS = 4,     // cos(pi t) I - i sin(pi t) X(x)X
  U2_ECR = 5,    // (I(x)X - X(x)Y) / sqrt(2)
  U2_DIAG = 6,   // diagonal
};

struct DevOp {
  int32_t kind;
  int32_t flags;
  int32_t r0, r1;    // register-bit indices (0..RB-1)
  int32_t mat;       // matrix offset in complex elements (U1: 4, U2: 16 entries)
  int32_t acc;       // first gradient accumulator of the pass, -1 if none
  int32_t aux;       // U2 grad: Pauli code pa | pb<<2 (1=X,2=Y,3=Z); DIAG: diag index; PERM: perm index
  int32_t sub;       // U2: U2Kind
};

struct DevStage {
  int32_t rbits[RB];   // tile-bit index held by each register bit
  int32_t op_begin, op_end;
  int32_t rsorted[RB]; // the same tile bits in increasing order
  int32_t flags;       // STAGE_GRAD_ONLY: every op only takes gradient sums; STAGE_DENSE: a full-layer matrix op
  int32_t dense_next[2];   // STAGE_DENSE: matrix of the pass's next such op forward [0] / backward [1], -1 if none
  int32_t fwd_next;        // stages to the next one the forward runs (gradient-only stages skipped)
};

// One diagonal op's tables: TL indexed by (tile bits 0..h-1, extra bits),
// TH by tile bits h..K-1.  Tables of ops whose angles are shared by every
// sample are built once per call for every tile position of the pass
// (k_diag_tables) and copied to LDS; ops with per-sample angles are built per
// workgroup from the term list.
struct DevDiag {
  int32_t term_begin, term_end;
  int32_t h;                        // split point in tile bits
  int32_t n_extra;
  int32_t extra[MAX_DIAG_EXTRA];    // tile-bit indices (>= h) appended to TL's index
  int32_t lds_off;                  // table offset in the diag-table LDS area (complex elements)
  int32_t gtab;                     // shared ops: offset of tile 0's tables in the prebuilt table
                                    // area (complex elements), TL then TH per tile; -1 otherwise
  int32_t pad[3];
};

// One shared diagonal op whose tables k_diag_tables builds: its pass, its
// index in the diagonal table, and the number of tile positions (log2).
struct DiagJob {
  int32_t pass, diag, tiles_log, entries;
};

// Diagonal term: phase e^{i phi(v)} with v = bit values (first bit more significant).
struct DevTerm {
  int32_t nbits;          // 1 or 2
  int32_t tb[2];          // tile-bit index, or -1 when the bit is a base (non-tile) bit
  int32_t gb[2];          // global bit position of each term bit
  int32_t ang;            // offset of 2^nbits angles (FP64) in the angle table
  int32_t per_sample;
  int32_t acc;            // accumulators: P_a, P_b, P_ab (2-bit) or P_a (1-bit); -1 none
  int32_t tab;            // 0: TL, 1: TH, 2: constant
};

// Gradient of one diagonal term as its op runs in one stage: the accumulator,
// the term's in-register bits as a register-bit pattern m (the index of its
// parity sum in the Walsh-Hadamard transform of the thread's 16 values), and
// the masks whose parities give the sign: tile bits held by the thread index
// (tmask, tile-bit positions) and bits outside the tile (gmask, state-index
// bits).  An OP_DIAG op with gradients lists its terms' entries from index
// mat, r1 of them.
struct DevTermGrad {
  int32_t acc, m;
  uint32_t tmask, gmask;
};

// Members of an OP_U1G group, by register bit: matrix offset and first gradient
// accumulator (3 per gate: the X, Y, Z Pauli sums), -1 when the bit has no gate
// or the gate no parameter.  OP_U2G uses slots 0 and 1 for its two pairs (one
// accumulator per gate).
struct DevGroup {
  int32_t mat[RB];
  int32_t acc[RB];
};

// Members of an OP_SEQ op: slots 0-1 the pair gates on (0,1), (2,3); 2-5 the
// 2x2 gates on bits 0-3; 6 the pair gate on (1,2); 7-8 the 2x2 gates on bits
// 1, 2.  Matrix offset and first gradient accumulator (-1: none).
constexpr int SEQ_SLOTS = 9;
struct DevSeq {
  int32_t mat[SEQ_SLOTS];
  int32_t acc[SEQ_SLOTS];
};

// In-tile permutation: dst tile index t takes src = xor of cols[i] over set bits i of t, ^ cxor.
struct DevPerm {
  uint32_t cols[KMAX];
  uint32_t cxor;
  int32_t pad[3];
};

enum LoadMode : int32_t { LOAD_GLOBAL = 0, LOAD_EMBED = 1, LOAD_NONE = 2 };

struct DevPass {
  int32_t K;                 // tile bits
  int32_t n;                 // qubits
  int32_t nv;                // qubits of the tile layout: max(n, RB); extra wires stay |0>
  int32_t spw_log;           // log2 samples per workgroup (K - n when n < K, else 0)
  int32_t tiles_log;         // log2 tiles per sample (n - K when n >= K, else 0)
  int32_t tpos[KMAX];        // global bit of each tile bit (state bits only; batch bits when spw_log>0)
  int32_t rest[NQMAX];       // global bits not in the tile, ascending (n-K of them)
  // GF(2)-affine maps on the state index: forward load gathers src = M(k)^c,
  // forward store scatters dst = M(k)^c.  Columns per tile bit and per rest bit.
  int32_t has_load_map, has_store_map;
  uint32_t load_tcol[KMAX], load_rcol[NQMAX], load_c;
  uint32_t store_tcol[KMAX], store_rcol[NQMAX], store_c;
  int32_t load_mode;         // forward: LOAD_GLOBAL / LOAD_EMBED
  int32_t embed_mat;         // embed: per-wire 2x2 matrices (column 0 is the wire state)
  int32_t embed_per_sample;
  int32_t n_stages;
  int32_t stage_begin;       // index into the stage table
  int32_t n_diag, diag_begin;
  int32_t n_acc;             // gradient accumulators of this pass
  int32_t acc_region;        // offset of this pass's partials (doubles)
  int32_t grad_stage_begin, n_grad_stages;   // backward-only tail stages (embed gradients)
  int32_t skip_bwd_store;    // backward of the first pass need not store
  int32_t diag_lds;          // complex elements of diag tables in LDS
  int32_t has_dense;         // 1 if the pass holds full-layer matrix ops (K = 10, DENSE_SUBS waves per tile)
  int32_t dense_first_mat[2];   // matrix of the first full-layer op forward [0] and backward [1], -1 if none
  // embedding pass, backward: state bits outside the tile whose embed gradients are
  // taken from the product-state environment (X, Y, Z sums per bit, ascending),
  // starting at accumulator outside_acc
  uint32_t outside_mask;
  int32_t outside_acc;
};

// Parameter-preparation program (run on the device per call, FP64).
enum PrepKind : int32_t {
  PREP_MAT1 = 1,    // product of 2x2 factors -> 2x2 matrix (dtype)
  PREP_MAT2 = 2,    // one 2-qubit gate -> 4x4 matrix (dtype)
  PREP_ANG = 3,     // diag term angles (FP64, 2^nbits)
  PREP_COEF1 = 4,   // Pauli coefficients (hx, hy, hz) of V G_k V^dag for factor k
  PREP_COEF2 = 5,   // U2 generator scale (c of G = c P(x)P)
  PREP_COEFD = 6,   // diag term class-sum coefficients (P_0, P_a[, P_b, P_ab])
  PREP_DENSE = 8,   // full layer matrix (2^nv x 2^nv, dtype) from the layer's gates; one thread per column
};

struct Factor {
  int32_t gate;     // tqs_gate
  int32_t src;      // tqs_source
  int32_t pidx;     // weight / feature index
  int32_t wires;    // dense layers: state bit of the first wire | (state bit of the second + 1) << 8
  double fixed;
};

struct PrepItem {
  int32_t kind;
  int32_t per_sample;
  int32_t out;          // output offset (complex elements for MAT, doubles otherwise)
  int32_t f_begin, f_end;
  int32_t k;            // COEF1: differentiated factor (absolute index)
  int32_t pad[2];
};

// Gradient contribution: grad[param] += sum_k coef[k] * A[acc + k]
struct Contrib {
  int32_t acc;          // global accumulator index
  int32_t n;            // number of accumulators (<= 4)
  int32_t coef;         // coefficient offset (doubles)
  int32_t coef_ps;      // coefficients are per sample
};

struct AccInfo {        // where a global accumulator's partials live
  int32_t pass;
  int32_t local;
};

struct PassGeom {       // per pass, for the finalize reduction
  int32_t region;       // offset (doubles) of the pass's partials
  int32_t n_wg;         // workgroups per launch (for the batch it was planned with) -- set at launch
  int32_t n_seg;        // segments per workgroup
  int32_t segs_per_sample;
  int32_t spw_log, tiles_log;
  int32_t pad[2];
};

}  // namespace tqs
