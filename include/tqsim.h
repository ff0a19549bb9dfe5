/*
 * tqsim.h -- C ABI of libtqsim, a batched state-vector simulator of layered
 * quantum-machine-learning circuits for AMD MI355X (gfx950).
 *
 * The operations follow the problem statement of arXiv 2506.04891 ("TQml
 * Simulator"): an n-qubit state is a vector psi of 2^n complex amplitudes
 * (Sec. 1); a circuit is an ordered list of layers of uniformly placed gates
 * (Sec. 1, Fig. 6); each layer evolves the state as psi' = U psi with U the
 * layer's 2^n x 2^n unitary (Sec. 2.2.1); the readout is the single-qubit
 * observables <Z_i> (Figs. 6 and 11); training needs the derivatives of the
 * readout with respect to the circuit's weights and its input features (Sec. 3).
 *
 * Conventions
 *   - Amplitude index j = sum_k b_k 2^(n-1-k): wire 0 is the most significant
 *     bit (the bit order of the binary counting matrix J, Sec. 2.4.1).
 *   - State buffers are [batch, 2^n] row-major, interleaved (re, im):
 *     TQS_C64 = 2 x float (8 bytes per amplitude), TQS_C128 = 2 x double.
 *   - Weights, features, expectation values and gradients are always double.
 *   - Gate matrices are those of the paper's Appendix A.  Rotation angles are
 *     radians; GPI / GPI2 phases and the MS angle are in turns.  ECR is read as
 *     (I(x)X - X(x)Y)/sqrt(2) (its printed rows 0-1; rows 2-3 as printed are not
 *     unitary) and MS as MS(0, 0, theta) = exp(-i pi theta X(x)X).
 *
 * Ownership and execution
 *   - The caller owns every device buffer and the stream.  Calls that take a
 *     stream only enqueue work on it (asynchronous, stream-ordered); they do not
 *     allocate device memory, do not synchronise and read no device data on the
 *     host, so they may be captured into a HIP graph once the circuit has been
 *     used outside capture (the first use uploads the circuit's plan).
 *   - A circuit is immutable after creation and may be used concurrently on
 *     different streams with distinct state and workspace buffers.
 *
 * Errors
 *   Every call returns a tqs_status.  Argument, layer-list and size errors give
 *   TQS_EINVAL before anything is enqueued; an undersized workspace gives
 *   TQS_ENOMEM; a HIP runtime or launch failure gives TQS_EDEVICE.
 *   tqs_last_error() returns a thread-local description of the last failure.
 */
#ifndef TQSIM_H
#define TQSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TQS_OK = 0,
  TQS_EINVAL = 1,        /* invalid argument, layer list or size            */
  TQS_ENOMEM = 2,        /* workspace smaller than tqs_workspace_size()     */
  TQS_EDEVICE = 3,       /* HIP runtime / launch failure                    */
  TQS_EUNSUPPORTED = 4   /* valid request that this build does not provide  */
} tqs_status;

typedef enum { TQS_C64 = 0, TQS_C128 = 1 } tqs_dtype;

/* Gates of the paper's Table 1 / Appendix A.  TQS_ROT is Appendix A's
 * Rot(theta, phi, lambda) = [[c, -e^{i lambda} s], [e^{i phi} s, e^{i(phi+lambda)} c]]
 * (c, s = cos, sin of theta/2; radians) and reads three parameters per gate.
 * TQS_MS is MS(phi0, phi1, theta) = exp(-i pi theta P(phi1) (x) P(phi0)) with
 * P(phi) = [[0, e^{-2 pi i phi}], [e^{2 pi i phi}, 0]]: its printed rows 0-2,
 * entry (3, 0) read as e^{+2 pi i (phi0 + phi1)} (as printed it would not be
 * unitary); the phases come from fixed_param2 / fixed_param3 (turns). */
typedef enum {
  TQS_RX = 0, TQS_RY = 1, TQS_RZ = 2, TQS_H = 3, TQS_X = 4, TQS_Z = 5, TQS_S = 6,
  TQS_SX = 7, TQS_GPI = 8, TQS_GPI2 = 9,                       /* 1-qubit */
  TQS_CNOT = 10, TQS_CZ = 11, TQS_SWAP = 12, TQS_ZZ = 13, TQS_MS = 14,
  TQS_ECR = 15,                                                /* 2-qubit */
  TQS_ROT = 16                                                 /* 1-qubit, 3 parameters */
} tqs_gate;

typedef enum {
  TQS_ALL = 0,         /* the 1-qubit gate on every wire 0..n-1                    */
  TQS_WIRE = 1,        /* one gate on `wire` (2-qubit: on (wire, wire2))           */
  TQS_RING = 2,        /* (i, i+1 mod n), i = 0..n-1 in order; n=2: (0,1); n=1: none */
  TQS_CHAIN = 3,       /* (i, i+1), i = 0..n-2 in order                            */
  TQS_PAIRS_EVEN = 4,  /* (2i, 2i+1); n even                                       */
  TQS_PAIRS_ODD = 5    /* (2i+1, 2i+2 mod n); n even                               */
} tqs_pattern;

typedef enum {
  TQS_FIXED = 0,       /* every gate of the layer uses fixed_param                 */
  TQS_WEIGHT = 1,      /* gate k of the layer uses weights[offset + k]             */
  TQS_INPUT = 2        /* gate k uses features[b * n_features + offset + k]        */
} tqs_source;          /* TQS_ROT: gate k uses (theta, phi, lambda) at offset + 3k,
                          + 3k + 1, + 3k + 2; FIXED: fixed_param, fixed_param2, 3 */

typedef struct {
  int32_t gate;        /* tqs_gate                                                 */
  int32_t pattern;     /* tqs_pattern                                              */
  int32_t source;      /* tqs_source (ignored for gates without a parameter)       */
  int32_t wire;        /* TQS_WIRE: the wire (first wire of a 2-qubit gate)        */
  int32_t wire2;       /* TQS_WIRE, 2-qubit gates: the second wire                 */
  int32_t offset;      /* first weight index / feature column of the layer         */
  double fixed_param;  /* parameter used when source == TQS_FIXED                  */
  double fixed_param2; /* TQS_MS: phi0 (turns); TQS_ROT with TQS_FIXED: phi         */
  double fixed_param3; /* TQS_MS: phi1 (turns); TQS_ROT with TQS_FIXED: lambda      */
} tqs_layer;

typedef struct tqs_circuit tqs_circuit;
typedef struct ihipStream_t *tqs_stream;   /* hipStream_t; NULL = default stream */

/* Validate a layer list and compile its execution plan (host only; no device
 * memory is touched until the first forward call or tqs_circuit_prepare).
 * The layer list is the paper's circuit model: uniform layers of gates, each
 * layer one unitary on the whole state (Sec. 1, Sec. 2.2.1); the plan picks a
 * technique per layer from its properties -- diagonal, permutation, real,
 * 1- or 2-qubit (Table 1, Sec. 3) -- and fuses layers into tile passes.
 * n_qubits in [1, 30];
 * parameters of a layer must fit in the weights / features implied by the
 * largest offset + count.  *out receives a new circuit (free with
 * tqs_circuit_destroy).  EINVAL for: n out of range, an unknown gate / pattern /
 * source, a pattern invalid for the gate's arity, repeated or out-of-range
 * wires, PAIRS patterns with odd n, negative offsets. */
tqs_status tqs_circuit_create(int32_t n_qubits, const tqs_layer *layers, int32_t n_layers,
                              tqs_dtype dtype, tqs_circuit **out);

/* Upload the circuit's plan to the current device (one allocation and a
 * synchronous copy) if it is not there yet, so that later calls enqueue work
 * only -- e.g. before the calls are captured into a HIP graph.  Options other
 * than "profile" cannot change afterwards.  EDEVICE on a HIP failure. */
tqs_status tqs_circuit_prepare(tqs_circuit *c);

/* Free a circuit and its device tables.  Safe on NULL. */
tqs_status tqs_circuit_destroy(tqs_circuit *c);

/* Number of weights and feature columns the circuit reads, and the state size
 * of one sample in bytes (2^n times 8 or 16).  Any pointer may be NULL. */
tqs_status tqs_circuit_info(const tqs_circuit *c, int32_t *n_weights, int32_t *n_features,
                            int64_t *state_bytes_per_sample);

/* Device workspace (bytes) needed by tqs_forward / tqs_expval_z /
 * tqs_adjoint_grad for `batch` samples; with_grad != 0 includes the adjoint
 * buffers.  The same workspace may serve all three calls in sequence. */
tqs_status tqs_workspace_size(const tqs_circuit *c, int32_t batch, int32_t with_grad,
                              size_t *bytes);

/* Forward pass: psi_b = U_L ... U_1 |0...0> for every sample -- each layer's
 * unitary applied in order to the state vector (Sec. 1, Sec. 2.2.1), the
 * features entering the input-driven layers (angle embedding, Sec. 3).
 * The first call on a circuit uploads its plan (one device allocation and a
 * synchronous copy) unless tqs_circuit_prepare ran before.
 *   weights_d   device, [n_weights] double (may be NULL if n_weights == 0)
 *   features_d  device, [batch, n_features] double row-major (NULL if none)
 *   state_d     device, [batch, 2^n] complex of the circuit's dtype; written
 *   ws_d        device workspace of ws_bytes >= tqs_workspace_size(batch, 0)
 * Enqueued on stream s. */
tqs_status tqs_forward(tqs_circuit *c, int32_t batch, const double *weights_d,
                       const double *features_d, void *state_d, void *ws_d, size_t ws_bytes,
                       tqs_stream s);

/* Readout: expz[b, i] = <psi_b| Z_i |psi_b> (Z_i = +1 on bit value 0 of wire i),
 * accumulated in double; norm[b] = <psi_b|psi_b> when norm_d != NULL.  This is
 * K_Rz^T |psi|^2 with K_Rz = 1 - 2J, J the binary counting matrix (Sec. 2.4.1);
 * the single-qubit observables of the paper's circuits (Figs. 6 and 11).
 *   state_d [batch, 2^n] (read only); expz_d [batch, n] double; norm_d [batch]. */
tqs_status tqs_expval_z(const tqs_circuit *c, int32_t batch, const void *state_d,
                        double *expz_d, double *norm_d, void *ws_d, size_t ws_bytes,
                        tqs_stream s);

/* tqs_expval_z without a workspace, for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same outputs and kernels as
 * tqs_expval_z; the readout partials, [batch][2^max(0, n-12)][13] doubles, sit
 * in a static 8 MiB device array that every GPU the library runs on holds
 * until the process ends.  Allocates nothing and calls no allocating routine.
 * The first call on a device looks the array's address up (once per device).
 *   state_d [batch, 2^n] (read only); expz_d [batch, n]; norm_d [batch] or NULL.
 * EINVAL when the partials exceed 8 MiB, i.e. batch * 2^max(0, n-12) > 80659.
 * Calls on one GPU share the array: calls that overlap in time on one GPU
 * (different streams, threads or processes' streams without ordering) race
 * and must be serialised by the caller. */
tqs_status tqs_expval_z_noalloc(const tqs_circuit *c, int32_t batch, const void *state_d,
                                double *expz_d, double *norm_d, tqs_stream s);

/* Adjoint gradient of L = sum_{b,i} g[b,i] <Z_i>_b (the adjoint method cited in
 * Sec. 2.1): lambda = (sum_i g_i Z_i) psi, then layer by layer in reverse the
 * derivative 2 Im <lambda|G|psi> of every parameter is accumulated (G the gate's
 * output-side generator) and psi, lambda are uncomputed with the inverse layer;
 * no intermediate state is stored.
 *   state_d        in: the final states of tqs_forward (same weights/features);
 *                  clobbered.
 *   grad_expz_d    [batch, n] double, upstream dL/d<Z_i>.
 *   grad_weights_d [n_weights] double, overwritten (may be NULL if n_weights == 0).
 *   grad_features_d [batch, n_features] double, overwritten; NULL to skip.
 *   ws_d           ws_bytes >= tqs_workspace_size(batch, 1). */
tqs_status tqs_adjoint_grad(tqs_circuit *c, int32_t batch, const double *weights_d,
                            const double *features_d, void *state_d, const double *grad_expz_d,
                            double *grad_weights_d, double *grad_features_d, void *ws_d,
                            size_t ws_bytes, tqs_stream s);

/* Per-segment column sums, FP64, rows in order (deterministic):
 *   out[s][c] = sum_{r = seg[s]}^{seg[s+1]-1} x[r][col_begin + c],
 * for s < n_seg and c < n_cols.  x_d [rows, ld] row-major device doubles;
 * seg_d device int32 [n_seg + 1], non-decreasing in [0, rows] (bounds are
 * clamped to that range); out_d device [n_seg, n_cols].  The batch reduction
 * of gradients when the rows of one launch belong to several requests (each
 * request's weight gradient is the sum over its samples, Sec. 3 training);
 * the serving loop uses it.  EINVAL for negative sizes or
 * col_begin + n_cols > ld. */
tqs_status tqs_segment_sum_rows(const double *x_d, int32_t rows, int32_t ld, int32_t col_begin,
                                int32_t n_cols, const int32_t *seg_d, int32_t n_seg, double *out_d,
                                tqs_stream s);

/* Dispatcher override, before the first forward call.  Keys:
 *   "mode"       0 = auto, 1 = per-layer passes (one technique per layer),
 *                2 = fused passes, 3 = dense: every layer without per-sample
 *                parameters applied as its full 2^n x 2^n matrix on the matrix
 *                cores (the unitary operation of Sec. 2.2.1); for n > 6 the
 *                plan falls back to fused passes
 *   "tile_bits"  0 = auto, else K in [10, 12] for multi-pass plans
 *   "hrz"        1 = H-Rz expansion (Sec. 2.5): RX, RY, GPI2 and Rot layers are
 *                rewritten as layers of H, RZ and phase gates (RX = H RZ H;
 *                RY = S H RZ H S^dag; GPI2(phi) = RZ(2 pi phi) H RZ(pi/2) H
 *                RZ(-2 pi phi)), each then applied by its own technique
 *   "fhwt"       1 (default) = Hadamard layers by the fast Walsh-Hadamard
 *                transform (add / subtract butterflies, one scale, Sec. 2.5);
 *                0 = as real 2x2 matrices
 *   "diag"       0 (default) = diagonal layers by split eigenphase tables (the
 *                eigenphase computation of Sec. 2.4.1 on the two halves of the
 *                tile, combined as a diagonal tensor product, Sec. 2.4.2);
 *                1 = diagonal Einsum (Sec. 2.4.3): gate by gate, one diagonal
 *                factor per gate
 *   "profile"    1 = time every kernel launch with HIP events (any time; not
 *                to be used while the stream is being captured into a graph)
 *   "backward"   0 = adjoint with uncompute (default): psi is rebuilt pass by
 *                pass with the inverse layers, two state sets at any depth;
 *                1 = stored states, the backpropagation of the paper's own
 *                training (Sec. 2.1, Sec. 3): tqs_forward keeps the output of
 *                every tile pass but the last in the workspace, and
 *                tqs_adjoint_grad reads psi from there and writes back only
 *                lambda -- it must get the workspace of the forward call, not
 *                modified in between (tqs_expval_z may run in between);
 *                2 = stored states when the adjoint's four state buffers
 *                exceed "stored_min" bytes (they stream from HBM instead of
 *                staying in the last-level cache: there the stored form is
 *                faster, measured) and the stored states fit "stored_cap"
 *                bytes; adjoint otherwise (decided per batch size, the same
 *                way by every call)
 *   "stored_cap" bytes the stored states may take under backward = 2
 *                (default 8 GiB)
 *   "stored_min" the adjoint state-set size above which backward = 2 stores
 *                (default 256 MiB, the MI355X last-level cache)
 * EINVAL for an unknown key or value, or for any key but "profile" after the
 * plan has been uploaded. */
tqs_status tqs_set_option(tqs_circuit *c, const char *key, int64_t value);

/* Per-kernel-kind launch statistics gathered while "profile" is on: waits for
 * the recorded events, then writes JSON {kind: {count, ms, bytes, flops}} where
 * bytes / flops are the algorithmic HBM bytes and arithmetic of the launches.
 * reset != 0 clears the statistics afterwards. */
tqs_status tqs_profile_report(tqs_circuit *c, int32_t reset, char *buf, size_t len);

/* JSON description of the execution plan (passes, tiles, stages, kernels). */
tqs_status tqs_plan_describe(const tqs_circuit *c, char *buf, size_t len);

const char *tqs_status_string(tqs_status st);
const char *tqs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TQSIM_H */
