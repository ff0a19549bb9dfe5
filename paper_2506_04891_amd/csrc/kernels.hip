// gfx950 kernels of libtqsim.
//
//   k_prep       -- FP64 gate matrices, diagonal phase angles and gradient
//                   coefficients from the weights / features (one thread per
//                   item and sample), rounded once to the state dtype.
//   k_pass       -- one HBM pass of the batched state: load a 2^K tile into LDS
//                   (or generate the embedded product state), run the pass's
//                   stages, store.  The backward instantiation uncomputes psi
//                   and lambda with the inverse ops and accumulates gradient
//                   partial sums before each inverse op.
//   k_expval     -- <Z_i> partial sums (the paper's K_Rz^T |psi|^2, Sec. 2.4.1).
//   k_adj_init   -- lambda = (sum_i g_i Z_i) psi.
//   k_acc_reduce / k_grad_combine / k_expval_final -- deterministic FP64
//                   reductions of the per-segment partial sums.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace tqs {

template <typename T>
struct __align__(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return cmk(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cplx<T> cjmul(cplx<T> a, cplx<T> b) {
  return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// s += sg * Im(conj(l) p) and s += sg * Re(conj(l) p) (sg = +-1) as two chained
// FMAs into the running sum: gradient sums accumulate without separate
// products and adds
template <typename T>
__device__ __forceinline__ void im_acc(T &s, cplx<T> l, cplx<T> p, T sg) {
  s = tfma(sg * l.x, p.y, s);
  s = tfma(-sg * l.y, p.x, s);
}
template <typename T>
__device__ __forceinline__ void re_acc(T &s, cplx<T> l, cplx<T> p, T sg) {
  s = tfma(sg * l.x, p.x, s);
  s = tfma(sg * l.y, p.y, s);
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
  return cmk(a.x, -a.y);
}
// m * a + n * b
template <typename T>
__device__ __forceinline__ cplx<T> cfma2(cplx<T> m, cplx<T> a, cplx<T> n, cplx<T> b) {
  cplx<T> r;
  r.x = m.x * a.x - m.y * a.y + n.x * b.x - n.y * b.y;
  r.y = m.x * a.y + m.y * a.x + n.x * b.y + n.y * b.x;
  return r;
}

// Plan tables, gate matrices and angles are read-only while a pass runs; they
// are addressed through the constant address space so that wave-uniform reads
// become scalar (SMEM) loads through the scalar cache.
#define TQS_CONST __attribute__((address_space(4)))
template <typename X>
using kptr = const TQS_CONST X *;
template <typename X>
__host__ __device__ __forceinline__ kptr<X> kc(const X *p) {
  return (kptr<X>)(uintptr_t)p;
}

template <typename T>
__device__ __forceinline__ cplx<T> kld(kptr<cplx<T>> p, long long i) {
  cplx<T> r;
  r.x = p[i].x;
  r.y = p[i].y;
  return r;
}

// LDS swizzle: XOR-fold the higher index groups into the lowest group so that
// 16 (8-byte) or 8 (16-byte) lanes walking any four / three distinct bit
// classes hit distinct banks.  GF(2)-linear, so swz(a ^ b) = swz(a) ^ swz(b).
template <typename T>
__device__ __forceinline__ int swz(int t);
template <>
__device__ __forceinline__ int swz<float>(int t) {
  return t ^ ((t >> 4) & 15) ^ ((t >> 8) & 15);
}
template <>
__device__ __forceinline__ int swz<double>(int t) {
  return t ^ ((t >> 3) & 7) ^ ((t >> 6) & 7) ^ ((t >> 9) & 7);
}

// Plan tables are read by every lane at the same address; readfirstlane makes
// the values wave-uniform (SGPRs) so that op dispatch stays scalar control flow.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uniu(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

struct UOp {
  int kind, flags, r0, r1, mat, acc, aux, sub;
};
__device__ __forceinline__ UOp load_op(kptr<DevOp> p) {
  UOp o;
  o.kind = uni(p->kind);
  o.flags = uni(p->flags);
  o.r0 = uni(p->r0);
  o.r1 = uni(p->r1);
  o.mat = uni(p->mat);
  o.acc = uni(p->acc);
  o.aux = uni(p->aux);
  o.sub = uni(p->sub);
  return o;
}
struct UStage {
  int rbits[RB];
  int rsorted[RB];
  int op_begin, op_end;
  int flags;
  int dense_next[2];
  int fwd_next;
};
__device__ __forceinline__ UStage load_stage(kptr<DevStage> p) {
  UStage s;
  s.rbits[0] = uni(p->rbits[0]);
  s.rbits[1] = uni(p->rbits[1]);
  s.rbits[2] = uni(p->rbits[2]);
  s.rbits[3] = uni(p->rbits[3]);
#pragma unroll
  for (int k = 0; k < RB; ++k) s.rsorted[k] = uni(p->rsorted[k]);
  s.op_begin = uni(p->op_begin);
  s.op_end = uni(p->op_end);
  s.flags = uni(p->flags);
  s.dense_next[0] = uni(p->dense_next[0]);
  s.dense_next[1] = uni(p->dense_next[1]);
  s.fwd_next = uni(p->fwd_next);
  return s;
}

// ---------------------------------------------------------------------------
// FP64 gate library (the paper's Appendix A; ECR and MS as read in tqsim.h)
// ---------------------------------------------------------------------------
struct zd {
  double x, y;
};
__device__ __forceinline__ zd zmk(double x, double y) {
  zd r;
  r.x = x;
  r.y = y;
  return r;
}
__device__ __forceinline__ zd zmul(zd a, zd b) { return zmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ zd zadd(zd a, zd b) { return zmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ zd zconj(zd a) { return zmk(a.x, -a.y); }
__device__ __forceinline__ zd zexpi(double t) {
  double s, c;
  sincos(t, &s, &c);
  return zmk(c, s);
}

enum GateId {
  G_RX = 0, G_RY = 1, G_RZ = 2, G_H = 3, G_X = 4, G_Z = 5, G_S = 6, G_SX = 7, G_GPI = 8, G_GPI2 = 9,
  G_CNOT = 10, G_CZ = 11, G_SWAP = 12, G_ZZ = 13, G_MS = 14, G_ECR = 15,
  G_GPI_DIAG = 100,  // diagonal factor of GPI: diag(e^{2 pi i phi}, e^{-2 pi i phi})
  G_PHASE = 101,     // diag(1, e^{i t}) (a factor of Rot)
  G_RZT = 102,       // RZ(2 pi t) (a factor of the H-Rz form of GPI2)
  G_RZNT = 103       // RZ(-2 pi t)
};

constexpr double PI = 3.14159265358979323846;
constexpr double RSQ2 = 0.70710678118654752440;

// 2x2 matrix (row-major) and its derivative with respect to the parameter.
__device__ void gate2(int g, double t, zd m[4], zd d[4]) {
  for (int i = 0; i < 4; ++i) {
    m[i] = zmk(0, 0);
    d[i] = zmk(0, 0);
  }
  double s, c;
  switch (g) {
    case G_RX:
      sincos(0.5 * t, &s, &c);
      m[0] = zmk(c, 0); m[1] = zmk(0, -s); m[2] = zmk(0, -s); m[3] = zmk(c, 0);
      d[0] = zmk(-0.5 * s, 0); d[1] = zmk(0, -0.5 * c); d[2] = zmk(0, -0.5 * c); d[3] = zmk(-0.5 * s, 0);
      break;
    case G_RY:
      sincos(0.5 * t, &s, &c);
      m[0] = zmk(c, 0); m[1] = zmk(-s, 0); m[2] = zmk(s, 0); m[3] = zmk(c, 0);
      d[0] = zmk(-0.5 * s, 0); d[1] = zmk(-0.5 * c, 0); d[2] = zmk(0.5 * c, 0); d[3] = zmk(-0.5 * s, 0);
      break;
    case G_RZ: {
      sincos(0.5 * t, &s, &c);
      m[0] = zmk(c, -s); m[3] = zmk(c, s);
      d[0] = zmk(-0.5 * s, -0.5 * c); d[3] = zmk(-0.5 * s, 0.5 * c);
      break;
    }
    case G_H:
      m[0] = zmk(RSQ2, 0); m[1] = zmk(RSQ2, 0); m[2] = zmk(RSQ2, 0); m[3] = zmk(-RSQ2, 0);
      break;
    case G_X:
      m[1] = zmk(1, 0); m[2] = zmk(1, 0);
      break;
    case G_Z:
      m[0] = zmk(1, 0); m[3] = zmk(-1, 0);
      break;
    case G_S:
      m[0] = zmk(1, 0); m[3] = zmk(0, 1);
      break;
    case G_SX:
      m[0] = zmk(0.5, 0.5); m[1] = zmk(0.5, -0.5); m[2] = zmk(0.5, -0.5); m[3] = zmk(0.5, 0.5);
      break;
    case G_GPI: {
      zd e = zexpi(2.0 * PI * t);
      m[1] = zconj(e); m[2] = e;
      d[1] = zmul(zmk(0, -2.0 * PI), zconj(e)); d[2] = zmul(zmk(0, 2.0 * PI), e);
      break;
    }
    case G_GPI2: {
      zd e = zexpi(2.0 * PI * t);
      m[0] = zmk(RSQ2, 0); m[3] = zmk(RSQ2, 0);
      m[1] = zmul(zmk(0, -RSQ2), zconj(e)); m[2] = zmul(zmk(0, -RSQ2), e);
      d[1] = zmul(zmk(-2.0 * PI * RSQ2, 0), zconj(e)); d[2] = zmul(zmk(2.0 * PI * RSQ2, 0), e);
      break;
    }
    case G_GPI_DIAG: {
      zd e = zexpi(2.0 * PI * t);
      m[0] = e; m[3] = zconj(e);
      d[0] = zmul(zmk(0, 2.0 * PI), e); d[3] = zmul(zmk(0, -2.0 * PI), zconj(e));
      break;
    }
    case G_PHASE: {
      zd e = zexpi(t);
      m[0] = zmk(1, 0); m[3] = e;
      d[3] = zmul(zmk(0, 1), e);
      break;
    }
    case G_RZT:
    case G_RZNT: {
      const double k = g == G_RZT ? PI : -PI;   // RZ(+-2 pi t): phases -+k t
      zd e = zexpi(k * t);
      m[0] = zconj(e); m[3] = e;
      d[0] = zmul(zmk(0, -k), zconj(e)); d[3] = zmul(zmk(0, k), e);
      break;
    }
    default:
      m[0] = zmk(1, 0); m[3] = zmk(1, 0);
  }
}

// 4x4 matrix (row-major; first wire = more significant bit).
__device__ void gate4(int g, double t, zd m[16]) {
  for (int i = 0; i < 16; ++i) m[i] = zmk(0, 0);
  switch (g) {
    case G_CNOT:
      m[0] = m[5] = m[11] = m[14] = zmk(1, 0);
      break;
    case G_CZ:
      m[0] = m[5] = m[10] = zmk(1, 0); m[15] = zmk(-1, 0);
      break;
    case G_SWAP:
      m[0] = m[6] = m[9] = m[15] = zmk(1, 0);
      break;
    case G_ZZ: {
      zd a = zexpi(-0.5 * t), b = zexpi(0.5 * t);
      m[0] = a; m[5] = b; m[10] = b; m[15] = a;
      break;
    }
    case G_MS: {
      double s, c;
      sincos(PI * t, &s, &c);
      m[0] = m[5] = m[10] = m[15] = zmk(c, 0);
      m[3] = m[6] = m[9] = m[12] = zmk(0, -s);
      break;
    }
    case G_ECR:
      m[1] = zmk(RSQ2, 0); m[3] = zmk(0, RSQ2);
      m[4] = zmk(RSQ2, 0); m[6] = zmk(0, -RSQ2);
      m[9] = zmk(0, RSQ2); m[11] = zmk(RSQ2, 0);
      m[12] = zmk(0, -RSQ2); m[14] = zmk(RSQ2, 0);
      break;
    default:
      m[0] = m[5] = m[10] = m[15] = zmk(1, 0);
  }
}

// Phase angles phi(v) of a diagonal gate, e^{i phi(v)}, v in bit order.
__device__ int diag_angles(int g, double t, double a[4], double da[4]) {
  for (int i = 0; i < 4; ++i) a[i] = da[i] = 0.0;
  switch (g) {
    case G_RZ: a[0] = -0.5 * t; a[1] = 0.5 * t; da[0] = -0.5; da[1] = 0.5; return 1;
    case G_Z: a[1] = PI; return 1;
    case G_S: a[1] = 0.5 * PI; return 1;
    case G_GPI_DIAG: a[0] = 2.0 * PI * t; a[1] = -2.0 * PI * t; da[0] = 2.0 * PI; da[1] = -2.0 * PI; return 1;
    case G_PHASE: a[1] = t; da[1] = 1.0; return 1;
    case G_RZT: a[0] = -PI * t; a[1] = PI * t; da[0] = -PI; da[1] = PI; return 1;
    case G_RZNT: a[0] = PI * t; a[1] = -PI * t; da[0] = PI; da[1] = -PI; return 1;
    case G_ZZ: a[0] = a[3] = -0.5 * t; a[1] = a[2] = 0.5 * t; da[0] = da[3] = -0.5; da[1] = da[2] = 0.5; return 2;
    case G_CZ: a[3] = PI; return 2;
  }
  return 1;
}

__device__ __forceinline__ double factor_param(const Factor &f, const double *w, const double *x,
                                               int nfeat, int b) {
  if (f.src == 1) return w[f.pidx];
  if (f.src == 2) return x[(size_t)b * nfeat + f.pidx];
  return f.fixed;
}

__device__ __forceinline__ void mat2mul(const zd a[4], const zd b[4], zd r[4]) {
  zd t[4];
  t[0] = zadd(zmul(a[0], b[0]), zmul(a[1], b[2]));
  t[1] = zadd(zmul(a[0], b[1]), zmul(a[1], b[3]));
  t[2] = zadd(zmul(a[2], b[0]), zmul(a[3], b[2]));
  t[3] = zadd(zmul(a[2], b[1]), zmul(a[3], b[3]));
  for (int i = 0; i < 4; ++i) r[i] = t[i];
}
// a * b^dagger
__device__ __forceinline__ void mat2mul_dag(const zd a[4], const zd b[4], zd r[4]) {
  zd t[4];
  t[0] = zadd(zmul(a[0], zconj(b[0])), zmul(a[1], zconj(b[1])));
  t[1] = zadd(zmul(a[0], zconj(b[2])), zmul(a[1], zconj(b[3])));
  t[2] = zadd(zmul(a[2], zconj(b[0])), zmul(a[3], zconj(b[1])));
  t[3] = zadd(zmul(a[2], zconj(b[2])), zmul(a[3], zconj(b[3])));
  for (int i = 0; i < 4; ++i) r[i] = t[i];
}

template <typename T>
struct PrepArgs {
  kptr<PrepItem> items;
  kptr<Factor> factors;
  int n_items;
  const double *w;
  const double *x;
  int nfeat;
  int batch;
  cplx<T> *mats;
  cplx<T> *mats_ps;
  int mats_ps_stride;
  double *dbl;       // angles and coefficients (shared)
  double *dbl_ps;    // per-sample
  int dbl_ps_stride;
  int nv;            // dense layer matrices are 2^nv x 2^nv
};

__device__ __forceinline__ PrepItem ld_item(kptr<PrepItem> p) {
  PrepItem r;
  r.kind = p->kind;
  r.per_sample = p->per_sample;
  r.out = p->out;
  r.f_begin = p->f_begin;
  r.f_end = p->f_end;
  r.k = p->k;
  return r;
}
__device__ __forceinline__ Factor ld_factor(kptr<Factor> p) {
  Factor f;
  f.gate = p->gate;
  f.src = p->src;
  f.pidx = p->pidx;
  f.wires = p->wires;
  f.fixed = p->fixed;
  return f;
}

template <typename T>
__global__ void __launch_bounds__(64) k_prep(PrepArgs<T> a) {
  const int item = blockIdx.y;
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (item >= a.n_items) return;
  const PrepItem it = ld_item(a.items + item);
  if (it.per_sample ? (b >= a.batch) : (b != 0)) return;
  const int bs = it.per_sample ? b : 0;
  switch (it.kind) {
    case PREP_MAT1: {
      zd m[4], d[4], f[4];
      m[0] = zmk(1, 0); m[1] = zmk(0, 0); m[2] = zmk(0, 0); m[3] = zmk(1, 0);
      for (int k = it.f_begin; k < it.f_end; ++k) {
        const Factor fc = ld_factor(a.factors + (k));
        gate2(fc.gate, factor_param(fc, a.w, a.x, a.nfeat, bs), f, d);
        mat2mul(f, m, m);
      }
      cplx<T> *o = it.per_sample ? a.mats_ps + (size_t)bs * a.mats_ps_stride + it.out : a.mats + it.out;
      for (int i = 0; i < 4; ++i) o[i] = cmk<T>((T)m[i].x, (T)m[i].y);
      break;
    }
    case PREP_MAT2: {
      zd m[16];
      const Factor fc = ld_factor(a.factors + (it.f_begin));
      gate4(fc.gate, factor_param(fc, a.w, a.x, a.nfeat, bs), m);
      cplx<T> *o = it.per_sample ? a.mats_ps + (size_t)bs * a.mats_ps_stride + it.out : a.mats + it.out;
      for (int i = 0; i < 16; ++i) o[i] = cmk<T>((T)m[i].x, (T)m[i].y);
      break;
    }
    case PREP_ANG: {
      double ang[4], da[4];
      const Factor fc = ld_factor(a.factors + (it.f_begin));
      int nb = diag_angles(fc.gate, factor_param(fc, a.w, a.x, a.nfeat, bs), ang, da);
      double *o = it.per_sample ? a.dbl_ps + (size_t)bs * a.dbl_ps_stride + it.out : a.dbl + it.out;
      for (int i = 0; i < (1 << nb); ++i) o[i] = ang[i];
      break;
    }
    case PREP_COEF1: {
      // h = V G V^dag with G = i dF F^dag of factor k and V the later factors.
      zd f[4], d[4], g[4], v[4], tmp[4];
      const Factor fk = ld_factor(a.factors + (it.k));
      gate2(fk.gate, factor_param(fk, a.w, a.x, a.nfeat, bs), f, d);
      mat2mul_dag(d, f, g);
      for (int i = 0; i < 4; ++i) g[i] = zmul(zmk(0, 1), g[i]);
      v[0] = zmk(1, 0); v[1] = zmk(0, 0); v[2] = zmk(0, 0); v[3] = zmk(1, 0);
      for (int k = it.k + 1; k < it.f_end; ++k) {
        const Factor fc = ld_factor(a.factors + (k));
        gate2(fc.gate, factor_param(fc, a.w, a.x, a.nfeat, bs), f, d);
        mat2mul(f, v, v);
      }
      mat2mul(v, g, tmp);
      mat2mul_dag(tmp, v, g);
      double *o = it.per_sample ? a.dbl_ps + (size_t)bs * a.dbl_ps_stride + it.out : a.dbl + it.out;
      o[0] = 2.0 * g[1].x;             // 2 hx
      o[1] = -2.0 * g[1].y;            // 2 hy
      o[2] = g[0].x - g[3].x;          // 2 hz
      break;
    }
    case PREP_COEF2: {
      // output-side generators: MS(theta) -> pi X(x)X, ZZ(theta) -> Z(x)Z / 2; the
      // kernel sums Im<l|P(x)P|p>, the coefficient is twice the generator scale.
      double *o = it.per_sample ? a.dbl_ps + (size_t)bs * a.dbl_ps_stride + it.out : a.dbl + it.out;
      o[0] = a.factors[it.f_begin].gate == G_MS ? 2.0 * PI : 1.0;
      break;
    }
    case PREP_COEFD: {
      double ang[4], da[4];
      const Factor fc = ld_factor(a.factors + (it.f_begin));
      int nb = diag_angles(fc.gate, factor_param(fc, a.w, a.x, a.nfeat, bs), ang, da);
      // dL/dtheta = -2 sum_v dphi(v) W(v) with W(v) = class sum; only the
      // parity sum over all term bits has a nonzero weight for these gates.
      double c = 0.0;
      for (int v = 0; v < (1 << nb); ++v) c += da[v] * ((__popc(v) & 1) ? -1.0 : 1.0);
      c *= -2.0 / (double)(1 << nb);
      double *o = it.per_sample ? a.dbl_ps + (size_t)bs * a.dbl_ps_stride + it.out : a.dbl + it.out;
      o[0] = c;
      break;
    }
    case PREP_DENSE:
      break;   // built by k_prep_dense
  }
}

// Full matrix of a dense layer (up to 64 x 64): one wave per column c.  Lane j
// holds amplitude j of U e_c in FP64; each gate of the layer, in order, mixes
// a lane with its partners across the gate's bits (lane shuffles), and the
// column is written rounded to the state dtype.
__device__ __forceinline__ zd shfl_xor_zd(zd v, int m) {
  zd r;
  r.x = __shfl_xor(v.x, m, 64);
  r.y = __shfl_xor(v.y, m, 64);
  return r;
}

template <typename T>
__global__ void __launch_bounds__(64) k_prep_dense(PrepArgs<T> a) {
  const int item = blockIdx.y;
  const int col = blockIdx.x;
  const int j = threadIdx.x;
  const int dim = 1 << a.nv;
  if (item >= a.n_items || col >= dim) return;
  const PrepItem it = ld_item(a.items + item);
  if (it.kind != PREP_DENSE) return;
  zd v = zmk(j == col ? 1.0 : 0.0, 0.0);
  for (int k = it.f_begin; k < it.f_end; ++k) {
    const Factor fc = ld_factor(a.factors + k);
    const double th = factor_param(fc, a.w, a.x, a.nfeat, 0);
    const int p0 = fc.wires & 0xff, p1 = (fc.wires >> 8) - 1;
    if (p1 < 0) {
      zd m[4], d[4];
      gate2(fc.gate, th, m, d);
      const int b0 = (j >> p0) & 1;
      const zd o = shfl_xor_zd(v, 1 << p0);
      // row b0 of the 2x2: own amplitude sits in column b0, partner in 1-b0
      v = zadd(zmul(m[b0 * 3], v), zmul(m[b0 ? 2 : 1], o));
    } else {
      zd m[16];
      gate4(fc.gate, th, m);
      const int m0 = 1 << p0, m1 = 1 << p1;
      const zd x1 = shfl_xor_zd(v, m1), x2 = shfl_xor_zd(v, m0), x3 = shfl_xor_zd(v, m0 | m1);
      const int r = 2 * ((j >> p0) & 1) + ((j >> p1) & 1);
      // partner at xor-mask q holds the amplitude of row index r ^ q'
      // (q' = 1 for the second wire, 2 for the first)
      zd acc = zmul(m[r * 4 + r], v);
      acc = zadd(acc, zmul(m[r * 4 + (r ^ 1)], x1));
      acc = zadd(acc, zmul(m[r * 4 + (r ^ 2)], x2));
      acc = zadd(acc, zmul(m[r * 4 + (r ^ 3)], x3));
      v = acc;
    }
  }
  if (j < dim) a.mats[it.out + (long long)j * dim + col] = cmk<T>((T)v.x, (T)v.y);
}

// ---------------------------------------------------------------------------
// register-level gate application on 16 amplitudes held by one thread
// ---------------------------------------------------------------------------
template <typename T, int R, bool ADJ>
__device__ __forceinline__ void u1_apply(cplx<T> (&v)[NREG], const cplx<T> m[4]) {
  cplx<T> m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
  if (ADJ) {
    m00 = cconj(m[0]); m01 = cconj(m[2]); m10 = cconj(m[1]); m11 = cconj(m[3]);
  }
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & (1 << R)) continue;
    const cplx<T> a = v[j], b = v[j | (1 << R)];
    v[j] = cfma2(m00, a, m01, b);
    v[j | (1 << R)] = cfma2(m10, a, m11, b);
  }
}

template <typename T, int R, bool ADJ>
__device__ __forceinline__ void u1_apply_real(cplx<T> (&v)[NREG], const cplx<T> m[4]) {
  T m00 = m[0].x, m01 = m[1].x, m10 = m[2].x, m11 = m[3].x;
  if (ADJ) {
    m01 = m[2].x; m10 = m[1].x;
  }
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & (1 << R)) continue;
    const cplx<T> a = v[j], b = v[j | (1 << R)];
    v[j] = cmk(m00 * a.x + m01 * b.x, m00 * a.y + m01 * b.y);
    v[j | (1 << R)] = cmk(m10 * a.x + m11 * b.x, m10 * a.y + m11 * b.y);
  }
}

template <typename T, int R, bool ADJ>
__device__ __forceinline__ void u1_apply_diag(cplx<T> (&v)[NREG], const cplx<T> m[4]) {
  const cplx<T> d0 = ADJ ? cconj(m[0]) : m[0], d1 = ADJ ? cconj(m[3]) : m[3];
#pragma unroll
  for (int j = 0; j < NREG; ++j) v[j] = cmul(v[j], (j & (1 << R)) ? d1 : d0);
}

// Pauli sums Im<l|X|p>, Im<l|Y|p>, Im<l|Z|p> over the pairs of register bit R.
template <typename T, int R>
__device__ __forceinline__ void u1_grad(const cplx<T> (&p)[NREG], const cplx<T> (&l)[NREG], T &sx,
                                        T &sy, T &sz) {
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & (1 << R)) continue;
    const cplx<T> pa = p[j], pb = p[j | (1 << R)], la = l[j], lb = l[j | (1 << R)];
    im_acc(sx, la, pb, T(1));    // Im(conj(la) pb) + Im(conj(lb) pa)
    im_acc(sx, lb, pa, T(1));
    re_acc(sy, lb, pa, T(1));    // Re(conj(lb) pa) - Re(conj(la) pb)
    re_acc(sy, la, pb, T(-1));
    im_acc(sz, la, pa, T(1));    // Im(conj(la) pa) - Im(conj(lb) pb)
    im_acc(sz, lb, pb, T(-1));
  }
}

template <typename T, int R0, int R1, bool ADJ>
__device__ __forceinline__ void u2_apply(cplx<T> (&v)[NREG], kptr<cplx<T>> mg) {
  // entry (r, c) of the applied matrix: U[r][c], or conj(U[c][r]) for the adjoint
#define TQS_M(r, c) (ADJ ? cconj(kld(mg, (c) * 4 + (r))) : kld(mg, (r) * 4 + (c)))
  const cplx<T> m00 = TQS_M(0, 0), m01 = TQS_M(0, 1), m02 = TQS_M(0, 2), m03 = TQS_M(0, 3);
  const cplx<T> m10 = TQS_M(1, 0), m11 = TQS_M(1, 1), m12 = TQS_M(1, 2), m13 = TQS_M(1, 3);
  const cplx<T> m20 = TQS_M(2, 0), m21 = TQS_M(2, 1), m22 = TQS_M(2, 2), m23 = TQS_M(2, 3);
  const cplx<T> m30 = TQS_M(3, 0), m31 = TQS_M(3, 1), m32 = TQS_M(3, 2), m33 = TQS_M(3, 3);
#undef TQS_M
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & ((1 << R0) | (1 << R1))) continue;
    const int i0 = j, i1 = j | (1 << R1), i2 = j | (1 << R0), i3 = j | (1 << R0) | (1 << R1);
    const cplx<T> a0 = v[i0], a1 = v[i1], a2 = v[i2], a3 = v[i3];
    v[i0] = cadd(cfma2(m00, a0, m01, a1), cfma2(m02, a2, m03, a3));
    v[i1] = cadd(cfma2(m10, a0, m11, a1), cfma2(m12, a2, m13, a3));
    v[i2] = cadd(cfma2(m20, a0, m21, a1), cfma2(m22, a2, m23, a3));
    v[i3] = cadd(cfma2(m30, a0, m31, a1), cfma2(m32, a2, m33, a3));
  }
}

// Structured 4x4 ops on the quads of register bits (R0 = more significant).
template <typename T, int R0, int R1, bool ADJ, int KIND>
__device__ __forceinline__ void u2s_apply(cplx<T> (&v)[NREG], kptr<cplx<T>> mg) {
  T c = 0, sn = 0;
  if (KIND == U2_MS) {
    c = mg[0].x;             // cos(pi t)
    sn = -mg[3].y;           // entry (0,3) = -i sin(pi t)
    if (ADJ) sn = -sn;
  }
  cplx<T> d0, d1, d2, d3;
  if (KIND == U2_DIAG) {
    d0 = kld(mg, 0); d1 = kld(mg, 5); d2 = kld(mg, 10); d3 = kld(mg, 15);
    if (ADJ) { d0 = cconj(d0); d1 = cconj(d1); d2 = cconj(d2); d3 = cconj(d3); }
  }
  const T r = (T)0.70710678118654752440;
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & ((1 << R0) | (1 << R1))) continue;
    const int i0 = j, i1 = j | (1 << R1), i2 = j | (1 << R0), i3 = j | (1 << R0) | (1 << R1);
    const cplx<T> a0 = v[i0], a1 = v[i1], a2 = v[i2], a3 = v[i3];
    if (KIND == U2_CNOT) {
      v[i2] = a3; v[i3] = a2;
    } else if (KIND == U2_SWAP) {
      v[i1] = a2; v[i2] = a1;
    } else if (KIND == U2_CZ) {
      v[i3] = cmk(-a3.x, -a3.y);
    } else if (KIND == U2_MS) {
      // out_k = c a_k - i s a_{k^3}
      v[i0] = cmk(c * a0.x + sn * a3.y, c * a0.y - sn * a3.x);
      v[i3] = cmk(c * a3.x + sn * a0.y, c * a3.y - sn * a0.x);
      v[i1] = cmk(c * a1.x + sn * a2.y, c * a1.y - sn * a2.x);
      v[i2] = cmk(c * a2.x + sn * a1.y, c * a2.y - sn * a1.x);
    } else if (KIND == U2_ECR) {
      // self-inverse: rows [0,1,0,i], [1,0,-i,0], [0,i,0,1], [-i,0,1,0] / sqrt(2)
      v[i0] = cmk((a1.x - a3.y) * r, (a1.y + a3.x) * r);
      v[i1] = cmk((a0.x + a2.y) * r, (a0.y - a2.x) * r);
      v[i2] = cmk((a3.x - a1.y) * r, (a3.y + a1.x) * r);
      v[i3] = cmk((a2.x + a0.y) * r, (a2.y - a0.x) * r);
    } else if (KIND == U2_DIAG) {
      v[i0] = cmul(a0, d0); v[i1] = cmul(a1, d1); v[i2] = cmul(a2, d2); v[i3] = cmul(a3, d3);
    }
  }
}

// Im<l| P(x)P |p> for P = X (code 1|1<<2) or Z (code 3|3<<2) on both bits.
template <typename T, int R0, int R1, bool XX>
__device__ __forceinline__ T u2s_grad(const cplx<T> (&p)[NREG], const cplx<T> (&l)[NREG]) {
  T acc = 0;
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & ((1 << R0) | (1 << R1))) continue;
    const int i0 = j, i1 = j | (1 << R1), i2 = j | (1 << R0), i3 = j | (1 << R0) | (1 << R1);
    if (XX) {
      im_acc(acc, l[i0], p[i3], T(1));
      im_acc(acc, l[i3], p[i0], T(1));
      im_acc(acc, l[i1], p[i2], T(1));
      im_acc(acc, l[i2], p[i1], T(1));
    } else {
      im_acc(acc, l[i0], p[i0], T(1));
      im_acc(acc, l[i1], p[i1], T(-1));
      im_acc(acc, l[i2], p[i2], T(-1));
      im_acc(acc, l[i3], p[i3], T(1));
    }
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ cplx<T> pauli_row(int code, int bit, cplx<T> a, cplx<T> b, T &sgn) {
  // returns (P psi) component for bit value `bit`, given psi components a (0) and b (1)
  switch (code) {
    case 1: return bit ? a : b;                                   // X
    case 2: return bit ? cmk(-a.y, a.x) : cmk(b.y, -b.x);         // Y: (-i b, i a)
    default: return bit ? cmk(-b.x, -b.y) : a;                    // Z
  }
}

// Im<l| P_a (x) P_b |p> over quads of register bits (R0 = more significant).
template <typename T, int R0, int R1>
__device__ __forceinline__ T u2_grad(const cplx<T> (&p)[NREG], const cplx<T> (&l)[NREG], int code) {
  const int ca = code & 3, cb = (code >> 2) & 3;
  T acc = 0;
  T dummy;
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    if (j & ((1 << R0) | (1 << R1))) continue;
    const int i0 = j, i1 = j | (1 << R1), i2 = j | (1 << R0), i3 = j | (1 << R0) | (1 << R1);
    // apply P_b on the low bit, then P_a on the high bit
    const cplx<T> q0 = pauli_row(cb, 0, p[i0], p[i1], dummy), q1 = pauli_row(cb, 1, p[i0], p[i1], dummy);
    const cplx<T> q2 = pauli_row(cb, 0, p[i2], p[i3], dummy), q3 = pauli_row(cb, 1, p[i2], p[i3], dummy);
    const cplx<T> r0 = pauli_row(ca, 0, q0, q2, dummy), r2 = pauli_row(ca, 1, q0, q2, dummy);
    const cplx<T> r1 = pauli_row(ca, 0, q1, q3, dummy), r3 = pauli_row(ca, 1, q1, q3, dummy);
    im_acc(acc, l[i0], r0, T(1));
    im_acc(acc, l[i1], r1, T(1));
    im_acc(acc, l[i2], r2, T(1));
    im_acc(acc, l[i3], r3, T(1));
  }
  return acc;
}

// ---------------------------------------------------------------------------
// pass kernel
// ---------------------------------------------------------------------------
template <typename T>
struct PassArgs {
  kptr<DevPass> pass;
  kptr<DevStage> stages;
  kptr<DevOp> ops;
  kptr<DevDiag> diags;
  kptr<DevTerm> terms;
  kptr<DevPerm> perms;
  kptr<DevGroup> groups;
  kptr<DevSeq> seqs;
  kptr<DevTermGrad> tgrads;
  kptr<cplx<T>> mats;
  kptr<cplx<T>> mats_ps;
  int mats_ps_stride;
  kptr<double> dbl;
  kptr<double> dbl_ps;
  int dbl_ps_stride;
  const cplx<T> *diag_tabs;   // prebuilt split tables of shared diagonal ops
  const cplx<T> *src0;
  cplx<T> *dst0;
  const cplx<T> *src1;
  cplx<T> *dst1;
  double *partials;       // FP64 gradient partials of every pass
  long long acc_region;   // first partial of this pass
  int units;              // partial units per sample of this pass
  int batch;
  // first backward pass: lambda = (sum_i g_i Z_i) psi is formed from psi as the
  // tile is loaded (no separate adjoint-init kernel, no lambda read); g [B, n]
  const double *g;
  int init_lambda;
  // backward: write the uncomputed psi back (0 when the next backward pass
  // reads psi from a state stored by the forward pass instead)
  int store_psi;
};

template <typename T>
__device__ __forceinline__ T seg_reduce(T v, int seg_log) {
  for (int m = 1; m < (1 << seg_log); m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// Cross-lane adds with DPP (no LDS traffic).  Steps 1-4 leave the sum of each
// aligned group of 2, 4, 8, 16 lanes in every lane of the group; step 5 leaves
// the 32-lane sums in lanes 16-31 and 48-63, step 6 the 64-lane sum in lanes 48-63.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, true);
  return v + __int_as_float(t);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, true);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// v + v of lane ^ 16 and v + v of lane ^ 32 with the CDNA4 row swaps: with both
// operands equal, the two results of a swap hold each lane's value and its
// partner's, in some order per lane, so their sum is the pair sum everywhere.
__device__ __forceinline__ float xor16_add(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor32_add(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xor16_add(double v) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | lo[0]) + __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ double xor32_add(double v) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | lo[0]) + __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// Three sums reduced over the 64 lanes of the wave as one transposed tree: the
// first two butterfly steps halve the number of values per lane (a lane keeps
// the value selected by its two low lane bits), the rest reduce that one value.
// Afterwards lane l holds the total of value l & 3 (x, y, z, 0).
template <typename T>
__device__ __forceinline__ T wave_sum3_transposed(T x, T y, T z, int lane) {
  const bool b0 = lane & 1, b1 = lane & 2;
  const T p = (b0 ? y : x) + dpp_mov<0xB1>(b0 ? x : y);        // quad_perm [1,0,3,2]
  const T q = (b0 ? T(0) : z) + dpp_mov<0xB1>(b0 ? z : T(0));
  T v = (b1 ? q : p) + dpp_mov<0x4E>(b1 ? p : q);               // quad_perm [2,3,0,1]
  v += dpp_mov<0x124>(v);                                        // row_ror:4
  v += dpp_mov<0x128>(v);                                        // row_ror:8
  v = xor16_add(v);
  v = xor32_add(v);
  return v;
}

// Eight sums reduced over the 64 lanes as one transposed tree: three butterfly
// steps over lane bits 0-2 halve the values per lane (a lane keeps the values
// its lane bits select; the bit-2 step pairs lane l with (l + 4) mod 16, which
// always holds the other half of the same values), then rotations and the
// CDNA4 row swaps reduce the one value left.  Afterwards lane l holds the total
// of value l & 7.
__device__ __forceinline__ double wave_sum8_transposed(const double (&v)[8], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  double h[4], q[2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    h[i] = (b0 ? v[2 * i + 1] : v[2 * i]) + dpp_mov<0xB1>(b0 ? v[2 * i] : v[2 * i + 1]);   // lane ^ 1
#pragma unroll
  for (int i = 0; i < 2; ++i)
    q[i] = (b1 ? h[2 * i + 1] : h[2 * i]) + dpp_mov<0x4E>(b1 ? h[2 * i] : h[2 * i + 1]);   // lane ^ 2
  double x = (b2 ? q[1] : q[0]) + dpp_mov<0x124>(b2 ? q[0] : q[1]);                      // row_ror:4
  x += dpp_mov<0x128>(x);                                                                 // row_ror:8
  x = xor16_add(x);
  x = xor32_add(x);
  return x;
}

// Sum over aligned segments of 2^seg_log lanes; valid in the last lane of each segment.
template <typename T>
__device__ __forceinline__ T seg_sum_dpp(T v, int seg_log) {
  if (seg_log >= 1) v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  if (seg_log >= 2) v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  if (seg_log >= 3) v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
  if (seg_log >= 4) v = dpp_add<0x140, 0xF>(v);  // row_mirror
  if (seg_log >= 5) v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  if (seg_log >= 6) v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum over the 64 lanes of the wave, straight-line; valid in lanes 48-63.
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
  v = dpp_add<0xB1, 0xF>(v);
  v = dpp_add<0x4E, 0xF>(v);
  v = dpp_add<0x141, 0xF>(v);
  v = dpp_add<0x140, 0xF>(v);
  v = dpp_add<0x142, 0xA>(v);
  v = dpp_add<0x143, 0xC>(v);
  return v;
}

template <typename T, int K>
struct Ctx {
  static constexpr int NT = 1 << (K - RB);
  int tid, lane;
  // passes with full-layer matrix ops: wave group `sub` of `nsub`, each running
  // every stage on its own copy of the tile; group 0 writes the tile and the
  // partials of the other ops, the gradient-only ops are shared out among the
  // groups (pwriter_own / pwriter3_own: the writer flags without that rule)
  int sub, nsub;
  int pwriter_own, pwriter3_own;
  int n, nv;
  int multi;            // several samples per workgroup
  int sample0;          // first sample of the workgroup
  uint32_t base;        // state-index bits of the tile (single-sample mode)
  int seg_log;          // log2 threads per reduction segment
  int units_wg_base;    // unit offset of this workgroup within its sample (single mode)
  // gradient partials (backward): the thread's slot for accumulator 0, the
  // distance between accumulators, and whether the thread writes its segment's sum
  double *pslot;
  long long pstride;
  int pwriter;
  // whole-wave segments: lanes 0-2 write the three sums of a transposed reduction
  double *pslot3;
  int pwriter3;
};

// Partial slot of the thread: partials[acc_region + (acc * batch + s) * units + u]
// for the sample s and unit u of the thread's reduction segment.
template <typename T, int K>
__device__ __forceinline__ void set_partial_slot(Ctx<T, K> &c, double *partials, long long acc_region, int batch,
                                                 int units) {
  const int segm = (1 << c.seg_log) - 1;
  const int seg = c.tid >> c.seg_log;
  int s, u;
  if (c.multi) {
    const int spt_log = (c.nv - RB) - c.seg_log;   // segments per sample (log2)
    s = c.sample0 + (seg >> spt_log);
    u = seg & ((1 << spt_log) - 1);
  } else {
    s = c.sample0;
    u = c.units_wg_base + seg;
  }
  c.pwriter = (c.tid & segm) == segm && s < batch;
  c.pslot = partials ? partials + acc_region + (long long)(s < batch ? s : 0) * units + u : partials;
  c.pstride = (long long)batch * units;
  c.pwriter3 = (c.tid & 63) < 3 && s < batch;
  c.pslot3 = partials ? c.pslot + (long long)(c.tid & 3) * c.pstride : partials;
}

// Sample of a thread in multi-sample mode: the sample bits are the top thread bits
// in every stage (register bits are always state bits).
template <typename T, int K>
__device__ __forceinline__ int thread_sample(const Ctx<T, K> &c, int batch) {
  const int s = c.multi ? c.sample0 + (c.tid >> (c.nv - RB)) : c.sample0;
  return s < batch ? s : batch - 1;   // padding samples of a ragged last workgroup
}

// Three sums of consecutive accumulators acc, acc+1, acc+2 (the Pauli sums of
// one single-qubit gradient), reduced together.  Each thread's sums over its
// own amplitudes arrive in the state's precision; they are widened to FP64
// before the cross-lane tree, so every sum over amplitudes beyond one thread's
// registers is FP64, and the partials are stored as FP64.
template <typename T, int K>
__device__ __forceinline__ void write_acc3(const Ctx<T, K> &c, const PassArgs<T> &a, T x, T y, T z, int acc) {
  double xd = (double)x, yd = (double)y, zd_ = (double)z;
  if (__builtin_amdgcn_readfirstlane(c.seg_log) == 6) {
    const double v = wave_sum3_transposed(xd, yd, zd_, c.lane);
    if (c.pwriter3) c.pslot3[(long long)acc * c.pstride] = v;
    return;
  } else {
    xd = seg_sum_dpp(xd, c.seg_log);
    yd = seg_sum_dpp(yd, c.seg_log);
    zd_ = seg_sum_dpp(zd_, c.seg_log);
  }
  if (c.pwriter) {
    double *p = c.pslot + (long long)acc * c.pstride;
    p[0] = xd;
    p[c.pstride] = yd;
    p[2 * c.pstride] = zd_;
  }
}

// One sum (a thread's share, any precision) reduced over its segment in FP64.
template <typename T, int K>
__device__ __forceinline__ void write_acc(const Ctx<T, K> &c, const PassArgs<T> &a, double v, int acc) {
  // one uniform test: whole-wave segments (every single-sample tile) take the
  // straight-line reduction
  if (__builtin_amdgcn_readfirstlane(c.seg_log) == 6)
    v = wave_sum_dpp(v);
  else
    v = seg_sum_dpp(v, c.seg_log);
  if (c.pwriter) c.pslot[(long long)acc * c.pstride] = v;
}

template <typename T>
__device__ __forceinline__ kptr<cplx<T>> op_mat(const PassArgs<T> &a, const UOp &op, int s) {
  return (op.flags & F_PERSAMPLE) ? a.mats_ps + (size_t)s * a.mats_ps_stride + op.mat : a.mats + op.mat;
}

// dispatch helpers on compile-time register bits.  Each case carries a distinct
// empty asm comment so that the optimiser cannot merge the case bodies into
// one body indexed through pointers (which would demote the register tile to
// scratch memory); the comment emits no instruction.
#define TQS_CASE_MARK(id) asm volatile("; tqs case " #id ::)
template <typename T, bool ADJ>
__device__ __forceinline__ void u1_dispatch(cplx<T> (&v)[NREG], const cplx<T> m[4], int r, int flags) {
  if (flags & F_DIAGONAL) {
    switch (r) {
      case 0: TQS_CASE_MARK(d0); u1_apply_diag<T, 0, ADJ>(v, m); TQS_CASE_MARK(ed0); break;
      case 1: TQS_CASE_MARK(d1); u1_apply_diag<T, 1, ADJ>(v, m); TQS_CASE_MARK(ed1); break;
      case 2: TQS_CASE_MARK(d2); u1_apply_diag<T, 2, ADJ>(v, m); TQS_CASE_MARK(ed2); break;
      default: TQS_CASE_MARK(d3); u1_apply_diag<T, 3, ADJ>(v, m); TQS_CASE_MARK(ed3); break;
    }
  } else if (flags & F_REAL) {
    switch (r) {
      case 0: TQS_CASE_MARK(r0); u1_apply_real<T, 0, ADJ>(v, m); TQS_CASE_MARK(er0); break;
      case 1: TQS_CASE_MARK(r1); u1_apply_real<T, 1, ADJ>(v, m); TQS_CASE_MARK(er1); break;
      case 2: TQS_CASE_MARK(r2); u1_apply_real<T, 2, ADJ>(v, m); TQS_CASE_MARK(er2); break;
      default: TQS_CASE_MARK(r3); u1_apply_real<T, 3, ADJ>(v, m); TQS_CASE_MARK(er3); break;
    }
  } else {
    switch (r) {
      case 0: TQS_CASE_MARK(c0); u1_apply<T, 0, ADJ>(v, m); TQS_CASE_MARK(ec0); break;
      case 1: TQS_CASE_MARK(c1); u1_apply<T, 1, ADJ>(v, m); TQS_CASE_MARK(ec1); break;
      case 2: TQS_CASE_MARK(c2); u1_apply<T, 2, ADJ>(v, m); TQS_CASE_MARK(ec2); break;
      default: TQS_CASE_MARK(c3); u1_apply<T, 3, ADJ>(v, m); TQS_CASE_MARK(ec3); break;
    }
  }
}

// A group of complex 2x2 gates on the register bits of MASK, each with its
// own matrix m[r]; straight-line code per mask.
template <typename T, int MASK, bool ADJ>
__device__ __forceinline__ void u1g_apply(cplx<T> (&v)[NREG], const cplx<T> (&m)[RB][4]) {
  if (MASK & 1) u1_apply<T, 0, ADJ>(v, m[0]);
  if (MASK & 2) u1_apply<T, 1, ADJ>(v, m[1]);
  if (MASK & 4) u1_apply<T, 2, ADJ>(v, m[2]);
  if (MASK & 8) u1_apply<T, 3, ADJ>(v, m[3]);
}

// Two structured gates of one kind on disjoint register-bit pairs (a,b), (c,d),
// the pair holding bit 0 first; key = a<<6 | b<<4 | c<<2 | d.
#define TQS_U2G_CASES(X)                                                                      \
  X(0, 1, 2, 3) X(0, 1, 3, 2) X(1, 0, 2, 3) X(1, 0, 3, 2) X(0, 2, 1, 3) X(0, 2, 3, 1) X(2, 0, 1, 3) \
  X(2, 0, 3, 1) X(0, 3, 1, 2) X(0, 3, 2, 1) X(3, 0, 1, 2) X(3, 0, 2, 1)

// One grouped op in one piece of straight-line code: in the backward pass the
// gradient sums at the group output, then the inverse gates on psi and lambda
// (fewer merge points in the op loop, so fewer register copies).
template <typename T, int K, bool BWD, int MASK>
__device__ __forceinline__ void u1g_step(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                         cplx<T> (&vl)[NREG], const cplx<T> (&m)[RB][4], const int (&ga)[RB],
                                         bool psi) {
  if (BWD) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (!((MASK >> r) & 1) || ga[r] < 0) continue;
      T sx = 0, sy = 0, sz = 0;
      if (r == 0) u1_grad<T, 0>(vp, vl, sx, sy, sz);
      if (r == 1) u1_grad<T, 1>(vp, vl, sx, sy, sz);
      if (r == 2) u1_grad<T, 2>(vp, vl, sx, sy, sz);
      if (r == 3) u1_grad<T, 3>(vp, vl, sx, sy, sz);
      write_acc3(c, a, sx, sy, sz, ga[r]);
    }
  }
  if (!BWD || psi) u1g_apply<T, MASK, BWD>(vp, m);
  if (BWD) u1g_apply<T, MASK, true>(vl, m);
}

template <typename T, int K, bool BWD>
__device__ __forceinline__ void u1g_run(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                        cplx<T> (&vl)[NREG], const cplx<T> (&m)[RB][4], const int (&ga)[RB],
                                        int mask, bool psi) {
  switch (mask) {
#define X(k) \
  case k: { TQS_CASE_MARK(G##k); u1g_step<T, K, BWD, k>(c, a, vp, vl, m, ga, psi); TQS_CASE_MARK(eG##k); break; }
    X(3) X(5) X(6) X(7) X(9) X(10) X(11) X(12) X(13) X(14) X(15)
#undef X
    default: break;
  }
}

template <typename T, int K, bool BWD, int KIND, int A, int B, int C, int D>
__device__ __forceinline__ void u2g_step(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                         cplx<T> (&vl)[NREG], kptr<cplx<T>> m0, kptr<cplx<T>> m1, int a0,
                                         int a1, bool psi) {
  if (BWD && KIND == U2_MS) {
    if (a0 >= 0) write_acc(c, a, u2s_grad<T, A, B, true>(vp, vl), a0);
    if (a1 >= 0) write_acc(c, a, u2s_grad<T, C, D, true>(vp, vl), a1);
  }
  if (!BWD || psi) {
    u2s_apply<T, A, B, BWD, KIND>(vp, m0);
    u2s_apply<T, C, D, BWD, KIND>(vp, m1);
  }
  if (BWD) {
    u2s_apply<T, A, B, true, KIND>(vl, m0);
    u2s_apply<T, C, D, true, KIND>(vl, m1);
  }
}

template <typename T, int K, bool BWD, int KIND>
__device__ __forceinline__ void u2g_run_k(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                          cplx<T> (&vl)[NREG], kptr<cplx<T>> m0, kptr<cplx<T>> m1, int a0,
                                          int a1, int key, bool psi) {
  switch (key) {
#define X(p, q, r, t)                                                                          \
  case (p << 6 | q << 4 | r << 2 | t): {                                                      \
    TQS_CASE_MARK(H##p##q##r##t##_##KIND);                                                    \
    u2g_step<T, K, BWD, KIND, p, q, r, t>(c, a, vp, vl, m0, m1, a0, a1, psi);                  \
    TQS_CASE_MARK(eH##p##q##r##t##_##KIND);                                                   \
    break;                                                                                    \
  }
    TQS_U2G_CASES(X)
#undef X
    default: break;
  }
}

// The brick-layer stage program (OP_SEQ), straight-line.  Forward: pair gates
// on (0,1),(2,3); 2x2 gates on bits 0-3; [pair gate on (1,2); [2x2 gates on
// bits 1, 2]].  Backward runs the steps in reverse, each step's gradients taken
// at its output before its inverse is applied to psi and lambda.
template <typename T, int K, bool BWD, int R>
__device__ __forceinline__ void seq_u1(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                       cplx<T> (&vl)[NREG], kptr<DevSeq> q, int slot) {
  const int mo = uni(q->mat[slot]);
  kptr<cplx<T>> ms = a.mats + mo;
  cplx<T> m[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) m[k] = kld(ms, k);
  if (BWD) {
    const int ga = uni(q->acc[slot]);
    if (ga >= 0) {
      T sx = 0, sy = 0, sz = 0;
      u1_grad<T, R>(vp, vl, sx, sy, sz);
      write_acc3(c, a, sx, sy, sz, ga);
    }
  }
  u1_apply<T, R, BWD>(vp, m);
  if (BWD) u1_apply<T, R, true>(vl, m);
}

template <typename T, int K, bool BWD, int KIND, int R0, int R1>
__device__ __forceinline__ void seq_u2(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                       cplx<T> (&vl)[NREG], kptr<DevSeq> q, int slot) {
  kptr<cplx<T>> mg = a.mats + uni(q->mat[slot]);
  if (BWD && KIND == U2_MS) {
    const int ga = uni(q->acc[slot]);
    if (ga >= 0) write_acc(c, a, u2s_grad<T, R0, R1, true>(vp, vl), ga);
  }
  u2s_apply<T, R0, R1, BWD, KIND>(vp, mg);
  if (BWD) u2s_apply<T, R0, R1, true, KIND>(vl, mg);
}

template <typename T, int K, bool BWD, int KIND, int LEN>
__device__ __forceinline__ void seq_step(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                         cplx<T> (&vl)[NREG], kptr<DevSeq> q) {
  if (!BWD) {
    seq_u2<T, K, false, KIND, 0, 1>(c, a, vp, vl, q, 0);
    seq_u2<T, K, false, KIND, 2, 3>(c, a, vp, vl, q, 1);
    seq_u1<T, K, false, 0>(c, a, vp, vl, q, 2);
    seq_u1<T, K, false, 1>(c, a, vp, vl, q, 3);
    seq_u1<T, K, false, 2>(c, a, vp, vl, q, 4);
    seq_u1<T, K, false, 3>(c, a, vp, vl, q, 5);
    if (LEN >= 3) seq_u2<T, K, false, KIND, 1, 2>(c, a, vp, vl, q, 6);
    if (LEN >= 4) {
      seq_u1<T, K, false, 1>(c, a, vp, vl, q, 7);
      seq_u1<T, K, false, 2>(c, a, vp, vl, q, 8);
    }
  } else {
    // gates acting on distinct bits commute: within a step the gradients can
    // be taken in any order, all at the step's output
    if (LEN >= 4) {
      seq_u1<T, K, true, 2>(c, a, vp, vl, q, 8);
      seq_u1<T, K, true, 1>(c, a, vp, vl, q, 7);
    }
    if (LEN >= 3) seq_u2<T, K, true, KIND, 1, 2>(c, a, vp, vl, q, 6);
    seq_u1<T, K, true, 3>(c, a, vp, vl, q, 5);
    seq_u1<T, K, true, 2>(c, a, vp, vl, q, 4);
    seq_u1<T, K, true, 1>(c, a, vp, vl, q, 3);
    seq_u1<T, K, true, 0>(c, a, vp, vl, q, 2);
    seq_u2<T, K, true, KIND, 2, 3>(c, a, vp, vl, q, 1);
    seq_u2<T, K, true, KIND, 0, 1>(c, a, vp, vl, q, 0);
  }
}

template <typename T, int K, bool BWD>
__device__ __forceinline__ void seq_run(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> (&vp)[NREG],
                                        cplx<T> (&vl)[NREG], kptr<DevSeq> q, int len, int sub) {
  switch (sub * 8 + len) {
#define X(kind, l) \
  case kind * 8 + l: { TQS_CASE_MARK(S##kind##l); seq_step<T, K, BWD, kind, l>(c, a, vp, vl, q); TQS_CASE_MARK(eS##kind##l); break; }
    X(U2_MS, 2) X(U2_MS, 3) X(U2_MS, 4) X(U2_ECR, 2) X(U2_ECR, 3) X(U2_ECR, 4)
#undef X
    default: break;
  }
}




template <typename T>
__device__ __forceinline__ void u1_grad_dispatch(const cplx<T> (&p)[NREG], const cplx<T> (&l)[NREG],
                                                 int r, T &sx, T &sy, T &sz) {
  switch (r) {
    case 0: TQS_CASE_MARK(g0); u1_grad<T, 0>(p, l, sx, sy, sz); TQS_CASE_MARK(eg0); break;
    case 1: TQS_CASE_MARK(g1); u1_grad<T, 1>(p, l, sx, sy, sz); TQS_CASE_MARK(eg1); break;
    case 2: TQS_CASE_MARK(g2); u1_grad<T, 2>(p, l, sx, sy, sz); TQS_CASE_MARK(eg2); break;
    default: TQS_CASE_MARK(g3); u1_grad<T, 3>(p, l, sx, sy, sz); TQS_CASE_MARK(eg3); break;
  }
}

#define TQS_U2_CASES(X) \
  X(0, 1) X(0, 2) X(0, 3) X(1, 0) X(1, 2) X(1, 3) X(2, 0) X(2, 1) X(2, 3) X(3, 0) X(3, 1) X(3, 2)

template <typename T, bool ADJ>
__device__ __forceinline__ void u2_dispatch(cplx<T> (&v)[NREG], kptr<cplx<T>> m, int r0, int r1) {
  switch (r0 * 4 + r1) {
#define X(a, b) \
  case a * 4 + b: TQS_CASE_MARK(u##a##b); u2_apply<T, a, b, ADJ>(v, m); TQS_CASE_MARK(eu##a##b); break;
    TQS_U2_CASES(X)
#undef X
  }
}

template <typename T, bool ADJ, int KIND>
__device__ __forceinline__ void u2s_dispatch_k(cplx<T> (&v)[NREG], kptr<cplx<T>> m, int r0, int r1) {
  switch (r0 * 4 + r1) {
#define X(a, b) \
  case a * 4 + b: TQS_CASE_MARK(s##a##b##_##KIND); u2s_apply<T, a, b, ADJ, KIND>(v, m); TQS_CASE_MARK(es##a##b##_##KIND); break;
    TQS_U2_CASES(X)
#undef X
  }
}

template <typename T, bool ADJ>
__device__ __forceinline__ void u2_apply_any(cplx<T> (&v)[NREG], kptr<cplx<T>> m, int r0, int r1, int sub) {
  switch (sub) {
    case U2_CNOT: u2s_dispatch_k<T, ADJ, U2_CNOT>(v, m, r0, r1); break;
    case U2_SWAP: u2s_dispatch_k<T, ADJ, U2_SWAP>(v, m, r0, r1); break;
    case U2_CZ: u2s_dispatch_k<T, ADJ, U2_CZ>(v, m, r0, r1); break;
    case U2_MS: u2s_dispatch_k<T, ADJ, U2_MS>(v, m, r0, r1); break;
    case U2_ECR: u2s_dispatch_k<T, ADJ, U2_ECR>(v, m, r0, r1); break;
    case U2_DIAG: u2s_dispatch_k<T, ADJ, U2_DIAG>(v, m, r0, r1); break;
    default: u2_dispatch<T, ADJ>(v, m, r0, r1); break;
  }
}


template <typename T, bool XX>
__device__ __forceinline__ T u2s_grad_dispatch(const cplx<T> (&p)[NREG], const cplx<T> (&l)[NREG], int r0,
                                               int r1) {
  switch (r0 * 4 + r1) {
#define X(a, b) \
  case a * 4 + b: { TQS_CASE_MARK(g##a##b##_##XX); const T r_ = u2s_grad<T, a, b, XX>(p, l); TQS_CASE_MARK(eg##a##b##_##XX); return r_; }
    TQS_U2_CASES(X)
#undef X
  }
  return T(0);
}

template <typename T>
__device__ __forceinline__ T u2_grad_dispatch(const cplx<T> (&p)[NREG], const cplx<T> (&l)[NREG], int r0,
                                              int r1, int code) {
  switch (r0 * 4 + r1) {
#define X(a, b) \
  case a * 4 + b: { TQS_CASE_MARK(q##a##b); const T r_ = u2_grad<T, a, b>(p, l, code); TQS_CASE_MARK(eq##a##b); return r_; }
    TQS_U2_CASES(X)
#undef X
  }
  return T(0);
}

// 16-point Walsh-Hadamard transform in registers: w[m] <- sum_j w[j] (-1)^{popc(j & m)}
template <typename T>
__device__ __forceinline__ void wht16(T (&w)[NREG]) {
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
      if (j & (1 << r)) continue;
      const T a = w[j], b = w[j | (1 << r)];
      w[j] = a + b;
      w[j | (1 << r)] = a - b;
    }
}

// The 16 register values as one vector: an element chosen by a wave-uniform
// index is then one indexed register move (no branch per pick).
template <typename T>
struct Vec16 {
  typedef T type __attribute__((ext_vector_type(16)));
};

// Phase angle of entry `idx` of a diagonal op's split tables (the TL entries
// first, then TH) for the tile whose bits outside the tile are `base`, and
// sample `smp` for terms with per-sample angles: the sum of the term angles
// (FP64) selected by the entry's bits.
__device__ __forceinline__ double diag_entry_angle(kptr<DevDiag> dg, kptr<DevTerm> terms, kptr<double> dbl,
                                                   kptr<double> dbl_ps, int dbl_ps_stride, uint32_t base,
                                                   int smp, int idx) {
  const int h = uni(dg->h), nx = uni(dg->n_extra);
  const int tbeg = uni(dg->term_begin), tend = uni(dg->term_end);
  const int ex0 = nx > 0 ? uni(dg->extra[0]) : -1, ex1 = nx > 1 ? uni(dg->extra[1]) : -1;
  const int nl = 1 << (h + nx);
  const bool low = idx < nl;
  const int e = low ? idx : idx - nl;
  double ang = 0.0;
  for (int ti = tbeg; ti < tend; ++ti) {
    kptr<DevTerm> tm = terms + ti;
    const int tab_id = uni(tm->tab);
    if (low ? (tab_id != 0) : (tab_id == 0)) continue;
    const int nb = uni(tm->nbits);
    int v = 0;
    for (int q = 0; q < nb; ++q) {
      int bit;
      const int tb = uni(tm->tb[q]);
      if (tb < 0) {
        bit = (base >> uni(tm->gb[q])) & 1;
      } else if (low) {
        if (tb < h)
          bit = (e >> tb) & 1;
        else
          bit = (e >> (h + (tb == ex0 ? 0 : (tb == ex1 ? 1 : 2)))) & 1;
      } else {
        bit = (e >> (tb - h)) & 1;
      }
      v = (v << 1) | bit;
    }
    const int ang_off = uni(tm->ang);
    kptr<double> an = uni(tm->per_sample) ? dbl_ps + (size_t)smp * dbl_ps_stride + ang_off : dbl + ang_off;
    ang += an[v];
  }
  return ang;
}

// The split phase tables of every diagonal op of the pass, in LDS: copied from
// the prebuilt tables of tile position `tile` for ops with shared angles,
// built here for ops with per-sample angles.
template <typename T, int K>
__device__ __forceinline__ void build_diag_tables(const Ctx<T, K> &c, const PassArgs<T> &a, cplx<T> *tab,
                                                  int tile) {
  kptr<DevPass> P = a.pass;
  const int nd = uni(P->n_diag), db = uni(P->diag_begin);
  for (int di = 0; di < nd; ++di) {
    kptr<DevDiag> dg = a.diags + db + di;
    const int h = uni(dg->h), nx = uni(dg->n_extra), off = uni(dg->lds_off), gt = uni(dg->gtab);
    const int n_ent = (1 << (h + nx)) + (1 << (K - h));
    if (gt >= 0) {
      const cplx<T> *src = a.diag_tabs + gt + (long long)tile * n_ent;
      for (int idx = c.tid + c.sub * Ctx<T, K>::NT; idx < n_ent; idx += Ctx<T, K>::NT * c.nsub)
        tab[off + idx] = src[idx];
      continue;
    }
    for (int idx = c.tid + c.sub * Ctx<T, K>::NT; idx < n_ent; idx += Ctx<T, K>::NT * c.nsub) {
      const double ang = diag_entry_angle(dg, a.terms, a.dbl, a.dbl_ps, a.dbl_ps_stride, c.base, c.sample0, idx);
      double s, co;
      sincos(ang, &s, &co);
      tab[off + idx] = cmk<T>((T)co, (T)s);
    }
  }
}

// Prebuilt split tables of the diagonal ops with shared angles, for every tile
// position of their pass (one thread per entry).  Run after k_prep, which
// writes the angles.
template <typename T>
struct DiagTabArgs {
  kptr<DevPass> passes;
  kptr<DevDiag> diags;
  kptr<DevTerm> terms;
  kptr<DiagJob> jobs;
  kptr<double> dbl;
  cplx<T> *out;
};

template <typename T>
__global__ void __launch_bounds__(256) k_diag_tables(DiagTabArgs<T> a) {
  kptr<DiagJob> j = a.jobs + blockIdx.y;
  const int entries = uni(j->entries), tiles_log = uni(j->tiles_log);
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= ((long long)entries << tiles_log)) return;
  const int tile = (int)(i / entries), idx = (int)(i % entries);
  kptr<DevPass> P = a.passes + uni(j->pass);
  uint32_t base = 0;
  for (int r = 0; r < tiles_log; ++r)
    if ((tile >> r) & 1) base |= 1u << uni(P->rest[r]);
  kptr<DevDiag> dg = a.diags + uni(j->diag);
  const double ang = diag_entry_angle(dg, a.terms, a.dbl, a.dbl, 0, base, 0, idx);
  double s, co;
  sincos(ang, &s, &co);
  a.out[uni(dg->gtab) + i] = cmk<T>((T)co, (T)s);
}

// Split-table phase of tile element t.  The extra index bits are passed in
// registers (x0..x2 = tile-bit positions, unused ones point at bit 31 of t,
// which is always 0).
struct DiagView {
  int h, nx, lds_off, th_off, x0, x1, x2;
};

__device__ __forceinline__ DiagView diag_view(kptr<DevDiag> dg) {
  DiagView v;
  v.h = uni(dg->h);
  v.nx = uni(dg->n_extra);
  v.lds_off = uni(dg->lds_off);
  v.th_off = v.lds_off + (1 << (v.h + v.nx));
  v.x0 = v.nx > 0 ? uni(dg->extra[0]) : 31;
  v.x1 = v.nx > 1 ? uni(dg->extra[1]) : 31;
  v.x2 = v.nx > 2 ? uni(dg->extra[2]) : 31;
  return v;
}

template <typename T>
__device__ __forceinline__ cplx<T> diag_phase(const DiagView &d, const cplx<T> *tab, int t) {
  const int il = (t & ((1 << d.h) - 1)) | (((t >> d.x0) & 1) << d.h) | (((t >> d.x1) & 1) << (d.h + 1)) |
                 (((t >> d.x2) & 1) << (d.h + 2));
  return cmul(tab[d.lds_off + il], tab[d.th_off + (t >> d.h)]);
}

// MFMA 16x16x4 (f32 and f64).  Operands: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; result register r of lane l is D[4*(l/16)+r][l%16] for f32
// and D[(l/16)+4r][l%16] for f64.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 V;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mfma<double> {
  typedef f64x4 V;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Ordering between two stages.  The next reader of an element may be another
// wave of the workgroup, so in general a workgroup barrier.  In passes with
// full-layer matrix ops (one wave per copy of the tile, NT = 64) every stage
// but the matrix ops touches only the wave's own copy, and a wave's LDS
// accesses complete in order: keeping the compiler from moving LDS accesses
// across this point suffices.
template <int K, bool DENSE>
__device__ __forceinline__ void stage_sync() {
  if constexpr (DENSE && (1 << (K - RB)) == 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Workgroup barrier for LDS traffic alone: global loads still in flight (the
// next matrix op's rows of U) are not waited for.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Registers carried between the full-layer matrix ops of a pass: the next op's
// rows of U (lane layout of dense_fetch), fetched while the current op runs.
template <typename T, bool DENSE>
struct DenseCarry {
  cplx<T> u[DENSE ? 16 : 1];
};

// The wave's MFMA A-operand of a 2^NV x 2^NV layer matrix: row block
// sub % (2^NV / 16), lane l holding row (l % 16) of the block and column
// 4 kb + l / 16 in u[kb].  Backward takes U^dagger: the same lanes read the
// transposed entry, and the conjugate is applied when the products are summed.
template <typename T, int K, int NV, bool BWD>
__device__ __forceinline__ void dense_fetch(const Ctx<T, K> &c, kptr<cplx<T>> Ug, cplx<T> (&u)[16]) {
  constexpr int DIM = 1 << NV, KB = DIM / 4, RBK = DIM / 16;
  const int ar = (c.sub % RBK) * 16 + (c.lane & 15);
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int kk = kb * 4 + (c.lane >> 4);
    u[kb] = kld(Ug, BWD ? kk * DIM + ar : ar * DIM + kk);
  }
  // every entry defined on every path, so that the carry stays in registers
#pragma unroll
  for (int kb = KB; kb < 16; ++kb) u[kb] = cmk<T>(0, 0);
}

template <typename T, int K, bool BWD>
__device__ __forceinline__ void dense_fetch_nv(const Ctx<T, K> &c, kptr<cplx<T>> Ug, cplx<T> (&u)[16]) {
  switch (c.nv) {
    case 4: dense_fetch<T, K, 4, BWD>(c, Ug, u); break;
    case 5: dense_fetch<T, K, 5, BWD>(c, Ug, u); break;
    default: dense_fetch<T, K, 6, BWD>(c, Ug, u); break;
  }
}

// A full-layer matrix op (the unitary operation of Sec. 2.2.1) on the matrix
// cores: X <- U X forward, U^dagger X backward (on psi and on lambda), for every
// sample of the tile: out[j][s] = sum_k U[j][k] X[k][s] with X[k][s] = tile
// element s * 2^NV + k.  A pass with such ops runs DENSE_SUBS waves per tile,
// each on its own copy of the tile (copies CS elements apart); with K = 10 the
// product has exactly DENSE_SUBS 16 x 16 output blocks (2^NV / 16 row blocks
// times 2^(K-NV) / 16 sample blocks), one per wave.  The wave's rows of U
// arrive in `carry` (fetched during the previous op, or before the first);
// the next op's rows (matrix offset `next`, -1 if none) are requested at once.
// Four independent real MFMA chains (re*re, im*im, re*im, im*re); once every
// wave has read its copy, each writes its block into all copies.  The reads
// are of the wave's own copy, written last by the wave itself or before the
// barrier that ends the previous matrix op.
template <typename T, int K, int NV, bool BWD>
__device__ __forceinline__ void dense_stage(const Ctx<T, K> &c, cplx<T> *Lp, cplx<T> *Ll, cplx<T> (&carry)[16],
                                            kptr<cplx<T>> mats, int next) {
  typedef typename Mfma<T>::V V;
  constexpr int DIM = 1 << NV, KB = DIM / 4, RBK = DIM / 16;
  static_assert(RBK * ((1 << (K - NV)) / 16) == DENSE_SUBS, "one 16 x 16 output block per wave");
  constexpr int CS = (BWD ? 2 : 1) << K;
  const int lane = c.lane;
  const int mb = c.sub % RBK, nb = c.sub / RBK;
  const int bj = nb * 16 + (lane & 15);
  cplx<T> u[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) u[kb] = carry[kb];
  if (next >= 0) dense_fetch<T, K, NV, BWD>(c, mats + next, carry);
  stage_sync<K, true>();
  const V z = {0, 0, 0, 0};
  V p0 = z, p1 = z, p2 = z, p3 = z, l0 = z, l1 = z, l2 = z, l3 = z;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int e = swz<T>(bj * DIM + kb * 4 + (lane >> 4));
    const cplx<T> x = Lp[e];
    p0 = Mfma<T>::run(u[kb].x, x.x, p0);
    p1 = Mfma<T>::run(u[kb].y, x.y, p1);
    p2 = Mfma<T>::run(u[kb].x, x.y, p2);
    p3 = Mfma<T>::run(u[kb].y, x.x, p3);
    if (BWD) {
      const cplx<T> y = Ll[e];
      l0 = Mfma<T>::run(u[kb].x, y.x, l0);
      l1 = Mfma<T>::run(u[kb].y, y.y, l1);
      l2 = Mfma<T>::run(u[kb].x, y.y, l2);
      l3 = Mfma<T>::run(u[kb].y, y.x, l3);
    }
  }
  lds_barrier();
  cplx<T> *base = Lp - (long long)c.sub * CS;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = swz<T>(bj * DIM + mb * 16 + Mfma<T>::row(lane, r));
    // backward: u holds U entries, the product is with their conjugates
    const cplx<T> vp = BWD ? cmk<T>(p0[r] + p1[r], p2[r] - p3[r]) : cmk<T>(p0[r] - p1[r], p2[r] + p3[r]);
#pragma unroll
    for (int q = 0; q < DENSE_SUBS; ++q) base[q * CS + e] = vp;
    if (BWD) {
      const cplx<T> vl = cmk<T>(l0[r] + l1[r], l2[r] - l3[r]);
#pragma unroll
      for (int q = 0; q < DENSE_SUBS; ++q) base[q * CS + (1 << K) + e] = vl;
    }
  }
  lds_barrier();
}

// Hadamard gates on the register bits of MASK as the fast Walsh-Hadamard
// transform: add / subtract butterflies, then one scale by 2^(-|MASK|/2).
template <typename T, int MASK>
__device__ __forceinline__ void wht_apply(cplx<T> (&v)[NREG]) {
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (!((MASK >> r) & 1)) continue;
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
      if (j & (1 << r)) continue;
      const cplx<T> a = v[j], b = v[j | (1 << r)];
      v[j] = cmk(a.x + b.x, a.y + b.y);
      v[j | (1 << r)] = cmk(a.x - b.x, a.y - b.y);
    }
  }
  constexpr int k = __builtin_popcount(MASK);
  const T sc = (k & 1) ? (T)(0.70710678118654752440 / (double)(1 << (k / 2))) : (T)(1.0 / (double)(1 << (k / 2)));
#pragma unroll
  for (int j = 0; j < NREG; ++j) v[j] = cmk(v[j].x * sc, v[j].y * sc);
}

template <typename T>
__device__ __forceinline__ void wht_dispatch(cplx<T> (&v)[NREG], int mask) {
  switch (mask) {
#define X(k) \
  case k: TQS_CASE_MARK(W##k); wht_apply<T, k>(v); TQS_CASE_MARK(eW##k); break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)
#undef X
    default: break;
  }
}

template <typename T, int K, bool BWD, bool DENSE, bool DIAG>
// psi_upto (backward): ops at processing position >= psi_upto skip the psi
// uncompute -- the pass's last stage when psi is neither stored nor needed
// afterwards (no later op of the stage takes a gradient from it).
__device__ __forceinline__ void run_stage(const Ctx<T, K> &c, const PassArgs<T> &a, const UStage &S, cplx<T> *Lp,
                          cplx<T> *Ll, const cplx<T> *tab, DenseCarry<T, DENSE> &dc, bool grad_only,
                          int psi_upto = 1 << 30) {
  constexpr int NT = Ctx<T, K>::NT;
  if constexpr (DENSE) {
    if (S.flags & STAGE_DENSE) {
      const int next = S.dense_next[BWD ? 1 : 0];
      switch (c.nv) {
        case 4: dense_stage<T, K, 4, BWD>(c, Lp, Ll, dc.u, a.mats, next); break;
        case 5: dense_stage<T, K, 5, BWD>(c, Lp, Ll, dc.u, a.mats, next); break;
        default: dense_stage<T, K, 6, BWD>(c, Lp, Ll, dc.u, a.mats, next); break;
      }
      return;
    }
  }
  const int op0_kind = uni(a.ops[S.op_begin].kind);
  if (op0_kind == OP_PERM) {
    // in-tile permutation: forward new[t] = old[src(t)], backward the inverse
    kptr<DevPerm> pm = a.perms + uni(a.ops[S.op_begin].aux);
    cplx<T> vp[NREG], vl[NREG];
    int srcs[NREG];
    uint32_t sthr = uniu(pm->cxor);
    for (int b = 0; b < K - RB; ++b) {
      const uint32_t col = uniu(pm->cols[b]);
      if ((c.tid >> b) & 1) sthr ^= col;
    }
    uint32_t rcol[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) rcol[b] = uniu(pm->cols[K - RB + b]);
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
      const int t = c.tid + i * NT;
      uint32_t s = sthr;
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if ((i >> b) & 1) s ^= rcol[b];
      srcs[i] = (int)s;
      const int rd = BWD ? t : (int)s;
      vp[i] = Lp[swz<T>(rd)];
      if (BWD) vl[i] = Ll[swz<T>(rd)];
    }
    stage_sync<K, DENSE>();
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
      const int t = c.tid + i * NT;
      const int wr = BWD ? srcs[i] : t;
      Lp[swz<T>(wr)] = vp[i];
      if (BWD) Ll[swz<T>(wr)] = vl[i];
    }
    stage_sync<K, DENSE>();
    return;
  }
  // thread tile base: the thread index spread over the non-register tile bits
  // in increasing order -- tid with a zero inserted at each register bit's
  // position, lowest first (each insertion sees the final positions below it)
  int tt = c.tid;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int p = S.rsorted[k];
    tt = ((tt >> p) << (p + 1)) | (tt & ((1 << p) - 1));
  }
  int toff[NREG], aoff[NREG];
  {
    const int o0 = 1 << S.rbits[0], o1 = 1 << S.rbits[1], o2 = 1 << S.rbits[2], o3 = 1 << S.rbits[3];
    const int st = swz<T>(tt), s0 = swz<T>(o0), s1 = swz<T>(o1), s2 = swz<T>(o2), s3 = swz<T>(o3);
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
      toff[j] = tt | ((j & 1) ? o0 : 0) | ((j & 2) ? o1 : 0) | ((j & 4) ? o2 : 0) | ((j & 8) ? o3 : 0);
      aoff[j] = st ^ ((j & 1) ? s0 : 0) ^ ((j & 2) ? s1 : 0) ^ ((j & 4) ? s2 : 0) ^ ((j & 8) ? s3 : 0);
    }
  }
  const int nops = S.op_end - S.op_begin;
  // gradient-only stage of a full-layer matrix pass: the wave group's own op,
  // requested before the tile is read
  const bool gonly = DENSE && (S.flags & STAGE_GRAD_ONLY);
  UOp own;
  if (gonly && c.sub < nops) own = load_op(a.ops + (BWD ? (S.op_end - 1 - c.sub) : (S.op_begin + c.sub)));
  cplx<T> vp[NREG], vl[NREG];
#pragma unroll
  for (int j = 0; j < NREG; ++j) {
    vp[j] = Lp[aoff[j]];
    if (BWD) vl[j] = Ll[aoff[j]];
  }
  const int s_thr = thread_sample(c, a.batch);
  for (int oi = 0; oi < nops; ++oi) {
    // gradient-only stages of full-layer matrix passes: the wave group takes
    // its own ops alone (see the ownership rule below)
    if (gonly && oi % c.nsub != c.sub) continue;
    const UOp op = (gonly && oi == c.sub) ? own : load_op(a.ops + (BWD ? (S.op_end - 1 - oi) : (S.op_begin + oi)));
    const bool upd_psi = oi < psi_upto;
    if (op.kind == OP_U1 || op.kind == OP_GRAD1) {
      kptr<cplx<T>> mg = op_mat(a, op, s_thr);
      if (BWD && (op.flags & F_GRAD)) {
        if (DENSE && op.kind == OP_GRAD1) {
          // a gradient-only op: taken by one wave group, in turn
          if (oi % c.nsub == c.sub) {
            Ctx<T, K> co = c;
            co.pwriter = c.pwriter_own;
            co.pwriter3 = c.pwriter3_own;
            T sx = 0, sy = 0, sz = 0;
            u1_grad_dispatch(vp, vl, op.r0, sx, sy, sz);
            write_acc3(co, a, sx, sy, sz, op.acc);
          }
        } else {
          T sx = 0, sy = 0, sz = 0;
          u1_grad_dispatch(vp, vl, op.r0, sx, sy, sz);
          write_acc3(c, a, sx, sy, sz, op.acc);
        }
      }
      if (op.kind == OP_U1) {
        cplx<T> m[4];
        if (op.flags & F_PERSAMPLE) {
          m[0] = kld(mg, 0); m[1] = kld(mg, 1); m[2] = kld(mg, 2); m[3] = kld(mg, 3);
        } else {
          // shared matrix: a uniform address, so scalar loads
          kptr<cplx<T>> ms = a.mats + op.mat;
          m[0] = kld(ms, 0); m[1] = kld(ms, 1); m[2] = kld(ms, 2); m[3] = kld(ms, 3);
        }
        if (!BWD || upd_psi) u1_dispatch<T, BWD>(vp, m, op.r0, op.flags);
        if (BWD) u1_dispatch<T, true>(vl, m, op.r0, op.flags);
      }
    } else if (op.kind == OP_U1G) {
      // the members commute, so every gradient is taken at the group's output
      kptr<DevGroup> gp = a.groups + op.aux;
      kptr<cplx<T>> mbase = (op.flags & F_PERSAMPLE) ? a.mats_ps + (size_t)s_thr * a.mats_ps_stride : a.mats;
      cplx<T> m[RB][4];
      int ga[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int mo = uni(gp->mat[r]);
        ga[r] = (op.flags & F_GRAD) ? uni(gp->acc[r]) : -1;
        kptr<cplx<T>> ms = mbase + (mo < 0 ? 0 : mo);
#pragma unroll
        for (int q = 0; q < 4; ++q) m[r][q] = kld(ms, q);
      }
      u1g_run<T, K, BWD>(c, a, vp, vl, m, ga, op.r0, upd_psi);
    } else if (op.kind == OP_WHT) {
      // H is its own inverse and has no parameter
      if (!BWD || upd_psi) wht_dispatch<T>(vp, op.r0);
      if (BWD) wht_dispatch<T>(vl, op.r0);
    } else if (op.kind == OP_SEQ) {
      seq_run<T, K, BWD>(c, a, vp, vl, a.seqs + op.aux, op.r0, op.sub);
    } else if (op.kind == OP_U2G) {
      kptr<DevGroup> gp = a.groups + op.aux;
      kptr<cplx<T>> m0 = a.mats + uni(gp->mat[0]), m1 = a.mats + uni(gp->mat[1]);
      const int a0 = (op.flags & F_GRAD) ? uni(gp->acc[0]) : -1, a1 = (op.flags & F_GRAD) ? uni(gp->acc[1]) : -1;
      if (op.sub == U2_MS)
        u2g_run_k<T, K, BWD, U2_MS>(c, a, vp, vl, m0, m1, a0, a1, op.r0, upd_psi);
      else
        u2g_run_k<T, K, BWD, U2_ECR>(c, a, vp, vl, m0, m1, a0, a1, op.r0, upd_psi);
    } else if (op.kind == OP_U2) {
      kptr<cplx<T>> mg = op_mat(a, op, s_thr);
      if (BWD && (op.flags & F_GRAD)) {
        T g;
        if (op.aux == (1 | (1 << 2)))
          g = u2s_grad_dispatch<T, true>(vp, vl, op.r0, op.r1);
        else if (op.aux == (3 | (3 << 2)))
          g = u2s_grad_dispatch<T, false>(vp, vl, op.r0, op.r1);
        else
          g = u2_grad_dispatch(vp, vl, op.r0, op.r1, op.aux);
        write_acc(c, a, g, op.acc);
      }
      if (!BWD || upd_psi) u2_apply_any<T, BWD>(vp, mg, op.r0, op.r1, op.sub);
      if (BWD) u2_apply_any<T, true>(vl, mg, op.r0, op.r1, op.sub);
    } else if (DENSE && op.kind == OP_GRAD2) {
      if (BWD && (op.flags & F_GRAD) && oi % c.nsub == c.sub) {
        Ctx<T, K> co = c;
        co.pwriter = c.pwriter_own;
        const T g = (op.aux == (1 | (1 << 2))) ? u2s_grad_dispatch<T, true>(vp, vl, op.r0, op.r1)
                                                : u2s_grad_dispatch<T, false>(vp, vl, op.r0, op.r1);
        write_acc(co, a, g, op.acc);
      }
    } else if (DIAG && op.kind == OP_DIAG) {
      kptr<DevDiag> dg = a.diags + uni(a.pass->diag_begin) + op.aux;
      const DiagView dv = diag_view(dg);
      if (BWD && (op.flags & F_GRAD)) {
        // w = Im(conj(l) p); parity sums over each term's bits via a register WHT
        T w[NREG];
#pragma unroll
        for (int j = 0; j < NREG; ++j) w[j] = vl[j].x * vp[j].y - vl[j].y * vp[j].x;
        wht16(w);
        // one entry per term with a parameter, laid out by the planner for this
        // stage: the parity-sum index m and the sign masks
        if (__builtin_amdgcn_readfirstlane(c.seg_log) == 6) {
          // whole-wave segments: the terms' sums reduced eight at a time as one
          // transposed tree; lane k of the wave writes term k of the chunk
          typename Vec16<T>::type wv;
#pragma unroll
          for (int j = 0; j < NREG; ++j) wv[j] = w[j];
          for (int k0 = 0; k0 < op.r1; k0 += 8) {
            double v8[8];
            int myacc = -1;
            // all eight descriptors requested at once (the planner pads the
            // table past the last op's terms); entries past r1 count zero
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              kptr<DevTermGrad> tg = a.tgrads + op.mat + k0 + q;
              const int tacc = uni(tg->acc), m = uni(tg->m) & (NREG - 1);
              const uint32_t tmask = uniu(tg->tmask), gmask = uniu(tg->gmask);
              const bool ok = k0 + q < op.r1;
              const int neg =
                  (__builtin_popcount(c.base & gmask) + __builtin_popcount((uint32_t)tt & tmask)) & 1;
              const double val = (double)wv[m];
              v8[q] = ok ? (neg ? -val : val) : 0.0;
              if (ok && (c.lane & 7) == q) myacc = tacc;
            }
            const double tot = wave_sum8_transposed(v8, c.lane);
            if (c.sub == 0 && c.lane < 8 && myacc >= 0) c.pslot[(long long)myacc * c.pstride] = tot;
          }
        } else {
          typename Vec16<T>::type wv;
#pragma unroll
          for (int j = 0; j < NREG; ++j) wv[j] = w[j];
          for (int k = 0; k < op.r1; ++k) {
            kptr<DevTermGrad> tg = a.tgrads + op.mat + k;
            const int tacc = uni(tg->acc), m = uni(tg->m) & (NREG - 1);
            const uint32_t tmask = uniu(tg->tmask), gmask = uniu(tg->gmask);
            const int neg = (__builtin_popcount(c.base & gmask) + __builtin_popcount((uint32_t)tt & tmask)) & 1;
            T val = wv[m];
            if (neg) val = -val;
            write_acc(c, a, val, tacc);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NREG; ++j) {
        cplx<T> d = diag_phase<T>(dv, tab, toff[j]);
        if (BWD) d = cconj(d);
        if (!BWD || upd_psi) vp[j] = cmul(vp[j], d);
        if (BWD) vl[j] = cmul(vl[j], d);
      }
    }
  }
  if (!grad_only) {
    const bool psi_live = !BWD || psi_upto > nops;
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
      if (psi_live) Lp[aoff[j]] = vp[j];
      if (BWD) Ll[aoff[j]] = vl[j];
    }
  }
  stage_sync<K, DENSE>();
}

// Embedding gradients of wires outside the embedding pass's tile, at the end of
// its backward (lambda in LDS is the adjoint state at the embedding output).
// The embedding output is a product state psi = (x)_k phi_k, so for an outside
// wire w (its bit fixed to beta_w in this tile)
//   <lambda| P_w |psi>|_tile = (P phi_w)(beta_w) * prod_{outside k != w} phi_k(beta_k)
//                              * sum_{tile} conj(lambda) psi_tile,
// with psi_tile the product over the tile's wires.  The last factor is a sum
// over the workgroup's elements, so each thread's share goes to write_acc.
template <typename T, int K>
__device__ __forceinline__ void outside_embed_grads(const Ctx<T, K> &c, const PassArgs<T> &a, kptr<DevPass> P,
                                                    const cplx<T> *Ll, uint32_t omask) {
  constexpr int NT = Ctx<T, K>::NT;
  const int n = c.n;
  const int emat = uni(P->embed_mat);
  kptr<cplx<T>> em = uni(P->embed_per_sample) ? a.mats_ps + (size_t)c.sample0 * a.mats_ps_stride + emat
                                              : a.mats + emat;
  // this thread's share of sum conj(lambda) psi_tile
  cplx<T> cth = cmk<T>(1, 0);
  for (int b = 0; b < K - RB; ++b) {
    const int p = uni(P->tpos[b]);
    cth = cmul(cth, kld(em + 4 * (n - 1 - p), ((c.tid >> b) & 1) ? 2 : 0));
  }
  cplx<T> f[RB][2];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    kptr<cplx<T>> m = em + 4 * (n - 1 - uni(P->tpos[K - RB + b]));
    f[b][0] = kld(m, 0);
    f[b][1] = kld(m, 2);
  }
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int i = 0; i < NREG; ++i) {
    cplx<T> v = cth;
#pragma unroll
    for (int b = 0; b < RB; ++b) v = cmul(v, f[b][(i >> b) & 1]);
    const cplx<T> l = Ll[swz<T>(c.tid + i * NT)];
    sx += (double)l.x * v.x + (double)l.y * v.y;     // conj(l) v
    sy += (double)l.x * v.y - (double)l.y * v.x;
  }
  const int tl = c.nv - K;
  int acc = uni(P->outside_acc);
  for (int q = 0; q < n; ++q) {
    if (!((omask >> q) & 1)) continue;
    const int beta = (c.base >> q) & 1;
    kptr<cplx<T>> mw = em + 4 * (n - 1 - q);
    const cplx<T> p0 = kld(mw, 0), p1 = kld(mw, 2);
    // product of the other outside wires' components (double)
    double rx = 1.0, ry = 0.0;
    for (int r = 0; r < tl; ++r) {
      const int k = uni(P->rest[r]);
      if (k == q) continue;
      const cplx<T> phi = kld(em + 4 * (n - 1 - k), ((c.base >> k) & 1) ? 2 : 0);
      const double nx = rx * phi.x - ry * phi.y, ny = rx * phi.y + ry * phi.x;
      rx = nx;
      ry = ny;
    }
    // (P phi)(beta) for P = X, Y, Z
    double cxr, cxi, cyr, cyi, czr, czi;
    if (beta) {
      cxr = p0.x; cxi = p0.y;           // X: phi_0
      cyr = -p0.y; cyi = p0.x;          // Y: i phi_0
      czr = -p1.x; czi = -p1.y;         // Z: -phi_1
    } else {
      cxr = p1.x; cxi = p1.y;           // X: phi_1
      cyr = p1.y; cyi = -p1.x;          // Y: -i phi_1
      czr = p0.x; czi = p0.y;           // Z: phi_0
    }
    const double cr[3] = {cxr, cyr, czr}, ci[3] = {cxi, cyi, czi};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double dr = cr[k] * rx - ci[k] * ry, di = cr[k] * ry + ci[k] * rx;
      write_acc(c, a, dr * sy + di * sx, acc + k);     // Im(D * S)
    }
    acc += 3;
  }
}

// Occupancy targets of the single-precision tile passes: forward 3 waves per
// SIMD (at most 168 registers), backward 2 (at most 256, shared by the
// architectural and accumulation registers).  Double precision and the
// matrix-core variant are left to the compiler.
template <typename T, bool BWD, bool DENSE>
struct PassOcc {
  static constexpr int waves = (sizeof(T) != 4 || DENSE) ? 1 : (BWD ? 2 : 3);
};

// DIAG = false: the variant for passes without diagonal layers (no phase
// tables, no diagonal op code).
template <typename T, int K, bool BWD, bool DENSE, bool DIAG>
__global__ void __launch_bounds__((1 << (K - RB)) * (DENSE ? DENSE_SUBS : 1))
__attribute__((amdgpu_waves_per_eu(PassOcc<T, BWD, DENSE>::waves))) k_pass(PassArgs<T> a) {
  constexpr int NT = 1 << (K - RB);
  constexpr int NE = 1 << K;
  constexpr int NSUB = DENSE ? DENSE_SUBS : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  Ctx<T, K> c;
  c.tid = NSUB > 1 ? (int)(threadIdx.x & (NT - 1)) : (int)threadIdx.x;
  c.lane = threadIdx.x & 63;
  c.sub = NSUB > 1 ? (int)(threadIdx.x >> (K - RB)) : 0;
  c.nsub = NSUB;
  // the wave group's copy of the tile: psi, then lambda (backward); the tables
  // after the last copy
  cplx<T> *Lp = reinterpret_cast<cplx<T> *>(smem) + (long long)c.sub * (BWD ? 2 : 1) * NE;
  cplx<T> *Ll = Lp + NE;
  cplx<T> *tab = reinterpret_cast<cplx<T> *>(smem) + NSUB * (BWD ? 2 : 1) * NE;
  kptr<DevPass> P = a.pass;

  c.n = uni(P->n);
  c.nv = uni(P->nv);
  c.multi = c.nv < K;
  c.base = 0;
  c.units_wg_base = 0;
  const int wg = blockIdx.x;
  if (!c.multi) {
    const int tl = c.nv - K;
    c.sample0 = wg >> tl;
    const uint32_t tile = (uint32_t)wg & ((1u << tl) - 1u);
    for (int r = 0; r < tl; ++r)
      if ((tile >> r) & 1) c.base |= 1u << uni(P->rest[r]);
    c.seg_log = (K - RB) < 6 ? (K - RB) : 6;
    c.units_wg_base = (int)tile * (NT >> c.seg_log);
  } else {
    c.sample0 = wg << (K - c.nv);
    const int tps = c.nv - RB;  // log2 threads per sample
    c.seg_log = tps < 6 ? tps : 6;
  }
  const int n = c.n;
  const long long sstride = 1ll << n;
  c.pslot = nullptr;
  c.pstride = 0;
  c.pwriter = 0;
  c.pslot3 = nullptr;
  c.pwriter3 = 0;
  if (BWD) set_partial_slot(c, a.partials, a.acc_region, a.batch, a.units);
  c.pwriter_own = c.pwriter;
  c.pwriter3_own = c.pwriter3;
  if (c.sub != 0) c.pwriter = c.pwriter3 = 0;

  if (DIAG && uni(P->n_diag) > 0)
    build_diag_tables<T, K>(c, a, tab, c.multi ? 0 : (int)((uint32_t)wg & ((1u << (c.nv - K)) - 1u)));

  // ---------------- load ----------------
  // Element e = tid + i * NT has tile index e; tile bits 0..K-RB-1 come from
  // tid and the top RB bits from i.
  uint32_t ptid = 0;
  for (int b = 0; b < K - RB; ++b)
    if ((c.tid >> b) & 1) ptid |= 1u << uni(P->tpos[b]);
  const int load_mode = uni(P->load_mode);
  const bool fwd_load_global = !BWD && load_mode == LOAD_GLOBAL;
  const bool fwd_embed = !BWD && load_mode == LOAD_EMBED;
  // map used for this direction's load and store
  const int lmap = uni(BWD ? P->has_store_map : P->has_load_map);
  const int smap = uni(BWD ? P->has_load_map : P->has_store_map);
  kptr<uint32_t> ltc = BWD ? P->store_tcol : P->load_tcol;
  kptr<uint32_t> lrc = BWD ? P->store_rcol : P->load_rcol;
  const uint32_t lc = uniu(BWD ? P->store_c : P->load_c);
  kptr<uint32_t> stc = BWD ? P->load_tcol : P->store_tcol;
  kptr<uint32_t> src_ = BWD ? P->load_rcol : P->store_rcol;
  const uint32_t sc = uniu(BWD ? P->load_c : P->store_c);
  uint32_t lbase = lc, lthr = 0, sbase = sc, sthr = 0;
  if (!c.multi) {
    const int tl = c.nv - K;
    const uint32_t tile = (uint32_t)wg & ((1u << tl) - 1u);
    for (int r = 0; r < tl; ++r) {
      const uint32_t l_ = uniu(lrc[r]), s_ = uniu(src_[r]);
      if ((tile >> r) & 1) {
        lbase ^= l_;
        sbase ^= s_;
      }
    }
    for (int b = 0; b < K - RB; ++b) {
      const uint32_t l_ = uniu(ltc[b]), s_ = uniu(stc[b]);
      if ((c.tid >> b) & 1) {
        lthr ^= l_;
        sthr ^= s_;
      }
    }
  }

  uint32_t treg[RB], lreg[RB], sreg[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    treg[b] = 1u << uni(P->tpos[K - RB + b]);
    lreg[b] = uniu(ltc[K - RB + b]);
    sreg[b] = uniu(stc[K - RB + b]);
  }
  const int embed_mat = uni(P->embed_mat), embed_ps = uni(P->embed_per_sample);

  if (fwd_embed) {
    // product state: amplitude = prod over wires of the wire's state component
    if (!c.multi) {
      kptr<cplx<T>> em = embed_ps ? a.mats_ps + (size_t)c.sample0 * a.mats_ps_stride + embed_mat
                                  : a.mats + embed_mat;
      // base (rest) bits and thread bits
      cplx<T> cth = cmk<T>(1, 0);
      for (int r = 0; r < c.nv - K; ++r) {
        const int p = uni(P->rest[r]);
        kptr<cplx<T>> m = em + 4 * (n - 1 - p);
        cth = cmul(cth, kld(m, ((c.base >> p) & 1) ? 2 : 0));
      }
      for (int b = 0; b < K - RB; ++b) {
        const int p = uni(P->tpos[b]);
        kptr<cplx<T>> m = em + 4 * (n - 1 - p);
        cth = cmul(cth, kld(m, ((c.tid >> b) & 1) ? 2 : 0));
      }
      cplx<T> f[RB][2];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int p = uni(P->tpos[K - RB + b]);
        kptr<cplx<T>> m = em + 4 * (n - 1 - p);
        f[b][0] = kld(m, 0);
        f[b][1] = kld(m, 2);
      }
#pragma unroll
      for (int i = 0; i < NREG; ++i) {
        cplx<T> v = cth;
#pragma unroll
        for (int b = 0; b < RB; ++b) v = cmul(v, f[b][(i >> b) & 1]);
        Lp[swz<T>(c.tid + i * NT)] = v;
      }
    } else {
#pragma unroll 4
      for (int i = 0; i < NREG; ++i) {
        const int t = c.tid + i * NT;
        const int s = c.sample0 + (t >> c.nv);
        const int j = t & ((1 << c.nv) - 1);
        cplx<T> v = cmk<T>(0, 0);
        if (s < a.batch && j < (1 << n)) {
          kptr<cplx<T>> em = embed_ps ? a.mats_ps + (size_t)s * a.mats_ps_stride + embed_mat
                                      : a.mats + embed_mat;
          v = cmk<T>(1, 0);
          for (int p = 0; p < n; ++p) {
            kptr<cplx<T>> m = em + 4 * (n - 1 - p);
            v = cmul(v, kld(m, ((j >> p) & 1) ? 2 : 0));
          }
        }
        Lp[swz<T>(t)] = v;
      }
    }
  } else if (fwd_load_global || BWD) {
    // every element of the thread is requested before any is waited for:
    // the tile's loads are in flight together (one memory latency per tile)
    cplx<T> tp[NREG], tl[NREG];
    if (!c.multi) {
      uint32_t kk[NREG];
      if (lmap) {
#pragma unroll
        for (int i = 0; i < NREG; ++i) {
          uint32_t k = lbase ^ lthr;
#pragma unroll
          for (int b = 0; b < RB; ++b)
            if ((i >> b) & 1) k ^= lreg[b];
          kk[i] = k;
        }
      } else {
#pragma unroll
        for (int i = 0; i < NREG; ++i) {
          uint32_t k = c.base | ptid;
#pragma unroll
          for (int b = 0; b < RB; ++b)
            if ((i >> b) & 1) k |= treg[b];
          kk[i] = k;
        }
      }
      const cplx<T> *s0 = a.src0 + (long long)c.sample0 * sstride;
#pragma unroll
      for (int i = 0; i < NREG; ++i) tp[i] = s0[kk[i]];
      if (BWD && uni(a.init_lambda)) {
        // lambda_k = psi_k * h(k), h(k) = sum_p g[n-1-p] (-1)^{bit p of k}.  The
        // element index is k_i = T0 ^ (xor of the columns selected by i), so h
        // is the 16-point Walsh-Hadamard transform of the weights grouped by
        // the pattern of bit p across the four columns.
        const uint32_t T0 = lmap ? (lbase ^ lthr) : (c.base | ptid);
        uint32_t col[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) col[b] = lmap ? lreg[b] : treg[b];
        kptr<double> gs = kc(a.g) + (long long)c.sample0 * n;
        double H[NREG];
#pragma unroll
        for (int q = 0; q < NREG; ++q) H[q] = 0.0;
        for (int p = 0; p < n; ++p) {
          const double wp = gs[n - 1 - p];
          const double v = ((T0 >> p) & 1) ? -wp : wp;
          int cp = 0;
#pragma unroll
          for (int b = 0; b < RB; ++b) cp |= (int)((col[b] >> p) & 1) << b;
          switch (uni(cp)) {
#define X(q) \
  case q: H[q] += v; break;
            X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)
#undef X
          }
        }
        wht16(H);
#pragma unroll
        for (int i = 0; i < NREG; ++i)
          tl[i] = cmk<T>((T)((double)tp[i].x * H[i]), (T)((double)tp[i].y * H[i]));
      } else if (BWD) {
        const cplx<T> *s1 = a.src1 + (long long)c.sample0 * sstride;
#pragma unroll
        for (int i = 0; i < NREG; ++i) tl[i] = s1[kk[i]];
      }
    } else {
      // several samples per workgroup: elements past the batch or the state
      // (virtual padding) read element 0 and are replaced by zero
      long long gg[NREG];
      bool ok[NREG];
#pragma unroll
      for (int i = 0; i < NREG; ++i) {
        const int t = c.tid + i * NT;
        const int smp = c.sample0 + (t >> c.nv);
        const int j = t & ((1 << c.nv) - 1);
        ok[i] = smp < a.batch && j < (1 << n);
        gg[i] = ok[i] ? (long long)smp * sstride + j : 0;
      }
#pragma unroll
      for (int i = 0; i < NREG; ++i) tp[i] = a.src0[gg[i]];
      if (BWD) {
#pragma unroll
        for (int i = 0; i < NREG; ++i) tl[i] = a.src1[gg[i]];
      }
#pragma unroll
      for (int i = 0; i < NREG; ++i) {
        if (!ok[i]) {
          tp[i] = cmk<T>(0, 0);
          tl[i] = cmk<T>(0, 0);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
      const int t = c.tid + i * NT;
      Lp[swz<T>(t)] = tp[i];
      if (BWD) Ll[swz<T>(t)] = tl[i];
    }
  }
  __syncthreads();

  // ---------------- stages ----------------
  const int ns = uni(P->n_stages), sb = uni(P->stage_begin);
  DenseCarry<T, DENSE> dc;
  if constexpr (DENSE) {
    const int m0 = uni(P->dense_first_mat[BWD ? 1 : 0]);
    if (m0 >= 0) dense_fetch_nv<T, K, BWD>(c, a.mats + m0, dc.u);
  }
  // backward: when psi is neither stored nor read after this pass (stored
  // states, or the first pass without embedding gradients), the psi uncompute
  // of the last stage is dead from its last gradient-taking op on
  const bool psi_dead_end = BWD && !DENSE && (!uni(a.store_psi) || uni(P->skip_bwd_store)) &&
                            uni(P->n_grad_stages) == 0 && uni(P->outside_mask) == 0;
  // full-layer matrix passes (one wave per SIMD) request the next stage's
  // descriptor while the current stage runs, and forward step over the
  // gradient-only stages
  UStage Snext;
  if (DENSE && ns > 0) Snext = load_stage(a.stages + sb + (BWD ? ns - 1 : 0));
  for (int si = 0; si < ns;) {
    UStage S;
    int step = 1;
    if constexpr (DENSE) {
      S = Snext;
      step = BWD ? 1 : S.fwd_next;
      if (si + step < ns) Snext = load_stage(a.stages + sb + (BWD ? (ns - 1 - si - step) : (si + step)));
    } else {
      S = load_stage(a.stages + sb + (BWD ? (ns - 1 - si) : si));
    }
    const int scur = si;
    si += step;
    int psi_upto = 1 << 30;
    if (psi_dead_end && scur == ns - 1) {
      // processing position of the last op that takes a gradient (-1: none);
      // brick-layer programs need psi between their inner steps
      const int nops = S.op_end - S.op_begin;
      int last = -1;
      bool seq = false;
      for (int oi = 0; oi < nops; ++oi) {
        const int k = S.op_end - 1 - oi;
        const int kind = uni(a.ops[k].kind), flags = uni(a.ops[k].flags);
        if (kind == OP_SEQ || kind == OP_PERM || kind == OP_DENSE) seq = true;
        if (flags & F_GRAD) last = oi;
      }
      if (!seq) psi_upto = last < 0 ? 0 : last;
    }
    // stages of gradient sums alone (full-layer matrix passes): nothing to do
    // forward, nothing to write back
    if (DENSE && (S.flags & STAGE_GRAD_ONLY)) {
      if (!BWD) continue;
      run_stage<T, K, BWD, DENSE, DIAG>(c, a, S, Lp, Ll, tab, dc, true);
      continue;
    }
    run_stage<T, K, BWD, DENSE, DIAG>(c, a, S, Lp, Ll, tab, dc, false, psi_upto);
  }
  if (BWD) {
    const int ng = uni(P->n_grad_stages), gsb = uni(P->grad_stage_begin);
    for (int si = 0; si < ng; ++si) {
      const UStage S = load_stage(a.stages + gsb + si);
      run_stage<T, K, BWD, DENSE, DIAG>(c, a, S, Lp, Ll, tab, dc, true);
    }
    const uint32_t omask = uniu(P->outside_mask);
    if (omask && !c.multi) outside_embed_grads(c, a, P, Ll, omask);
    if (uni(P->skip_bwd_store)) return;
  }

  // ---------------- store ----------------
  if (NSUB > 1 && c.sub != 0) return;   // every copy holds the same tile
  // an opaque copy of the thread's index bits: otherwise the compiler keeps the
  // load phase's element indices alive through every stage to reuse them here
  uint32_t ptid_s = ptid;
  asm volatile("" : "+v"(ptid_s));
  cplx<T> tp[NREG], tl[NREG];
#pragma unroll
  for (int i = 0; i < NREG; ++i) {
    const int t = c.tid + i * NT;
    tp[i] = Lp[swz<T>(t)];
    if (BWD) tl[i] = Ll[swz<T>(t)];
  }
  if (!c.multi) {
    uint32_t kk[NREG];
    if (smap) {
#pragma unroll
      for (int i = 0; i < NREG; ++i) {
        uint32_t k = sbase ^ sthr;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if ((i >> b) & 1) k ^= sreg[b];
        kk[i] = k;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NREG; ++i) {
        uint32_t k = c.base | ptid_s;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if ((i >> b) & 1) k |= treg[b];
        kk[i] = k;
      }
    }
    cplx<T> *d0 = a.dst0 + (long long)c.sample0 * sstride;
    if (!BWD || uni(a.store_psi)) {
#pragma unroll
      for (int i = 0; i < NREG; ++i) d0[kk[i]] = tp[i];
    }
    if (BWD) {
      cplx<T> *d1 = a.dst1 + (long long)c.sample0 * sstride;
#pragma unroll
      for (int i = 0; i < NREG; ++i) d1[kk[i]] = tl[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
      const int t = c.tid + i * NT;
      const int smp = c.sample0 + (t >> c.nv);
      const int j = t & ((1 << c.nv) - 1);
      if (smp < a.batch && j < (1 << n)) {
        const long long g = (long long)smp * sstride + j;
        if (!BWD || a.store_psi) a.dst0[g] = tp[i];
        if (BWD) a.dst1[g] = tl[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// readout and adjoint init: tiles of 2^KE consecutive amplitudes of [B, 2^n]
// ---------------------------------------------------------------------------
constexpr int KE = 12;
constexpr int NTE = 1 << (KE - RB);

template <typename T>
struct ReadArgs {
  const cplx<T> *psi;
  cplx<T> *lam;
  const double *g;      // [B, n] upstream (adj init)
  double *partials;     // expval: [B][units][KE+1]
  int n, batch;
};

// Element layout of the readout kernels: a workgroup covers 2^KE consecutive
// amplitudes of the (virtually padded) index space; thread tid holds the 16
// consecutive amplitudes 16*tid .. 16*tid+15, so its register bits are state
// bits 0..3 and every thread belongs to exactly one sample.
struct RdCtx {
  int nv, multi, tps_log;
  long long sample0;
  uint32_t jbase;
};

__device__ __forceinline__ RdCtx rd_ctx(int n) {
  RdCtx c;
  c.nv = n < RB ? RB : n;
  c.multi = c.nv < KE;
  if (c.multi) {
    c.sample0 = (long long)blockIdx.x << (KE - c.nv);
    c.jbase = 0;
    c.tps_log = c.nv - RB;
  } else {
    const int tl = c.nv - KE;
    c.sample0 = (long long)blockIdx.x >> tl;
    c.jbase = (uint32_t)(blockIdx.x & ((1u << tl) - 1u)) << KE;
    c.tps_log = KE - RB;
  }
  return c;
}

__device__ __forceinline__ bool rd_elem(const RdCtx &c, int n, int batch, int t, long long &g) {
  long long s;
  uint32_t j;
  if (c.multi) {
    s = c.sample0 + (t >> c.nv);
    j = (uint32_t)t & ((1u << c.nv) - 1u);
  } else {
    s = c.sample0;
    j = c.jbase | (uint32_t)t;
  }
  if (s >= batch || j >= (1u << n)) return false;
  g = (s << n) | j;
  return true;
}

// Per sample and tile: total probability and the signed sum over each tile bit.
// COAL: a sample spans whole tiles; element i*NTE + tid (lane-contiguous loads),
// register bits are tile bits KE-4..KE-1.  Otherwise thread tid holds
// elements 16*tid .. 16*tid+15 (register bits 0..3) so that no thread mixes
// samples.
template <typename T, bool COAL>
__global__ void __launch_bounds__(NTE) k_expval(ReadArgs<T> a) {
  const int n = a.n;
  const int tid = threadIdx.x;
  const RdCtx c = rd_ctx(n);
  constexpr int RB0 = COAL ? KE - RB : 0;      // first register tile bit
  double tot = 0.0;
  double sr[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) sr[b] = 0.0;
  long long gi[NREG];
  bool ok[NREG];
  cplx<T> v[NREG];
#pragma unroll
  for (int i = 0; i < NREG; ++i) {
    const int t = COAL ? tid + i * NTE : tid * NREG + i;
    ok[i] = rd_elem(c, n, a.batch, t, gi[i]);
    if (!ok[i]) gi[i] = 0;
  }
#pragma unroll
  for (int i = 0; i < NREG; ++i) v[i] = a.psi[gi[i]];
#pragma unroll
  for (int i = 0; i < NREG; ++i) {
    const double p = ok[i] ? (double)v[i].x * (double)v[i].x + (double)v[i].y * (double)v[i].y : 0.0;
    tot += p;
#pragma unroll
    for (int b = 0; b < RB; ++b) sr[b] += ((i >> b) & 1) ? -p : p;
  }
  // values: 0 = total, 1 + b = signed sum over tile bit b
  double vals[KE + 1];
  vals[0] = tot;
#pragma unroll
  for (int b = 0; b < KE; ++b) {
    if (b >= RB0 && b < RB0 + RB)
      vals[1 + b] = sr[b - RB0];
    else {
      const int tb = COAL ? b : b - RB;        // thread-index bit of tile bit b
      vals[1 + b] = ((tid >> tb) & 1) ? -tot : tot;
    }
  }
  const int seg_log = c.tps_log < 6 ? c.tps_log : 6;
#pragma unroll
  for (int v = 0; v <= KE; ++v) vals[v] = seg_sum_dpp(vals[v], seg_log);
  const int segm = (1 << seg_log) - 1;
  const long long units = c.multi ? 1 : (1ll << (c.nv - KE));
  const long long u = c.multi ? 0 : ((long long)blockIdx.x & (units - 1));
  if (c.tps_log >= 6) {
    // a sample spans whole waves: combine its waves through LDS
    __shared__ double red[(NTE / 64) * (KE + 1)];
    const int wave = tid >> 6;
    if ((tid & 63) == 63)
      for (int v = 0; v <= KE; ++v) red[wave * (KE + 1) + v] = vals[v];
    __syncthreads();
    const int wps = 1 << (c.tps_log - 6);          // waves per sample
    const int spt = (NTE / 64) / wps;               // samples in this tile
    if (tid < spt * (KE + 1)) {
      const int sl = tid / (KE + 1), v = tid % (KE + 1);
      double s = 0.0;
      for (int w = 0; w < wps; ++w) s += red[(sl * wps + w) * (KE + 1) + v];
      const long long smp = c.sample0 + sl;
      if (smp < a.batch) a.partials[(smp * units + u) * (KE + 1) + v] = s;
    }
  } else if ((tid & segm) == segm) {
    const long long smp = c.sample0 + (tid >> seg_log);
    if (smp < a.batch)
      for (int v = 0; v <= KE; ++v) a.partials[(smp * units + u) * (KE + 1) + v] = vals[v];
  }
}

// Sum of a double across the 64 lanes of a wave, in a fixed order; valid in lane 63.
__device__ __forceinline__ double wave_sum(double v) { return seg_sum_dpp(v, 6); }

constexpr int NTR = 256;   // threads per block of the grouped reduction kernels

// expz[b, i] and norm[b] from the partials; wire i <-> state bit p = n-1-i.
// A group of 2^gl lanes per output (b, i); i == n gives the norm.
#ifndef TQS_PASS_TU   // defined once, in the translation unit of the host API
__global__ void __launch_bounds__(NTR) k_expval_final(const double *partials, double *expz, double *norm, int n,
                                                      int batch, int gl) {
  const long long o = ((long long)blockIdx.x * NTR + threadIdx.x) >> gl;
  const int g = threadIdx.x & ((1 << gl) - 1);
  const bool valid = o < (long long)batch * (n + 1);
  double s = 0.0;
  const int b = (int)(o / (n + 1)), i = (int)(o % (n + 1));
  if (valid) {
    const long long units = n > KE ? (1ll << (n - KE)) : 1;
    const int p = n - 1 - i;
    for (long long u = g; u < units; u += (1 << gl)) {
      const double *q = partials + ((long long)b * units + u) * (KE + 1);
      if (i == n)
        s += q[0];
      else if (p < KE)
        s += q[1 + p];
      else
        s += ((u >> (p - KE)) & 1) ? -q[0] : q[0];
    }
  }
  s = seg_sum_dpp(s, gl);
  if (valid && g == (1 << gl) - 1) {
    if (i == n) {
      if (norm) norm[b] = s;
    } else {
      expz[(long long)b * n + i] = s;
    }
  }
}
#endif

// lambda = psi * h with h(j) = sum_i g_i (1 - 2 b_i(j)), per sample
template <typename T, bool COAL>
__global__ void __launch_bounds__(NTE) k_adj_init(ReadArgs<T> a) {
  const int n = a.n;
  const int tid = threadIdx.x;
  const RdCtx c = rd_ctx(n);
  constexpr int RB0 = COAL ? KE - RB : 0;
  long long g0;
  if (!rd_elem(c, n, a.batch, COAL ? tid : tid * NREG, g0)) return;   // padding / past the batch
  const long long s = g0 >> n;
  const double *gg = a.g + s * n;
  const uint32_t j0 = (uint32_t)(g0 & ((1ll << n) - 1));
  // thread part: every state bit except the register bits
  double hthr = 0.0;
  for (int p = 0; p < n; ++p) {
    if (p >= RB0 && p < RB0 + RB) continue;
    hthr += ((j0 >> p) & 1) ? -gg[n - 1 - p] : gg[n - 1 - p];
  }
  // all loads first (one memory latency per thread), then the products
  long long gi[NREG];
  bool ok[NREG];
  cplx<T> v[NREG];
#pragma unroll
  for (int i = 0; i < NREG; ++i) {
    const int t = COAL ? tid + i * NTE : tid * NREG + i;
    ok[i] = rd_elem(c, n, a.batch, t, gi[i]);
    if (!ok[i]) gi[i] = g0;
  }
#pragma unroll
  for (int i = 0; i < NREG; ++i) v[i] = a.psi[gi[i]];
#pragma unroll
  for (int i = 0; i < NREG; ++i) {
    double h = hthr;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int p = RB0 + b;
      if (p < n) h += ((i >> b) & 1) ? -gg[n - 1 - p] : gg[n - 1 - p];
    }
    if (ok[i]) a.lam[gi[i]] = cmk<T>((T)(v[i].x * h), (T)(v[i].y * h));
  }
}

// A[acc][b] = sum of the pass partials of sample b (FP64, fixed order); one wave per (acc, b).
// Deterministic grouped reductions: 2^gl lanes per output (gl chosen on the
// host from the longest sum), each lane summing a fixed stride of the terms in
// order, then a fixed DPP tree within the group.  Blocks of NTR threads.

#ifndef TQS_PASS_TU   // defined once, in the translation unit of the host API
__global__ void __launch_bounds__(NTR) k_acc_reduce(const double *partials, const long long *acc_static,
                                                    const int *acc_units, int n_acc, int batch, double *A,
                                                    int gl) {
  const long long o = ((long long)blockIdx.x * NTR + threadIdx.x) >> gl;
  const int g = threadIdx.x & ((1 << gl) - 1);
  const bool valid = o < (long long)n_acc * batch;
  double s = 0.0;
  if (valid) {
    const int acc = (int)(o / batch), b = (int)(o % batch);
    const int U = acc_units[acc];
    const double *p = partials + acc_static[acc] * batch + (long long)b * U;
    for (int u = g; u < U; u += (1 << gl)) s += p[u];
  }
  s = seg_sum_dpp(s, gl);
  if (valid && g == (1 << gl) - 1) A[o] = s;
}
#endif

// weight gradients: sum over samples of the accumulator combinations; one
// group of 2^gl lanes per weight, lanes striding over the batch
#ifndef TQS_PASS_TU   // defined once, in the translation unit of the host API
__global__ void __launch_bounds__(NTR) k_grad_weights(const int *cptr, const Contrib *contribs, const double *A,
                                                      const double *dbl, const double *dbl_ps, int dbl_ps_stride,
                                                      int n_w, int batch, double *gw, int gl) {
  const long long o = ((long long)blockIdx.x * NTR + threadIdx.x) >> gl;
  const int g = threadIdx.x & ((1 << gl) - 1);
  const bool valid = o < n_w;
  double s = 0.0;
  if (valid) {
    const int p = (int)o;
    const int G = 1 << gl;
    // contributions outermost: the loads of the batch loops below do not wait
    // on one another, so four of them are kept in flight per lane
    for (int ci = cptr[p]; ci < cptr[p + 1]; ++ci) {
      const Contrib cb = contribs[ci];
      for (int k = 0; k < cb.n; ++k) {
        const double *Ak = A + (long long)(cb.acc + k) * batch;
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        if (cb.coef_ps) {
          const double *co = dbl_ps + cb.coef + k;
          int b = g;
          for (; b + 3 * G < batch; b += 4 * G) {
            t0 += co[(size_t)b * dbl_ps_stride] * Ak[b];
            t1 += co[(size_t)(b + G) * dbl_ps_stride] * Ak[b + G];
            t2 += co[(size_t)(b + 2 * G) * dbl_ps_stride] * Ak[b + 2 * G];
            t3 += co[(size_t)(b + 3 * G) * dbl_ps_stride] * Ak[b + 3 * G];
          }
          for (; b < batch; b += G) t0 += co[(size_t)b * dbl_ps_stride] * Ak[b];
          s += (t0 + t1) + (t2 + t3);
        } else {
          // a shared coefficient: the batch sum first
          int b = g;
          for (; b + 3 * G < batch; b += 4 * G) {
            t0 += Ak[b];
            t1 += Ak[b + G];
            t2 += Ak[b + 2 * G];
            t3 += Ak[b + 3 * G];
          }
          for (; b < batch; b += G) t0 += Ak[b];
          s += dbl[cb.coef + k] * ((t0 + t1) + (t2 + t3));
        }
      }
    }
  }
  s = seg_sum_dpp(s, gl);
  if (valid && g == (1 << gl) - 1) gw[o] = s;
}
#endif

// Sums of column blocks over row segments (FP64, rows in order): out[s][c] =
// sum over rows r in [seg[s], seg[s+1]) of x[r][c0 + c].  The serving loop's
// per-request weight gradients: the rows of one launch are the samples of
// several requests.  Segment bounds are clamped to [0, rows].
#ifndef TQS_PASS_TU   // defined once, in the translation unit of the host API
__global__ void __launch_bounds__(NTR) k_segment_sum(const double *x, int rows, int ld, int c0, int nc,
                                                     const int *seg, int n_seg, double *out) {
  const long long t = (long long)blockIdx.x * NTR + threadIdx.x;
  if (t >= (long long)n_seg * nc) return;
  const int sg = (int)(t / nc), cc = (int)(t % nc);
  const int r0 = min(max(seg[sg], 0), rows), r1 = min(max(seg[sg + 1], r0), rows);
  double acc = 0.0;
  for (int r = r0; r < r1; ++r) acc += x[(long long)r * ld + c0 + cc];
  out[t] = acc;
}
#endif

// feature gradients: one thread per (sample, feature)
#ifndef TQS_PASS_TU   // defined once, in the translation unit of the host API
__global__ void __launch_bounds__(NTR) k_grad_features(const int *cptr, const Contrib *contribs, const double *A,
                                                       const double *dbl, const double *dbl_ps, int dbl_ps_stride,
                                                       int n_w, int n_x, int batch, double *gx) {
  const long long j = (long long)blockIdx.x * NTR + threadIdx.x;
  if (j >= (long long)n_x * batch) return;
  const int b = (int)(j / n_x), f = (int)(j % n_x);
  const int p = n_w + f;
  double s = 0.0;
  for (int ci = cptr[p]; ci < cptr[p + 1]; ++ci) {
    const Contrib cb = contribs[ci];
    const double *co = cb.coef_ps ? dbl_ps + (size_t)b * dbl_ps_stride + cb.coef : dbl + cb.coef;
    for (int k = 0; k < cb.n; ++k) s += co[k] * A[(long long)(cb.acc + k) * batch + b];
  }
  gx[(long long)b * n_x + f] = s;
}
#endif

}  // namespace tqs
