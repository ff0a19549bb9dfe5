// libtqsim C ABI: circuit objects, workspace layout and launch sequencing.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hip"
#include "pass_launch.h"
#include "planner.h"
#include "tqsim.h"

using namespace tqs;

static thread_local std::string g_last_error;

// Scratch of tqs_expval_z_noalloc: the readout partials live in this
// file-scope device array instead of a caller workspace.  Every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends; host code must use the address hipGetSymbolAddress returns for the
// current device, never the array's name (a host-side stand-in).
static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];


static tqs_status fail(tqs_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

static tqs_status from_msg(const std::string &m) {
  if (m.rfind("EINVAL", 0) == 0) return fail(TQS_EINVAL, m);
  return fail(TQS_EUNSUPPORTED, m);
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(TQS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

// Optional per-launch timing with HIP events (option "profile"): every kernel
// launch is bracketed by two events on its stream; tqs_profile_report waits for
// them and aggregates duration and algorithmic bytes / flops per kernel kind.
struct ProfRec {
  int kind;
  double bytes, flops;
  hipEvent_t e0, e1;
};
struct ProfAgg {
  long long count = 0;
  double ms = 0, bytes = 0, flops = 0;
};

struct tqs_circuit {
  Plan plan;
  bool profile = false;
  std::mutex pmu;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> kind_names;
  std::vector<ProfAgg> agg;
  std::vector<LayerSpec> layers;
  int n = 0, dtype = 0;
  PlanOptions opts;
  // backward: 0 = adjoint with uncompute (psi rebuilt pass by pass with the
  // inverse layers), 1 = stored states (every forward pass keeps its output;
  // the backward reads psi from there and writes only lambda), 2 = stored when
  // the adjoint's four state buffers exceed stored_min bytes (they no longer
  // stay in the last-level cache), the stored states fit stored_cap bytes and
  // the plan has at most STORED_AUTO_MAX_PASSES forward passes; adjoint otherwise
  int backward = 0;
  long long stored_cap = 8ll << 30;
  long long stored_min = 256ll << 20;
  std::mutex mu;
  bool uploaded = false;
  int device = -1;
  void *dmem = nullptr;
  DevPass *d_pass = nullptr;
  DevStage *d_stage = nullptr;
  DevOp *d_op = nullptr;
  DevDiag *d_diag = nullptr;
  DiagJob *d_djob = nullptr;
  DevTerm *d_term = nullptr;
  DevPerm *d_perm = nullptr;
  DevGroup *d_group = nullptr;
  DevSeq *d_seq = nullptr;
  DevTermGrad *d_tgrad = nullptr;
  PrepItem *d_prep = nullptr;
  Factor *d_fac = nullptr;
  Contrib *d_contrib = nullptr;
  int *d_cptr = nullptr;
  long long *d_acc_static = nullptr;
  int *d_acc_units = nullptr;
  int max_units = 1;   // longest per-sample accumulator sum
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// log2 of the lanes given to a sum of `n` terms: ceil(log2 n), at most a wave
int ceil_log2(long long n) {
  int l = 0;
  while (l < 6 && (1ll << l) < n) ++l;
  return l;
}

template <typename V>
size_t bytes_of(const std::vector<V> &v) {
  return v.size() * sizeof(V);
}

std::once_flag g_attr_once;

void set_all_attrs() {
  pass_attrs_f32_fwd();
  pass_attrs_f32_bwd();
  pass_attrs_f64_fwd();
  pass_attrs_f64_bwd();
}

tqs_status upload(tqs_circuit *c) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->uploaded) return TQS_OK;
  c->max_units = 1;
  for (int u : c->plan.acc_units) c->max_units = std::max(c->max_units, u);
  std::call_once(g_attr_once, set_all_attrs);
  const Plan &P = c->plan;
  struct Part {
    const void *src;
    size_t bytes;
    void **dst;
  };
  std::vector<Part> parts = {
      {P.dpass.data(), bytes_of(P.dpass), (void **)&c->d_pass},
      {P.dstage.data(), bytes_of(P.dstage), (void **)&c->d_stage},
      {P.dop.data(), bytes_of(P.dop), (void **)&c->d_op},
      {P.ddiag.data(), bytes_of(P.ddiag), (void **)&c->d_diag},
      {P.diag_jobs.data(), bytes_of(P.diag_jobs), (void **)&c->d_djob},
      {P.dterm.data(), bytes_of(P.dterm), (void **)&c->d_term},
      {P.dperm.data(), bytes_of(P.dperm), (void **)&c->d_perm},
      {P.dgroup.data(), bytes_of(P.dgroup), (void **)&c->d_group},
      {P.dseq.data(), bytes_of(P.dseq), (void **)&c->d_seq},
      {P.dtgrad.data(), bytes_of(P.dtgrad), (void **)&c->d_tgrad},
      {P.prep.data(), bytes_of(P.prep), (void **)&c->d_prep},
      {P.factors.data(), bytes_of(P.factors), (void **)&c->d_fac},
      {P.contribs.data(), bytes_of(P.contribs), (void **)&c->d_contrib},
      {P.cptr.data(), bytes_of(P.cptr), (void **)&c->d_cptr},
      {P.acc_static.data(), bytes_of(P.acc_static), (void **)&c->d_acc_static},
      {P.acc_units.data(), bytes_of(P.acc_units), (void **)&c->d_acc_units},
  };
  size_t total = 0;
  for (auto &p : parts) total += align256(p.bytes ? p.bytes : 1);
  HIP_TRY(hipGetDevice(&c->device));
  HIP_TRY(hipMalloc(&c->dmem, total));
  size_t off = 0;
  std::vector<char> host(total, 0);
  for (auto &p : parts) {
    *p.dst = static_cast<char *>(c->dmem) + off;
    if (p.bytes) std::memcpy(host.data() + off, p.src, p.bytes);
    off += align256(p.bytes ? p.bytes : 1);
  }
  HIP_TRY(hipMemcpy(c->dmem, host.data(), total, hipMemcpyHostToDevice));
  c->uploaded = true;
  return TQS_OK;
}

struct WsLayout {
  size_t x = 0, la = 0, lb = 0, st = 0, mats = 0, mats_ps = 0, dbl = 0, dbl_ps = 0, dtab = 0, partials = 0, A = 0,
         ev = 0;
  size_t total = 0, state = 0;
  bool has_x = false, has_lb = false, stored = false;
  int n_stored = 0;   // forward pass outputs kept in the workspace (all but the last)
};

size_t expval_partials_bytes(const Plan &P, int B);

int forward_passes(const Plan &P) {
  int m = 0;
  for (const PlanPass &pp : P.passes) m += !pp.bwd_only;
  return m;
}

// Stored-state backward with more forward passes than this is not chosen
// automatically (option backward = 2).
constexpr int STORED_AUTO_MAX_PASSES = 64;

// Whether the stored-state backward serves batch B: the workspace layout of
// forward and backward calls depends on it, and both derive it from (plan, B).
bool use_stored(const tqs_circuit *c, int B) {
  if (c->backward == 1) return true;
  if (c->backward != 2) return false;
  const Plan &P = c->plan;
  const int m = forward_passes(P);
  const double state = (double)((size_t)B << P.n) * (P.dtype ? 16.0 : 8.0);
  return m <= STORED_AUTO_MAX_PASSES && (double)(m - 1) * state <= (double)c->stored_cap &&
         4.0 * state > (double)c->stored_min;
}

WsLayout layout(const Plan &P, int B, bool grad, bool stored) {
  WsLayout L;
  const size_t es = P.dtype ? 16 : 8;
  const size_t state = ((size_t)B << P.n) * es;
  L.state = state;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes ? bytes : 1);
    return o;
  };
  L.stored = stored;
  L.has_x = P.any_oop;
  L.has_lb = grad && P.any_oop;
  if (L.has_x) L.x = take(state);
  if (stored) {
    // outputs of forward passes 0 .. m-2 (the last pass writes the caller's state)
    L.n_stored = std::max(0, forward_passes(P) - 1);
    L.st = take(state * (size_t)L.n_stored);
  }
  if (grad) L.la = take(state);
  if (L.has_lb) L.lb = take(state);
  L.mats = take((size_t)P.n_mats * es);
  L.mats_ps = take((size_t)B * P.n_mats_ps * es);
  L.dbl = take((size_t)P.n_dbl * 8);
  L.dbl_ps = take((size_t)B * P.n_dbl_ps * 8);
  L.dtab = take((size_t)P.n_diag_tab * es);
  if (grad) {
    L.partials = take((size_t)B * (size_t)P.units_total * sizeof(double));
    L.A = take((size_t)P.n_acc * B * 8);
  }
  L.ev = take(expval_partials_bytes(P, B));
  L.total = off;
  return L;
}

// Workgroups of one pass launch, in 64-bit arithmetic (B near INT32_MAX with
// several samples per workgroup must not wrap).
long long pass_grid(const DevPass &d, int B) {
  if (d.nv >= d.K) return (long long)B << (d.nv - d.K);
  const long long spw = 1ll << (d.K - d.nv);
  return ((long long)B + spw - 1) / spw;
}

int prof_kind(tqs_circuit *c, const std::string &name) {
  for (size_t i = 0; i < c->kind_names.size(); ++i)
    if (c->kind_names[i] == name) return (int)i;
  c->kind_names.push_back(name);
  c->agg.emplace_back();
  return (int)c->kind_names.size() - 1;
}

hipEvent_t prof_event(tqs_circuit *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch; call begin() before and end() after the launch.
struct ProfScope {
  tqs_circuit *c;
  hipStream_t s;
  ProfRec r;
  bool on;
  ProfScope(tqs_circuit *c_, hipStream_t s_, const std::string &name, double bytes, double flops)
      : c(c_), s(s_), on(c_->profile) {
    if (!on) return;
    std::lock_guard<std::mutex> lk(c->pmu);
    r.kind = prof_kind(c, name);
    r.bytes = bytes;
    r.flops = flops;
    r.e0 = prof_event(c);
    r.e1 = prof_event(c);
    if (!r.e0 || !r.e1) {
      on = false;
      return;
    }
    (void)hipEventRecord(r.e0, s);
  }
  void end() {
    if (!on) return;
    (void)hipEventRecord(r.e1, s);
    std::lock_guard<std::mutex> lk(c->pmu);
    c->pending.push_back(r);
    on = false;
  }
};

template <typename T, bool BWD>
tqs_status launch_pass(tqs_circuit *c, int pi, int B, const cplx<T> *src0, cplx<T> *dst0,
                       const cplx<T> *src1, cplx<T> *dst1, char *ws, const WsLayout &L,
                       hipStream_t s, const double *g_init = nullptr, bool store_psi = true) {
  const Plan &P = c->plan;
  const DevPass &d = P.dpass[pi];
  PassArgs<T> a;
  a.pass = kc(c->d_pass + pi);
  a.stages = kc(c->d_stage);
  a.ops = kc(c->d_op);
  a.diags = kc(c->d_diag);
  a.terms = kc(c->d_term);
  a.perms = kc(c->d_perm);
  a.groups = kc(c->d_group);
  a.seqs = kc(c->d_seq);
  a.tgrads = kc(c->d_tgrad);
  a.mats = kc(reinterpret_cast<const cplx<T> *>(ws + L.mats));
  a.mats_ps = kc(reinterpret_cast<const cplx<T> *>(ws + L.mats_ps));
  a.mats_ps_stride = P.n_mats_ps;
  a.dbl = kc(reinterpret_cast<const double *>(ws + L.dbl));
  a.dbl_ps = kc(reinterpret_cast<const double *>(ws + L.dbl_ps));
  a.dbl_ps_stride = P.n_dbl_ps;
  a.diag_tabs = reinterpret_cast<const cplx<T> *>(ws + L.dtab);
  a.src0 = src0;
  a.dst0 = dst0;
  a.src1 = src1;
  a.dst1 = dst1;
  a.partials = BWD ? reinterpret_cast<double *>(ws + L.partials) : nullptr;
  a.acc_region = (long long)B * P.pass_prefix[pi];
  a.units = P.pass_units[pi];
  a.batch = B;
  a.g = g_init;
  a.init_lambda = g_init != nullptr;
  a.store_psi = store_psi ? 1 : 0;
  const long long grid_ll = pass_grid(d, B);
  if (grid_ll > INT32_MAX) return fail(TQS_EINVAL, "batch too large: pass grid exceeds 2^31 - 1 workgroups");
  const int grid = (int)grid_ll;
  const size_t es = sizeof(cplx<T>);
  // one copy of the tile (psi, and lambda backward) per wave group: DENSE_SUBS
  // copies in passes with full-layer matrix ops
  const size_t copies = d.has_dense ? DENSE_SUBS : 1;
  const size_t lds = (copies * (BWD ? 2 : 1) * ((size_t)1 << d.K) + (size_t)d.diag_lds) * es;
  if (lds > 160 * 1024) return fail(TQS_EUNSUPPORTED, "pass needs more than 160 KiB of LDS");
  double bytes = 0, flops = 0;
  if (c->profile) {
    const double amps = (double)B * (double)(1ll << P.n);
    if (BWD)
      bytes = amps * es * ((g_init ? 1.0 : 2.0) + (d.skip_bwd_store ? 0.0 : (store_psi ? 2.0 : 1.0)));
    else
      bytes = amps * es * ((d.load_mode == LOAD_GLOBAL ? 1.0 : 0.0) + 1.0);
    double ff = 0, fb = 0;
    pass_flops(P, pi, &ff, &fb);
    const double f = BWD ? fb : ff;
    flops = amps * f;
  }
  ProfScope ps(c, s, std::string(BWD ? "pass_bwd_K" : "pass_fwd_K") + std::to_string(d.K) +
                         (sizeof(T) == 8 ? "_c128" : "_c64"), bytes, flops);
  // passes holding full-layer matrix ops use their own instantiation, so that
  // the matrix-core code does not raise the register use of the others
  if (!PassLaunch<T, BWD>::run(a, d.K, d.has_dense != 0, d.n_diag > 0, grid, lds, s))
    return fail(TQS_EUNSUPPORTED, d.has_dense ? "dense layers need a 10-bit tile" : "tile size not built");
  ps.end();
  HIP_TRY(hipGetLastError());
  return TQS_OK;
}

template <typename T>
tqs_status do_prep(tqs_circuit *c, int B, const double *w, const double *x, char *ws, const WsLayout &L,
                   hipStream_t s) {
  const Plan &P = c->plan;
  if (P.prep.empty() && P.diag_jobs.empty()) return TQS_OK;
  PrepArgs<T> a;
  a.items = kc(c->d_prep);
  a.factors = kc(c->d_fac);
  a.n_items = (int)P.prep.size();
  a.w = w;
  a.x = x;
  a.nfeat = P.n_features;
  a.batch = B;
  a.mats = reinterpret_cast<cplx<T> *>(ws + L.mats);
  a.mats_ps = reinterpret_cast<cplx<T> *>(ws + L.mats_ps);
  a.mats_ps_stride = P.n_mats_ps;
  a.dbl = reinterpret_cast<double *>(ws + L.dbl);
  a.dbl_ps = reinterpret_cast<double *>(ws + L.dbl_ps);
  a.dbl_ps_stride = P.n_dbl_ps;
  a.nv = P.nv;
  dim3 grid((B + 63) / 64, (unsigned)P.prep.size());
  ProfScope ps(c, s, "prep", 0.0, 0.0);
  if (!P.prep.empty()) hipLaunchKernelGGL((k_prep<T>), grid, dim3(64), 0, s, a);
  if (P.dense && !P.prep.empty()) hipLaunchKernelGGL((k_prep_dense<T>), dim3(1u << P.nv, (unsigned)P.prep.size()), dim3(64), 0, s, a);
  if (!P.diag_jobs.empty()) {
    // split phase tables of the diagonal ops with shared angles, every tile position
    DiagTabArgs<T> t;
    t.passes = kc(c->d_pass);
    t.diags = kc(c->d_diag);
    t.terms = kc(c->d_term);
    t.jobs = kc(c->d_djob);
    t.dbl = kc(reinterpret_cast<const double *>(ws + L.dbl));
    t.out = reinterpret_cast<cplx<T> *>(ws + L.dtab);
    long long most = 1;
    for (const DiagJob &j : P.diag_jobs) most = std::max(most, (long long)j.entries << j.tiles_log);
    hipLaunchKernelGGL((k_diag_tables<T>), dim3((unsigned)((most + 255) / 256), (unsigned)P.diag_jobs.size()),
                       dim3(256), 0, s, t);
  }
  ps.end();
  HIP_TRY(hipGetLastError());
  return TQS_OK;
}

template <typename T>
tqs_status forward_t(tqs_circuit *c, int B, const double *w, const double *x, void *state, char *ws,
                     const WsLayout &L, hipStream_t s) {
  const Plan &P = c->plan;
  tqs_status st = do_prep<T>(c, B, w, x, ws, L, s);
  if (st != TQS_OK) return st;
  std::vector<int> fwd;
  for (size_t p = 0; p < P.passes.size(); ++p)
    if (!P.passes[p].bwd_only) fwd.push_back((int)p);
  int k = 0;
  for (size_t i = 1; i < fwd.size(); ++i)
    if (P.passes[fwd[i]].has_load || P.passes[fwd[i]].has_store) ++k;
  cplx<T> *S = reinterpret_cast<cplx<T> *>(state);
  cplx<T> *X = L.has_x ? reinterpret_cast<cplx<T> *>(ws + L.x) : nullptr;
  if (L.stored) {
    // every pass out of place into its own buffer; the last into the caller's
    cplx<T> *ST = reinterpret_cast<cplx<T> *>(ws + L.st);
    const size_t elems = (size_t)B << P.n;
    cplx<T> *prev = nullptr;
    for (size_t i = 0; i < fwd.size(); ++i) {
      cplx<T> *dst = (i + 1 == fwd.size()) ? S : ST + i * elems;
      st = launch_pass<T, false>(c, fwd[i], B, i == 0 ? dst : prev, dst, nullptr, nullptr, ws, L, s);
      if (st != TQS_OK) return st;
      prev = dst;
    }
    return TQS_OK;
  }
  cplx<T> *cur = (k % 2 == 0) ? S : X;
  for (size_t i = 0; i < fwd.size(); ++i) {
    const PlanPass &pp = P.passes[fwd[i]];
    const bool oop = pp.has_load || pp.has_store;
    cplx<T> *src = cur, *dst = cur;
    if (i > 0 && oop) dst = (cur == S) ? X : S;
    st = launch_pass<T, false>(c, fwd[i], B, src, dst, nullptr, nullptr, ws, L, s);
    if (st != TQS_OK) return st;
    cur = dst;
  }
  return TQS_OK;
}

// Bytes of readout partials that <Z_i> and the norm need for `B` samples:
// [B][units][KE + 1] doubles, units = 2^(n - KE) per sample (one below that).
size_t expval_partials_bytes(const Plan &P, int B) {
  const size_t ev_units = P.n > KE ? ((size_t)1 << (P.n - KE)) : 1;
  return (size_t)B * ev_units * (KE + 1) * sizeof(double);
}

template <typename T>
tqs_status expval_t(const tqs_circuit *c, int B, const void *state, double *expz, double *norm, double *partials,
                    hipStream_t s, bool prof = true) {
  const Plan &P = c->plan;
  ReadArgs<T> a;
  a.psi = reinterpret_cast<const cplx<T> *>(state);
  a.lam = nullptr;
  a.g = nullptr;
  a.partials = partials;
  a.n = P.n;
  a.batch = B;
  const long long padded = (long long)B << P.nv;
  const long long blocks = (padded + (1ll << KE) - 1) >> KE;
  tqs_circuit *cm = const_cast<tqs_circuit *>(c);
  const bool was = cm->profile;
  if (!prof) cm->profile = false;
  ProfScope ps(cm, s, "expval", (double)B * (double)(1ll << P.n) * sizeof(cplx<T>),
               (double)B * (double)(1ll << P.n) * (4.0 + P.n));   // |psi|^2 and n signed sums
  if (!prof) cm->profile = was;
  if (P.nv >= KE)
    hipLaunchKernelGGL((k_expval<T, true>), dim3((unsigned)blocks), dim3(NTE), 0, s, a);
  else
    hipLaunchKernelGGL((k_expval<T, false>), dim3((unsigned)blocks), dim3(NTE), 0, s, a);
  ps.end();
  HIP_TRY(hipGetLastError());
  const long long tot = (long long)B * (P.n + 1);
  const int gl = std::min(6, std::max(0, P.n - KE));   // lanes per output: the unit count, up to 64
  hipLaunchKernelGGL(k_expval_final, dim3((unsigned)(((tot << gl) + NTR - 1) / NTR)), dim3(NTR), 0, s,
                     (const double *)partials, expz, norm, P.n, B, gl);
  HIP_TRY(hipGetLastError());
  return TQS_OK;
}

template <typename T>
tqs_status adjoint_t(tqs_circuit *c, int B, const double *w, const double *x, void *state, const double *g,
                     double *gw, double *gx, char *ws, const WsLayout &L, hipStream_t s) {
  const Plan &P = c->plan;
  tqs_status st = do_prep<T>(c, B, w, x, ws, L, s);
  if (st != TQS_OK) return st;
  cplx<T> *S = reinterpret_cast<cplx<T> *>(state);
  cplx<T> *X = L.has_x ? reinterpret_cast<cplx<T> *>(ws + L.x) : nullptr;
  cplx<T> *LA = reinterpret_cast<cplx<T> *>(ws + L.la);
  cplx<T> *LB = L.has_lb ? reinterpret_cast<cplx<T> *>(ws + L.lb) : nullptr;
  // when the first backward pass holds one sample per workgroup it forms
  // lambda itself as it loads psi; otherwise a separate kernel does
  const int last = (int)P.passes.size() - 1;
  const bool fused_init = P.nv > P.dpass[last].K;
  if (!fused_init) {
    ReadArgs<T> a;
    a.psi = S;
    a.lam = LA;
    a.g = g;
    a.partials = nullptr;
    a.n = P.n;
    a.batch = B;
    const long long padded = (long long)B << P.nv;
    const long long blocks = (padded + (1ll << KE) - 1) >> KE;
    ProfScope ps(c, s, "adj_init", 2.0 * (double)B * (double)(1ll << P.n) * sizeof(cplx<T>),
                 (double)B * (double)(1ll << P.n) * 4.0);
    if (P.nv >= KE)
      hipLaunchKernelGGL((k_adj_init<T, true>), dim3((unsigned)blocks), dim3(NTE), 0, s, a);
    else
      hipLaunchKernelGGL((k_adj_init<T, false>), dim3((unsigned)blocks), dim3(NTE), 0, s, a);
    ps.end();
    HIP_TRY(hipGetLastError());
  }
  if (L.stored) {
    // psi of each forward pass comes from its stored output; only lambda is
    // written back, except where a gradient-only pass needs the uncomputed psi
    cplx<T> *ST = reinterpret_cast<cplx<T> *>(ws + L.st);
    const size_t elems = (size_t)B << P.n;
    std::vector<int> fidx(P.passes.size(), -1);
    int m = 0;
    for (size_t p = 0; p < P.passes.size(); ++p)
      if (!P.passes[p].bwd_only) fidx[p] = m++;
    cplx<T> *pc = nullptr, *lc = LA;
    for (int p = (int)P.passes.size() - 1; p >= 0; --p) {
      const PlanPass &pp = P.passes[p];
      const bool oop = pp.has_load || pp.has_store;
      cplx<T> *psrc = pp.bwd_only ? pc : (fidx[p] == m - 1 ? S : ST + (size_t)fidx[p] * elems);
      const bool store = pp.bwd_only || (p > 0 && P.passes[p - 1].bwd_only);
      cplx<T> *pdst = (store && oop) ? (psrc == X ? S : X) : psrc;
      cplx<T> *ld = oop ? ((lc == LA) ? LB : LA) : lc;
      st = launch_pass<T, true>(c, p, B, psrc, pdst, lc, ld, ws, L, s, (fused_init && p == last) ? g : nullptr,
                                store);
      if (st != TQS_OK) return st;
      pc = pdst;
      lc = ld;
    }
  } else {
  cplx<T> *pc = S, *lc = LA;
  for (int p = (int)P.passes.size() - 1; p >= 0; --p) {
    const PlanPass &pp = P.passes[p];
    const bool oop = pp.has_load || pp.has_store;
    cplx<T> *pd = pc, *ld = lc;
    if (oop) {
      pd = (pc == S) ? X : S;
      ld = (lc == LA) ? LB : LA;
    }
    st = launch_pass<T, true>(c, p, B, pc, pd, lc, ld, ws, L, s, (fused_init && p == last) ? g : nullptr);
    if (st != TQS_OK) return st;
    pc = pd;
    lc = ld;
  }
  }
  double *A = reinterpret_cast<double *>(ws + L.A);
  ProfScope psf(c, s, "grad_finalize", 0.0, 0.0);
  if (P.n_acc > 0) {
    const long long tot = (long long)P.n_acc * B;
    const int gl = ceil_log2(c->max_units);
    hipLaunchKernelGGL(k_acc_reduce, dim3((unsigned)(((tot << gl) + NTR - 1) / NTR)), dim3(NTR), 0, s,
                       reinterpret_cast<const double *>(ws + L.partials), (const long long *)c->d_acc_static,
                       (const int *)c->d_acc_units, P.n_acc, B, A, gl);
    HIP_TRY(hipGetLastError());
  }
  if (P.n_weights > 0 && gw) {
    const int gl = ceil_log2(B);
    hipLaunchKernelGGL(k_grad_weights, dim3((unsigned)((((long long)P.n_weights << gl) + NTR - 1) / NTR)),
                       dim3(NTR), 0, s, (const int *)c->d_cptr, (const Contrib *)c->d_contrib, (const double *)A,
                       (const double *)(ws + L.dbl), (const double *)(ws + L.dbl_ps), P.n_dbl_ps, P.n_weights, B,
                       gw, gl);
    HIP_TRY(hipGetLastError());
  }
  const long long totx = (long long)P.n_features * B;
  if (totx > 0 && gx) {
    hipLaunchKernelGGL(k_grad_features, dim3((unsigned)((totx + NTR - 1) / NTR)), dim3(NTR), 0, s,
                       (const int *)c->d_cptr, (const Contrib *)c->d_contrib, (const double *)A,
                       (const double *)(ws + L.dbl), (const double *)(ws + L.dbl_ps), P.n_dbl_ps, P.n_weights,
                       P.n_features, B, gx);
    HIP_TRY(hipGetLastError());
  }
  psf.end();
  return TQS_OK;
}

tqs_status check_batch(const tqs_circuit *c, int B) {
  if (!c) return fail(TQS_EINVAL, "circuit is NULL");
  if (B <= 0) return fail(TQS_EINVAL, "batch must be positive");
  const int es_log = c->dtype ? 4 : 3;
  if (c->n + es_log + 31 - __builtin_clz((unsigned)B) >= 62)
    return fail(TQS_EINVAL, "batch * 2^n * element size overflows int64");
  if ((long long)B * (1ll << c->plan.nv) > (1ll << 40)) return fail(TQS_EINVAL, "state too large");
  for (const DevPass &d : c->plan.dpass)
    if (pass_grid(d, B) > INT32_MAX) return fail(TQS_EINVAL, "batch too large: a pass grid exceeds 2^31 - 1");
  return TQS_OK;
}

tqs_status rebuild(tqs_circuit *c) {
  Plan P;
  std::string e = build_plan(P, c->n, c->layers.data(), (int)c->layers.size(), c->dtype, c->opts);
  if (!e.empty()) return from_msg(e);
  c->plan = std::move(P);
  return TQS_OK;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
tqs_status scratch_for_current_device(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(TQS_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TQS_EDEVICE, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TQS_OK;
}

}  // namespace

extern "C" {

tqs_status tqs_circuit_create(int32_t n_qubits, const tqs_layer *layers, int32_t n_layers, tqs_dtype dtype,
                              tqs_circuit **out) {
  if (!out) return fail(TQS_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != TQS_C64 && dtype != TQS_C128) return fail(TQS_EINVAL, "unknown dtype");
  if (n_layers < 0 || (n_layers > 0 && !layers)) return fail(TQS_EINVAL, "bad layer array");
  tqs_circuit *c = new (std::nothrow) tqs_circuit();
  if (!c) return fail(TQS_ENOMEM, "host allocation failed");
  c->n = n_qubits;
  c->dtype = dtype;
  for (int i = 0; i < n_layers; ++i) {
    LayerSpec L;
    L.gate = layers[i].gate;
    L.pattern = layers[i].pattern;
    L.source = layers[i].source;
    L.wire = layers[i].wire;
    L.wire2 = layers[i].wire2;
    L.offset = layers[i].offset;
    L.fixed = layers[i].fixed_param;
    L.fixed2 = layers[i].fixed_param2;
    L.fixed3 = layers[i].fixed_param3;
    c->layers.push_back(L);
  }
  tqs_status st = rebuild(c);
  if (st != TQS_OK) {
    delete c;
    return st;
  }
  *out = c;
  return TQS_OK;
}

tqs_status tqs_circuit_prepare(tqs_circuit *c) {
  if (!c) return fail(TQS_EINVAL, "circuit is NULL");
  return upload(c);
}

tqs_status tqs_circuit_destroy(tqs_circuit *c) {
  if (!c) return TQS_OK;
  for (auto &r : c->pending) {
    (void)hipEventSynchronize(r.e1);
    c->pool.push_back(r.e0);
    c->pool.push_back(r.e1);
  }
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->dmem) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (c->device >= 0 && cur != c->device) (void)hipSetDevice(c->device);
    (void)hipFree(c->dmem);
    if (cur >= 0 && cur != c->device) (void)hipSetDevice(cur);
  }
  delete c;
  return TQS_OK;
}

tqs_status tqs_circuit_info(const tqs_circuit *c, int32_t *n_weights, int32_t *n_features,
                            int64_t *state_bytes_per_sample) {
  if (!c) return fail(TQS_EINVAL, "circuit is NULL");
  if (n_weights) *n_weights = c->plan.n_weights;
  if (n_features) *n_features = c->plan.n_features;
  if (state_bytes_per_sample) *state_bytes_per_sample = (int64_t(1) << c->n) * (c->dtype ? 16 : 8);
  return TQS_OK;
}

tqs_status tqs_workspace_size(const tqs_circuit *c, int32_t batch, int32_t with_grad, size_t *bytes) {
  tqs_status st = check_batch(c, batch);
  if (st != TQS_OK) return st;
  if (!bytes) return fail(TQS_EINVAL, "bytes is NULL");
  *bytes = layout(c->plan, batch, with_grad != 0, use_stored(c, batch)).total;
  return TQS_OK;
}

tqs_status tqs_forward(tqs_circuit *c, int32_t batch, const double *weights_d, const double *features_d,
                       void *state_d, void *ws_d, size_t ws_bytes, tqs_stream s) {
  tqs_status st = check_batch(c, batch);
  if (st != TQS_OK) return st;
  if (!state_d || !ws_d) return fail(TQS_EINVAL, "state or workspace is NULL");
  if (c->plan.n_weights > 0 && !weights_d) return fail(TQS_EINVAL, "weights are NULL");
  if (c->plan.n_features > 0 && !features_d) return fail(TQS_EINVAL, "features are NULL");
  const WsLayout L = layout(c->plan, batch, false, use_stored(c, batch));
  if (ws_bytes < L.total) return fail(TQS_ENOMEM, "workspace too small");
  st = upload(c);
  if (st != TQS_OK) return st;
  char *ws = static_cast<char *>(ws_d);
  if (c->dtype == TQS_C64)
    return forward_t<float>(c, batch, weights_d, features_d, state_d, ws, L, (hipStream_t)s);
  return forward_t<double>(c, batch, weights_d, features_d, state_d, ws, L, (hipStream_t)s);
}

tqs_status tqs_expval_z(const tqs_circuit *c, int32_t batch, const void *state_d, double *expz_d,
                        double *norm_d, void *ws_d, size_t ws_bytes, tqs_stream s) {
  tqs_status st = check_batch(c, batch);
  if (st != TQS_OK) return st;
  if (!state_d || !expz_d || !ws_d) return fail(TQS_EINVAL, "state, expz or workspace is NULL");
  const WsLayout L = layout(c->plan, batch, false, use_stored(c, batch));
  if (ws_bytes < L.total) return fail(TQS_ENOMEM, "workspace too small");
  char *ws = static_cast<char *>(ws_d);
  double *part = reinterpret_cast<double *>(ws + L.ev);
  if (c->dtype == TQS_C64) return expval_t<float>(c, batch, state_d, expz_d, norm_d, part, (hipStream_t)s);
  return expval_t<double>(c, batch, state_d, expz_d, norm_d, part, (hipStream_t)s);
}

tqs_status tqs_expval_z_noalloc(const tqs_circuit *c, int32_t batch, const void *state_d, double *expz_d,
                                double *norm_d, tqs_stream s) {
  tqs_status st = check_batch(c, batch);
  if (st != TQS_OK) return st;
  if (!state_d || !expz_d) return fail(TQS_EINVAL, "state or expz is NULL");
  const size_t need = expval_partials_bytes(c->plan, batch);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(TQS_EINVAL, "readout partials of " + std::to_string(need) + " bytes exceed the " +
                                std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte static scratch");
  void *part = nullptr;
  st = scratch_for_current_device(&part);
  if (st != TQS_OK) return st;
  if (c->dtype == TQS_C64)
    return expval_t<float>(c, batch, state_d, expz_d, norm_d, static_cast<double *>(part), (hipStream_t)s, false);
  return expval_t<double>(c, batch, state_d, expz_d, norm_d, static_cast<double *>(part), (hipStream_t)s, false);
}

tqs_status tqs_adjoint_grad(tqs_circuit *c, int32_t batch, const double *weights_d, const double *features_d,
                            void *state_d, const double *grad_expz_d, double *grad_weights_d,
                            double *grad_features_d, void *ws_d, size_t ws_bytes, tqs_stream s) {
  tqs_status st = check_batch(c, batch);
  if (st != TQS_OK) return st;
  if (!state_d || !ws_d || !grad_expz_d) return fail(TQS_EINVAL, "state, upstream or workspace is NULL");
  if (c->plan.n_weights > 0 && (!weights_d || !grad_weights_d))
    return fail(TQS_EINVAL, "weights or weight gradients are NULL");
  if (c->plan.n_features > 0 && !features_d) return fail(TQS_EINVAL, "features are NULL");
  const WsLayout L = layout(c->plan, batch, true, use_stored(c, batch));
  if (ws_bytes < L.total) return fail(TQS_ENOMEM, "workspace too small");
  st = upload(c);
  if (st != TQS_OK) return st;
  char *ws = static_cast<char *>(ws_d);
  if (c->dtype == TQS_C64)
    return adjoint_t<float>(c, batch, weights_d, features_d, state_d, grad_expz_d, grad_weights_d,
                            grad_features_d, ws, L, (hipStream_t)s);
  return adjoint_t<double>(c, batch, weights_d, features_d, state_d, grad_expz_d, grad_weights_d,
                           grad_features_d, ws, L, (hipStream_t)s);
}

tqs_status tqs_segment_sum_rows(const double *x_d, int32_t rows, int32_t ld, int32_t col_begin, int32_t n_cols,
                                const int32_t *seg_d, int32_t n_seg, double *out_d, tqs_stream s) {
  if (rows < 0 || n_cols < 0 || n_seg < 0 || col_begin < 0 || (long long)col_begin + n_cols > ld)
    return fail(TQS_EINVAL, "bad segment-sum sizes");
  if ((long long)n_seg * n_cols == 0) return TQS_OK;
  if (!seg_d || !out_d || (rows > 0 && !x_d)) return fail(TQS_EINVAL, "segment-sum pointer is NULL");
  const long long tot = (long long)n_seg * n_cols;
  if ((tot + NTR - 1) / NTR > INT32_MAX) return fail(TQS_EINVAL, "segment-sum too large");
  hipLaunchKernelGGL(k_segment_sum, dim3((unsigned)((tot + NTR - 1) / NTR)), dim3(NTR), 0, (hipStream_t)s, x_d, rows,
                     ld, col_begin, n_cols, (const int *)seg_d, n_seg, out_d);
  HIP_TRY(hipGetLastError());
  return TQS_OK;
}

tqs_status tqs_set_option(tqs_circuit *c, const char *key, int64_t value) {
  if (!c || !key) return fail(TQS_EINVAL, "circuit or key is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  if (std::strcmp(key, "profile") != 0 && c->uploaded)
    return fail(TQS_EINVAL, "options must be set before the first forward call");
  if (std::strcmp(key, "profile") == 0) {
    c->profile = value != 0;
    return TQS_OK;
  }
  if (std::strcmp(key, "mode") == 0) {
    if (value < 0 || value > 3) return fail(TQS_EINVAL, "mode must be 0..3");
    c->opts.mode = (int)value;
  } else if (std::strcmp(key, "hrz") == 0 || std::strcmp(key, "fhwt") == 0 || std::strcmp(key, "diag") == 0) {
    if (value < 0 || value > 1) return fail(TQS_EINVAL, std::string(key) + " must be 0 or 1");
    (key[0] == 'h' ? c->opts.hrz : key[0] == 'f' ? c->opts.fhwt : c->opts.diag) = (int)value;
  } else if (std::strcmp(key, "backward") == 0) {
    if (value < 0 || value > 2) return fail(TQS_EINVAL, "backward must be 0..2");
    c->backward = (int)value;
    return TQS_OK;
  } else if (std::strcmp(key, "stored_cap") == 0 || std::strcmp(key, "stored_min") == 0) {
    if (value < 0) return fail(TQS_EINVAL, std::string(key) + " must be >= 0");
    (key[7] == 'c' ? c->stored_cap : c->stored_min) = value;
    return TQS_OK;
  } else if (std::strcmp(key, "tile_bits") == 0) {
    if (value != 0 && (value < KMIN || value > KMAX)) return fail(TQS_EINVAL, "tile_bits must be 0 or 10..12");
    c->opts.tile_bits = (int)value;
  } else {
    return fail(TQS_EINVAL, std::string("unknown option ") + key);
  }
  return rebuild(c);
}

tqs_status tqs_plan_describe(const tqs_circuit *c, char *buf, size_t len) {
  if (!c || !buf || len == 0) return fail(TQS_EINVAL, "bad arguments");
  const std::string s = describe_plan(c->plan);
  if (s.size() + 1 > len) return fail(TQS_ENOMEM, "buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return TQS_OK;
}

tqs_status tqs_profile_report(tqs_circuit *c, int32_t reset, char *buf, size_t len) {
  if (!c || !buf || len == 0) return fail(TQS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(c->pmu);
  for (auto &r : c->pending) {
    HIP_TRY(hipEventSynchronize(r.e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.e0, r.e1));
    ProfAgg &a = c->agg[r.kind];
    a.count += 1;
    a.ms += ms;
    a.bytes += r.bytes;
    a.flops += r.flops;
    c->pool.push_back(r.e0);
    c->pool.push_back(r.e1);
  }
  c->pending.clear();
  std::string out = "{";
  for (size_t i = 0; i < c->agg.size(); ++i) {
    char tmp[256];
    snprintf(tmp, sizeof tmp, "%s\"%s\":{\"count\":%lld,\"ms\":%.6f,\"bytes\":%.0f,\"flops\":%.0f}",
             i ? "," : "", c->kind_names[i].c_str(), c->agg[i].count, c->agg[i].ms, c->agg[i].bytes,
             c->agg[i].flops);
    out += tmp;
  }
  out += "}";
  if (reset)
    for (auto &a : c->agg) a = ProfAgg();
  if (out.size() + 1 > len) return fail(TQS_ENOMEM, "buffer too small");
  std::memcpy(buf, out.c_str(), out.size() + 1);
  return TQS_OK;
}

const char *tqs_status_string(tqs_status st) {
  switch (st) {
    case TQS_OK: return "TQS_OK";
    case TQS_EINVAL: return "TQS_EINVAL";
    case TQS_ENOMEM: return "TQS_ENOMEM";
    case TQS_EDEVICE: return "TQS_EDEVICE";
    case TQS_EUNSUPPORTED: return "TQS_EUNSUPPORTED";
  }
  return "TQS_UNKNOWN";
}

const char *tqs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
