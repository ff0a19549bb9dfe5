// Launchers of the tile-pass kernels.  Each (element type, direction) pair of
// k_pass instantiations is compiled in a translation unit of its own
// (pass_*.hip, built in parallel); the host API calls them through these.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace tqs {

template <typename T>
struct PassArgs;

// Launch k_pass<T, K, BWD, dense, diag> (dense: the matrix-core variant, K = 10
// only; diag = false, the variant without diagonal layers, is built for K = 12
// and the other sizes use the diag variant).  Returns false for a tile size
// that is not built.
bool launch_pass_f32_fwd(const PassArgs<float> &a, int K, bool dense, bool diag, int grid, size_t lds,
                         hipStream_t s);
bool launch_pass_f32_bwd(const PassArgs<float> &a, int K, bool dense, bool diag, int grid, size_t lds,
                         hipStream_t s);
bool launch_pass_f64_fwd(const PassArgs<double> &a, int K, bool dense, bool diag, int grid, size_t lds,
                         hipStream_t s);
bool launch_pass_f64_bwd(const PassArgs<double> &a, int K, bool dense, bool diag, int grid, size_t lds,
                         hipStream_t s);

// Allow the kernels of one unit the full 160 KiB of LDS.
void pass_attrs_f32_fwd();
void pass_attrs_f32_bwd();
void pass_attrs_f64_fwd();
void pass_attrs_f64_bwd();

template <typename T, bool BWD>
struct PassLaunch;
template <>
struct PassLaunch<float, false> {
  static bool run(const PassArgs<float> &a, int K, bool d, bool dg, int g, size_t l, hipStream_t s) {
    return launch_pass_f32_fwd(a, K, d, dg, g, l, s);
  }
};
template <>
struct PassLaunch<float, true> {
  static bool run(const PassArgs<float> &a, int K, bool d, bool dg, int g, size_t l, hipStream_t s) {
    return launch_pass_f32_bwd(a, K, d, dg, g, l, s);
  }
};
template <>
struct PassLaunch<double, false> {
  static bool run(const PassArgs<double> &a, int K, bool d, bool dg, int g, size_t l, hipStream_t s) {
    return launch_pass_f64_fwd(a, K, d, dg, g, l, s);
  }
};
template <>
struct PassLaunch<double, true> {
  static bool run(const PassArgs<double> &a, int K, bool d, bool dg, int g, size_t l, hipStream_t s) {
    return launch_pass_f64_bwd(a, K, d, dg, g, l, s);
  }
};

}  // namespace tqs
