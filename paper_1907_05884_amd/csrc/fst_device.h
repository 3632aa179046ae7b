// Device-side helpers shared by the HIP sources of the library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fst_internal.h"

namespace fst {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

static inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
static inline void check_launch(const char* what) { check_hip(hipGetLastError(), what); }

// 16 x 16 x 4 MFMA steps: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the four
// accumulator values of lane l sit in column l % 16 and in the rows given by row(l / 16, v).
template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
  typedef floatx4 V;
  static __device__ inline V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int g, int v) { return 4 * g + v; }
};
template <> struct MfmaAcc<double> {
  typedef doublex4 V;
  static __device__ inline V mfma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int g, int v) { return g + 4 * v; }
};

// ------------------------------------------------------------------------------ basis
// Orthonormal Legendre recurrence phi_{m+1} = a_m t phi_m - b_m phi_{m-1}, phi_0 = 1,
// phi_1 = sqrt(3) t, from Bonnet's recurrence with phi_m = sqrt(2m+1) P_m:
//   a_m = sqrt((2m+1)(2m+3)) / (m+1),  b_m = m sqrt(2m+3) / ((m+1) sqrt(2m-1)).
template <typename T>
struct Recurrence {
  T a[kMaxBasis];
  T b[kMaxBasis];
};
template <typename T>
static inline Recurrence<T> make_recurrence() {
  Recurrence<T> r;
  for (int m = 0; m < kMaxBasis; ++m) {
    double a = std::sqrt((2.0 * m + 1.0) * (2.0 * m + 3.0)) / (m + 1.0);
    double b = m == 0 ? 0.0 : m * std::sqrt(2.0 * m + 3.0) / ((m + 1.0) * std::sqrt(2.0 * m - 1.0));
    r.a[m] = (T)a;
    r.b[m] = (T)b;
  }
  return r;
}

template <typename T>
struct ModeMap {   // xi = (y - lo) * scale - 1, scale = 2 / (hi - lo)
  T lo[kMaxModes];
  T scale[kMaxModes];
};
template <typename T>
static inline ModeMap<T> make_map(const fst_model* m) {
  ModeMap<T> mm;
  for (int k = 0; k < kMaxModes; ++k) {
    mm.lo[k] = (T)m->lo[k];
    mm.scale[k] = (T)(2.0 / (m->hi[k] - m->lo[k]));
  }
  return mm;
}

static inline int pad8(int r) { return (r + 7) / 8 * 8; }

// lower-triangle tile t -> (bi, bj), bj <= bi, t = bi (bi + 1) / 2 + bj
__device__ inline void tri_tile(int64_t t, int64_t& bi, int64_t& bj) {
  int64_t b = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (b * (b + 1) / 2 > t) --b;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  bi = b;
  bj = t - b * (b + 1) / 2;
}

}  // namespace fst
