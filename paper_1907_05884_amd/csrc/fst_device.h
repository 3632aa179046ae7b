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

// 16-bit operands, MFMA 16x16x32 with FP32 accumulation: lane l supplies 8 consecutive k of
// row l % 16 (k group l / 16); output layout as MfmaAcc<float> (lane l: D[4 (l / 16) + v][l % 16])
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx8 __attribute__((ext_vector_type(8)));

template <typename H> struct Mfma16;
template <> struct Mfma16<__bf16> {
  typedef bf16x8 V8;
  static __device__ inline floatx4 mfma(V8 a, V8 b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <> struct Mfma16<_Float16> {
  typedef halfx8 V8;
  static __device__ inline floatx4 mfma(V8 a, V8 b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
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

// Wavelet details of one mode (W_{s,q} beside P_p): for reference coordinate t, calls
// f(row, value) for the q + 1 functions psi_{l,c,m}(t) of the point's cell c at every level
// l < s, with row = (q + 1)(2^l - 1 + c) + m the detail row of the coefficient matrix.
// psi_{l,c,m}(t) = 2^(l/2) psi_m(x), x = 2^l (t + 1) - 2c - 1, c = floor((t + 1) 2^(l-1))
// clamped to the level's cells; psi_m(x) = sqrt(2) sum_n wave[(m * 2 + half) * 8 + n]
// phi_n(2x -+ 1) on the half of [-1, 1] that holds x.  Loops run to the largest degree with
// predicates, so every array index is static.
template <typename T, typename F>
__device__ inline void for_each_detail(T t, int s, int q, const T* __restrict__ wave, const Recurrence<T>& rec,
                                       F&& f) {
  T scale = T(1.4142135623730951);   // sqrt(2) 2^(l/2) at level l
  for (int l = 0; l < s; ++l) {
    const int ncell = 1 << l;
    T cf = floor((t + T(1)) * T(0.5) * T(ncell));
    cf = cf < T(0) ? T(0) : (cf > T(ncell - 1) ? T(ncell - 1) : cf);
    const int c = (int)cf;
    const T x = (t + T(1)) * T(ncell) - T(2 * c + 1);
    const int half = x >= T(0) ? 1 : 0;
    const T y = half ? T(2) * x - T(1) : T(2) * x + T(1);
    T ph[kMaxWaveDegree + 1];
    ph[0] = T(1);
    {
      T pm1 = T(1), pm = y * rec.a[0];
#pragma unroll
      for (int n = 1; n <= kMaxWaveDegree; ++n) {
        ph[n] = pm;
        const T pn = rec.a[n] * y * pm - rec.b[n] * pm1;
        pm1 = pm;
        pm = pn;
      }
    }
    const int base = (q + 1) * (ncell - 1 + c);
#pragma unroll
    for (int m = 0; m <= kMaxWaveDegree; ++m) {
      if (m > q) break;
      const T* w = wave + (m * 2 + half) * (kMaxWaveDegree + 1);
      T v = T(0);
#pragma unroll
      for (int n = 0; n <= kMaxWaveDegree; ++n)
        if (n <= q) v += w[n] * ph[n];
      f(base + m, scale * v);
    }
    scale *= T(1.4142135623730951);
  }
}

// u[j] += sum over the point's detail functions of mode k of detail_k[row][j] psi(t), j < RP
// (detail_k: [kMaxDetail][kMaxRank]); u stays in registers (static indices only)
template <typename T, int RP>
__device__ __forceinline__ void add_details(T (&u)[RP], T t, int s, int q, const T* __restrict__ wave,
                                            const T* __restrict__ detail_k, const Recurrence<T>& rec) {
  for_each_detail(t, s, q, wave, rec, [&](int row, T v) {
    const T* dr = detail_k + row * kMaxRank;
#pragma unroll
    for (int j = 0; j < RP; ++j) u[j] += dr[j] * v;
  });
}

// lower-triangle tile t -> (bi, bj), bj <= bi, t = bi (bi + 1) / 2 + bj
__device__ inline void tri_tile(int64_t t, int64_t& bi, int64_t& bj) {
  int64_t b = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (b * (b + 1) / 2 > t) --b;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  bi = b;
  bj = t - b * (b + 1) / 2;
}

}  // namespace fst
