// Materialised design rows and the d-way form of the hot path for gfx950: Algorithm 2 and the
// reconstruction of eq. (1) for models with d = 4 modes (Sec. 2 states the format for any d;
// Sec. 6 compresses data in three space dimensions plus time), and the dense route of the
// 3-way Gram.  The d-way refit also takes 3-way models (r4 = 1).
//
//   k_factor_eval      eq. (2) at the M sampled rows for the d modes (fst_kernels.hip)
//   k_design_rows      rows of W in eq. (6) for a chunk of sampled rows, written transposed:
//                      A^T[j][q] = U1[q][j1] U2[q][j2] U3[q][j3] U4[q][j4],
//                      j = ((j1 r2 + j2) r3 + j3) r4 + j4
//   k_design_rows_vec  the same for 3-way models, 16 / sizeof(T) rows per thread
//   k_design_rows16    3-way rows in BF16 or scaled FP16 for the precision form
//   k_gram_dense       G += A^T A (lower triangle) of the chunk on MFMA, and h += A^T v
//                      (fst_mix.hip; k_gram_dense16 for 16-bit rows)
//   k_eval4            eq. (1) at points of interest
//
// A chunk of C rows is R C values, written once at HBM speed, against 2 R^2 C flop of Gram
// work on them, so the write costs about 1% of the contraction at R = 13,824-20,736, and the
// dense Gram, whose operands come straight from LDS, runs faster than the Khatri-Rao Gram of
// fst_kernels.hip, which forms the entries inside its MFMA loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

// ------------------------------------------------------------------------------ design rows
// One thread per row q of the chunk (q < Sp, rows mc .. Sp-1 are zero), each workgroup on one
// (j1, j2) pair: the product u1 u2 is formed once, the r4 values of U4 are held in registers
// (RP of them, clamped past r4; RP = 1 and u4 = 1 for a 3-way model) and every (j3, j4)
// column is a coalesced run of 256 entries of A^T.  The workgroups of pair 0 also write b.
template <typename T>
struct DesignArgs {
  const T* U;      // [sum r][M] factor values of the sampled rows (feature-major)
  const T* vs;     // [M] sampled values
  T* At;           // [R][Sp]
  T* b;            // [Sp]
  int64_t M, q0, mc, Sp;
  int32_t r[kMaxModes], off[kMaxModes];
};

constexpr int DR_THREADS = 256;

// Workgroup order: super-blocks of DR_SUPER row blocks of DR_THREADS rows; inside one, the
// (j1, j2) pairs, and inside a pair the row blocks.  The factor values of a super-block
// (sum r x 2048 entries) stay in L2 while all pairs read them, and each design row still
// receives runs of DR_SUPER x DR_THREADS contiguous entries.  sb0: first super-block of this
// launch.
constexpr int64_t DR_SUPER = 8;

template <typename T, int RP>
__global__ __launch_bounds__(DR_THREADS) void k_design_rows(DesignArgs<T> a, int64_t sb0) {
  const int64_t P = (int64_t)a.r[0] * a.r[1], nb = (a.Sp + DR_THREADS - 1) / DR_THREADS;
  const int64_t sb = sb0 + (int64_t)blockIdx.x / (P * DR_SUPER), rem = (int64_t)blockIdx.x % (P * DR_SUPER);
  const int64_t w = min(DR_SUPER, nb - sb * DR_SUPER);
  if (w <= 0) return;
  const int64_t pr = rem / w, cb = sb * DR_SUPER + rem % w;
  if (pr >= P) return;
  const int64_t q = cb * DR_THREADS + threadIdx.x;
  if (q >= a.Sp) return;
  const bool live = q < a.mc;
  const int64_t col = a.q0 + (live ? q : a.mc - 1);
  const int pair = (int)pr;
  const int j1 = pair / a.r[1], j2 = pair - j1 * a.r[1];
  const T* U = a.U;
  const T p12 = U[(int64_t)(a.off[0] + j1) * a.M + col] * U[(int64_t)(a.off[1] + j2) * a.M + col];
  const T pm = live ? p12 : T(0);
  T u4[RP];
#pragma unroll
  for (int j4 = 0; j4 < RP; ++j4)
    u4[j4] = RP == 1 ? T(1) : U[(int64_t)(a.off[3] + min(j4, a.r[3] - 1)) * a.M + col];
  T* dst = a.At + (int64_t)pair * a.r[2] * a.r[3] * a.Sp + q;
  for (int j3 = 0; j3 < a.r[2]; ++j3) {
    const T p = pm * U[(int64_t)(a.off[2] + j3) * a.M + col];
#pragma unroll
    for (int j4 = 0; j4 < RP; ++j4)
      if (j4 < a.r[3]) dst[(int64_t)(j3 * a.r[3] + j4) * a.Sp] = p * u4[j4];
  }
  if (pair == 0 && a.b) a.b[q] = live ? a.vs[col] : T(0);
}

constexpr int64_t DW_CHUNK = 16384;   // sampled rows per materialised chunk
static_assert(DW_CHUNK % GD_SP_MULTIPLE == 0, "chunks must be whole Gram chunks");

struct DwayLayout {
  int64_t Sc;                   // rows of the largest chunk, padded
  size_t U, vs, At, b, total;   // byte offsets in the workspace
};

static DwayLayout dway_layout(const fst_model* m, int dtype, int64_t M) {
  const size_t es = dtype == FST_F64 ? 8 : 4;
  DwayLayout L;
  L.Sc = std::min<int64_t>(DW_CHUNK, (M + GD_SP_MULTIPLE - 1) / GD_SP_MULTIPLE * GD_SP_MULTIPLE);
  size_t off = 0;
  L.U = off;
  off += align_up(es * (size_t)m->sum_r() * (size_t)M);
  L.vs = off;
  off += align_up(es * (size_t)M);
  L.At = off;
  off += align_up(es * (size_t)m->R() * (size_t)L.Sc);
  L.b = off;
  off += align_up(es * (size_t)L.Sc);
  L.total = off;
  return L;
}

size_t dway_workspace_bytes(const fst_model* m, int dtype, int64_t M) { return dway_layout(m, dtype, M).total; }

// 3-way models: each thread forms 16 / sizeof(T) consecutive rows with 16-byte loads of the
// factor values and 16-byte stores of A^T (same products in the same order as k_design_rows);
// threads that reach past the chunk's last row take their rows one by one.  Needs U rows and
// the chunk start aligned to the vector width (M and q0 multiples of it).  Workgroup order as
// in k_design_rows, with super-blocks of DRV_SUPER blocks of DR_THREADS vectors.
constexpr int64_t DRV_SUPER = 4;

template <typename T>
__global__ __launch_bounds__(DR_THREADS) void k_design_rows_vec(DesignArgs<T> a, int64_t sb0) {
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T TV __attribute__((ext_vector_type(VW)));
  const int64_t P = (int64_t)a.r[0] * a.r[1], nb = (a.Sp + DR_THREADS * VW - 1) / (DR_THREADS * VW);
  const int64_t sb = sb0 + (int64_t)blockIdx.x / (P * DRV_SUPER), rem = (int64_t)blockIdx.x % (P * DRV_SUPER);
  const int64_t w = min(DRV_SUPER, nb - sb * DRV_SUPER);
  if (w <= 0) return;
  const int64_t pr = rem / w, cb = sb * DRV_SUPER + rem % w;
  if (pr >= P) return;
  const int64_t q = (cb * DR_THREADS + threadIdx.x) * VW;
  if (q >= a.Sp) return;
  const int j1 = (int)(pr / a.r[1]), j2 = (int)(pr - (int64_t)j1 * a.r[1]);
  const T* U1 = a.U + (int64_t)(a.off[0] + j1) * a.M + a.q0;
  const T* U2 = a.U + (int64_t)(a.off[1] + j2) * a.M + a.q0;
  const T* U3 = a.U + (int64_t)a.off[2] * a.M + a.q0;
  T* dst = a.At + pr * a.r[2] * a.Sp + q;
  const bool full = q + VW <= a.mc;
  TV p12;
  if (full) {
    p12 = *reinterpret_cast<const TV*>(U1 + q) * *reinterpret_cast<const TV*>(U2 + q);
  } else {
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int64_t c = min(q + e, a.mc - 1);
      p12[e] = q + e < a.mc ? U1[c] * U2[c] : T(0);
    }
  }
  for (int j3 = 0; j3 < a.r[2]; ++j3) {
    const T* u3 = U3 + (int64_t)j3 * a.M;
    TV f;
    if (full) {
      f = *reinterpret_cast<const TV*>(u3 + q);
    } else {
#pragma unroll
      for (int e = 0; e < VW; ++e) f[e] = u3[min(q + e, a.mc - 1)];
    }
    *reinterpret_cast<TV*>(dst + (int64_t)j3 * a.Sp) = p12 * f;
  }
  if (pr == 0 && a.b) {
    TV bv;
#pragma unroll
    for (int e = 0; e < VW; ++e) bv[e] = q + e < a.mc ? a.vs[a.q0 + q + e] : T(0);
    *reinterpret_cast<TV*>(a.b + q) = bv;
  }
}

template <typename T>
static void design_launch_vec(const DesignArgs<T>& a, void* stream) {
  constexpr int VW = 16 / (int)sizeof(T);
  const int64_t P = (int64_t)a.r[0] * a.r[1], nb = (a.Sp + DR_THREADS * VW - 1) / (DR_THREADS * VW);
  const int64_t nsb = (nb + DRV_SUPER - 1) / DRV_SUPER, per = std::max<int64_t>(1, (int64_t(1) << 30) / (P * DRV_SUPER));
  for (int64_t sb0 = 0; sb0 < nsb; sb0 += per) {
    const int64_t n = std::min(per, nsb - sb0);
    hipLaunchKernelGGL(k_design_rows_vec<T>, dim3((unsigned)(n * P * DRV_SUPER)), dim3(DR_THREADS), 0, S(stream), a,
                       sb0);
    check_launch("k_design_rows_vec");
  }
}

// 16-bit design rows of a 3-way model for the precision form: entry ((u1 u2) scale) u3 formed
// in FP32 and rounded to H (the scale a power of two, 1 for BF16), as the Khatri-Rao
// precision-form Gram forms its operands; 8 consecutive rows per thread, one 16-byte store per
// design column; rows past mc are zero.  Workgroup order as k_design_rows_vec.
template <typename H>
__global__ __launch_bounds__(DR_THREADS) void k_design_rows16(DesignArgs<float> a, H* At, float scale, int64_t sb0) {
  constexpr int VW = 8;
  typedef H HV __attribute__((ext_vector_type(8)));
  typedef float F4 __attribute__((ext_vector_type(4)));
  const int64_t P = (int64_t)a.r[0] * a.r[1], nb = (a.Sp + DR_THREADS * VW - 1) / (DR_THREADS * VW);
  const int64_t sb = sb0 + (int64_t)blockIdx.x / (P * DRV_SUPER), rem = (int64_t)blockIdx.x % (P * DRV_SUPER);
  const int64_t w = min(DRV_SUPER, nb - sb * DRV_SUPER);
  if (w <= 0) return;
  const int64_t pr = rem / w, cb = sb * DRV_SUPER + rem % w;
  if (pr >= P) return;
  const int64_t q = (cb * DR_THREADS + threadIdx.x) * VW;
  if (q >= a.Sp) return;
  const int j1 = (int)(pr / a.r[1]), j2 = (int)(pr - (int64_t)j1 * a.r[1]);
  const float* U1 = a.U + (int64_t)(a.off[0] + j1) * a.M;
  const float* U2 = a.U + (int64_t)(a.off[1] + j2) * a.M;
  const float* U3 = a.U + (int64_t)a.off[2] * a.M;
  const bool vec = q + VW <= a.mc && a.M % 4 == 0;
  float p12[VW];
  if (vec) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const F4 x = *reinterpret_cast<const F4*>(U1 + q + 4 * h), y = *reinterpret_cast<const F4*>(U2 + q + 4 * h);
#pragma unroll
      for (int e = 0; e < 4; ++e) p12[4 * h + e] = x[e] * y[e] * scale;
    }
  } else {
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int64_t c = min(q + e, a.mc - 1);
      p12[e] = q + e < a.mc ? U1[c] * U2[c] * scale : 0.0f;
    }
  }
  H* dst = At + pr * a.r[2] * a.Sp + q;
  for (int j3 = 0; j3 < a.r[2]; ++j3) {
    const float* u3 = U3 + (int64_t)j3 * a.M;
    float f[VW];
    if (vec) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const F4 z = *reinterpret_cast<const F4*>(u3 + q + 4 * h);
#pragma unroll
        for (int e = 0; e < 4; ++e) f[4 * h + e] = z[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < VW; ++e) f[e] = u3[min(q + e, a.mc - 1)];
    }
    HV hv;
#pragma unroll
    for (int e = 0; e < VW; ++e) hv[e] = (H)(p12[e] * f[e]);
    *reinterpret_cast<HV*>(dst + (int64_t)j3 * a.Sp) = hv;
  }
}

template <typename T, int RP>
static void design_launch(const DesignArgs<T>& a, void* stream) {
  const int64_t P = (int64_t)a.r[0] * a.r[1], nb = (a.Sp + DR_THREADS - 1) / DR_THREADS;
  const int64_t nsb = (nb + DR_SUPER - 1) / DR_SUPER, per = std::max<int64_t>(1, (int64_t(1) << 30) / (P * DR_SUPER));
  for (int64_t sb0 = 0; sb0 < nsb; sb0 += per) {
    // the last super-block may hold fewer row blocks: its pairs take P w workgroups, and the
    // launch's tail of P (DR_SUPER - w) workgroups finds nothing to do
    const int64_t n = std::min(per, nsb - sb0);
    hipLaunchKernelGGL((k_design_rows<T, RP>), dim3((unsigned)(n * P * DR_SUPER)), dim3(DR_THREADS), 0, S(stream),
                       a, sb0);
    check_launch("k_design_rows");
  }
}

template <typename T>
static DesignArgs<T> design_args(const fst_model* m, const T* U, const T* vs, int64_t M, T* At, T* b) {
  DesignArgs<T> a;
  a.U = U;
  a.vs = vs;
  a.At = At;
  a.b = b;
  a.M = M;
  int off = 0;
  for (int k = 0; k < kMaxModes; ++k) {
    a.r[k] = k < m->d ? m->rank[k] : 1;
    a.off[k] = off;
    off += k < m->d ? m->rank[k] : 0;
  }
  return a;
}

// rows q0 .. q0 + mc - 1 written as columns 0 .. mc - 1 of At (R x Sp), columns mc .. Sp - 1 zero
template <typename T>
static void design_chunk(const fst_model* m, DesignArgs<T>& a, int64_t q0, int64_t mc, int64_t Sp, void* stream) {
  a.q0 = q0;
  a.mc = mc;
  a.Sp = Sp;
  constexpr int VW = 16 / (int)sizeof(T);
  if (m->d == 3 && a.M % VW == 0 && q0 % VW == 0) {
    design_launch_vec(a, stream);
    return;
  }
  switch (m->d == 4 ? pad8(m->rank[3]) : 1) {
    case 1: design_launch<T, 1>(a, stream); break;
    case 8: design_launch<T, 8>(a, stream); break;
    case 16: design_launch<T, 16>(a, stream); break;
    case 24: design_launch<T, 24>(a, stream); break;
    default: design_launch<T, 32>(a, stream); break;
  }
}

// G = A^T A and h = A^T v_S (either may be NULL) over M rows given by their factor values,
// `chunk` rows at a time materialised in At (and b)
template <typename T>
static void rows_normal_equations(const fst_model* m, const T* U, const T* vs, int64_t M, T* At, T* b,
                                  int64_t chunk, double* G, double* h, void* stream) {
  DesignArgs<T> a = design_args(m, U, vs, M, At, b);
  for (int64_t q0 = 0; q0 < M; q0 += chunk) {
    const int64_t mc = std::min<int64_t>(chunk, M - q0);
    const int64_t Sp = (mc + GD_SP_MULTIPLE - 1) / GD_SP_MULTIPLE * GD_SP_MULTIPLE;
    design_chunk(m, a, q0, mc, Sp, stream);
    dense_normal_equations(sizeof(T) == 8 ? FST_F64 : FST_F32, At, b, m->R(), Sp, G, h, q0 > 0, stream);
  }
}

size_t dense_rows_bytes(const fst_model* m, int dtype, int64_t chunk) {
  return align_up((dtype == FST_F64 ? 8 : 4) * (size_t)m->R() * (size_t)chunk);
}

void dense_gram_from_rows(const fst_model* m, int dtype, int64_t mrows, const void* U, double* G, void* At,
                          int64_t chunk, void* stream) {
  if (chunk <= 0 || chunk % GD_SP_MULTIPLE != 0) fail(FST_E_INVAL, "dense Gram: bad chunk");
  if (m->R() * chunk >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "dense Gram: chunk of A^T too large");
  if (dtype == FST_F64)
    rows_normal_equations<double>(m, (const double*)U, nullptr, mrows, (double*)At, nullptr, chunk, G, nullptr,
                                  stream);
  else
    rows_normal_equations<float>(m, (const float*)U, nullptr, mrows, (float*)At, nullptr, chunk, G, nullptr,
                                 stream);
}

void design_rows(const fst_model* m, int dtype, int64_t mrows, const void* U, const void* vs, int64_t Sp, void* At,
                 void* b, void* stream) {
  if (Sp < mrows || Sp % GD_SP_MULTIPLE != 0) fail(FST_E_INVAL, "design rows: Sp must be a multiple of 64 >= mrows");
  if (m->R() * Sp >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "design rows: A^T too large");
  if (b && !vs) fail(FST_E_INVAL, "design rows: b needs the sampled values");
  if (mrows < 1) fail(FST_E_INVAL, "design rows: mrows must be >= 1");
  if (dtype == FST_F64) {
    DesignArgs<double> a = design_args(m, (const double*)U, (const double*)vs, mrows, (double*)At, (double*)b);
    design_chunk(m, a, 0, mrows, Sp, stream);
  } else {
    DesignArgs<float> a = design_args(m, (const float*)U, (const float*)vs, mrows, (float*)At, (float*)b);
    design_chunk(m, a, 0, mrows, Sp, stream);
  }
}

void design_rows16(const fst_model* m, int gram_prec, int64_t mrows, const float* U, int64_t Sp, void* At, float scale,
                   void* stream) {
  if (m->d != 3 || mrows < 1 || Sp < mrows || Sp % 8 != 0) fail(FST_E_INVAL, "16-bit design rows: bad sizes");
  DesignArgs<float> a = design_args<float>(m, U, nullptr, mrows, nullptr, nullptr);
  a.q0 = 0;
  a.mc = mrows;
  a.Sp = Sp;
  const int64_t P = (int64_t)a.r[0] * a.r[1], nb = (Sp + DR_THREADS * 8 - 1) / (DR_THREADS * 8);
  const int64_t nsb = (nb + DRV_SUPER - 1) / DRV_SUPER, per = std::max<int64_t>(1, (int64_t(1) << 30) / (P * DRV_SUPER));
  for (int64_t sb0 = 0; sb0 < nsb; sb0 += per) {
    const dim3 g((unsigned)(std::min(per, nsb - sb0) * P * DRV_SUPER));
    if (gram_prec == FST_GRAM_BF16)
      hipLaunchKernelGGL(k_design_rows16<__bf16>, g, dim3(DR_THREADS), 0, S(stream), a, (__bf16*)At, scale, sb0);
    else
      hipLaunchKernelGGL(k_design_rows16<_Float16>, g, dim3(DR_THREADS), 0, S(stream), a, (_Float16*)At, scale, sb0);
    check_launch("k_design_rows16");
  }
}

void dway_normal_equations(const fst_model* m, int dtype, const void* const* coords, const void* v,
                           const int32_t* idx, int64_t M, void* ws, size_t ws_bytes, double* G, double* h,
                           void* stream) {
  const DwayLayout L = dway_layout(m, dtype, M);
  if (ws_bytes < L.total) fail(FST_E_NOMEM, "d-way rows: workspace too small");
  if (m->R() * L.Sc >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "d-way rows: chunk of A^T too large");
  if ((int64_t)m->sum_r() * M >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "d-way rows: too many factor values");
  char* w = (char*)ws;
  const DeviceModel& dm = device_model(m, dtype);
  // Algorithm 2 step 1 at the sampled rows: factor functions of the d modes and the values
  launch_factor_eval_d(m, dm, dtype, coords, v, idx, M, w + L.U, w + L.vs, stream);
  // step 5: normal equations of the sampled rows, chunk by chunk
  if (dtype == FST_F64)
    rows_normal_equations<double>(m, (const double*)(w + L.U), (const double*)(w + L.vs), M, (double*)(w + L.At),
                                  (double*)(w + L.b), L.Sc, G, h, stream);
  else
    rows_normal_equations<float>(m, (const float*)(w + L.U), (const float*)(w + L.vs), M, (float*)(w + L.At),
                                 (float*)(w + L.b), L.Sc, G, h, stream);
}

// ------------------------------------------------------------------------------ subset gather
// The interpolation subset of Algorithm 1 (D coordinates and the value of each chosen point)
// copied into one FP64 array for the host steps.
struct GatherArgs {
  const void* c[kMaxModes];
  const void* v;
  const int32_t* idx;
  double* out;
  int64_t K;
  int32_t D, f64;
};

__global__ void k_gather_d(GatherArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.K) return;
  const int64_t i = a.idx[t];
  double* o = a.out + (a.D + 1) * t;
  for (int k = 0; k <= a.D; ++k) {
    const void* src = k < a.D ? a.c[k] : a.v;
    o[k] = a.f64 ? ((const double*)src)[i] : (double)((const float*)src)[i];
  }
}

size_t gather_workspace_bytes(int64_t K, int D) {
  return align_up(sizeof(int32_t) * (size_t)K) + sizeof(double) * (size_t)(D + 1) * (size_t)K;
}

void gather_points_d(int dtype, int64_t K, const int64_t* idx_host, int D, const void* const* coords, const void* v,
                     double* out_host, void* ws, size_t ws_bytes, void* stream) {
  if (ws_bytes < gather_workspace_bytes(K, D)) fail(FST_E_NOMEM, "gather: workspace too small");
  if (K <= 0) return;
  std::vector<int32_t> idx32((size_t)K);
  for (int64_t t = 0; t < K; ++t) idx32[(size_t)t] = (int32_t)idx_host[t];
  GatherArgs a;
  for (int k = 0; k < kMaxModes; ++k) a.c[k] = k < D ? coords[k] : nullptr;
  a.v = v;
  a.idx = (int32_t*)ws;
  a.out = (double*)((char*)ws + align_up(sizeof(int32_t) * (size_t)K));
  a.K = K;
  a.D = D;
  a.f64 = dtype == FST_F64 ? 1 : 0;
  copy_h2d((void*)a.idx, idx32.data(), sizeof(int32_t) * (size_t)K, stream);
  hipLaunchKernelGGL(k_gather_d, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, S(stream), a);
  check_launch("k_gather_d");
  copy_d2h(out_host, a.out, sizeof(double) * (size_t)(D + 1) * (size_t)K, stream);
}

// ------------------------------------------------------------------------------ reconstruction
// eq. (1) for d = 4: f = sum_{j1 j2} u1[j1] u2[j2] sum_{j3} u3[j3] sum_{j4} alpha[j1 j2 j3 j4] u4[j4].
// One thread per point.  The basis values of modes 1 and 2 and the factor values u3, u4 (RP of
// each, zero past r3, r4) stay in registers; u1 and u2 are formed per (j1, j2) pair from the
// coefficients, read with wave-uniform addresses.  The core is staged in LDS as RP x RP slices
// per (j1, j2) pair (zero-padded), as many pairs per slice as fit in 64 KB; every thread reads
// the same LDS word at a time (a broadcast).  The sums run in a fixed order.
template <typename TIn, typename T>
struct Eval4Args {
  const TIn* c[kMaxModes];
  const T* coefs;   // [kMaxModes][kMaxBasis][kMaxRank]
  const T* core;    // R, C order
  TIn* out;
  int64_t n;
  int32_t r[kMaxModes];
  int32_t pair_chunk;
  ModeMap<T> map;
  Recurrence<T> rec;
};

constexpr size_t EVAL4_LDS_BUDGET = 64 * 1024;

template <typename TIn, typename T, int NP, int RP>
__global__ __launch_bounds__(256) void k_eval4(Eval4Args<TIn, T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);   // [pair_chunk][RP][RP]
  const T* __restrict__ C1 = a.coefs;
  const T* __restrict__ C2 = a.coefs + kMaxBasis * kMaxRank;
  const T* __restrict__ C3 = a.coefs + 2 * kMaxBasis * kMaxRank;
  const T* __restrict__ C4 = a.coefs + 3 * kMaxBasis * kMaxRank;
  const int r2 = a.r[1], r3 = a.r[2], r4 = a.r[3];
  const int npairs = a.r[0] * r2;
  const int nchunk = (npairs + a.pair_chunk - 1) / a.pair_chunk;
  auto load_chunk = [&](int c) {
    const int p0 = c * a.pair_chunk;
    const int rows = min(a.pair_chunk, npairs - p0);
    for (int e = threadIdx.x; e < rows * RP * RP; e += blockDim.x) {
      const int pp = e / (RP * RP), j3 = (e / RP) % RP, j4 = e % RP;
      sA[e] = (j3 < r3 && j4 < r4) ? a.core[((int64_t)(p0 + pp) * r3 + j3) * r4 + j4] : T(0);
    }
  };
  if (nchunk == 1) load_chunk(0);
  __syncthreads();

  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nround = (a.n + stride - 1) / stride;
  for (int64_t rnd = 0; rnd < nround; ++rnd) {
    const int64_t q = rnd * stride + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = q < a.n;
    const int64_t i = live ? q : 0;
    T t[kMaxModes];
#pragma unroll
    for (int k = 0; k < kMaxModes; ++k) t[k] = ((T)a.c[k][i] - a.map.lo[k]) * a.map.scale[k] - T(1);
    T phi1[NP], phi2[NP];
    {
      T pm1 = T(1), pm = t[0] * a.rec.a[0], rm1 = T(1), rm = t[1] * a.rec.a[0];
      phi1[0] = T(1);
      phi2[0] = T(1);
#pragma unroll
      for (int m = 1; m < NP; ++m) {
        phi1[m] = pm;
        phi2[m] = rm;
        const T pn = a.rec.a[m] * t[0] * pm - a.rec.b[m] * pm1;
        pm1 = pm;
        pm = pn;
        const T rn = a.rec.a[m] * t[1] * rm - a.rec.b[m] * rm1;
        rm1 = rm;
        rm = rn;
      }
    }
    T u3[RP], u4[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) {
      u3[j] = C3[j];
      u4[j] = C4[j];
    }
    {
      T pm1 = T(1), pm = t[2] * a.rec.a[0], rm1 = T(1), rm = t[3] * a.rec.a[0];
#pragma unroll
      for (int m = 1; m < NP; ++m) {
#pragma unroll
        for (int j = 0; j < RP; ++j) {
          u3[j] += C3[m * kMaxRank + j] * pm;
          u4[j] += C4[m * kMaxRank + j] * rm;
        }
        const T pn = a.rec.a[m] * t[2] * pm - a.rec.b[m] * pm1;
        pm1 = pm;
        pm = pn;
        const T rn = a.rec.a[m] * t[3] * rm - a.rec.b[m] * rm1;
        rm1 = rm;
        rm = rn;
      }
    }
    T acc = T(0);
    for (int c = 0; c < nchunk; ++c) {
      if (nchunk > 1) {
        __syncthreads();
        load_chunk(c);
        __syncthreads();
      }
      const int p0 = c * a.pair_chunk;
      const int rows = min(a.pair_chunk, npairs - p0);
      int j1_prev = -1;
      T u1 = T(0);
      for (int pp = 0; pp < rows; ++pp) {
        const int p = p0 + pp, j1 = p / r2, j2 = p - j1 * r2;
        if (j1 != j1_prev) {   // uniform across the workgroup
          u1 = T(0);
#pragma unroll
          for (int m = 0; m < NP; ++m) u1 += C1[m * kMaxRank + j1] * phi1[m];
          j1_prev = j1;
        }
        T u2 = T(0);
#pragma unroll
        for (int m = 0; m < NP; ++m) u2 += C2[m * kMaxRank + j2] * phi2[m];
        const T* ap = &sA[pp * RP * RP];
        T s = T(0);
#pragma unroll
        for (int j3 = 0; j3 < RP; ++j3) {
          T w = T(0);
#pragma unroll
          for (int j4 = 0; j4 < RP; ++j4) w += ap[j3 * RP + j4] * u4[j4];
          s += w * u3[j3];
        }
        acc += (u1 * u2) * s;
      }
    }
    if (live) a.out[q] = (TIn)acc;
  }
}

template <typename TIn, typename T, int NP, int RP>
static void eval4_launch(Eval4Args<TIn, T>& a, void* stream) {
  const size_t per_pair = sizeof(T) * RP * RP;
  const int npairs = a.r[0] * a.r[1];
  a.pair_chunk = (int)std::min<size_t>((size_t)npairs, std::max<size_t>(1, EVAL4_LDS_BUDGET / per_pair));
  const size_t lds = per_pair * (size_t)a.pair_chunk;
  const int64_t blocks = std::min<int64_t>((a.n + 255) / 256, (int64_t)device_cu_count() * 8);
  if (blocks < 1) return;
  hipLaunchKernelGGL((k_eval4<TIn, T, NP, RP>), dim3((unsigned)blocks), dim3(256), lds, S(stream), a);
  check_launch("k_eval4");
}

template <typename TIn, typename T>
static void eval4_t(const fst_model* m, const DeviceModel& dm, int64_t n, const void* const* coords, void* out,
                    void* stream) {
  Eval4Args<TIn, T> a;
  for (int k = 0; k < kMaxModes; ++k) {
    a.c[k] = (const TIn*)coords[k];
    a.r[k] = m->rank[k];
  }
  a.coefs = (const T*)dm.coefs;
  a.core = (const T*)dm.core;
  a.out = (TIn*)out;
  a.n = n;
  a.map = make_map<T>(m);
  a.rec = make_recurrence<T>();
  const int rp = (std::max(m->rank[2], m->rank[3]) + 3) / 4 * 4;
  const bool np16 = m->degree[0] < 16 && m->degree[1] < 16 && m->degree[2] < 16 && m->degree[3] < 16;
#define FST_EVAL4_RP(NPV)                                       \
  switch (rp) {                                                 \
    case 4: eval4_launch<TIn, T, NPV, 4>(a, stream); break;     \
    case 8: eval4_launch<TIn, T, NPV, 8>(a, stream); break;     \
    case 12: eval4_launch<TIn, T, NPV, 12>(a, stream); break;   \
    case 16: eval4_launch<TIn, T, NPV, 16>(a, stream); break;   \
    case 20: eval4_launch<TIn, T, NPV, 20>(a, stream); break;   \
    case 24: eval4_launch<TIn, T, NPV, 24>(a, stream); break;   \
    case 28: eval4_launch<TIn, T, NPV, 28>(a, stream); break;   \
    default: eval4_launch<TIn, T, NPV, 32>(a, stream); break;   \
  }
  if (np16) {
    FST_EVAL4_RP(16)
  } else {
    FST_EVAL4_RP(32)
  }
#undef FST_EVAL4_RP
}

// ------------------------------------------------------------------------------ wavelet models
// eq. (1) for models whose modes hold wavelet details (d = 3 or 4), one thread per point and
// no cross-thread work: the thread builds the factor values of each mode in its own LDS
// column (basis values, then the Legendre sums, then the detail sums of the point's cells),
// keeps the last mode's RP values in registers (rows past r zero) and contracts the core in
// a fixed order, reading core entries with wave-uniform addresses (indices clamped into the
// core, where they meet a zero factor value).  With residual != 0 it writes v[idx[q]] - f.
template <typename TIn, typename T>
struct EvalWaveArgs {
  const TIn* c[kMaxModes];
  const TIn* v;
  const int32_t* idx;
  const T* coefs;     // [kMaxModes][kMaxBasis][kMaxRank]
  const T* detail;    // [kMaxModes][kMaxDetail][kMaxRank]
  const T* wave;      // [kMaxModes][kWaveTable]
  const T* core;
  void* out;          // TIn (eval) or T (residual)
  int64_t n;
  int32_t d, residual;
  int32_t r[kMaxModes], nb[kMaxModes], wl[kMaxModes], wq[kMaxModes], off[kMaxModes];
  ModeMap<T> map;
  Recurrence<T> rec;
};

constexpr int EW_THREADS = 64;

template <typename TIn, typename T, int RP>
__global__ __launch_bounds__(EW_THREADS) void k_eval_wave(EvalWaveArgs<TIn, T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int st = blockDim.x, me = threadIdx.x;
  T* sPhi = reinterpret_cast<T*>(smem_raw) + me;     // [kMaxBasis][st]
  T* sU = reinterpret_cast<T*>(smem_raw) + (size_t)kMaxBasis * st + me;   // [rows][st]
  const int last = a.d - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.n; q += stride) {
    const int64_t i = a.idx ? (int64_t)a.idx[q] : q;
    for (int k = 0; k < a.d; ++k) {
      const T t = ((T)a.c[k][i] - a.map.lo[k]) * a.map.scale[k] - T(1);
      {
        T pm1 = T(1), pm = t * a.rec.a[0];
        sPhi[0] = T(1);
        for (int m = 1; m < a.nb[k]; ++m) {
          sPhi[m * st] = pm;
          const T pn = a.rec.a[m] * t * pm - a.rec.b[m] * pm1;
          pm1 = pm;
          pm = pn;
        }
      }
      T* col = sU + (size_t)a.off[k] * st;
      const T* Ck = a.coefs + (size_t)k * kMaxBasis * kMaxRank;
      const int rows = k == last ? RP : a.r[k];
      for (int j = 0; j < rows; ++j) {
        T u = T(0);
        if (j < a.r[k])
          for (int m = 0; m < a.nb[k]; ++m) u += Ck[m * kMaxRank + j] * sPhi[m * st];
        col[j * st] = u;
      }
      if (a.wl[k] > 0) {
        const T* dk = a.detail + (size_t)k * kMaxDetail * kMaxRank;
        const int rk = a.r[k];
        for_each_detail(t, a.wl[k], a.wq[k], a.wave + k * kWaveTable, a.rec, [&](int row, T val) {
          const T* dr = dk + row * kMaxRank;
          for (int j = 0; j < rk; ++j) col[j * st] += dr[j] * val;
        });
      }
    }
    T ul[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) ul[j] = sU[(size_t)(a.off[last] + j) * st];
    const int rl = a.r[last];
    // sum over the leading modes (two for d = 3, three for d = 4) of their factor values times
    // the inner contraction with the last mode
    const int64_t lead = a.d == 3 ? (int64_t)a.r[0] * a.r[1] : (int64_t)a.r[0] * a.r[1] * a.r[2];
    T acc = T(0);
    for (int64_t p = 0; p < lead; ++p) {
      T w = T(1);
      int64_t rem = p;
      for (int k = a.d - 2; k >= 0; --k) {
        const int jk = (int)(rem % a.r[k]);
        rem /= a.r[k];
        w *= sU[(size_t)(a.off[k] + jk) * st];
      }
      const T* cp = a.core + p * rl;
      T s = T(0);
#pragma unroll
      for (int j = 0; j < RP; ++j) s += cp[j < rl ? j : rl - 1] * ul[j];
      acc += w * s;
    }
    if (a.residual)
      reinterpret_cast<T*>(a.out)[q] = (T)a.v[i] - acc;
    else
      reinterpret_cast<TIn*>(a.out)[q] = (TIn)acc;
  }
}

template <typename TIn, typename T>
static void eval_wave_t(const fst_model* m, const DeviceModel& dm, int64_t n, const void* const* coords,
                        const int32_t* idx, const void* v, void* out, bool residual, void* stream) {
  if (!dm.detail || !dm.wave) fail(FST_E_DEVICE, "reconstruction: wavelet tables missing");
  EvalWaveArgs<TIn, T> a;
  a.d = m->d;
  int off = 0;
  for (int k = 0; k < kMaxModes; ++k) {
    const bool live = k < m->d;
    a.c[k] = live ? (const TIn*)coords[k] : nullptr;
    a.r[k] = live ? m->rank[k] : 1;
    a.nb[k] = live ? m->degree[k] + 1 : 0;
    a.wl[k] = live ? m->wlevel[k] : 0;
    a.wq[k] = live ? m->wdegree[k] : 0;
    a.off[k] = off;
    off += live ? (k == m->d - 1 ? kMaxRank : m->rank[k]) : 0;
  }
  a.v = (const TIn*)v;
  a.idx = idx;
  a.coefs = (const T*)dm.coefs;
  a.detail = (const T*)dm.detail;
  a.wave = (const T*)dm.wave;
  a.core = (const T*)dm.core;
  a.out = out;
  a.n = n;
  a.residual = residual ? 1 : 0;
  a.map = make_map<T>(m);
  a.rec = make_recurrence<T>();
  const size_t lds = sizeof(T) * (size_t)EW_THREADS * (kMaxBasis + off);
  const int64_t blocks = std::min<int64_t>((n + EW_THREADS - 1) / EW_THREADS, (int64_t)device_cu_count() * 16);
  if (blocks < 1) return;
  const int rp = pad8(m->rank[m->d - 1]);
  const dim3 g((unsigned)blocks), b(EW_THREADS);
  switch (rp) {
    case 8: hipLaunchKernelGGL((k_eval_wave<TIn, T, 8>), g, b, lds, S(stream), a); break;
    case 16: hipLaunchKernelGGL((k_eval_wave<TIn, T, 16>), g, b, lds, S(stream), a); break;
    case 24: hipLaunchKernelGGL((k_eval_wave<TIn, T, 24>), g, b, lds, S(stream), a); break;
    default: hipLaunchKernelGGL((k_eval_wave<TIn, T, 32>), g, b, lds, S(stream), a); break;
  }
  check_launch("k_eval_wave");
}

void launch_eval_wave(const fst_model* m, const DeviceModel& dm, int dtype, int in_dtype, int64_t n,
                      const void* const* coords, const int32_t* idx, const void* v, void* out, bool residual,
                      void* stream) {
  if (dtype == FST_F64 && in_dtype == FST_F64)
    eval_wave_t<double, double>(m, dm, n, coords, idx, v, out, residual, stream);
  else if (dtype == FST_F64)
    eval_wave_t<float, double>(m, dm, n, coords, idx, v, out, residual, stream);
  else
    eval_wave_t<float, float>(m, dm, n, coords, idx, v, out, residual, stream);
}

void launch_eval_d(const fst_model* m, const DeviceModel& dm, int dtype, int64_t n, const void* const* coords,
                   void* out, void* stream) {
  if (m->has_wavelets()) {
    launch_eval_wave(m, dm, dtype, dtype, n, coords, nullptr, nullptr, out, false, stream);
    return;
  }
  if (m->d == 3) {
    launch_eval(m, dm, dtype, n, coords[0], coords[1], coords[2], nullptr, nullptr, out, stream);
    return;
  }
  if (dtype == FST_F64)
    eval4_t<double, double>(m, dm, n, coords, out, stream);
  else
    eval4_t<float, float>(m, dm, n, coords, out, stream);
}

}  // namespace fst
