// Factor evaluation of eq. (2) with the contraction on MFMA (gfx950):
//
//   U_k[j, q] = sum_m C_k[m, j] phi_m(xi_k(x_q)),   m < n_k = p_k + 1 <= 32,  j < r_k <= 32
//
// Per 64 sampled rows and mode, U_k (64 x r_k) = Phi (64 x n_k) C_k (n_k x r_k) is a GEMM with
// K = n_k <= 32: one step of MFMA 16x16x32 FP16 per 16 x 16 block, over operands split in two
// FP16 terms each (x = hi + lo: hi = x rounded to FP16, lo = x - hi exact in FP32 and rounded
// to FP16, 22 significant bits; hi*hi + hi*lo + lo*hi, FP32 accumulation; the dropped lo*lo is
// below 2^-22 of the product).  FP32 MFMA would take four times the matrix-core time and, on
// this chip, does not run alongside the VALU work of the wave (the basis recurrence), while
// the 16-bit MFMAs do.
//
// Basis: a factor function of eq. (2) is a polynomial of degree n_k - 1; the kernel evaluates
// it in the Chebyshev basis, sum_m C[m, j] phi_m = sum_i D[i, j] T_i, with D formed in FP64
// when the model is placed on the device (phi_m = sqrt(2m+1) P_m = sum_i L[m, i] T_i,
// D = L^T C; sum_i |D_i| <= sum_m sqrt(2m+1) |C_m|, so the Chebyshev form is no worse
// conditioned than the Legendre one).  T_{i+1} = 2 t T_i - T_{i-1} is one VALU operation per
// degree (the Legendre recurrence takes two).  |T_i(t)| <= rho^i with
// rho = |t| + sqrt(t^2 - 1) (rho = 1 inside the box), so starting the recurrence at 2^xs with
// xs = 14 - ceil((n_k - 1) log2 rho) keeps every value the mode uses below 2^15, in FP16
// range (values past n_k, whose coefficients are zero, are clamped into it).  The
// coefficients of a mode come scaled by one power of two (largest to [2^14, 2^15), applied
// with D); both scales are undone on the accumulators through a per-point factor.
//
// Per wave and round of 64 rows, lane l takes row q0 + l and, for each mode:
//   1. runs the recurrence for the 32 basis values of its row and splits them into FP16 terms
//      (16 pairs per term);
//   2. a 4 x 4 transpose of 16-lane blocks (v_permlane16_swap, v_permlane32_swap) per pair
//      position turns them into the A operands of the four 16-row tiles (lane group g: the
//      basis values 8 g .. 8 g + 7 of rows 16 t + li, the k-slot g);
//   3. three MFMAs per tile and 16-column block; the B operands (coefficients 8 g .. 8 g + 7 of
//      column 16 jb + li, both terms) come from an LDS copy with 80-byte rows (conflict-free).
// Lane l then holds U_k[16 jb + l % 16] at rows 16 t + 4 (l / 16) + v, v = 0..3.  A store of
// that layout would touch 16 columns of U (mrows apart) with 64 bytes each, and the store path
// spends its time on the per-column requests; so each 16-column block goes through a per-wave
// LDS tile [16 columns][64 rows] and leaves as four stores of four whole column segments
// (lanes 16 G .. 16 G + 15 write rows q0 .. q0 + 63 of one column: 256 contiguous bytes).
// A wave loads the coordinates of up to eight rounds at once (through the row index of a
// gather) and parks them in LDS before computing them, so no load waits behind its stores
// (vector memory counts loads and stores in one queue).  The sampled values v_S are gathered by
// a separate first pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

constexpr int FM_WAVES = 4, FM_THREADS = 64 * FM_WAVES, FM_ROWS = 64, FM_PARK = 6, FM_TPAD = 68;

typedef float fm_floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t fm_uintx4 __attribute__((ext_vector_type(4)));
// buffer offset of a dropped store, and the largest U (bytes) that the kernel writes
constexpr uint32_t kFmSkip = 0x80000000u;
// cache policy of the U stores: non-temporal (U is streamed to HBM for a later kernel; 10%
// faster than stores that allocate in L2)
constexpr int kFmNontemporal = 2;
constexpr int64_t kFmMaxUBytes = 0x7FFFFF00;

template <typename TIn>
struct FactorMfmaArgs {
  const TIn* c[kMaxModes];
  const TIn* v;
  const int32_t* idx;
  const float* coefs;   // Chebyshev coefficients D 2^xc, [kMaxModes][kMaxBasis][kMaxRank]
  float* U;
  float* vs;
  int64_t mrows, nrounds, ubytes;
  int32_t d;
  int32_t rank[kMaxModes], nb[kMaxModes], off[kMaxModes];
  int32_t xc[kMaxModes];   // the coefficients' scale exponents
  // -1, passed at run time: the compiler then forms lo = x - hi as one mixed-precision FMA
  // (v_fma_mix_f32, hi read as FP16) instead of a conversion back to FP32 and a subtraction
  float minus_one;
  ModeMap<float> map;
};

constexpr int FM_BPAD = 40;   // halfs per staged coefficient row (80 bytes)
// scale exponents: xs in [-100, 14] (rows up to |t| of about 6 stay in FP16 range, about
// where FP32 values of degree 31 overflow too), xc in [-20, 26] (largest coefficient between
// 2^-12 and 2^34); the unscale 2^-(xs + xc) is then a normal float
constexpr int FM_XSMIN = -100, FM_XCMIN = -20, FM_XCMAX = 26;

typedef _Float16 fm_half2 __attribute__((ext_vector_type(2)));
typedef _Float16 fm_half8 __attribute__((ext_vector_type(8)));

// JB: blocks of 16 columns (ceil(max r_k / 16)); NQ: basis values evaluated (16 or 32, at
// least max n_k); VEC: the row count is a multiple of 4 (16-byte stores).
template <typename TIn, int D, int JB, int NQ, bool VEC>
__global__ __launch_bounds__(FM_THREADS) __attribute__((amdgpu_waves_per_eu(D == 3 ? 3 : 2))) void k_factor_eval_mfma(
    FactorMfmaArgs<TIn> a) {
  __shared__ __align__(16) _Float16 sB[2][D][32][FM_BPAD];   // [term][mode][column j][degree m]
  __shared__ __align__(16) float sPark[FM_WAVES][FM_PARK][D][64];
  __shared__ __align__(16) float sUs[FM_WAVES][64];            // per-point unscale of the mode
  __shared__ __align__(16) float sT[FM_WAVES][16][FM_TPAD];      // column block on its way out
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  for (int e = threadIdx.x; e < D * 32 * FM_BPAD; e += FM_THREADS) {
    const int k = e / (32 * FM_BPAD), j = (e / FM_BPAD) % 32, m = e % FM_BPAD;
    const float x = (m < a.nb[k] && j < a.rank[k]) ? a.coefs[(k * kMaxBasis + m) * kMaxRank + j] : 0.0f;
    const _Float16 hi = (_Float16)x;
    sB[0][k][j][m] = hi;
    sB[1][k][j][m] = (_Float16)(x - (float)hi);
  }
  // values of the sampled rows (a gather when idx is given)
  if (a.vs) {
    for (int64_t q = (int64_t)blockIdx.x * FM_THREADS + threadIdx.x; q < a.mrows; q += (int64_t)gridDim.x * FM_THREADS)
      a.vs[q] = (float)a.v[a.idx ? (int64_t)a.idx[q] : q];
  }
  __syncthreads();
  int xc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xc[k] = a.xc[k];
  // U through a buffer resource: a store whose offset is past the end (kFmSkip) is dropped by
  // the hardware, so the stores need no branches
  const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.U, (short)0, (int)(uint32_t)(a.ubytes), 0x00020000);
  // Each wave takes up to FM_PARK rounds per pass (rounds w, w + W, .. of the pass, W = all
  // waves of the grid): their coordinates are loaded first and parked in LDS, then the rounds
  // are computed and stored with no load in between (loads and stores share one counter of
  // outstanding requests, so a load after stores waits for them).
  float (*park)[D][64] = sPark[wave];
  float* us = sUs[wave];
  float (*tt)[FM_TPAD] = sT[wave];
  const int64_t wtot = (int64_t)gridDim.x * FM_WAVES, w = (int64_t)blockIdx.x * FM_WAVES + wave;
  for (int64_t pass0 = w; pass0 < a.nrounds; pass0 += wtot * FM_PARK) {
    int nr = 0;
    uint32_t rows[FM_PARK];
#pragma unroll
    for (int i = 0; i < FM_PARK; ++i) {   // rows past the end read the last row (never stored)
      const int64_t r = pass0 + wtot * i;
      const int64_t q = min(r * FM_ROWS + lane, a.mrows - 1);
      rows[i] = a.idx ? (uint32_t)a.idx[q] : (uint32_t)q;
      nr += r < a.nrounds ? 1 : 0;
    }
#pragma unroll
    for (int i = 0; i < FM_PARK; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) park[i][k][lane] = (float)a.c[k][rows[i]];
    for (int i = 0; i < nr; ++i) {
      const int64_t r = pass0 + wtot * i;
      float cur[D];
#pragma unroll
      for (int k = 0; k < D; ++k) cur[k] = park[i][k][lane];
      const int64_t q0 = r * FM_ROWS;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float t = (cur[k] - a.map.lo[k]) * a.map.scale[k] - 1.0f;
        // 1. the basis of this lane's row, started at 2^xs, split into FP16 terms.  The scale is
        //    set by the mode's own degree n_k - 1; a mode with n_k < NQ runs the recurrence on
        //    past n_k, where it may leave FP16 range: those values are clamped into it (their
        //    coefficients are zero)
        const int nbk = a.nb[k];
        const float at = fabsf(t);
        const float rho = fmaxf(1.0f, at + sqrtf(fmaxf(at * at - 1.0f, 0.0f)));   // 1 inside the box
        const int xs = std::max(FM_XSMIN, 14 - (int)ceilf((float)(nbk - 1) * __log2f(rho)));
        uint32_t wh[16], wl[16];
        auto basis = [&](auto full) {
          const float t2 = t + t;
          float prev = 0.0f, now = ldexpf(1.0f, xs);
          const float m1 = a.minus_one;
#pragma unroll
          for (int pr = 0; pr < 16; ++pr) {
            if (2 * pr < NQ) {
              float x[2];
#pragma unroll
              for (int i = 0; i < 2; ++i) {
                const int m = 2 * pr + i;
                // past n_k the coefficients are zero; the value only has to stay finite in FP16
                x[i] = decltype(full)::value ? now : __builtin_amdgcn_fmed3f(now, -65504.0f, 65504.0f);
                const float next = m == 0 ? t * now : fmaf(t2, now, -prev);
                prev = now;
                now = next;
              }
              // hi = x rounded to FP16, lo = x - hi (exact in FP32), then rounded to FP16
              const fm_half2 h = {(_Float16)x[0], (_Float16)x[1]};
              wh[pr] = __builtin_bit_cast(uint32_t, h);
              wl[pr] = __builtin_bit_cast(uint32_t, fm_half2{(_Float16)__builtin_fmaf((float)h[0], m1, x[0]),
                                                             (_Float16)__builtin_fmaf((float)h[1], m1, x[1])});
            } else {
              wh[pr] = 0u;
              wl[pr] = 0u;
            }
          }
        };
        if (nbk == NQ) basis(std::true_type{});
        else basis(std::false_type{});
        us[lane] = ldexpf(1.0f, -(xs + xc[k]));
        // 2. pairs -> A operands: register t of lane group g holds pairs 4 g .. 4 g + 3 of rows
        //    16 t + li
        uint32_t ah[4][4], al[4][4];
        auto transpose = [&](const uint32_t (&wd)[16], uint32_t (&o)[4][4]) {
#pragma unroll
          for (int pw = 0; pw < 4; ++pw) {
            auto p0 = __builtin_amdgcn_permlane16_swap(wd[pw], wd[4 + pw], false, false);
            auto p1 = __builtin_amdgcn_permlane16_swap(wd[8 + pw], wd[12 + pw], false, false);
            auto q0 = __builtin_amdgcn_permlane32_swap(p0[0], p1[0], false, false);
            auto q1 = __builtin_amdgcn_permlane32_swap(p0[1], p1[1], false, false);
            o[0][pw] = q0[0];
            o[2][pw] = q0[1];
            o[1][pw] = q1[0];
            o[3][pw] = q1[1];
          }
        };
        transpose(wh, ah);
        transpose(wl, al);
        // 3. MFMA: B operands of the mode's column blocks, three products per tile and block
        fm_floatx4 acc[4][JB];
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const fm_half8 bh = *reinterpret_cast<const fm_half8*>(&sB[0][k][16 * jb + li][8 * g]);
          const fm_half8 bl = *reinterpret_cast<const fm_half8*>(&sB[1][k][16 * jb + li][8 * g]);
#pragma unroll
          for (int tile = 0; tile < 4; ++tile) {
            const fm_half8 xh = __builtin_bit_cast(fm_half8, fm_uintx4{ah[tile][0], ah[tile][1], ah[tile][2], ah[tile][3]});
            const fm_half8 xl = __builtin_bit_cast(fm_half8, fm_uintx4{al[tile][0], al[tile][1], al[tile][2], al[tile][3]});
            fm_floatx4 c = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bh, fm_floatx4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bl, c, 0, 0, 0);
            acc[tile][jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl, bh, c, 0, 0, 0);
          }
        }
        // per-point unscale: rows 16 t + 4 g + v of this lane
#pragma unroll
        for (int tile = 0; tile < 4; ++tile) {
          const fm_floatx4 f = *reinterpret_cast<const fm_floatx4*>(&us[16 * tile + 4 * g]);
#pragma unroll
          for (int jb = 0; jb < JB; ++jb) acc[tile][jb] *= f;
        }
        // 4. per column block: through the LDS tile (lane (li, g) writes rows 16 t + 4 g .. + 3 of
        //    column li; lane (p, G) reads rows 4 p .. 4 p + 3 of column 4 s + G) and out, four
        //    columns per store
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
#pragma unroll
          for (int tile = 0; tile < 4; ++tile)
            *reinterpret_cast<fm_floatx4*>(&tt[li][16 * tile + 4 * g]) = acc[tile][jb];
#pragma unroll
          for (int sc = 0; sc < 4; ++sc) {
            const fm_floatx4 v = *reinterpret_cast<const fm_floatx4*>(&tt[4 * sc + g][4 * li]);
            const int j = 16 * jb + 4 * sc + g;
            const bool jv = j < a.rank[k];
            const int64_t row = q0 + 4 * li;
            const uint32_t base = (uint32_t)(((int64_t)(a.off[k] + j) * a.mrows + row) * 4);
            if (VEC) {   // mrows % 4 == 0: four consecutive rows are all inside or all past the end
              __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(fm_uintx4, v), urs,
                                                     jv && row < a.mrows ? base : kFmSkip, 0, kFmNontemporal);
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                // (the element is copied to a float first: a bit cast of a vector-element lvalue
                // compiles to a read of element 0)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, (float)v[e]), urs,
                                                      jv && row + e < a.mrows ? base + 4u * e : kFmSkip, 0,
                                                      kFmNontemporal);
            }
          }
        }
      }
    }
  }
}

bool factor_eval_mfma_applies(const fst_model* m, int64_t mrows) {
  if (m->has_wavelets() || (m->d != 3 && m->d != 4)) return false;
  int64_t sr = 0;
  for (int k = 0; k < m->d; ++k) sr += m->rank[k];
  if (sr * mrows * 4 > kFmMaxUBytes) return false;
  for (int k = 0; k < m->d; ++k)
    if (m->rank[k] > kMaxRank || m->degree[k] + 1 > kMaxBasis) return false;
  return true;
}

// a persistent grid: as many workgroups as the occupancy of the instance allows on every CU
template <typename TIn, int D, int JB, int NQ, bool VEC>
static void launch_one(const FactorMfmaArgs<TIn>& a, void* stream) {
  static std::atomic<int> occupancy(0);
  int per_cu = occupancy.load();
  if (!per_cu) {
    int nb = 0;
    check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_factor_eval_mfma<TIn, D, JB, NQ, VEC>, FM_THREADS, 0),
              "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    per_cu = nb > 0 ? nb : 1;
    occupancy.store(per_cu);
  }
  const int64_t blocks =
      std::min<int64_t>((a.nrounds + FM_WAVES - 1) / FM_WAVES, (int64_t)device_cu_count() * per_cu);
  hipLaunchKernelGGL((k_factor_eval_mfma<TIn, D, JB, NQ, VEC>), dim3((unsigned)blocks), dim3(FM_THREADS), 0, S(stream),
                     a);
}

template <typename TIn, int D, bool VEC>
static void launch_d(const FactorMfmaArgs<TIn>& a, int jb, int nq, void* stream) {
  if (jb == 1) {
    if (nq <= 16) launch_one<TIn, D, 1, 16, VEC>(a, stream);
    else launch_one<TIn, D, 1, 32, VEC>(a, stream);
  } else {
    if (nq <= 16) launch_one<TIn, D, 2, 16, VEC>(a, stream);
    else launch_one<TIn, D, 2, 32, VEC>(a, stream);
  }
}

void launch_factor_eval_mfma(const fst_model* m, const DeviceModel& dm, const void* const* coords, const void* v,
                             const int32_t* idx, int64_t mrows, void* U, void* vs, void* stream) {
  if (mrows <= 0) return;
  if (!factor_eval_mfma_applies(m, mrows)) fail(FST_E_INVAL, "factor evaluation on MFMA: unsupported model or size");
  FactorMfmaArgs<float> a;
  a.v = (const float*)v;
  a.idx = idx;
  if (!dm.cheb) fail(FST_E_UNSUPPORTED, "factor evaluation on MFMA: no Chebyshev coefficients on the device");
  a.coefs = (const float*)dm.cheb;
  a.U = (float*)U;
  a.vs = (float*)vs;
  a.mrows = mrows;
  a.nrounds = (mrows + FM_ROWS - 1) / FM_ROWS;
  a.d = m->d;
  a.ubytes = 0;
  for (int k = 0; k < m->d; ++k) a.ubytes += (int64_t)m->rank[k] * mrows * 4;
  int off = 0, rmax = 1, nbmax = 1;
  for (int k = 0; k < kMaxModes; ++k) {
    const bool live = k < m->d;
    a.c[k] = live ? (const float*)coords[k] : nullptr;
    a.rank[k] = live ? m->rank[k] : 0;
    a.nb[k] = live ? m->degree[k] + 1 : 0;
    a.off[k] = off;
    off += a.rank[k];
    rmax = std::max(rmax, a.rank[k]);
    nbmax = std::max(nbmax, a.nb[k]);
  }
  a.map = make_map<float>(m);
  a.minus_one = -1.0f;
  for (int k = 0; k < kMaxModes; ++k) a.xc[k] = dm.cheb_xc[k];
  const int jb = (rmax + 15) / 16, nq = nbmax;
  const bool vec = mrows % 4 == 0;
  if (m->d == 3) {
    if (vec) launch_d<float, 3, true>(a, jb, nq, stream);
    else launch_d<float, 3, false>(a, jb, nq, stream);
  } else {
    if (vec) launch_d<float, 4, true>(a, jb, nq, stream);
    else launch_d<float, 4, false>(a, jb, nq, stream);
  }
  check_launch("k_factor_eval_mfma");
}

}  // namespace fst
