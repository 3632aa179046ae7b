// Reconstruction of eq. (1) on MFMA (gfx950):
//
//   f(x_q) = sum_{j1, j2} u1[q, j1] u2[q, j2] T[q, (j1 j2)],   T = U3 alpha^T,
//   U3[q, j3] = u3_{j3}(x_q),  alpha^T[j3, (j1 j2)] = alpha[j1, j2, j3]
//
// Both contractions with K <= 32 run on MFMA 16x16x32 FP16 with FP32 accumulation over
// operands split in two FP16 terms each (x = hi + lo, 22 significant bits; hi*hi + hi*lo +
// lo*hi, the dropped lo*lo is below 2^-22 of the product): the factor functions of eq. (2)
// (basis against coefficients, per mode) and T (u3 against the core).  FP32 MFMA would take
// three to four times the matrix-core time and, on this chip, does not run alongside the VALU
// work of the wave, while the 16-bit MFMAs do.  The factor functions are evaluated in the
// Chebyshev basis, with the coefficients converted when the model is placed on the device
// (T_{i+1} = 2 t T_i - T_{i-1}: one VALU operation per degree; the polynomials are the same).
// Powers of two keep every term in FP16 range: the basis of a point from its growth bound
// (|T_i(t)| <= rho^i), the coefficients per mode (applied with the conversion) and the core
// per workgroup (largest entry to [2^14, 2^15)), u3 per point (its largest value likewise).
// All of them are undone at once, exactly, by one per-point exponent applied to the u1 table
// with ldexp.
//
// Each wave takes one 64-point tile per round; the LDS holds one workgroup per CU.
//   phase 1 (lane l: point l): per mode, the 32 basis values, split and transposed into the
//     A operands of the four 16-point blocks (v_permlane16_swap, v_permlane32_swap), then
//     three MFMAs per block and 16-column block of ranks.  Mode 3 first: u3 goes through a
//     per-wave LDS tile [point][j3] and comes back in the A-operand layout of phase 2 (lane
//     group g: u3[8 g .. 8 g + 7] of a point), where it is scaled and split, which completes
//     the point's exponent; then u1 (unscaled by it) and u2 go to per-wave tables [j][point],
//     each as soon as it is formed;
//   phase 2: T of the tile, 16 columns (j1 j2) per block on MFMA, then f += u1 u2 T from the
//     accumulators, with the LDS reads of the next blocks issued half a block pair ahead.
//
// LDS: coefficients as two FP16 planes [2][3][RP][40]; 16 bytes for the core's scale
// exponent; alpha as two FP16 planes [2][r1 r2 padded to 16][40] (80-byte rows: the 16-byte
// reads of 16 consecutive rows fall in distinct banks); the column table [r1 r2 padded] of
// (j1, j2) table offsets; four floats for the workgroup's maximum; per wave the point
// exponents [2][64] and a region that holds the u3 tile [64][36] and then the tables
// u1 [r1][68], u2 [r2][68].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

constexpr int EM_WAVES = 4, EM_THREADS = 64 * EM_WAVES, EM_TSTRIDE = 68, EM_APAD = 40, EM_CPAD = 40, EM_SPAD = 36;
// scale exponents: point basis in [-100, 14] (rows up to |t| of about 6 stay in range),
// coefficients in [-20, 26], core and u3 in [-60, 60]; the per-point exponent is applied with
// ldexp, so their sum needs no range of its own
constexpr int EM_XSMIN = -100, EM_XCMIN = -20, EM_XCMAX = 26, EM_XMAX = 60;
constexpr size_t EM_LDS_LIMIT = 160 * 1024;

struct EvalMfmaArgs {
  const float *x, *y, *z, *v;
  const int32_t* idx;
  const float* coefs;   // Chebyshev coefficients D 2^xc, [3][kMaxBasis][kMaxRank]
  const float* core;    // R, C order
  float* out;
  int64_t n, ntiles;
  int32_t r1, r2, r3, r12p, residual, rounds;
  int32_t nb[3];              // n_k = degree + 1
  int32_t xc[3];              // the coefficients' scale exponents
  // -1, passed at run time: the compiler then forms lo = x - hi as one mixed-precision FMA
  // (v_fma_mix, hi read as FP16) instead of a conversion back to FP32 and a subtraction
  float minus_one;
  ModeMap<float> map;
};

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef uint32_t uint32x4 __attribute__((ext_vector_type(4)));
typedef int int4v __attribute__((ext_vector_type(4)));

static inline int em_rp(int r1, int r2, int r3) { return pad8(std::max(std::max(r1, r2), r3)); }
__host__ __device__ inline size_t em_wave_bytes(int r1, int r2) {
  const size_t tables = (size_t)(r1 + r2) * EM_TSTRIDE * 4, stage = (size_t)64 * EM_SPAD * 4;
  return 512 + (tables > stage ? tables : stage);
}
static size_t em_lds_bytes(int r1, int r2, int r3) {
  const size_t r12p = ((size_t)r1 * r2 + 15) / 16 * 16, rp = (size_t)em_rp(r1, r2, r3);
  return 480 * rp + 16 + 160 * r12p + 8 * r12p + 16 + EM_WAVES * em_wave_bytes(r1, r2);
}

// hi = x rounded to FP16, lo = x - hi (exact in FP32) rounded to FP16; m1 = -1
__device__ __forceinline__ void em_split2(float x0, float x1, float m1, uint32_t& hi, uint32_t& lo) {
  const half2v h = {(_Float16)x0, (_Float16)x1};
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, half2v{(_Float16)__builtin_fmaf((float)h[0], m1, x0),
                                           (_Float16)__builtin_fmaf((float)h[1], m1, x1)});
}

// RP: ranks padded to 8 (JB = 16-column blocks of the factor products)
template <int RP>
__global__ __launch_bounds__(EM_THREADS) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_eval_mfma(
    EvalMfmaArgs a) {
  constexpr int JB = (RP + 15) / 16;
  extern __shared__ __align__(16) float em_smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  const int r1 = a.r1, r2 = a.r2, r3 = a.r3, R12 = r1 * r2, nbs = a.r12p / 16;
  char* base = reinterpret_cast<char*>(em_smem);
  _Float16* sCB = reinterpret_cast<_Float16*>(base);                       // [2][3][RP][EM_CPAD]
  int* sXa = reinterpret_cast<int*>(base + 480 * RP);                       // [4], [0]: the core's scale
  _Float16* sA16 = reinterpret_cast<_Float16*>(base + 480 * RP + 16);       // [2][r12p][EM_APAD]
  const int plane = a.r12p * EM_APAD;
  int2* sCol = reinterpret_cast<int2*>(sA16 + 2 * plane);                   // [r12p]
  float* sRed = reinterpret_cast<float*>(sCol + a.r12p);                    // [EM_WAVES]
  char* wb = reinterpret_cast<char*>(sRed + EM_WAVES) + (size_t)wave * em_wave_bytes(r1, r2);
  int* sE = reinterpret_cast<int*>(wb);          // [64] per-point exponent of the u1 table
  int* sQ = sE + 64;                              // [64] per-point scale exponent of u3
  float* sU1 = reinterpret_cast<float*>(wb + 512);   // [r1][68]
  float* sU2 = sU1 + r1 * EM_TSTRIDE;                  // [r2][68]
  float* sStage = sU1;                                  // [64][36], before the tables are written

  // ---- staging: the scale of the core (largest entry to [2^14, 2^15)); the coefficients come
  // scaled
  {
    float amax = 0.0f;
    for (int e = threadIdx.x; e < R12 * r3; e += EM_THREADS) amax = fmaxf(amax, fabsf(a.core[e]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    if (lane == 0) sRed[wave] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
      float v = 0.0f;
      for (int w = 0; w < EM_WAVES; ++w) v = fmaxf(v, sRed[w]);
      sXa[0] = std::min(EM_XMAX, std::max(-EM_XMAX, 15 - __builtin_amdgcn_frexp_expf(v)));
    }
    __syncthreads();
  }
  const int xa = sXa[0];
  int xc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) xc[k] = a.xc[k];
  const float m1 = a.minus_one;
  {
    const float sa = ldexpf(1.0f, xa);
    for (int e = threadIdx.x; e < plane; e += EM_THREADS) {
      const int c = e / EM_APAD, j3 = e - c * EM_APAD;
      const float x = (c < R12 && j3 < r3) ? a.core[(int64_t)c * r3 + j3] * sa : 0.0f;
      const _Float16 hi = (_Float16)x;
      sA16[e] = hi;
      sA16[plane + e] = (_Float16)(x - (float)hi);
    }
    for (int e = threadIdx.x; e < 3 * RP * EM_CPAD; e += EM_THREADS) {
      const int k = e / (RP * EM_CPAD), j = (e / EM_CPAD) % RP, m = e % EM_CPAD;
      const int rk = k == 0 ? r1 : (k == 1 ? r2 : r3);
      const float x = (m < a.nb[k] && j < rk) ? a.coefs[(k * kMaxBasis + m) * kMaxRank + j] : 0.0f;
      const _Float16 hi = (_Float16)x;
      sCB[e] = hi;
      sCB[3 * RP * EM_CPAD + e] = (_Float16)(x - (float)hi);
    }
    // columns past r1 r2 point at row 0 of both tables (finite values; their alpha rows are zero)
    for (int c = threadIdx.x; c < a.r12p; c += EM_THREADS)
      sCol[c] = c < R12 ? make_int2((c / r2) * EM_TSTRIDE, (c % r2) * EM_TSTRIDE) : make_int2(0, 0);
  }
  __syncthreads();

  // coordinates of the lane's point in the wave's tile of round rnd (clamped into the input)
  auto load_coords = [&](int rnd, float (&c)[3]) {
    const int64_t tile = ((int64_t)rnd * gridDim.x + blockIdx.x) * EM_WAVES + wave;
    const int64_t q = std::min<int64_t>(tile * 64 + lane, a.n - 1);
    const int64_t i = a.idx ? (int64_t)a.idx[q] : q;
    c[0] = a.x[i];
    c[1] = a.y[i];
    c[2] = a.z[i];
  };
  // 4 x 4 transpose of 16-lane blocks for each of the four pairs of a k-slot: register t of
  // lane group g then holds pairs 4 g .. 4 g + 3 of points 16 t + li
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

  // ---- phase 2 operands of the tile being contracted (point block mb; hi, lo terms)
  halfx8 ah[4], al[4];
  // phase 1 of the tile whose point coordinates the lane holds in c.  Mode 3 first: its factor
  // values go through the stage into the A operands of phase 2 and fix the point's u3 scale,
  // which completes the per-point exponent; then modes 1 and 2, each written to its table as
  // soon as it is formed (one mode's products live at a time)
  auto phase1 = [&](const float (&c)[3]) {
    float tk[3];
    int xs[3];
    int esum = xa;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      tk[k] = (c[k] - a.map.lo[k]) * a.map.scale[k] - 1.0f;
      const float at = fabsf(tk[k]);
      const float rho = fmaxf(1.0f, at + sqrtf(fmaxf(at * at - 1.0f, 0.0f)));   // 1 inside the box
      xs[k] = std::max(EM_XSMIN, 14 - (int)ceilf((float)(a.nb[k] - 1) * __log2f(rho)));
      esum += xs[k] + xc[k];
    }
    // the factor values of mode k on MFMA: lane (li, g) gets U_k[points 16 t + 4 g + v][ranks 16 jb + li]
    auto factor = [&](int k, floatx4 (&U)[4][JB]) {
      uint32_t wh[16], wl[16];
      {
        const float t2 = tk[k] + tk[k];
        float prev = 0.0f, now = ldexpf(1.0f, xs[k]);
#pragma unroll
        for (int pr = 0; pr < 16; ++pr) {
          float x[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int m = 2 * pr + i;
            // past n_k the coefficients are zero: the value only has to stay finite in FP16
            x[i] = __builtin_amdgcn_fmed3f(now, -65504.0f, 65504.0f);
            const float next = m == 0 ? tk[k] * now : fmaf(t2, now, -prev);
            prev = now;
            now = next;
          }
          em_split2(x[0], x[1], m1, wh[pr], wl[pr]);
        }
      }
      uint32_t th[4][4], tl[4][4];
      transpose(wh, th);
      transpose(wl, tl);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int row = std::min(16 * jb + li, RP - 1);   // columns past RP are never used
        const _Float16* bp = sCB + ((size_t)k * RP + row) * EM_CPAD + 8 * g;
        const halfx8 bh = *reinterpret_cast<const halfx8*>(bp);
        const halfx8 bl = *reinterpret_cast<const halfx8*>(bp + 3 * RP * EM_CPAD);
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
          const halfx8 xh = __builtin_bit_cast(halfx8, uint32x4{th[t4][0], th[t4][1], th[t4][2], th[t4][3]});
          const halfx8 xl = __builtin_bit_cast(halfx8, uint32x4{tl[t4][0], tl[t4][1], tl[t4][2], tl[t4][3]});
          floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bh, floatx4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bl, acc, 0, 0, 0);
          U[t4][jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl, bh, acc, 0, 0, 0);
        }
      }
    };
    {
      floatx4 U[4][JB];
      factor(2, U);
      __builtin_amdgcn_s_waitcnt(0xC07F);   // earlier reads of the wave's region done (lgkmcnt(0))
      // u3 to the stage [point][j3] (zeros from RP on), back as the A operands of phase 2
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            sStage[(16 * t4 + 4 * g + v) * EM_SPAD + 16 * jb + li] = 16 * jb + li < RP ? U[t4][jb][v] : 0.0f;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const float* sp = sStage + (16 * mb + li) * EM_SPAD + 8 * g;
      floatx4 p0 = *reinterpret_cast<const floatx4*>(sp), p1 = *reinterpret_cast<const floatx4*>(sp + 4);
      if (8 * g >= 16 * JB) {   // k-slots past the ranks of the factor products
        p0 = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        p1 = p0;
      }
      float mq = 0.0f;
#pragma unroll
      for (int e = 0; e < 4; ++e) mq = fmaxf(mq, fmaxf(fabsf(p0[e]), fabsf(p1[e])));
      mq = fmaxf(mq, __shfl_xor(mq, 16, 64));
      mq = fmaxf(mq, __shfl_xor(mq, 32, 64));
      const int xq = std::min(EM_XMAX, std::max(-EM_XMAX, 15 - __builtin_amdgcn_frexp_expf(mq)));
      const float sq = ldexpf(1.0f, xq);
      uint32_t hw[4], lw[4];
      em_split2(p0[0] * sq, p0[1] * sq, m1, hw[0], lw[0]);
      em_split2(p0[2] * sq, p0[3] * sq, m1, hw[1], lw[1]);
      em_split2(p1[0] * sq, p1[1] * sq, m1, hw[2], lw[2]);
      em_split2(p1[2] * sq, p1[3] * sq, m1, hw[3], lw[3]);
      ah[mb] = __builtin_bit_cast(halfx8, uint32x4{hw[0], hw[1], hw[2], hw[3]});
      al[mb] = __builtin_bit_cast(halfx8, uint32x4{lw[0], lw[1], lw[2], lw[3]});
      if (g == 0) sQ[16 * mb + li] = xq;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    sE[lane] = esum + sQ[lane];   // every scale of this point, undone on its u1 values
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    // u1 (scaled back by the point exponents), then u2, to the tables over the stage
    {
      floatx4 U[4][JB];
      factor(0, U);
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4) {
        const int4v E = *reinterpret_cast<const int4v*>(&sE[16 * t4 + 4 * g]);
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int col = 16 * jb + li;
          if (col < r1)
            *reinterpret_cast<floatx4*>(&sU1[col * EM_TSTRIDE + 16 * t4 + 4 * g]) =
                floatx4{ldexpf(U[t4][jb][0], -E[0]), ldexpf(U[t4][jb][1], -E[1]), ldexpf(U[t4][jb][2], -E[2]),
                        ldexpf(U[t4][jb][3], -E[3])};
        }
      }
    }
    {
      floatx4 U[4][JB];
      factor(1, U);
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int col = 16 * jb + li;
          if (col < r2) *reinterpret_cast<floatx4*>(&sU2[col * EM_TSTRIDE + 16 * t4 + 4 * g]) = U[t4][jb];
        }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);   // the tables written before they are read
    __builtin_amdgcn_wave_barrier();
  };

  // ---- phase 2: LDS reads of column block nb (clamped into the blocks): B operands (k-slot g
  // of column 16 nb + li, both terms), the column's rows of the u1 and u2 tables, and the
  // products u1 u2 of the lane's 16 points
  auto loadb = [&](int nb, halfx8 (&b)[2]) {
    const _Float16* bp = sA16 + (std::min(nb, nbs - 1) * 16 + li) * EM_APAD + 8 * g;
    b[0] = *reinterpret_cast<const halfx8*>(bp);
    b[1] = *reinterpret_cast<const halfx8*>(bp + plane);
  };
  auto loadcol = [&](int nb) { return sCol[std::min(nb, nbs - 1) * 16 + li]; };
  auto loadx = [&](int2 off, floatx4 (&x1)[4], floatx4 (&x2)[4]) {
    const float* w1 = sU1 + off.x + 4 * g;
    const float* w2 = sU2 + off.y + 4 * g;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      x1[mb] = *reinterpret_cast<const floatx4*>(w1 + 16 * mb);
      x2[mb] = *reinterpret_cast<const floatx4*>(w2 + 16 * mb);
    }
  };
  auto product = [&](const floatx4 (&x1)[4], const floatx4 (&x2)[4], floatx4 (&w)[4]) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) w[mb] = x1[mb] * x2[mb];
  };
  auto mfma = [&](const halfx8 (&b)[2], floatx4 (&acc)[4]) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[mb], b[0], floatx4{0, 0, 0, 0}, 0, 0, 0);
      acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[mb], b[1], acc[mb], 0, 0, 0);
      acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[mb], b[0], acc[mb], 0, 0, 0);
    }
  };
  float f[4][4];
  auto reduce = [&](const floatx4 (&acc)[4], const floatx4 (&w)[4]) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) f[mb][v] = fmaf(w[mb][v], acc[mb][v], f[mb][v]);
  };

  float cn[3];
  load_coords(0, cn);
  const int nit = (nbs - 1) / 2;
  for (int rnd = 0; rnd < a.rounds; ++rnd) {
    phase1(cn);
    load_coords(rnd + 1, cn);   // the next tile's coordinates, used by the next round
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) f[mb][v] = 0.0f;
    // pipeline state at the top of an iteration (nb even): accA = block nb issued, wA its
    // products; bB and colB of block nb + 1 read
    floatx4 accA[4], accB[4], x1[4], x2[4], wA[4], wB[4];
    halfx8 bA[2], bB[2];
    int2 colA = loadcol(0), colB;
    loadb(0, bA);
    loadx(colA, x1, x2);
    product(x1, x2, wA);
    colB = loadcol(1);
    loadb(1, bB);
    mfma(bA, accA);
    int nb = 0;
    for (int it = 0; it < nit; ++it) {
      // block nb + 1 into accB; reads for blocks nb + 1 (u1 u2) and nb + 2 (B, column)
      loadx(colB, x1, x2);
      loadb(nb + 2, bA);
      colA = loadcol(nb + 2);
      mfma(bB, accB);
      reduce(accA, wA);
      product(x1, x2, wB);
      // block nb + 2 into accA; reads for blocks nb + 2 (u1 u2) and nb + 3 (B, column)
      loadx(colA, x1, x2);
      loadb(nb + 3, bB);
      colB = loadcol(nb + 3);
      mfma(bA, accA);
      reduce(accB, wB);
      product(x1, x2, wA);
      nb += 2;
    }
    if (nb + 1 < nbs) {   // one block left over
      loadx(colB, x1, x2);
      product(x1, x2, wB);
      mfma(bB, accB);
      reduce(accA, wA);
      reduce(accB, wB);
    } else {
      reduce(accA, wA);
    }
    // the 16 lanes of a lane group hold partial sums of the same points over different columns
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s = f[mb][v];
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 8, 64);
        f[mb][v] = s;
      }
    // lanes li < 4 of lane group g store points 16 mb + 4 g + li: 16 consecutive points per mb
    const int64_t tile = ((int64_t)rnd * gridDim.x + blockIdx.x) * EM_WAVES + wave;
    if (li < 4) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const float val = li == 0 ? f[mb][0] : (li == 1 ? f[mb][1] : (li == 2 ? f[mb][2] : f[mb][3]));
        const int64_t q = tile * 64 + 16 * mb + 4 * g + li;
        if (q < a.n) {
          if (a.residual) {
            const int64_t i = a.idx ? (int64_t)a.idx[q] : q;
            a.out[q] = a.v[i] - val;
          } else {
            a.out[q] = val;
          }
        }
      }
    }
  }
}

bool eval_mfma_applies(const fst_model* m) {
  if (m->d != 3 || m->has_wavelets()) return false;
  for (int k = 0; k < 3; ++k)
    if (m->rank[k] > kMaxRank || m->degree[k] + 1 > kMaxBasis) return false;
  return em_lds_bytes(m->rank[0], m->rank[1], m->rank[2]) <= EM_LDS_LIMIT;
}

template <int RP>
static void em_launch(const EvalMfmaArgs& a, size_t lds, int blocks, void* stream) {
  hipLaunchKernelGGL((k_eval_mfma<RP>), dim3((unsigned)blocks), dim3(EM_THREADS), lds, S(stream), a);
  check_launch("k_eval_mfma");
}

void launch_eval_mfma(const fst_model* m, const DeviceModel& dm, int64_t n, const float* x, const float* y,
                      const float* z, const int32_t* idx, const float* v, float* out, bool residual, void* stream) {
  if (!eval_mfma_applies(m)) fail(FST_E_UNSUPPORTED, "MFMA reconstruction: model shape not supported");
  if (n <= 0) return;
  EvalMfmaArgs a;
  a.x = x;
  a.y = y;
  a.z = z;
  a.v = v;
  a.idx = idx;
  if (!dm.cheb) fail(FST_E_UNSUPPORTED, "MFMA reconstruction: no Chebyshev coefficients on the device");
  a.coefs = (const float*)dm.cheb;
  a.core = (const float*)dm.core;
  a.out = out;
  a.n = n;
  a.ntiles = (n + 63) / 64;
  a.r1 = m->rank[0];
  a.r2 = m->rank[1];
  a.r3 = m->rank[2];
  a.r12p = (a.r1 * a.r2 + 15) / 16 * 16;
  a.residual = residual ? 1 : 0;
  a.map = make_map<float>(m);
  for (int k = 0; k < 3; ++k) a.nb[k] = m->degree[k] + 1;
  for (int k = 0; k < 3; ++k) a.xc[k] = dm.cheb_xc[k];
  a.minus_one = -1.0f;
  const size_t lds = em_lds_bytes(a.r1, a.r2, a.r3);
  const int64_t per_block = EM_WAVES;
  const int blocks = (int)std::min<int64_t>((a.ntiles + per_block - 1) / per_block, (int64_t)device_cu_count());
  a.rounds = (int)((a.ntiles + (int64_t)blocks * per_block - 1) / ((int64_t)blocks * per_block));
  switch (em_rp(a.r1, a.r2, a.r3)) {
    case 8: em_launch<8>(a, lds, blocks, stream); break;
    case 16: em_launch<16>(a, lds, blocks, stream); break;
    case 24: em_launch<24>(a, lds, blocks, stream); break;
    default: em_launch<32>(a, lds, blocks, stream); break;
  }
}

}  // namespace fst
