// Reconstruction of eq. (1) with the core contraction on FP32 MFMA (gfx950):
//
//   f(x_q) = sum_{j1, j2} u1[q, j1] u2[q, j2] T[q, (j1 j2)],   T = U3 alpha^T,
//   U3[q, j3] = u3_{j3}(x_q),  alpha^T[j3, (j1 j2)] = alpha[j1, j2, j3]
//
// For a tile of 64 points, T (64 x r1 r2) is a GEMM with K = r3 <= 32: 2 R flop per point, the
// bulk of the work, on MFMA 16x16x32 FP16 with FP32 accumulation over operands split in two
// FP16 terms each (x = hi + lo, 22 significant bits): hi*hi + hi*lo + lo*hi per product (the
// dropped lo*lo is below 2^-22 of it), so T is as accurate as an FP32 product while taking a
// third of the matrix-core time of FP32 MFMA 16x16x4, and (unlike FP32 MFMA on this chip) the
// 16-bit MFMAs run alongside the wave's VALU work.  Scaling by powers of two keeps the terms in
// FP16 range: alpha by one factor per workgroup (its largest entry to [2^14, 2^15)), u3 by one
// factor per point (its largest value likewise); both are undone in the u1 table, exactly.
// The weighted reduction over (j1, j2), 3 r1 r2 flop per point, runs on the VALU from the MFMA
// accumulators.
//
// Each wave takes one 64-point tile per round; lane l evaluates point l of a tile.
//   phase 1 (VALU): the factor functions of eq. (2) at the lane's point, the three modes advanced
//     together one degree per step by the monic Legendre recurrence p_{m+1} = t p_m - beta_m
//     p_{m-1} (the normalisation c_m of phi_m = c_m p_m is folded into the staged coefficients,
//     which every lane reads from LDS at the same address);
//   phase 2 (MFMA): T of the tile, 16 columns (j1 j2) per block, then f += u1 u2 T.
// The LDS holds one workgroup per CU, so a SIMD runs one wave; the two phases overlap inside
// the wave instead: the loop over T's column blocks carries the degree steps of the NEXT
// tile's phase 1 (SPH degree steps per block), so the VALU works while the matrix core runs.
// U3 reaches the MFMA A operand without LDS: lane l holds the 16 FP16 pairs of u3 (each term)
// of point l; for each of the four pairs of a lane group's k-slot, a 4 x 4 transpose of
// 16-lane blocks (v_permlane16_swap, v_permlane32_swap) hands lane group g of point block mb
// the pairs 4 g .. 4 g + 3 of the points 16 mb + li, i.e. u3[8 g .. 8 g + 7], which is the
// k-slot g of the A operand; B takes alpha[column][8 g .. 8 g + 7] in the same slot.  u1 and u2
// go to per-wave LDS tables (points contiguous, float4 reads), and a per-column table gives
// each column's rows of them.
//
// LDS: coefficients [3][kMaxBasis][kMaxRank] (scaled by c_m); beta [kMaxBasis]; alpha as two
// FP16 planes [2][r1 r2 padded to 16][40] with j3 fastest (80-byte rows: the 16-byte reads of
// 16 consecutive rows fall in distinct banks); the column table [r1 r2 padded]; four floats for
// the workgroup's maximum; per wave u1 [r1][68] and u2 [r2][68].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

constexpr int EM_WAVES = 4, EM_THREADS = 64 * EM_WAVES, EM_TSTRIDE = 68, EM_APAD = 40;
// power-of-two scale exponents are kept within +-60, so the unscale 2^-(xa + xq) is a normal float
constexpr int EM_XMAX = 60;
constexpr size_t EM_LDS_LIMIT = 160 * 1024;

struct EvalMfmaArgs {
  const float *x, *y, *z, *v;
  const int32_t* idx;
  const float* coefs;   // [3][kMaxBasis][kMaxRank]
  const float* core;    // R, C order
  float* out;
  int64_t n, ntiles;
  int32_t r1, r2, r3, r12p, residual, rounds, nst;
  ModeMap<float> map;
  float beta[kMaxBasis];     // beta_m of the monic recurrence (beta_0 = 0)
  double cscale[kMaxBasis];  // c_m
};

constexpr int EM_CSIZE = 3 * kMaxBasis * kMaxRank;
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef uint32_t uint32x4 __attribute__((ext_vector_type(4)));   // coefficient matrices, staged once per workgroup

static size_t em_lds_bytes(int r1, int r2) {
  const size_t r12p = ((size_t)r1 * r2 + 15) / 16 * 16;
  return sizeof(float) * (EM_CSIZE + kMaxBasis + EM_WAVES + (size_t)EM_WAVES * (r1 + r2) * EM_TSTRIDE) +
         2 * sizeof(_Float16) * r12p * EM_APAD + 8 * r12p;
}

// RP: ranks padded to 8 (the factor values held per mode); SPH: degree steps of the next
// tile per column block.
template <int RP, int SPH>
__global__ __launch_bounds__(EM_THREADS) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_eval_mfma(
    EvalMfmaArgs a) {
  constexpr int NW = RP / 2;   // FP16 pairs of u3 per point and term
  extern __shared__ __align__(16) float em_smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  const int r1 = a.r1, r2 = a.r2, r3 = a.r3, R12 = r1 * r2, nbs = a.r12p / 16, nst = a.nst;
  const int plane = a.r12p * EM_APAD;
  float* sC = em_smem;                                                  // [3][kMaxBasis][kMaxRank]
  float* sBeta = sC + EM_CSIZE;                                         // [kMaxBasis]
  _Float16* sA16 = reinterpret_cast<_Float16*>(sBeta + kMaxBasis);      // [2][r12p][EM_APAD]
  int2* sCol = reinterpret_cast<int2*>(sA16 + 2 * plane);               // [r12p]
  float* sRed = reinterpret_cast<float*>(sCol + a.r12p);                // [EM_WAVES]
  float* sU1 = sRed + EM_WAVES + (size_t)wave * (r1 + r2) * EM_TSTRIDE;  // [r1][68]
  float* sU2 = sU1 + r1 * EM_TSTRIDE;                                   // [r2][68]
  // the scale of alpha: its largest magnitude to [2^14, 2^15)
  float amax = 0.0f;
  for (int e = threadIdx.x; e < R12 * r3; e += EM_THREADS) amax = fmaxf(amax, fabsf(a.core[e]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) sRed[wave] = amax;
  __syncthreads();
  amax = fmaxf(fmaxf(sRed[0], sRed[1]), fmaxf(sRed[2], sRed[3]));
  const int xa = std::min(EM_XMAX, std::max(-EM_XMAX, 15 - __builtin_amdgcn_frexp_expf(amax)));
  const float sa = ldexpf(1.0f, xa);
  for (int e = threadIdx.x; e < plane; e += EM_THREADS) {
    const int c = e / EM_APAD, j3 = e - c * EM_APAD;
    const float x = (c < R12 && j3 < r3) ? a.core[(int64_t)c * r3 + j3] * sa : 0.0f;
    const _Float16 hi = (_Float16)x;
    sA16[e] = hi;
    sA16[plane + e] = (_Float16)(x - (float)hi);
  }
  for (int e = threadIdx.x; e < EM_CSIZE; e += EM_THREADS)
    sC[e] = (float)(a.cscale[(e / kMaxRank) % kMaxBasis] * (double)a.coefs[e]);
  if (threadIdx.x < kMaxBasis) sBeta[threadIdx.x] = a.beta[threadIdx.x];
  // columns past r1 r2 point at row 0 of both tables (finite values; their alpha rows are zero)
  for (int c = threadIdx.x; c < a.r12p; c += EM_THREADS)
    sCol[c] = c < R12 ? make_int2((c / r2) * EM_TSTRIDE, (c % r2) * EM_TSTRIDE) : make_int2(0, 0);
  __syncthreads();

  // ---- phase 1 state: the lane's point of the tile being evaluated
  float tt[3], pm[3], pm1[3], u[3][RP];
  auto start = [&](const float (&c)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      tt[k] = (c[k] - a.map.lo[k]) * a.map.scale[k] - 1.0f;
      pm[k] = 1.0f;
      pm1[k] = 0.0f;
#pragma unroll
      for (int j = 0; j < RP; ++j) u[k][j] = 0.0f;
    }
  };
  // degree m of all three modes: the coefficient rows (and beta_m) are read first, then used
  typedef floatx4 CoefRows[3][RP / 4];
  auto loadc = [&](int m, CoefRows& c, float& bm) {
    const float* cm = sC + m * kMaxRank;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < RP / 4; ++q) c[k][q] = *reinterpret_cast<const floatx4*>(cm + k * kMaxBasis * kMaxRank + 4 * q);
    bm = sBeta[m];
  };
  auto stepc = [&](const CoefRows& c, float bm) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < RP; ++j) u[k][j] = fmaf(c[k][j / 4][j % 4], pm[k], u[k][j]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float pn = fmaf(tt[k], pm[k], -bm * pm1[k]);
      pm1[k] = pm[k];
      pm[k] = pn;
    }
  };
  CoefRows cr;
  float crb;
  auto step = [&](int m) {
    loadc(m, cr, crb);
    stepc(cr, crb);
  };
  // coordinates of the lane's point in the wave's tile of round rnd (clamped into the input)
  auto load_coords = [&](int rnd, float (&c)[3]) {
    const int64_t tile = ((int64_t)rnd * gridDim.x + blockIdx.x) * EM_WAVES + wave;
    const int64_t q = std::min<int64_t>(tile * 64 + lane, a.n - 1);
    const int64_t i = a.idx ? (int64_t)a.idx[q] : q;
    c[0] = a.x[i];
    c[1] = a.y[i];
    c[2] = a.z[i];
  };
  // ---- phase 2 state: A operands of the tile being contracted (point block mb; hi, lo terms)
  halfx8 ah[4], al[4];
  // end of a tile's phase 1: u1 (with the unscale of both factors) and u2 to the wave's tables;
  // u3 scaled, split in two FP16 terms and transposed into the A operands
  auto finish = [&]() {
    float mq = 0.0f;
#pragma unroll
    for (int j = 0; j < RP; ++j) mq = fmaxf(mq, fabsf(u[2][j]));
    const int xq = std::min(EM_XMAX, std::max(-EM_XMAX, 15 - __builtin_amdgcn_frexp_expf(mq)));
    const float sq = ldexpf(1.0f, xq), unscale = ldexpf(1.0f, -(xa + xq));
    __builtin_amdgcn_s_waitcnt(0xC07F);   // earlier reads of the tables done (lgkmcnt(0))
#pragma unroll
    for (int j = 0; j < RP; ++j) {
      if (j < r1) sU1[j * EM_TSTRIDE + lane] = u[0][j] * unscale;
      if (j < r2) sU2[j * EM_TSTRIDE + lane] = u[1][j];
    }
    uint32_t wh[16], wl[16];   // FP16 pairs (2 w, 2 w + 1) of each term; zero past RP
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      if (w < NW) {
        const float x0 = u[2][2 * w] * sq, x1 = u[2][2 * w + 1] * sq;
        const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
        const _Float16 l0 = (_Float16)(x0 - (float)h0), l1 = (_Float16)(x1 - (float)h1);
        wh[w] = __builtin_bit_cast(uint32_t, half2v{h0, h1});
        wl[w] = __builtin_bit_cast(uint32_t, half2v{l0, l1});
      } else {
        wh[w] = 0u;
        wl[w] = 0u;
      }
    }
    uint32x4 th[4], tl[4];   // [point block mb] words 0..3 of the k-slot of this lane group
    auto transpose = [&](const uint32_t (&wd)[16], uint32x4 (&t)[4]) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        // lane group mb holds pair 4 g' + w of its points in register g'; afterwards lane group g
        // holds pair 4 g + w of the points of block mb in register mb
        auto p0 = __builtin_amdgcn_permlane16_swap(wd[w], wd[4 + w], false, false);
        auto p1 = __builtin_amdgcn_permlane16_swap(wd[8 + w], wd[12 + w], false, false);
        auto q0 = __builtin_amdgcn_permlane32_swap(p0[0], p1[0], false, false);
        auto q1 = __builtin_amdgcn_permlane32_swap(p0[1], p1[1], false, false);
        t[0][w] = q0[0];
        t[2][w] = q0[1];
        t[1][w] = q1[0];
        t[3][w] = q1[1];
      }
    };
    transpose(wh, th);
    transpose(wl, tl);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      ah[mb] = __builtin_bit_cast(halfx8, th[mb]);
      al[mb] = __builtin_bit_cast(halfx8, tl[mb]);
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);   // the tables written before they are read
    __builtin_amdgcn_wave_barrier();
  };
  // LDS reads of column block nb (clamped into the blocks): B operands (k-slot g of column
  // 16 nb + li, both terms), the column's rows of the u1 and u2 tables, and the products u1 u2
  // of the lane's 16 points
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
  // one half-iteration as the scheduler should order it: its LDS reads first, then each MFMA
  // followed by a share of the VALU work (hints only: no effect on the results)
  auto schedule = [&]() {
    __builtin_amdgcn_sched_group_barrier(0x100, 40, 0);   // LDS reads
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);  // VALU
    }
  };

  // prologue: phase 1 of the wave's first tile on its own
  float cn[3];
  load_coords(0, cn);
  start(cn);
  for (int m = 0; m < nst; ++m) step(m);
  finish();
  load_coords(1, cn);
  // the column blocks go in pairs; the first npair_s pairs carry 2 SPH degree steps of the
  // next tile, the steps left over run after the blocks
  const int nit = (nbs - 1) / 2, nit_s = std::min(nit, nst / (2 * SPH));
  for (int rnd = 0; rnd < a.rounds; ++rnd) {
    start(cn);                  // phase 1 of the next tile
    load_coords(rnd + 2, cn);   // coordinates of the tile after it
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
    int nb = 0, m = 0;
    auto iteration = [&](auto with_steps) {
      // block nb + 1 into accB; reads for blocks nb + 1 (u1 u2) and nb + 2 (B, column)
      loadx(colB, x1, x2);
      loadb(nb + 2, bA);
      colA = loadcol(nb + 2);
      if (decltype(with_steps)::value) loadc(m, cr, crb);
      mfma(bB, accB);
      reduce(accA, wA);
      if (decltype(with_steps)::value) {
        stepc(cr, crb);
#pragma unroll
        for (int s = 1; s < SPH; ++s) step(m + s);
      }
      product(x1, x2, wB);
      schedule();
      __builtin_amdgcn_sched_barrier(0);
      // block nb + 2 into accA; reads for blocks nb + 2 (u1 u2) and nb + 3 (B, column)
      loadx(colA, x1, x2);
      loadb(nb + 3, bB);
      colB = loadcol(nb + 3);
      if (decltype(with_steps)::value) loadc(m + SPH, cr, crb);
      mfma(bA, accA);
      reduce(accB, wB);
      if (decltype(with_steps)::value) {
        stepc(cr, crb);
#pragma unroll
        for (int s = 1; s < SPH; ++s) step(m + SPH + s);
      }
      product(x1, x2, wA);
      schedule();
      __builtin_amdgcn_sched_barrier(0);
      nb += 2;
      if (decltype(with_steps)::value) m += 2 * SPH;
    };
    int it = 0;
    for (; it < nit_s; ++it) iteration(std::true_type{});
    for (; it < nit; ++it) iteration(std::false_type{});
    if (nb + 1 < nbs) {   // one block left over
      loadx(colB, x1, x2);
      product(x1, x2, wB);
      mfma(bB, accB);
      reduce(accA, wA);
      reduce(accB, wB);
    } else {
      reduce(accA, wA);
    }
    for (; m < nst; ++m) step(m);   // degree steps left over
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
    finish();   // the next tile's tables and A operands
  }
}

bool eval_mfma_applies(const fst_model* m) {
  if (m->d != 3 || m->has_wavelets()) return false;
  for (int k = 0; k < 3; ++k)
    if (m->rank[k] > kMaxRank || m->degree[k] + 1 > kMaxBasis) return false;
  return em_lds_bytes(m->rank[0], m->rank[1]) <= EM_LDS_LIMIT;
}

template <int RP, int SPH>
static void em_launch(const EvalMfmaArgs& a, size_t lds, int blocks, void* stream) {
  hipLaunchKernelGGL((k_eval_mfma<RP, SPH>), dim3((unsigned)blocks), dim3(EM_THREADS), lds, S(stream), a);
  check_launch("k_eval_mfma");
}
template <int RP>
static void em_launch_sb(const EvalMfmaArgs& a, int sb, size_t lds, int blocks, void* stream) {
  if (RP == 32 || sb == 1) em_launch<RP, 1>(a, lds, blocks, stream);
  else if (sb == 2) em_launch<RP, 2>(a, lds, blocks, stream);
  else em_launch<RP, 4>(a, lds, blocks, stream);
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
  a.coefs = (const float*)dm.coefs;
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
  a.nst = 1;
  for (int k = 0; k < 3; ++k) a.nst = std::max(a.nst, m->degree[k] + 1);
  // monic Legendre recurrence: phi_{m+1} = A_m t phi_m - B_m phi_{m-1} with phi_m = c_m p_m,
  // c_0 = 1, c_{m+1} = A_m c_m gives p_{m+1} = t p_m - beta_m p_{m-1}, beta_m = B_m / (A_m A_{m-1})
  {
    auto A = [](int k) { return std::sqrt((2.0 * k + 1.0) * (2.0 * k + 3.0)) / (k + 1.0); };
    auto B = [](int k) { return k == 0 ? 0.0 : k * std::sqrt(2.0 * k + 3.0) / ((k + 1.0) * std::sqrt(2.0 * k - 1.0)); };
    double c = 1.0;
    for (int k = 0; k < kMaxBasis; ++k) {
      a.cscale[k] = c;
      a.beta[k] = k == 0 ? 0.0f : (float)(B(k) / (A(k) * A(k - 1)));
      c *= A(k);
    }
  }
  const size_t lds = em_lds_bytes(a.r1, a.r2);
  const int64_t per_block = EM_WAVES;
  const int blocks = (int)std::min<int64_t>((a.ntiles + per_block - 1) / per_block, (int64_t)device_cu_count());
  a.rounds = (int)((a.ntiles + (int64_t)blocks * per_block - 1) / ((int64_t)blocks * per_block));
  // degree steps per column block (pairs of blocks after the first carry them): 1, 2 or 4,
  // the nearest to steps / blocks
  const int carriers = std::max(1, (a.r12p / 16 - 1) / 2 * 2);
  const double ratio = (double)a.nst / carriers;
  const int rp = pad8(std::max(std::max(a.r1, a.r2), a.r3));
  // (at RP = 32 more steps per block do not fit the registers)
  const int sb = rp == 32 || ratio < 1.5 ? 1 : (ratio < 3.0 ? 2 : 4);
  switch (rp) {
    case 8: em_launch_sb<8>(a, sb, lds, blocks, stream); break;
    case 16: em_launch_sb<16>(a, sb, lds, blocks, stream); break;
    case 24: em_launch_sb<24>(a, sb, lds, blocks, stream); break;
    default: em_launch_sb<32>(a, sb, lds, blocks, stream); break;
  }
}

}  // namespace fst
