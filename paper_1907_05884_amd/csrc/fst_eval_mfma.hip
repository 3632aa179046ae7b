// Reconstruction of eq. (1) with the core contraction on FP32 MFMA (gfx950):
//
//   f(x_q) = sum_{j1, j2} u1[q, j1] u2[q, j2] T[q, (j1 j2)],   T = U3 alpha^T,
//   U3[q, j3] = u3_{j3}(x_q),  alpha^T[j3, (j1 j2)] = alpha[j1, j2, j3]
//
// For a tile of 64 points, T (64 x r1 r2) is a GEMM with K = r3 on MFMA 16x16x4 (FP32 in,
// FP32 accumulation): 2 R flop per point, the bulk of the work.  The weighted reduction over
// (j1, j2), 3 r1 r2 flop per point, runs on the VALU from the MFMA accumulators.
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
// U3 reaches the MFMA A operand without LDS: a 4 x 4 transpose of 16-lane blocks
// (v_permlane16_swap, v_permlane32_swap) turns lane l's u3[4s .. 4s+3] into the operands of
// the four 16-point blocks.  u1 and u2 go to per-wave LDS tables (points contiguous, float4
// reads), and a per-column table gives each column's rows of them.
//
// LDS: coefficients [3][kMaxBasis][kMaxRank] (scaled by c_m); alpha [r1 r2 padded to 16][r3s]
// with j3 fastest (r3s = r3 rounded up to 4 and to 2 mod 4, so 16 consecutive rows read at
// one column fall in distinct bank pairs); the column table [r1 r2 padded]; per wave
// u1 [r1][68] and u2 [r2][68].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

constexpr int EM_WAVES = 4, EM_THREADS = 64 * EM_WAVES, EM_TSTRIDE = 68;
constexpr size_t EM_LDS_LIMIT = 160 * 1024;

struct EvalMfmaArgs {
  const float *x, *y, *z, *v;
  const int32_t* idx;
  const float* coefs;   // [3][kMaxBasis][kMaxRank]
  const float* core;    // R, C order
  float* out;
  int64_t n, ntiles;
  int32_t r1, r2, r3, r3s, r12p, residual, rounds, nst;
  ModeMap<float> map;
  float beta[kMaxBasis];     // beta_m of the monic recurrence (beta_0 = 0)
  double cscale[kMaxBasis];  // c_m
};

static inline int em_r3s(int r3) {
  int s = (r3 + 3) / 4 * 4;
  return s % 4 == 2 ? s : s + 2;
}

constexpr int EM_CSIZE = 3 * kMaxBasis * kMaxRank;   // coefficient matrices, staged once per workgroup

static size_t em_lds_bytes(int r1, int r2, int r3) {
  const size_t r3s = (size_t)em_r3s(r3), r12p = ((size_t)r1 * r2 + 15) / 16 * 16;
  return sizeof(float) * (EM_CSIZE + kMaxBasis + r12p * r3s + (size_t)EM_WAVES * (r1 + r2) * EM_TSTRIDE) + 8 * r12p;
}

// RP: ranks padded to 8 (KS = RP / 4 MFMA k-steps and the factor values held per mode);
// SPH: degree steps of the next tile per column block.
template <int RP, int SPH>
__global__ __launch_bounds__(EM_THREADS) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_eval_mfma(
    EvalMfmaArgs a) {
  constexpr int KS = RP / 4;
  extern __shared__ __align__(16) float em_smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  const int r1 = a.r1, r2 = a.r2, r3 = a.r3, r3s = a.r3s, R12 = r1 * r2, nbs = a.r12p / 16, nst = a.nst;
  float* sC = em_smem;                                           // [3][kMaxBasis][kMaxRank]
  float* sBeta = sC + EM_CSIZE;                                  // [kMaxBasis]
  float* sAlpha = sBeta + kMaxBasis;                             // [r12p][r3s]
  int2* sCol = reinterpret_cast<int2*>(sAlpha + (size_t)a.r12p * r3s);   // [r12p]
  float* sU1 = reinterpret_cast<float*>(sCol + a.r12p) + (size_t)wave * (r1 + r2) * EM_TSTRIDE;   // [r1][68]
  float* sU2 = sU1 + r1 * EM_TSTRIDE;                                                              // [r2][68]
  for (int e = threadIdx.x; e < a.r12p * r3s; e += EM_THREADS) {
    const int c = e / r3s, j3 = e - c * r3s;
    sAlpha[e] = (c < R12 && j3 < r3) ? a.core[(int64_t)c * r3 + j3] : 0.0f;
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
  // ---- phase 2 state: A operands of the tile being contracted, the f partials
  float av[4][KS];
  // end of a tile's phase 1: u1, u2 to the wave's tables, u3 transposed into the A operands
  // (lane group mb of register i holds u3[4 s + i] of points 16 mb + li; afterwards register mb of
  // lane group i holds it, as the A operand of point block mb wants)
  auto finish = [&]() {
    __builtin_amdgcn_s_waitcnt(0xC07F);   // earlier reads of the tables done (lgkmcnt(0))
#pragma unroll
    for (int j = 0; j < RP; ++j) {
      if (j < r1) sU1[j * EM_TSTRIDE + lane] = u[0][j];
      if (j < r2) sU2[j * EM_TSTRIDE + lane] = u[1][j];
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      uint32_t x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = __builtin_bit_cast(uint32_t, u[2][4 * s + i]);
      auto p0 = __builtin_amdgcn_permlane16_swap(x[0], x[1], false, false);
      auto p1 = __builtin_amdgcn_permlane16_swap(x[2], x[3], false, false);
      auto q0 = __builtin_amdgcn_permlane32_swap(p0[0], p1[0], false, false);
      auto q1 = __builtin_amdgcn_permlane32_swap(p0[1], p1[1], false, false);
      av[0][s] = __builtin_bit_cast(float, (uint32_t)q0[0]);
      av[2][s] = __builtin_bit_cast(float, (uint32_t)q0[1]);
      av[1][s] = __builtin_bit_cast(float, (uint32_t)q1[0]);
      av[3][s] = __builtin_bit_cast(float, (uint32_t)q1[1]);
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);   // the tables written before they are read
    __builtin_amdgcn_wave_barrier();
  };
  const int ks3 = (r3 + 3) / 4 - 1;   // last k-step with alpha columns (av is zero past r3)
  // LDS reads of column block nb (clamped into the blocks): B operands, the column's rows of
  // the u1 and u2 tables, and the products u1 u2 of the lane's 16 points
  auto loadb = [&](int nb, float (&b)[KS]) {
    const float* bp = sAlpha + (std::min(nb, nbs - 1) * 16 + li) * r3s + g;
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = bp[4 * std::min(s, ks3)];
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
  auto mfma = [&](const float (&b)[KS], floatx4 (&acc)[4]) {
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb][s], b[s], s == 0 ? floatx4{0, 0, 0, 0} : acc[mb], 0, 0, 0);
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
    for (int i = 0; i < 4 * KS; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);   // VALU
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
    float bA[KS], bB[KS];
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
  return em_lds_bytes(m->rank[0], m->rank[1], m->rank[2]) <= EM_LDS_LIMIT;
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
  a.r3s = em_r3s(a.r3);
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
  const size_t lds = em_lds_bytes(a.r1, a.r2, a.r3);
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
