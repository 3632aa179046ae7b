// Reconstruction of eq. (1) with the core contraction on FP32 MFMA (gfx950):
//
//   f(x_q) = sum_{j1, j2} u1[q, j1] u2[q, j2] T[q, (j1 j2)],   T = U3 alpha^T,
//   U3[q, j3] = u3_{j3}(x_q),  alpha^T[j3, (j1 j2)] = alpha[j1, j2, j3]
//
// For a tile of 64 points, T (64 x r1 r2) is a GEMM with K = r3 on MFMA 16x16x4 (FP32 in,
// FP32 accumulation): 2 R flop per point, the bulk of the work.  The weighted reduction over
// (j1, j2), 3 r1 r2 flop per point, runs on the VALU from the MFMA accumulators.
//
// Layout (per workgroup of four waves, each wave one 64-point tile per round):
//   LDS alpha   [r1 r2 padded to 16][r3s]   the core with j3 fastest, r3s = r3 rounded up to
//                                           4 and to 2 mod 4 (16 consecutive rows read at one
//                                           column fall in distinct bank pairs)
//   LDS U3      [64 points][r3s]            factor values of mode 3 (MFMA A operand)
//   LDS U1T/U2T [r1 | r2][68]               modes 1 and 2, points contiguous (float4 reads)
// Phase 1: each lane evaluates the Legendre basis and the three factor functions of one
// point (eq. (2); coefficients staged in LDS, read as broadcasts) and writes them to the tables.
// Phase 2: for every 16 columns (j1 j2) of T, K = r3 / 4 MFMA steps per 16-point block, then
// f += u1 u2 T in registers; a 16-lane butterfly sums each point's 16 column partials.
#include <hip/hip_runtime.h>

#include <algorithm>

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
  int32_t r1, r2, r3, r3s, r12p, residual, rounds;
  ModeMap<float> map;
  Recurrence<float> rec;
};

static inline int em_r3s(int r3) {
  int s = (r3 + 3) / 4 * 4;
  return s % 4 == 2 ? s : s + 2;
}

constexpr int EM_CSIZE = 3 * kMaxBasis * kMaxRank;   // coefficient matrices, staged once per workgroup

static size_t em_lds_bytes(int r1, int r2, int r3) {
  const size_t r3s = (size_t)em_r3s(r3), r12p = ((size_t)r1 * r2 + 15) / 16 * 16;
  return sizeof(float) * (EM_CSIZE + r12p * r3s + EM_WAVES * (64 * r3s + (size_t)(r1 + r2) * EM_TSTRIDE));
}

template <int NP, int RP>
__global__ __launch_bounds__(EM_THREADS) void k_eval_mfma(EvalMfmaArgs a) {
  extern __shared__ __align__(16) float em_smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  const int r1 = a.r1, r2 = a.r2, r3 = a.r3, r3s = a.r3s;
  float* sC = em_smem;                                            // [3][kMaxBasis][kMaxRank]
  float* sAlpha = sC + EM_CSIZE;                                  // [r12p][r3s]
  float* sW = sAlpha + (size_t)a.r12p * r3s + (size_t)wave * (64 * r3s + (r1 + r2) * EM_TSTRIDE);
  float* sU3 = sW;                                                 // [64][r3s]
  float* sU1 = sW + 64 * r3s;                                      // [r1][68]
  float* sU2 = sU1 + r1 * EM_TSTRIDE;                              // [r2][68]
  const int R12 = r1 * r2;
  for (int e = threadIdx.x; e < a.r12p * r3s; e += EM_THREADS) {
    const int c = e / r3s, j3 = e - c * r3s;
    sAlpha[e] = (c < R12 && j3 < r3) ? a.core[(int64_t)c * r3 + j3] : 0.0f;
  }
  for (int e = threadIdx.x; e < EM_CSIZE; e += EM_THREADS) sC[e] = a.coefs[e];
  const int KS = (r3 + 3) / 4;
  __syncthreads();

  for (int rnd = 0; rnd < a.rounds; ++rnd) {
    const int64_t tile = ((int64_t)rnd * gridDim.x + blockIdx.x) * EM_WAVES + wave;
    // ---- phase 1: this lane's point
    {
      int64_t q = tile * 64 + lane;
      q = q < a.n ? q : a.n - 1;
      q = q < 0 ? 0 : q;
      const int64_t i = a.idx ? (int64_t)a.idx[q] : q;
      // one mode at a time: basis values, then the factor values (coefficients by scalar loads)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float c = k == 0 ? a.x[i] : (k == 1 ? a.y[i] : a.z[i]);
        const float t = (c - a.map.lo[k]) * a.map.scale[k] - 1.0f;
        const float* Ck = sC + k * kMaxBasis * kMaxRank;   // same address in every lane: broadcast reads
        float u[RP];
#pragma unroll
        for (int j = 0; j < RP; ++j) u[j] = Ck[j];
        float pm1 = 1.0f, pm = t * a.rec.a[0];
#pragma unroll 2
        for (int m = 1; m < NP; ++m) {
#pragma unroll
          for (int j = 0; j < RP; ++j) u[j] += Ck[m * kMaxRank + j] * pm;
          const float pn = a.rec.a[m] * t * pm - a.rec.b[m] * pm1;
          pm1 = pm;
          pm = pn;
        }
        if (k == 0) {
#pragma unroll
          for (int j = 0; j < RP; ++j)
            if (j < r1) sU1[j * EM_TSTRIDE + lane] = u[j];
        } else if (k == 1) {
#pragma unroll
          for (int j = 0; j < RP; ++j)
            if (j < r2) sU2[j * EM_TSTRIDE + lane] = u[j];
        } else {
#pragma unroll
          for (int j = 0; j < RP; ++j)
            if (j < r3s) sU3[lane * r3s + j] = j < r3 ? u[j] : 0.0f;
        }
      }
      for (int j = RP; j < r3s; ++j) sU3[lane * r3s + j] = 0.0f;
    }
    __syncthreads();
    // ---- phase 2: T = U3 alpha^T on MFMA, 16 columns at a time, reduced with u1 u2
    float av[4][RP / 4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int s = 0; s < RP / 4; ++s) av[mb][s] = s < KS ? sU3[(16 * mb + li) * r3s + 4 * s + g] : 0.0f;
    float f[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) f[mb][v] = 0.0f;
    // T blocks of 16 columns on MFMA, two in flight: the MFMAs of block nb + 1 are issued before
    // the VALU reduction of block nb reads its accumulators
    auto block = [&](int nb, floatx4 (&acc)[4]) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) acc[mb] = floatx4{0, 0, 0, 0};
      const float* bp = sAlpha + (nb * 16 + li) * r3s + g;
#pragma unroll
      for (int s = 0; s < RP / 4; ++s) {
        if (s < KS) {
          const float b = bp[4 * s];
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb][s], b, acc[mb], 0, 0, 0);
        }
      }
    };
    int j1 = li / r2, j2 = li - (li / r2) * r2;
    auto reduce = [&](const floatx4 (&acc)[4]) {
      if (j1 < r1) {
        const float* w1 = sU1 + j1 * EM_TSTRIDE + 4 * g;
        const float* w2 = sU2 + j2 * EM_TSTRIDE + 4 * g;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const floatx4 x1 = *reinterpret_cast<const floatx4*>(w1 + 16 * mb);
          const floatx4 x2 = *reinterpret_cast<const floatx4*>(w2 + 16 * mb);
#pragma unroll
          for (int v = 0; v < 4; ++v) f[mb][v] += x1[v] * x2[v] * acc[mb][v];
        }
      }
      j2 += 16;
      while (j2 >= r2) {
        j2 -= r2;
        ++j1;
      }
    };
    const int nbs = a.r12p / 16;
    floatx4 accA[4], accB[4];
    block(0, accA);
    for (int nb = 0; nb < nbs; nb += 2) {
      if (nb + 1 < nbs) block(nb + 1, accB);
      reduce(accA);
      if (nb + 1 >= nbs) break;
      if (nb + 2 < nbs) block(nb + 2, accA);
      reduce(accB);
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
    if (li == 0) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t q = tile * 64 + 16 * mb + 4 * g + v;
          if (q < a.n) {
            if (a.residual) {
              const int64_t i = a.idx ? (int64_t)a.idx[q] : q;
              a.out[q] = a.v[i] - f[mb][v];
            } else {
              a.out[q] = f[mb][v];
            }
          }
        }
    }
    __syncthreads();
  }
}

bool eval_mfma_applies(const fst_model* m) {
  if (m->d != 3 || m->has_wavelets()) return false;
  for (int k = 0; k < 3; ++k)
    if (m->rank[k] > kMaxRank || m->degree[k] + 1 > kMaxBasis) return false;
  return em_lds_bytes(m->rank[0], m->rank[1], m->rank[2]) <= EM_LDS_LIMIT;
}

template <int NP, int RP>
static void em_launch(const EvalMfmaArgs& a, size_t lds, int blocks, void* stream) {
  hipLaunchKernelGGL((k_eval_mfma<NP, RP>), dim3((unsigned)blocks), dim3(EM_THREADS), lds, S(stream), a);
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
  a.rec = make_recurrence<float>();
  const size_t lds = em_lds_bytes(a.r1, a.r2, a.r3);
  const int64_t per_block = EM_WAVES;
  const int blocks = (int)std::min<int64_t>((a.ntiles + per_block - 1) / per_block, (int64_t)device_cu_count());
  a.rounds = (int)((a.ntiles + (int64_t)blocks * per_block - 1) / ((int64_t)blocks * per_block));
  const int rp = pad8(std::max(std::max(a.r1, a.r2), a.r3));
  const bool np16 = m->degree[0] < 16 && m->degree[1] < 16 && m->degree[2] < 16;
#define FST_EM_CASE(NPV, RPV) em_launch<NPV, RPV>(a, lds, blocks, stream)
  if (np16) {
    switch (rp) {
      case 8: FST_EM_CASE(16, 8); break;
      case 16: FST_EM_CASE(16, 16); break;
      case 24: FST_EM_CASE(16, 24); break;
      default: FST_EM_CASE(16, 32); break;
    }
  } else {
    switch (rp) {
      case 8: FST_EM_CASE(32, 8); break;
      case 16: FST_EM_CASE(32, 16); break;
      case 24: FST_EM_CASE(32, 24); break;
      default: FST_EM_CASE(32, 32); break;
    }
  }
#undef FST_EM_CASE
}

}  // namespace fst
