// Factor evaluation of eq. (2) with the contraction on FP32 MFMA (gfx950):
//
//   U_k[j, q] = sum_m C_k[m, j] phi_m(xi_k(x_q)),   m < n_k = p_k + 1 <= 32,  j < r_k <= 32
//
// Per 64 sampled rows and mode, U_k (64 x r_k) = Phi (64 x n_k) C_k (n_k x r_k) is a GEMM
// with K = n_k: on MFMA 16x16x4 (FP32 in, FP32 accumulation) that is 2 n_k r_k flop per point
// at the matrix-core rate instead of one VALU FMA and one LDS broadcast per term, which is
// what bounded the one-thread-per-point form.
//
// Per wave and round of 64 rows, lane l takes row q0 + l, and for each mode and each MFMA
// k-step s:
//   1. the lane advances the monic three-term recurrence of the Legendre polynomials
//      (coefficients folded into the code as constants; the normalisation of the orthonormal
//      basis goes into the staged coefficients) by four degrees, holding p_{4s .. 4s+3} of
//      its own row in four registers;
//   2. a 4 x 4 transpose of 16-lane blocks across those registers (two v_permlane16_swap and
//      two v_permlane32_swap) turns them into the A operands of the four 16-row tiles: lane
//      group g of tile t's register holds p_{4s+g} of rows 16 t .. 16 t + 15;
//   3. one MFMA per tile and 16-column block; the B operand (c_m C_k, zero past n_k and r_k) comes
//      from a per-workgroup LDS copy, swizzled [m][j ^ 16 ((m / 2) % 2)] so that the reads of 4
//      consecutive m at 16 consecutive j fall in 64 distinct banks.
// The basis never goes through LDS, so recurrence (VALU) and MFMA interleave within a wave.
// Lane l then holds U_k[16 jb + l % 16] at rows 16 t + 4 (l / 16) + v, v = 0..3: four
// consecutive rows of one column, one 16-byte store.
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

constexpr int FM_WAVES = 4, FM_THREADS = 64 * FM_WAVES, FM_ROWS = 64, FM_PARK = 8;

typedef float fm_floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t fm_uintx4 __attribute__((ext_vector_type(4)));
// buffer offset of a dropped store, and the largest U (bytes) that the kernel writes
constexpr uint32_t kFmSkip = 0x80000000u;
constexpr int64_t kFmMaxUBytes = 0x7FFFFF00;

template <typename TIn>
struct FactorMfmaArgs {
  const TIn* c[kMaxModes];
  const TIn* v;
  const int32_t* idx;
  const float* coefs;   // [kMaxModes][kMaxBasis][kMaxRank]
  float* U;
  float* vs;
  int64_t mrows, nrounds, ubytes;
  int32_t d;
  int32_t rank[kMaxModes], nb[kMaxModes], off[kMaxModes];
  ModeMap<float> map;
};

// The orthonormal Legendre basis satisfies phi_{m+1} = A_m t phi_m - B_m phi_{m-1} with
// A_m = sqrt((2m+1)(2m+3)) / (m+1), B_m = m sqrt(2m+3) / ((m+1) sqrt(2m-1)).  Writing
// phi_m = c_m p_m with c_0 = 1, c_{m+1} = A_m c_m gives the monic recurrence
// p_{m+1} = t p_m - beta_m p_{m-1}, beta_m = B_m / (A_m A_{m-1}): two VALU operations per degree.
// The kernel runs it and folds c_m into the staged coefficients (C'[m][j] = c_m C[m][j]).
// Square roots by Newton's iteration at compile time.
constexpr double fm_sqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 200; ++i) r = 0.5 * (r + x / r);
  return r;
}
constexpr double fm_rec_a(int m) { return fm_sqrt((2.0 * m + 1.0) * (2.0 * m + 3.0)) / (m + 1.0); }
constexpr double fm_rec_b(int m) {
  return m == 0 ? 0.0 : m * fm_sqrt(2.0 * m + 3.0) / ((m + 1.0) * fm_sqrt(2.0 * m - 1.0));
}
struct FmMonic {
  float beta[kMaxBasis];    // beta_m (beta_0 = 0)
  double scale[kMaxBasis];  // c_m
};
constexpr FmMonic fm_monic() {
  FmMonic t{};
  double c = 1.0;
  for (int m = 0; m < kMaxBasis; ++m) {
    t.scale[m] = c;
    t.beta[m] = m == 0 ? 0.0f : (float)(fm_rec_b(m) / (fm_rec_a(m) * fm_rec_a(m - 1)));
    c *= fm_rec_a(m);
  }
  return t;
}
// c_m for the coefficient staging (a plain device table: indexed at run time)
__constant__ double fm_scale_table[kMaxBasis] = {
#define FM_S(m) fm_monic().scale[m]
    FM_S(0),  FM_S(1),  FM_S(2),  FM_S(3),  FM_S(4),  FM_S(5),  FM_S(6),  FM_S(7),  FM_S(8),  FM_S(9),  FM_S(10),
    FM_S(11), FM_S(12), FM_S(13), FM_S(14), FM_S(15), FM_S(16), FM_S(17), FM_S(18), FM_S(19), FM_S(20), FM_S(21),
    FM_S(22), FM_S(23), FM_S(24), FM_S(25), FM_S(26), FM_S(27), FM_S(28), FM_S(29), FM_S(30), FM_S(31)};
#undef FM_S
static_assert(kMaxBasis == 32, "scale table size");
// bound on the recurrence state when n_k is not a multiple of 4: rows past n_k are then
// evaluated too (their coefficients are zero) and must stay finite; far outside the box the
// state would overflow, so it is clamped there (values at that size are not representable in
// the field either)
constexpr float kFmClamp = 1e30f;

// JB: blocks of 16 columns (ceil(max r_k / 16)); KS: MFMA k-steps (ceil(max n_k / 4));
// VEC: the row count is a multiple of 4 (16-byte stores).
template <typename TIn, int D, int JB, int KS, bool VEC>
__global__ __launch_bounds__(FM_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_factor_eval_mfma(
    FactorMfmaArgs<TIn> a) {
  __shared__ float sC[D][4 * KS][32];
  __shared__ float sPark[FM_WAVES][FM_PARK][D][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  static_assert(D * 4 * KS * 32 % FM_THREADS == 0, "staging loop");
#pragma unroll   // all loads issued before the first wait
  for (int e0 = 0; e0 < D * 4 * KS * 32; e0 += FM_THREADS) {
    const int e = e0 + threadIdx.x;
    const int k = e / (4 * KS * 32), m = (e / 32) % (4 * KS), j = e % 32;
    sC[k][m][j ^ (16 * ((m >> 1) & 1))] =
        (m < a.nb[k] && j < a.rank[k]) ? (float)(fm_scale_table[m] * a.coefs[(k * kMaxBasis + m) * kMaxRank + j]) : 0.0f;
  }
  // values of the sampled rows (a gather when idx is given)
  if (a.vs) {
    for (int64_t q = (int64_t)blockIdx.x * FM_THREADS + threadIdx.x; q < a.mrows; q += (int64_t)gridDim.x * FM_THREADS)
      a.vs[q] = (float)a.v[a.idx ? (int64_t)a.idx[q] : q];
  }
  __syncthreads();
  // U through a buffer resource: a store whose offset is past the end (kFmSkip) is dropped by
  // the hardware, so the stores need no branches
  const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.U, (short)0, (int)(uint32_t)(a.ubytes), 0x00020000);
  // Each wave takes up to FM_PARK rounds per pass (rounds w, w + W, .. of the pass, W = all
  // waves of the grid): their coordinates are loaded first and parked in LDS, then the rounds
  // are computed and stored with no load in between, so no wait on the stores is needed until
  // the next pass.
  float (*park)[D][64] = sPark[wave];
  const int64_t wtot = (int64_t)gridDim.x * FM_WAVES, w = (int64_t)blockIdx.x * FM_WAVES + wave;
  for (int64_t pass0 = 0; pass0 < a.nrounds; pass0 += wtot * FM_PARK) {
    int nr = 0;
    uint32_t rows[FM_PARK];
#pragma unroll
    for (int i = 0; i < FM_PARK; ++i) {   // rows past the end read the last row (never stored)
      const int64_t r = pass0 + w + i * wtot;
      const int64_t q = min(r * FM_ROWS + lane, a.mrows - 1);
      rows[i] = a.idx ? (uint32_t)a.idx[q] : (uint32_t)q;
      nr += r < a.nrounds ? 1 : 0;
    }
#pragma unroll
    for (int i = 0; i < FM_PARK; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) park[i][k][lane] = (float)a.c[k][rows[i]];
    for (int i = 0; i < nr; ++i) {
      const int64_t r = pass0 + w + i * wtot;
      float cur[D];
#pragma unroll
      for (int k = 0; k < D; ++k) cur[k] = park[i][k][lane];
      const int64_t q0 = r * FM_ROWS;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        constexpr FmMonic rec = fm_monic();
        const float t = (cur[k] - a.map.lo[k]) * a.map.scale[k] - 1.0f;
        fm_floatx4 acc[4][JB];
#pragma unroll
        for (int tile = 0; tile < 4; ++tile)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb) acc[tile][jb] = fm_floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        auto contract = [&](auto clamp) {
          float prev = 0.0f, now = 1.0f;   // p_{m-1}, p_m of this lane's row
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            // 1. p_{4s .. 4s+3} of this lane's row
            uint32_t x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int m = 4 * s + i;
              x[i] = __builtin_bit_cast(uint32_t, now);
              float next = fmaf(t, now, -rec.beta[m] * prev);
              if (decltype(clamp)::value) next = fminf(fmaxf(next, -kFmClamp), kFmClamp);
              prev = now;
              now = next;
            }
            // 2. blocks (row group t, degree g) -> (tile t, lane group g)
            {
              auto p0 = __builtin_amdgcn_permlane16_swap(x[0], x[1], false, false);
              auto p1 = __builtin_amdgcn_permlane16_swap(x[2], x[3], false, false);
              auto q0 = __builtin_amdgcn_permlane32_swap(p0[0], p1[0], false, false);
              auto q1 = __builtin_amdgcn_permlane32_swap(p0[1], p1[1], false, false);
              x[0] = q0[0];
              x[2] = q0[1];
              x[1] = q1[0];
              x[3] = q1[1];
            }
            // 3. MFMA
            float bv[JB];
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) bv[jb] = sC[k][4 * s + g][(16 * jb + li) ^ (16 * ((g >> 1) & 1))];
#pragma unroll
            for (int tile = 0; tile < 4; ++tile)
#pragma unroll
              for (int jb = 0; jb < JB; ++jb)
                acc[tile][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_bit_cast(float, x[tile]), bv[jb],
                                                                     acc[tile][jb], 0, 0, 0);
          }
        };
        if (a.nb[k] == 4 * KS) contract(std::false_type{});
        else contract(std::true_type{});
        // 3. lane l: column 16 jb + l % 16, rows q0 + 16 tile + 4 g + (0..3)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int j = 16 * jb + li;
          const bool jv = j < a.rank[k];
          const uint32_t base = (uint32_t)(((int64_t)(a.off[k] + j) * a.mrows + q0 + 4 * g) * 4);
          if (VEC) {   // n % 4 == 0: four consecutive rows are all inside or all past the end
#pragma unroll
            for (int tile = 0; tile < 4; ++tile) {
              const bool ok = jv && q0 + 16 * tile + 4 * g < a.mrows;
              __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(fm_uintx4, acc[tile][jb]), urs,
                                                     ok ? base + 64u * tile : kFmSkip, 0, 0);
            }
          } else {
#pragma unroll
            for (int tile = 0; tile < 4; ++tile)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                // (the element is copied to a float first: a bit cast of a vector-element lvalue
                // compiles to a read of element 0)
                const bool ok = jv && q0 + 16 * tile + 4 * g + v < a.mrows;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, (float)acc[tile][jb][v]), urs,
                                                      ok ? base + 64u * tile + 4u * v : kFmSkip, 0, 0);
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

// one resident workgroup per slot (grid-stride over the rounds): as many workgroups as the
// occupancy of the instance allows on every CU
template <typename TIn, int D, int JB, int KS, bool VEC>
static void launch_one(const FactorMfmaArgs<TIn>& a, void* stream) {
  static std::atomic<int> occupancy(0);
  int per_cu = occupancy.load();
  if (!per_cu) {
    int nb = 0;
    check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_factor_eval_mfma<TIn, D, JB, KS, VEC>, FM_THREADS, 0),
              "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    per_cu = nb > 0 ? nb : 1;
    occupancy.store(per_cu);
  }
  const int64_t blocks =
      std::min<int64_t>((a.nrounds + FM_WAVES - 1) / FM_WAVES, (int64_t)device_cu_count() * per_cu);
  hipLaunchKernelGGL((k_factor_eval_mfma<TIn, D, JB, KS, VEC>), dim3((unsigned)blocks), dim3(FM_THREADS), 0, S(stream),
                     a);
}

template <typename TIn, int D, bool VEC>
static void launch_d(const FactorMfmaArgs<TIn>& a, int jb, int ks, void* stream) {
  if (jb == 1) {
    if (ks <= 4) launch_one<TIn, D, 1, 4, VEC>(a, stream);
    else launch_one<TIn, D, 1, 8, VEC>(a, stream);
  } else {
    if (ks <= 4) launch_one<TIn, D, 2, 4, VEC>(a, stream);
    else launch_one<TIn, D, 2, 8, VEC>(a, stream);
  }
}

void launch_factor_eval_mfma(const fst_model* m, const DeviceModel& dm, const void* const* coords, const void* v,
                             const int32_t* idx, int64_t mrows, void* U, void* vs, void* stream) {
  if (mrows <= 0) return;
  if (!factor_eval_mfma_applies(m, mrows)) fail(FST_E_INVAL, "factor evaluation on MFMA: unsupported model or size");
  FactorMfmaArgs<float> a;
  a.v = (const float*)v;
  a.idx = idx;
  a.coefs = (const float*)dm.coefs;
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
  const int jb = (rmax + 15) / 16, ks = (nbmax + 3) / 4;
  const bool vec = mrows % 4 == 0;
  if (m->d == 3) {
    if (vec) launch_d<float, 3, true>(a, jb, ks, stream);
    else launch_d<float, 3, false>(a, jb, ks, stream);
  } else {
    if (vec) launch_d<float, 4, true>(a, jb, ks, stream);
    else launch_d<float, 4, false>(a, jb, ks, stream);
  }
  check_launch("k_factor_eval_mfma");
}

}  // namespace fst
