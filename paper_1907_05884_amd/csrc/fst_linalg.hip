// FP64 linear algebra of the core solve (Algorithm 2, normal equations (6)) for gfx950:
// blocked Cholesky factorisation G = L L^T in place, and the two triangular solves.
//
//   diagonal block      factor + inverse of a 64 x 64 block, one wave     k_potrf_diag
//   panel               L21 = A21 inv(L11)^T, FP64 MFMA                   k_trsm_panel
//   trailing update     G -= L21 L21^T on the lower triangle, FP64 MFMA   k_syrk_tile
//   solves              block forward / backward substitution            k_trsv_*
//
// Storage: G is row-major R x R; only its lower triangle is read.  On return L is in the
// lower triangle, and the strict upper triangle of every 64 x 64 diagonal block holds the
// inverse of that block of L, transposed: G[k0 + c][k0 + r] = inv(L_bb)[r][c] for r > c (the
// diagonal of the inverse is 1 / L_rr and is not stored).  The rest of the upper triangle is
// not touched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

// ------------------------------------------------------------------------------ Cholesky
// Right-looking blocked Cholesky in FP64 with 64-column blocks inside 256-column panels:
// factor the diagonal block, solve the panel below it, update the rest of the 256-column
// panel (K = 64), and once a panel is done update the trailing lower triangle with K = 256.
constexpr int CH_NB = 64;

__device__ inline double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __hiloint2double(hi, lo);
}

// Diagonal block, four waves.  A pivot counts as a breakdown when it is not above
// tol * (its diagonal entry before the factorisation), tol = R * 2^-52: at that size the
// Schur complement is rounding noise and the sampled system is numerically rank deficient.
// With drop_tol > 0 such a column is dropped instead (semidefinite factorisation): L_jj = +inf
// makes its column of L, its solution entry and its row and column of the block inverse
// exactly zero in every later step.
//
// Lane i of wave w holds row i, columns 16 w .. 16 w + 15, in registers.  Column j: the wave
// that owns it reads the pivot from lane j, scales the entries below and publishes the
// column through LDS (two alternating buffers, one barrier per column); every wave then
// applies the rank-1 update to its columns right of j.  1 / L_jj comes from the hardware
// reciprocal square root refined by two Newton steps, and L_jj = d / sqrt(d) from it with
// one more Newton correction.
//
// inv(L11) is then formed by the first wave in 16 x 16 blocks X_ij: the diagonal blocks by
// forward substitution (lane 16 b + c forms column c of X_bb), the others level by level
// (i - j = 1, 2, 3) as X_ij = -X_ii sum_{j <= k < i} L_ik X_kj on FP64 MFMA.  The accumulator
// of a 16 x 16 x 4 product holds in lane l the rows l / 16 + 4 v of column l % 16, which is
// the B operand of the next product's k-step v, so the second product reads no LDS for it.
// The block goes back to G with coalesced row writes.  A short last block (nb < 64) is
// padded with the identity.
__device__ inline double rsqrt_f64(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_potrf_diag(
    double* G, int64_t R, int64_t k0, int nb, int64_t* info, const double* diag0, double tol, double drop_tol) {
  __shared__ double sA[CH_NB][CH_NB + 1];
  __shared__ double sX[CH_NB][CH_NB + 1];
  __shared__ double scol[2][CH_NB];
  __shared__ double srd[CH_NB];
  __shared__ int64_t sinfo[4][2];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  {
    // 16 rows per wave, all loads in flight (clamped rows and columns), padding selected after
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = 16 * w + u;
      v[u] = G[(k0 + (r < nb ? r : 0)) * R + k0 + (l < nb ? l : 0)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = 16 * w + u;
      sA[r][l] = (r < nb && l <= r) ? v[u] : (r == l ? 1.0 : 0.0);
    }
  }
  const double thr = (tol > drop_tol ? tol : drop_tol) * diag0[k0 + (l < nb ? l : 0)];
  __syncthreads();
  double a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = sA[l][16 * w + c];
  int64_t brk = 0, ndrop = 0;
#pragma unroll
  for (int j = 0; j < CH_NB; ++j) {
    const int jb = j >> 4, jc = j & 15, buf = j & 1;
    if (w == jb) {
      // pivot logic without branches (uniform values)
      const double d = readlane_f64(a[jc], j);
      const double t = readlane_f64(thr, j);
      const bool fin = isfinite(d);
      const bool ok = j >= nb || (d > t && fin);
      const bool drop = !ok && drop_tol > 0.0 && fin;
      const double dd = ok ? d : 1.0;
      const double y = rsqrt_f64(dd);
      double sq = dd * y;
      sq = fma(0.5 * y, fma(-sq, sq, dd), sq);
      const double ljj = ok ? sq : (drop ? INFINITY : 1.0);
      const double inv = ok ? y : (drop ? 0.0 : 1.0);
      ndrop += drop ? 1 : 0;
      brk = (!ok && !drop && brk == 0) ? k0 + j + 1 : brk;
      const double lij = l > j ? a[jc] * inv : (l == j ? ljj : a[jc]);
      a[jc] = lij;
      scol[buf][l] = lij;
      if (l == 0) srd[j] = inv;
    }
    __syncthreads();
    if (w >= jb) {
      const double lj = scol[buf][l];
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (w > jb || c > jc) a[c] -= lj * scol[buf][16 * w + c];
    }
  }
  if (l == 0) {
    sinfo[w][0] = brk;
    sinfo[w][1] = ndrop;
  }
#pragma unroll
  for (int c = 0; c < 16; ++c)
    if (16 * w + c <= l) sA[l][16 * w + c] = a[c];
  __syncthreads();
  if (w == 0) {
    {
      // diagonal 16 x 16 blocks of the inverse: lane 16 b + c forms column c of X_bb
      const int b = l >> 4, c = l & 15, o = 16 * b;
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double xi = (i == c ? 1.0 : x[i]) * srd[o + i];
        x[i] = i < c ? 0.0 : xi;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (r > i) x[r] -= sA[o + r][o + i] * x[i];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) sX[o + r][o + c] = x[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int li = l & 15, g = l >> 4;
#pragma unroll
    for (int dd = 1; dd < 4; ++dd) {
#pragma unroll
      for (int j = 0; j + dd < 4; ++j) {
        const int i = j + dd;
        doublex4 t = doublex4{0, 0, 0, 0};
#pragma unroll
        for (int k = j; k < i; ++k)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            t = MfmaAcc<double>::mfma(sA[16 * i + li][16 * k + 4 * s4 + g], sX[16 * k + 4 * s4 + g][16 * j + li], t);
        doublex4 xij = doublex4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) xij = MfmaAcc<double>::mfma(sX[16 * i + li][16 * i + 4 * s4 + g], t[s4], xij);
#pragma unroll
        for (int v = 0; v < 4; ++v) sX[16 * i + MfmaAcc<double>::row(g, v)][16 * j + li] = -xij[v];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  }
  __syncthreads();
  // row r of the block: L[r][0..r] below and on the diagonal, inv(L11)[c][r] right of it
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int r = 16 * w + u;
    if (r < nb && l < nb) G[(k0 + r) * R + k0 + l] = l <= r ? sA[r][l] : sX[l][r];
  }
  if (threadIdx.x == 0) {
    int64_t b0 = 0, nd = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (b0 == 0) b0 = sinfo[q][0];
      nd += sinfo[q][1];
    }
    if (b0 != 0 && info[0] == 0) info[0] = b0;
    info[1] += nd;
  }
}

// Panel: rows i >= k0 + 64 solve L21[i, :] L11^T = A21[i, :], formed as A21[i, :] W with
// W = inv(L11)^T read from the block's upper triangle (W[k][j] = inv(L11)[j][k], zero for
// k > j), on FP64 MFMA.  16 rows per wave.  The contraction index of a 16 x 16 x 4 step is
// only summed over, so lane group g = lane / 16 takes the 16 consecutive columns
// 16 g .. 16 g + 15 of its row and reads the matching rows of W from LDS; each wave reads
// its rows completely before it overwrites them.
__global__ __launch_bounds__(256) void k_trsm_panel(double* G, int64_t R, int64_t k0) {
  __shared__ double sW[CH_NB][CH_NB + 1];
  for (int e = threadIdx.x; e < CH_NB * CH_NB; e += 256) {
    const int k = e / CH_NB, j = e % CH_NB;
    double v = 0.0;
    if (j > k) v = G[(k0 + k) * R + k0 + j];
    else if (j == k) v = 1.0 / G[(k0 + k) * R + k0 + k];
    sW[k][j] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t row0 = k0 + CH_NB + ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (row0 >= R) return;
  const int64_t row = row0 + li;
  const bool ok = row < R;
  const double* src = G + (ok ? row : row0) * R + k0 + 16 * g;
  double av[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const double t = src[s];
    av[s] = ok ? t : 0.0;
  }
  doublex4 acc[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) acc[n] = doublex4{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 16; ++s)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[n] = MfmaAcc<double>::mfma(av[s], sW[16 * g + s][16 * n + li], acc[n]);
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = row0 + MfmaAcc<double>::row(g, v);
      if (r < R) G[r * R + k0 + 16 * n + li] = acc[n][v];
    }
}

// Trailing update G[i, j] -= sum_{c < K} L[i, kL + c] L[j, kL + c] for base <= j <= i < R,
// j < col_end, on FP64 MFMA.  Workgroup tile 128 x 128: sixteen waves, each 32 x 32 (2 x 2
// blocks of 16 x 16), K staged 8 columns at a time through double-buffered LDS with a
// register prefetch of the next slice; two workgroups fit on a CU, so eight waves per SIMD
// hide the LDS, barrier and global latency (measured faster than fewer, larger wave tiles).
// The loads go through buffer resources whose extent ends at the last row of the matrix, so
// rows past R read as zero.  In a 16 x 16 x 4 step the contraction index is only summed
// over, so lane group g = lane / 16 takes the consecutive columns KS g .. KS g + KS - 1 of
// each staged row (16-byte LDS reads).  Tiles: the lower triangle of row/column blocks
// (nbc == 0), numbered so that each XCD (workgroups are dealt to the eight XCDs in turn)
// gets a contiguous run of tiles that share row blocks in its L2; or an nbc x nblk rectangle
// of column x row blocks whose tiles above the diagonal exit at once.
constexpr int SY_WM = 4, SY_WN = 4, SY_BM = 2, SY_BN = 2, SY_KC = 8;
constexpr int SY_THREADS = 64 * SY_WM * SY_WN, SY_TM = SY_WM * SY_BM * 16, SY_TN = SY_WN * SY_BN * 16;
constexpr int SY_Q = SY_TM / SY_TN, SY_KCP = SY_KC + 2, SY_RPP = SY_THREADS / SY_KC;
constexpr int SY_PA = SY_TM / SY_RPP, SY_PB = SY_TN / SY_RPP, SY_KS = SY_KC / 4;
static_assert(SY_TM % SY_TN == 0 && SY_KS % 2 == 0, "tile shape");
struct SyrkArgs {
  double* G;
  int64_t R, kL, base, col_end;
  int32_t K, nbc;
};
// lower-triangle tile t -> (bi, bj): row block bi (SY_TM rows) holds SY_Q (bi + 1) column
// blocks (SY_TN columns) and is preceded by SY_Q bi (bi + 1) / 2 tiles
__device__ inline void syrk_tile_of(int64_t t, int64_t& bi, int64_t& bj) {
  int64_t b = (int64_t)((sqrt(8.0 * (double)t / SY_Q + 1.0) - 1.0) * 0.5);
  while (SY_Q * b * (b + 1) / 2 > t) --b;
  while (SY_Q * (b + 1) * (b + 2) / 2 <= t) ++b;
  bi = b;
  bj = t - SY_Q * b * (b + 1) / 2;
}
__host__ __device__ inline int64_t syrk_tiles(int64_t nbr) { return SY_Q * nbr * (nbr + 1) / 2; }
constexpr int kXcds = 8;

__global__ __launch_bounds__(SY_THREADS) void k_syrk_tile(SyrkArgs a) {
  __shared__ double sA[2][SY_TM][SY_KCP];
  __shared__ double sB[2][SY_TN][SY_KCP];
  int64_t bi, bj;
  if (a.nbc > 0) {
    bj = blockIdx.x % a.nbc;
    bi = blockIdx.x / a.nbc;
  } else {
    // the grid is the tile count rounded up to a multiple of kXcds
    const int64_t per = gridDim.x / kXcds, t = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int64_t nbr = (a.R - a.base + SY_TM - 1) / SY_TM;
    if (t >= syrk_tiles(nbr)) return;
    syrk_tile_of(t, bi, bj);
  }
  const int64_t r0 = a.base + bi * SY_TM, c0 = a.base + bj * SY_TN;
  // nothing to do above the diagonal or right of the last column; a column block starting at
  // or past R would also give its buffer resource a non-positive extent
  if (c0 > r0 + SY_TM - 1 || c0 >= a.R || c0 >= a.col_end) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave / SY_WN, wc = wave % SY_WN;
  const int li = lane & 15, g = lane >> 4;
  const int64_t wrow0 = r0 + wr * SY_BM * 16, wcol0 = c0 + wc * SY_BN * 16;
  const bool active = wrow0 < a.R && wrow0 + SY_BM * 16 - 1 >= wcol0;
  const int64_t rowsA = std::min<int64_t>(SY_TM, a.R - r0), rowsB = std::min<int64_t>(SY_TN, a.R - c0);
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(a.G + r0 * a.R + a.kL), (short)0, (int)(rowsA * a.R * 8), 0x00020000);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(a.G + c0 * a.R + a.kL), (short)0, (int)(rowsB * a.R * 8), 0x00020000);
  const int fr = threadIdx.x / SY_KC, fc = threadIdx.x % SY_KC;
  const int Rb = (int)a.R * 8;
  double pa[SY_PA], pb[SY_PB];
  auto fetch = [&](int k) {
#pragma unroll
    for (int u = 0; u < SY_PA; ++u)
      pa[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rA, (fr + SY_RPP * u) * Rb + (k + fc) * 8, 0, 0));
#pragma unroll
    for (int u = 0; u < SY_PB; ++u)
      pb[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rB, (fr + SY_RPP * u) * Rb + (k + fc) * 8, 0, 0));
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int u = 0; u < SY_PA; ++u) sA[b][fr + SY_RPP * u][fc] = pa[u];
#pragma unroll
    for (int u = 0; u < SY_PB; ++u) sB[b][fr + SY_RPP * u][fc] = pb[u];
  };
  doublex4 acc[SY_BM][SY_BN];
#pragma unroll
  for (int x = 0; x < SY_BM; ++x)
#pragma unroll
    for (int y = 0; y < SY_BN; ++y) acc[x][y] = doublex4{0, 0, 0, 0};
  const int nk = a.K / SY_KC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int b = kc & 1;
    if (kc + 1 < nk) fetch((kc + 1) * SY_KC);
    if (active) {
#pragma unroll
      for (int h = 0; h < SY_KS / 2; ++h) {   // k-steps 2 h and 2 h + 1 of the chunk
        double2 av[SY_BM], bv[SY_BN];
#pragma unroll
        for (int x = 0; x < SY_BM; ++x)
          av[x] = *reinterpret_cast<const double2*>(&sA[b][wr * SY_BM * 16 + x * 16 + li][SY_KS * g + 2 * h]);
#pragma unroll
        for (int y = 0; y < SY_BN; ++y)
          bv[y] = *reinterpret_cast<const double2*>(&sB[b][wc * SY_BN * 16 + y * 16 + li][SY_KS * g + 2 * h]);
#pragma unroll
        for (int x = 0; x < SY_BM; ++x)
#pragma unroll
          for (int y = 0; y < SY_BN; ++y) acc[x][y] = MfmaAcc<double>::mfma(av[x].x, bv[y].x, acc[x][y]);
#pragma unroll
        for (int x = 0; x < SY_BM; ++x)
#pragma unroll
          for (int y = 0; y < SY_BN; ++y) acc[x][y] = MfmaAcc<double>::mfma(av[x].y, bv[y].y, acc[x][y]);
      }
    }
    if (kc + 1 < nk) stash(b ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int x = 0; x < SY_BM; ++x)
#pragma unroll
    for (int y = 0; y < SY_BN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = wrow0 + x * 16 + MfmaAcc<double>::row(g, v);
        const int64_t col = wcol0 + y * 16 + li;
        if (row < a.R && col <= row && col < a.col_end) a.G[row * a.R + col] -= acc[x][y][v];
      }
}

__global__ void k_copy_diag(const double* G, int64_t R, double* d) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < R) d[t] = G[t * R + t];
}

size_t cholesky_workspace_bytes(int64_t R) { return 256 + align_up(sizeof(double) * (size_t)R); }

__global__ void k_shift_diag(double* G, int64_t R, double f) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < R) G[t * R + t] *= f;
}

__global__ void k_zero_info(int64_t* info) {
  if (threadIdx.x < 2) info[threadIdx.x] = 0;
}

int64_t cholesky(int64_t R, double* G, void* ws, size_t ws_bytes, void* stream, double drop_tol,
                 int64_t* dropped, double shift) {
  if (ws_bytes < cholesky_workspace_bytes(R)) fail(FST_E_NOMEM, "cholesky: workspace too small");
  int64_t* d_info = (int64_t*)ws;   // [0] first breakdown (1-based), [1] dropped pivots
  double* d_diag = (double*)((char*)ws + 256);
  const double tol = (double)R * 2.220446049250313e-16;
  hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, S(stream), d_info);
  check_launch("k_zero_info");
  hipLaunchKernelGGL(k_copy_diag, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, S(stream), G, R, d_diag);
  check_launch("k_copy_diag");
  if (shift > 0.0) {
    hipLaunchKernelGGL(k_shift_diag, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, S(stream), G, R, 1.0 + shift);
    check_launch("k_shift_diag");
  }
  constexpr int64_t OUTER = 4 * CH_NB;
  for (int64_t K0 = 0; K0 < R; K0 += OUTER) {
    const int64_t P = std::min<int64_t>(OUTER, R - K0);
    const int64_t panel_end = K0 + P;
    for (int64_t k0 = K0; k0 < panel_end; k0 += CH_NB) {
      int nb = (int)std::min<int64_t>(CH_NB, R - k0);
      hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, S(stream), G, R, k0, nb, d_info, d_diag, tol,
                         drop_tol);
      check_launch("k_potrf_diag");
      const int64_t rest = R - k0 - nb;
      if (rest <= 0) break;
      hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)((rest + 63) / 64)), dim3(256), 0, S(stream), G, R, k0);
      check_launch("k_trsm_panel");
      const int64_t base = k0 + CH_NB;
      if (base < panel_end) {
        SyrkArgs sa;
        sa.G = G;
        sa.R = R;
        sa.kL = k0;
        sa.K = CH_NB;
        sa.base = base;
        sa.col_end = panel_end;
        sa.nbc = (int)((panel_end - base + SY_TN - 1) / SY_TN);
        const int64_t nbr = (R - base + SY_TM - 1) / SY_TM;
        hipLaunchKernelGGL(k_syrk_tile, dim3((unsigned)(sa.nbc * nbr)), dim3(SY_THREADS), 0, S(stream), sa);
        check_launch("k_syrk_tile(panel)");
      }
    }
    if (panel_end < R) {
      SyrkArgs sa;
      sa.G = G;
      sa.R = R;
      sa.kL = K0;
      sa.K = (int)P;
      sa.base = panel_end;
      sa.col_end = R;
      sa.nbc = 0;
      const int64_t nbr = (R - panel_end + SY_TM - 1) / SY_TM;
      const int64_t grid = (syrk_tiles(nbr) + kXcds - 1) / kXcds * kXcds;
      hipLaunchKernelGGL(k_syrk_tile, dim3((unsigned)grid), dim3(SY_THREADS), 0, S(stream), sa);
      check_launch("k_syrk_tile(trailing)");
    }
  }
  int64_t info[2] = {0, 0};
  copy_d2h(info, d_info, sizeof(info), stream);
  if (dropped) *dropped = info[1];
  return info[0];
}

// ------------------------------------------------------------------------------ no-allocation form
// Scratch of the Cholesky (breakdown flags, then the original diagonal) for callers that
// cannot allocate device memory: a file-scope device array, one copy per GPU, held until the
// process ends.  Host code reaches a GPU's copy only through the address hipGetSymbolAddress
// returns on that GPU (the array's name in host code is not a device address).  Every call on
// a GPU uses the same copy, so calls that overlap on one GPU race.
static __device__ __align__(256) unsigned char scratch[256 + 8 * FST_CHOLESKY_NOALLOC_MAX_R];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device ordinal -> address of its copy

static void* scratch_address() {
  const int dev = current_device();
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!p) fail(FST_E_DEVICE, "no device address for the Cholesky scratch array");
  g_scratch_ptr[dev] = p;
  return p;
}

int64_t cholesky_static_scratch(int64_t R, double* G, void* stream, double shift) {
  if (R < 1 || R > FST_CHOLESKY_NOALLOC_MAX_R)
    fail(FST_E_INVAL, "fst_cholesky_noalloc: R = " + std::to_string(R) + " is outside [1, " +
                          std::to_string((long long)FST_CHOLESKY_NOALLOC_MAX_R) + "]");
  return cholesky(R, G, scratch_address(), sizeof(scratch), stream, 0.0, nullptr, shift);
}

// ------------------------------------------------------------------------------ solves
// Stage the 64 x 64 diagonal block (L below the diagonal, the stored inverse above) in LDS;
// blockDim.x must be a multiple of 64.
__device__ inline void stage_block(const double* L, int64_t R, int64_t k0, int nb, double (*sB)[CH_NB + 1]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r0 = w * 16; r0 < CH_NB; r0 += nw * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      int r = r0 + u;
      bool in = r < nb && l < nb;
      double t = L[in ? (k0 + r) * R + k0 + l : 0];
      v[u] = in ? t : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) sB[r0 + u][l] = v[u];
  }
}

// y = inv(L_bb) r (forward) or inv(L_bb)^T r (backward) from the staged block; first wave,
// lane i forms entry i.
__device__ inline void block_inverse_apply(const double (*sB)[CH_NB + 1], int nb, bool transposed,
                                           const double* sr, double* sy) {
  const int i = threadIdx.x;
  if (i >= 64) return;
  double acc = 0.0;
  if (i < nb) {
    acc = sr[i] / sB[i][i];
    if (!transposed) {
      for (int c = 0; c < i; ++c) acc += sB[c][i] * sr[c];        // inv[i][c] stored at [c][i]
    } else {
      for (int c = i + 1; c < nb; ++c) acc += sB[i][c] * sr[c];   // inv[c][i] stored at [i][c]
    }
  }
  sy[i] = acc;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One block step of the forward solve: with r_b final (all earlier blocks applied), every
// workgroup forms y_b = inv(L_bb) r_b and subtracts L[row, block] y_b from its 64 rows below.
// y_b itself is written by k_trsv_blocks afterwards, so no workgroup overwrites r_b while
// another still reads it.  Each wave handles 16 rows with all 16 row loads in flight.
constexpr int TS_ROWS = 64;
__global__ __launch_bounds__(256) void k_trsv_fwd_step(const double* L, int64_t R, int64_t k0, int nb, double* x) {
  __shared__ double sB[CH_NB][CH_NB + 1];
  __shared__ double sr[CH_NB], sy[CH_NB];
  stage_block(L, R, k0, nb, sB);
  if (threadIdx.x < CH_NB) sr[threadIdx.x] = threadIdx.x < nb ? x[k0 + threadIdx.x] : 0.0;
  __syncthreads();
  block_inverse_apply(sB, nb, false, sr, sy);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double yl = lane < nb ? sy[lane] : 0.0;
  const int64_t rbeg = k0 + nb + (int64_t)blockIdx.x * TS_ROWS + wave * 16;
  double p[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    int64_t row = rbeg + u;
    bool ok = row < R && lane < nb;
    double t = L[ok ? row * R + k0 + lane : 0];
    p[u] = ok ? t * yl : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    double q = wave_sum(p[u]);
    int64_t row = rbeg + u;
    if (lane == 0 && row < R) x[row] -= q;
  }
}

// One block step of the backward solve (L^T x = y): every workgroup forms
// x_b = inv(L_bb)^T r_b and subtracts (L[block, i])^T x_b from its rows i above the block.
__global__ __launch_bounds__(256) void k_trsv_bwd_step(const double* L, int64_t R, int64_t k0, int nb, double* x) {
  __shared__ double sB[CH_NB][CH_NB + 1];
  __shared__ double sr[CH_NB], sy[CH_NB];
  stage_block(L, R, k0, nb, sB);
  if (threadIdx.x < CH_NB) sr[threadIdx.x] = threadIdx.x < nb ? x[k0 + threadIdx.x] : 0.0;
  __syncthreads();
  block_inverse_apply(sB, nb, true, sr, sy);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k0) return;
  double s = 0.0;
#pragma unroll 16
  for (int c = 0; c < CH_NB; ++c) {
    double t = c < nb ? L[(k0 + c) * R + i] : 0.0;
    s += t * sy[c];
  }
  x[i] -= s;
}

// Final pass of either sweep: every block's solution from its (final) right-hand side.
__global__ __launch_bounds__(64) void k_trsv_blocks(const double* L, int64_t R, double* x, int transposed) {
  __shared__ double sB[CH_NB][CH_NB + 1];
  __shared__ double sr[CH_NB], sy[CH_NB];
  const int64_t k0 = (int64_t)blockIdx.x * CH_NB;
  const int nb = (int)((R - k0) < CH_NB ? (R - k0) : CH_NB);
  stage_block(L, R, k0, nb, sB);
  sr[threadIdx.x] = (int)threadIdx.x < nb ? x[k0 + threadIdx.x] : 0.0;
  __syncthreads();
  block_inverse_apply(sB, nb, transposed != 0, sr, sy);
  __syncthreads();
  if ((int)threadIdx.x < nb) x[k0 + threadIdx.x] = sy[threadIdx.x];
}

__global__ void k_copy(int64_t n, const double* a, double* b) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

void cholesky_solve(int64_t R, const double* L, const double* b, double* x, void* stream) {
  if (b != x) {
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, S(stream), R, b, x);
    check_launch("k_copy");
  }
  const int64_t nblk = (R + CH_NB - 1) / CH_NB;
  for (int64_t bk = 0; bk + 1 < nblk; ++bk) {
    const int64_t k0 = bk * CH_NB;
    const int64_t rest = R - k0 - CH_NB;
    hipLaunchKernelGGL(k_trsv_fwd_step, dim3((unsigned)((rest + TS_ROWS - 1) / TS_ROWS)), dim3(256), 0, S(stream),
                       L, R, k0, CH_NB, x);
    check_launch("k_trsv_fwd_step");
  }
  hipLaunchKernelGGL(k_trsv_blocks, dim3((unsigned)nblk), dim3(64), 0, S(stream), L, R, x, 0);
  check_launch("k_trsv_blocks(fwd)");
  for (int64_t bk = nblk - 1; bk >= 1; --bk) {
    const int64_t k0 = bk * CH_NB;
    const int nb = (int)std::min<int64_t>(CH_NB, R - k0);
    hipLaunchKernelGGL(k_trsv_bwd_step, dim3((unsigned)((k0 + 255) / 256)), dim3(256), 0, S(stream), L, R, k0, nb, x);
    check_launch("k_trsv_bwd_step");
  }
  hipLaunchKernelGGL(k_trsv_blocks, dim3((unsigned)nblk), dim3(64), 0, S(stream), L, R, x, 1);
  check_launch("k_trsv_blocks(bwd)");
}

// Host mask of the columns a semidefinite factorisation skipped (L_jj = +inf).
std::vector<uint8_t> dropped_mask(const double* L, int64_t R, void* ws, void* stream) {
  double* d = (double*)ws;
  hipLaunchKernelGGL(k_copy_diag, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, S(stream), L, R, d);
  check_launch("k_copy_diag");
  std::vector<double> diag((size_t)R);
  copy_d2h(diag.data(), d, sizeof(double) * (size_t)R, stream);
  std::vector<uint8_t> mask((size_t)R);
  for (int64_t j = 0; j < R; ++j) mask[(size_t)j] = std::isinf(diag[(size_t)j]) ? 1 : 0;
  return mask;
}
}  // namespace fst
