// Mixed least-squares rows of Algorithm 2 (steps 1-5 with the randomised transform) for
// gfx950: the design matrix W (N x R, rows past n zero) and the values u are multiplied by
// random signs D and mixed by the normalised Walsh-Hadamard transform F = H_N / sqrt(N) (the
// real orthogonal stand-in for the FFT), S rows of F D W and F D u are kept, and the normal
// equations of that sampled problem are formed.
//
//   k_mix_lo     the r3 design columns of one (j1, j2) pair (Khatri-Rao products of three
//                factor rows, times the sign of each row) in blocks of 4096 rows: the signed
//                product u1 u2 is formed once per row and each column multiplies it by its u3;
//                the 12 butterfly stages inside a block, 4 in registers and 8 through LDS (in
//                passes of up to three stages, each a register butterfly of 8 elements)
//   k_mix_hi     the remaining stages across blocks (strides 4096 .. N/2) through LDS (up to
//                three per pass, as above), the 1/sqrt(N) scale, and a scatter of the sampled
//                rows into A^T from a list of the samples that fall into the workgroup's rows
//   k_gram_dense G = A^T A (lower triangle) from the materialised sampled rows, MFMA
//   k_atv_dense  h = A^T b
//
// N is the smallest power of two >= max(n, 4096).  The transform of a column touches every
// one of its N entries twice (one read and one write per pass), so the mixing is bound by
// HBM; the Gram of the S x R sampled rows is the same MFMA work as the unmixed one, read from
// a dense A^T instead of being formed from factor values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

constexpr int MX_B1 = 4096;        // rows of one block of the first pass
constexpr int MX_THREADS = 256;
constexpr int MX_MAX_LOG2N = 23;   // N <= 2^23 (the second pass holds 2^(log2 N - 12) rows per offset)
constexpr int64_t kSignsStream = 5;

// Output i (from 0) of the SplitMix64 stream started at `state`: mix(state + (i + 1) gamma);
// the row sign is -1 when its top bit is set.
__device__ inline int row_sign_negative(uint64_t state, int64_t i) {
  uint64_t z = state + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (int)(z >> 63);
}

template <typename T>
struct MixArgs {
  const T* U;            // [SR][n] factor values at all points
  const T* v;            // values (with `values` set)
  int64_t n, N, R;
  int32_t r1, r2, r3, L, lgL, H, values;
  int64_t c0;            // first design column of this launch (a multiple of r3)
  uint64_t sign_state;
  T* buf;                // [columns of the launch][N]
  const int32_t* sel;    // per second-pass workgroup: (LDS element, sample position) pairs
  const int32_t* sel_off;
  T* At;                 // [R][Sp]
  T* b;                  // [Sp]
  int64_t Sp;
  T scale;
};

// Workgroup (x, y): rows x 4096 .. x 4096 + 4095 of the r3 columns of pair y of the launch
// (or of the value column).
template <typename T>
__global__ __launch_bounds__(MX_THREADS) void k_mix_lo(MixArgs<T> a) {
  __shared__ T s[MX_B1];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * MX_B1;
  const int64_t j0 = a.c0 + (int64_t)blockIdx.y * a.r3;   // column of j3 = 0
  const int64_t j12 = j0 / a.r3;
  const T* p1 = a.U + (j12 / a.r2) * a.n;
  const T* p2 = a.U + (a.r1 + j12 % a.r2) * a.n;
  const T* p3 = a.U + (int64_t)(a.r1 + a.r2) * a.n;
  T pr[16];   // sign x u1 u2 (or sign x value) of the thread's rows
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = base + t + 256 * k;
    T x = T(0);
    if (i < a.n) {
      x = a.values ? a.v[i] : p1[i] * p2[i];
      if (row_sign_negative(a.sign_state, i)) x = -x;
    }
    pr[k] = x;
  }
  const int ncol = a.values ? 1 : a.r3;
  // u3 of the next column is loaded while the current one goes through the LDS stages
  T u3[16];
  auto load_u3 = [&](int jj) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t i = base + t + 256 * k;
      u3[k] = (!a.values && i < a.n) ? p3[(int64_t)jj * a.n + i] : T(1);
    }
  };
  load_u3(0);
  for (int jj = 0; jj < ncol; ++jj) {
    T w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = pr[k] * u3[k];
    if (jj + 1 < ncol) load_u3(jj + 1);
    // strides 256 .. 2048 (bits 8 .. 11 of the row): partners among this thread's elements
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (!(k & (1 << sb))) {
          const T x = w[k], y = w[k | (1 << sb)];
          w[k] = x + y;
          w[k | (1 << sb)] = x - y;
        }
#pragma unroll
    for (int k = 0; k < 16; ++k) s[t + 256 * k] = w[k];
    __syncthreads();
    // strides 1 .. 128 (bits 0 .. 7), in passes of three, three and two stages: a thread takes
    // the 2^NB elements base + m 2^lh of a group, applies NB stages in registers and writes
    // them back
    auto pass = [&](auto lhc, auto nbits) {
      constexpr int LH = decltype(lhc)::value, NB = decltype(nbits)::value, G = 1 << NB;
#pragma unroll
      for (int q = 0; q < (MX_B1 >> NB) / MX_THREADS; ++q) {
        const int p = t + MX_THREADS * q;
        const int base = ((p >> LH) << (LH + NB)) | (p & ((1 << LH) - 1));
        T v[G];
#pragma unroll
        for (int m = 0; m < G; ++m) v[m] = s[base + (m << LH)];
#pragma unroll
        for (int sb = 0; sb < NB; ++sb)
#pragma unroll
          for (int m = 0; m < G; ++m)
            if (!(m & (1 << sb))) {
              const T x = v[m], y = v[m | (1 << sb)];
              v[m] = x + y;
              v[m | (1 << sb)] = x - y;
            }
#pragma unroll
        for (int m = 0; m < G; ++m) s[base + (m << LH)] = v[m];
      }
      __syncthreads();
    };
    pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{});
    pass(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{});
    pass(std::integral_constant<int, 6>{}, std::integral_constant<int, 2>{});
    T* out = a.buf + ((int64_t)blockIdx.y * ncol + jj) * a.N + base;
#pragma unroll
    for (int k = 0; k < 16; ++k) out[t + 256 * k] = s[t + 256 * k];
    __syncthreads();   // s is rewritten by the next column
  }
}

// Workgroup (x, c): offsets x L .. x L + L - 1 inside the 4096-row blocks of column c of the
// launch, all K = 2^H blocks (LDS element k L + l is row k 4096 + x L + l).
template <typename T>
__global__ __launch_bounds__(MX_THREADS) void k_mix_hi(MixArgs<T> a) {
  extern __shared__ __align__(16) unsigned char mx_smem[];
  T* s = reinterpret_cast<T*>(mx_smem);   // [K][L]
  const int c = blockIdx.y;
  const int64_t j = a.values ? a.R : a.c0 + c;
  const int L = a.L, lgL = a.lgL, E = L << a.H;
  const int l0 = blockIdx.x * L;
  const T* col = a.buf + (int64_t)c * a.N;
  // L and 2^H are powers of two: every index below is shifts and masks
  for (int e = threadIdx.x; e < E; e += MX_THREADS) s[e] = col[(int64_t)(e >> lgL) * MX_B1 + l0 + (e & (L - 1))];
  __syncthreads();
  // the H cross-block stages (they commute) up to three at a time: a thread takes the 2^NB
  // elements of a group (blocks k = base + m 2^lh, m < 2^NB, one offset l), applies NB stages
  // in registers and writes them back, so each pass reads and writes the column once
  auto pass = [&](int lh, auto nbits) {
    constexpr int NB = decltype(nbits)::value, G = 1 << NB;
    const int lo = (1 << lh) - 1;
    for (int p = threadIdx.x; p < (E >> NB); p += MX_THREADS) {
      const int pk = p >> lgL, l = p & (L - 1);
      const int base = ((pk >> lh) << (lh + NB)) | (pk & lo);
      T w[G];
#pragma unroll
      for (int m = 0; m < G; ++m) w[m] = s[(base + (m << lh)) * L + l];
#pragma unroll
      for (int sb = 0; sb < NB; ++sb)
#pragma unroll
        for (int m = 0; m < G; ++m)
          if (!(m & (1 << sb))) {
            const T x = w[m], y = w[m | (1 << sb)];
            w[m] = x + y;
            w[m | (1 << sb)] = x - y;
          }
#pragma unroll
      for (int m = 0; m < G; ++m) s[(base + (m << lh)) * L + l] = w[m];
    }
    __syncthreads();
  };
  for (int lh = 0; lh < a.H; lh += 3) {
    const int nb = a.H - lh < 3 ? a.H - lh : 3;
    if (nb == 3) pass(lh, std::integral_constant<int, 3>{});
    else if (nb == 2) pass(lh, std::integral_constant<int, 2>{});
    else pass(lh, std::integral_constant<int, 1>{});
  }
  const int beg = a.sel_off[blockIdx.x], end = a.sel_off[blockIdx.x + 1];
  for (int q = beg + threadIdx.x; q < end; q += MX_THREADS) {
    const int e = a.sel[2 * q], p = a.sel[2 * q + 1];
    const T val = s[e] * a.scale;
    if (j < a.R)
      a.At[j * a.Sp + p] = val;
    else
      a.b[p] = val;
  }
}

// zero entries [S, Sp) of every row of A^T and of b (the padding of the last K chunk)
template <typename T>
__global__ void k_zero_tail(T* At, T* b, int64_t R, int64_t S, int64_t Sp) {
  const int64_t w = Sp - S;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (R + 1) * w) return;
  const int64_t r = e / w, q = S + e % w;
  if (r < R)
    At[r * Sp + q] = T(0);
  else
    b[q] = T(0);
}

// G = A^T A for the lower triangle of 128 x 128 tiles: sixteen waves of 32 x 32 (2 x 2
// MFMA blocks), KC points of the tile's 128 row-block and 128 column-block rows of A^T staged
// through double-buffered LDS with 16-byte loads (rows of A^T are Sp long, Sp a multiple of
// KC, so every chunk is whole).  As in the Khatri-Rao Gram, lane group g takes the points
// g KC/4 + s, and FP32 accumulation is folded into FP64 registers every chunk.  With
// accumulate != 0 the tile is added to the G already there (row chunks of a larger A).
template <typename T> struct DenseKC;
template <> struct DenseKC<float> { static constexpr int KC = 64; };
template <> struct DenseKC<double> { static constexpr int KC = 32; };
constexpr int GD_TILE = 128, GD_THREADS = 1024;
static_assert(GD_SP_MULTIPLE % DenseKC<float>::KC == 0 && GD_SP_MULTIPLE % DenseKC<double>::KC == 0,
              "padded row counts must hold whole chunks");

template <typename T>
__global__ __launch_bounds__(GD_THREADS) void k_gram_dense(const T* At, int64_t R, int64_t Sp, double* G,
                                                          int accumulate) {
  constexpr int KC = DenseKC<T>::KC, KCP = KC + 16 / (int)sizeof(T), VW = 16 / (int)sizeof(T);
  constexpr int PIECES = 2 * GD_TILE * KC / VW / GD_THREADS;   // 16-byte pieces per thread per chunk
  typedef T T4 __attribute__((ext_vector_type(4)));
  typedef T TV __attribute__((ext_vector_type(16 / sizeof(T))));
  typedef typename MfmaAcc<T>::V V;
  constexpr bool kFold = sizeof(T) == 4;
  __shared__ __align__(16) T sA[2][2 * GD_TILE][KCP];
  int64_t bi, bj;
  tri_tile(blockIdx.x, bi, bj);
  const int64_t r0 = bi * GD_TILE, c0 = bj * GD_TILE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3, li = lane & 15, g = lane >> 4;
  const int row0 = wr * 32, col0 = wc * 32;
  const bool active = c0 + col0 <= r0 + row0 + 31;
  TV pf[PIECES];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const int e = threadIdx.x + GD_THREADS * u;
      const int r = e / (KC / VW), pc = e % (KC / VW);
      const int64_t gr = r < GD_TILE ? r0 + r : c0 + (r - GD_TILE);
      TV val = TV{};
      if (gr < R) val = *reinterpret_cast<const TV*>(&At[gr * Sp + k0 + pc * VW]);
      pf[u] = val;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const int e = threadIdx.x + GD_THREADS * u;
      const int r = e / (KC / VW), pc = e % (KC / VW);
      *reinterpret_cast<TV*>(&sA[b][r][pc * VW]) = pf[u];
    }
  };
  V acc[2][2];
  double dacc[kFold ? 2 : 1][kFold ? 2 : 1][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = V{0, 0, 0, 0};
  if (kFold) {
#pragma unroll
    for (int x = 0; x < (kFold ? 2 : 1); ++x)
#pragma unroll
      for (int y = 0; y < (kFold ? 2 : 1); ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[x][y][v] = 0.0;
  }
  const int64_t nch = Sp / KC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int b = (int)(ch & 1);
    if (ch + 1 < nch) fetch((ch + 1) * KC);
    if (active) {
#pragma unroll
      for (int s0 = 0; s0 < KC / 4; s0 += 4) {
        const int p = g * (KC / 4) + s0;
        T4 av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = *reinterpret_cast<const T4*>(&sA[b][row0 + x * 16 + li][p]);
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = *reinterpret_cast<const T4*>(&sA[b][GD_TILE + col0 + y * 16 + li][p]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = MfmaAcc<T>::mfma(av[x][s], bv[y][s], acc[x][y]);
      }
      if (kFold) {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
#pragma unroll
            for (int v = 0; v < 4; ++v) dacc[kFold ? x : 0][kFold ? y : 0][v] += (double)acc[x][y][v];
            acc[x][y] = V{0, 0, 0, 0};
          }
      }
    }
    if (ch + 1 < nch) stash(b ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + row0 + x * 16 + MfmaAcc<T>::row(g, v);
        const int64_t col = c0 + col0 + y * 16 + li;
        const double val = kFold ? dacc[kFold ? x : 0][kFold ? y : 0][v] : (double)acc[x][y][v];
        if (row < R && col <= row) G[row * R + col] = accumulate ? G[row * R + col] + val : val;
      }
}

// The same Gram from 16-bit rows (BF16, or FP16 already scaled by a power of two): chunks of
// GD16_KC = 128 points through double-buffered LDS, MFMA 16x16x32 with lane group g taking
// the points 32 ks + 8 g .. + 7 of step ks, FP32 accumulation folded into FP64 every chunk,
// G = sums x unscale.  This is the arithmetic of the Khatri-Rao precision-form kernel on the
// same 16-bit entries.  Sp: a multiple of GD16_KC.
constexpr int GD16_KC = 128;

template <typename H>
__global__ __launch_bounds__(GD_THREADS) void k_gram_dense16(const H* At, int64_t R, int64_t Sp, double* G,
                                                            double unscale, int accumulate) {
  typedef typename Mfma16<H>::V8 V8;
  constexpr int KC = GD16_KC, KCP = KC + 8, VW = 8;
  constexpr int PIECES = 2 * GD_TILE * KC / VW / GD_THREADS;   // 16-byte pieces per thread per chunk
  __shared__ __align__(16) H sA[2][2 * GD_TILE][KCP];
  int64_t bi, bj;
  tri_tile(blockIdx.x, bi, bj);
  const int64_t r0 = bi * GD_TILE, c0 = bj * GD_TILE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3, li = lane & 15, g = lane >> 4;
  const int row0 = wr * 32, col0 = wc * 32;
  const bool active = c0 + col0 <= r0 + row0 + 31;
  V8 pf[PIECES];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const int e = threadIdx.x + GD_THREADS * u;
      const int r = e / (KC / VW), pc = e % (KC / VW);
      const int64_t gr = r < GD_TILE ? r0 + r : c0 + (r - GD_TILE);
      V8 val = V8{};
      if (gr < R) val = *reinterpret_cast<const V8*>(&At[gr * Sp + k0 + pc * VW]);
      pf[u] = val;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const int e = threadIdx.x + GD_THREADS * u;
      const int r = e / (KC / VW), pc = e % (KC / VW);
      *reinterpret_cast<V8*>(&sA[b][r][pc * VW]) = pf[u];
    }
  };
  floatx4 acc[2][2];
  double dacc[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      acc[x][y] = floatx4{0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[x][y][v] = 0.0;
    }
  const int64_t nch = Sp / KC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int b = (int)(ch & 1);
    if (ch + 1 < nch) fetch((ch + 1) * KC);
    if (active) {
#pragma unroll
      for (int ks = 0; ks < KC / 32; ++ks) {
        const int p = ks * 32 + g * 8;
        V8 av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = *reinterpret_cast<const V8*>(&sA[b][row0 + x * 16 + li][p]);
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = *reinterpret_cast<const V8*>(&sA[b][GD_TILE + col0 + y * 16 + li][p]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = Mfma16<H>::mfma(av[x], bv[y], acc[x][y]);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
#pragma unroll
          for (int v = 0; v < 4; ++v) dacc[x][y][v] += (double)acc[x][y][v];
          acc[x][y] = floatx4{0, 0, 0, 0};
        }
    }
    if (ch + 1 < nch) stash(b ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + row0 + x * 16 + MfmaAcc<float>::row(g, v);
        const int64_t col = c0 + col0 + y * 16 + li;
        const double val = dacc[x][y][v] * unscale;
        if (row < R && col <= row) G[row * R + col] = accumulate ? G[row * R + col] + val : val;
      }
}

void dense_gram16(int gram_prec, const void* At, int64_t R, int64_t Sp, double* G, double unscale, void* stream) {
  if (Sp % GD16_KC != 0 || Sp <= 0) fail(FST_E_INVAL, "dense 16-bit Gram: row count not padded");
  const int64_t nt = (R + GD_TILE - 1) / GD_TILE;
  const dim3 gg((unsigned)(nt * (nt + 1) / 2));
  if (gram_prec == FST_GRAM_BF16)
    hipLaunchKernelGGL(k_gram_dense16<__bf16>, gg, dim3(GD_THREADS), 0, S(stream), (const __bf16*)At, R, Sp, G,
                       unscale, 0);
  else
    hipLaunchKernelGGL(k_gram_dense16<_Float16>, gg, dim3(GD_THREADS), 0, S(stream), (const _Float16*)At, R, Sp, G,
                       unscale, 0);
  check_launch("k_gram_dense16");
}

// h[j] = sum_q A^T[j][q] b[q] in FP64 (added to h[j] with accumulate != 0), one wave per row,
// lanes striding over q in a fixed order
template <typename T>
__global__ __launch_bounds__(256) void k_atv_dense(const T* At, const T* b, int64_t R, int64_t Sp, double* h,
                                                   int accumulate) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= R) return;
  const T* row = At + j * Sp;
  double s = 0.0;
  for (int64_t q = lane; q < Sp; q += 64) s += (double)row[q] * (double)b[q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) h[j] = accumulate ? h[j] + s : s;
}

void dense_normal_equations(int dtype, const void* At, const void* b, int64_t R, int64_t Sp, double* G, double* h,
                            bool accumulate, void* stream) {
  if (Sp % GD_SP_MULTIPLE != 0) fail(FST_E_INVAL, "dense Gram: row count not padded");
  const int64_t nt = (R + GD_TILE - 1) / GD_TILE;
  const dim3 gg((unsigned)(nt * (nt + 1) / 2)), ga((unsigned)((R + 3) / 4));
  if (dtype == FST_F64) {
    if (G) {
      hipLaunchKernelGGL(k_gram_dense<double>, gg, dim3(GD_THREADS), 0, S(stream), (const double*)At, R, Sp, G,
                         accumulate ? 1 : 0);
      check_launch("k_gram_dense");
    }
    if (h) {
      hipLaunchKernelGGL(k_atv_dense<double>, ga, dim3(256), 0, S(stream), (const double*)At, (const double*)b, R,
                         Sp, h, accumulate ? 1 : 0);
      check_launch("k_atv_dense");
    }
  } else {
    if (G) {
      hipLaunchKernelGGL(k_gram_dense<float>, gg, dim3(GD_THREADS), 0, S(stream), (const float*)At, R, Sp, G,
                         accumulate ? 1 : 0);
      check_launch("k_gram_dense");
    }
    if (h) {
      hipLaunchKernelGGL(k_atv_dense<float>, ga, dim3(256), 0, S(stream), (const float*)At, (const float*)b, R, Sp,
                         h, accumulate ? 1 : 0);
      check_launch("k_atv_dense");
    }
  }
}

// ------------------------------------------------------------------------------ host side
int64_t mixed_length(int64_t n) {
  int64_t N = MX_B1;
  while (N < n) N *= 2;
  return N;
}

// Second-pass geometry: offsets per workgroup L (32 KB of LDS hold L 2^H values)
static int mix_H(int64_t N) {
  int H = 0;
  while ((int64_t(MX_B1) << H) < N) ++H;
  return H;
}
static int mix_L(int dtype, int H) {
  const int64_t elems = dtype == FST_F64 ? 4096 : 8192;   // 32 KB of LDS
  return (int)std::min<int64_t>(MX_B1, elems >> H);
}

struct MixLayout {
  int64_t N, Sp, C;
  int H, L;
  size_t U, buf, sel, sel_off, At, b, total;
};
static MixLayout mix_layout(const fst_model* m, int dtype, int64_t n, int64_t nsamp) {
  const size_t es = dtype == FST_F64 ? 8 : 4;
  MixLayout L;
  L.N = mixed_length(n);
  L.Sp = (nsamp + 63) / 64 * 64;
  L.H = mix_H(L.N);
  L.L = mix_L(dtype, L.H);
  // columns per launch: whole (j1, j2) pairs, about 1 GB of transform buffer
  const int64_t r3 = m->rank[2];
  const int64_t cmax = std::max<int64_t>(1, std::min<int64_t>(256, (int64_t(1) << 30) / (L.N * (int64_t)es)));
  L.C = std::max<int64_t>(1, cmax / r3) * r3;
  size_t off = 0;
  L.U = off;
  off += align_up(es * (size_t)m->sum_r() * (size_t)n);
  L.buf = off;
  off += align_up(es * (size_t)L.C * (size_t)L.N);
  L.sel = off;
  off += align_up(8 * (size_t)nsamp);
  L.sel_off = off;
  off += align_up(4 * (size_t)(MX_B1 / L.L + 1));
  L.At = off;
  off += align_up(es * (size_t)m->R() * (size_t)L.Sp);
  L.b = off;
  off += align_up(es * (size_t)L.Sp);
  L.total = off;
  return L;
}

size_t mixed_workspace_bytes(const fst_model* m, int dtype, int64_t n, int64_t nsamp) {
  return mix_layout(m, dtype, n, nsamp).total;
}

template <typename T>
static void mixed_normal_equations_t(const fst_model* m, const DeviceModel& dm, int64_t n, const void* x,
                                     const void* y, const void* z, const void* v, int64_t nsamp, uint64_t seed,
                                     void* ws, double* G, double* h, void* stream) {
  const int dtype = sizeof(T) == 8 ? FST_F64 : FST_F32;
  const MixLayout L = mix_layout(m, dtype, n, nsamp);
  char* w = (char*)ws;
  T* U = (T*)(w + L.U);
  T* buf = (T*)(w + L.buf);
  int32_t* sel = (int32_t*)(w + L.sel);
  int32_t* sel_off = (int32_t*)(w + L.sel_off);
  T* At = (T*)(w + L.At);
  T* b = (T*)(w + L.b);
  const int64_t R = m->R(), N = L.N;

  // Algorithm 2 step 4 over the N mixed rows: S rows uniformly without replacement (stream
  // 2), listed per second-pass workgroup as (LDS element, sample position).  The normal
  // equations do not depend on the order of the rows, so when they are formed here the rows
  // of a workgroup take consecutive positions (its writes are coalesced); the rows handed to
  // the caller keep the order of the draw.
  {
    const bool grouped = G || h;
    std::vector<int64_t> idx((size_t)nsamp);
    sample_indices(seed, FST_STREAM_LS, N, nsamp, idx.data());
    const int nblk = MX_B1 / L.L;
    std::vector<int32_t> off((size_t)nblk + 1, 0), fill((size_t)nblk, 0), list((size_t)(2 * nsamp));
    for (int64_t q = 0; q < nsamp; ++q) ++off[(size_t)((idx[(size_t)q] % MX_B1) / L.L) + 1];
    for (int bk = 0; bk < nblk; ++bk) off[(size_t)bk + 1] += off[(size_t)bk];
    for (int64_t q = 0; q < nsamp; ++q) {
      const int64_t i = idx[(size_t)q];
      const int bk = (int)((i % MX_B1) / L.L);
      const int64_t e = (i / MX_B1) * L.L + (i % MX_B1 - (int64_t)bk * L.L);
      const int32_t t = off[(size_t)bk] + fill[(size_t)bk]++;
      list[(size_t)(2 * t)] = (int32_t)e;
      list[(size_t)(2 * t + 1)] = grouped ? t : (int32_t)q;
    }
    copy_h2d(sel, list.data(), sizeof(int32_t) * list.size(), stream);
    copy_h2d(sel_off, off.data(), sizeof(int32_t) * off.size(), stream);
  }
  // step 1: factor functions at every point
  launch_factor_eval(m, dm, dtype, n, x, y, z, nullptr, nullptr, n, U, nullptr, stream);
  // steps 2-4: signs, transform, sampled rows; whole (j1, j2) pairs per launch, then the values
  MixArgs<T> a;
  a.U = U;
  a.v = (const T*)v;
  a.n = n;
  a.N = N;
  a.R = R;
  a.r1 = m->rank[0];
  a.r2 = m->rank[1];
  a.r3 = m->rank[2];
  a.H = L.H;
  a.L = L.L;
  a.lgL = 0;
  while ((1 << a.lgL) < L.L) ++a.lgL;
  a.sign_state = seed * 256u + (uint64_t)kSignsStream;
  a.buf = buf;
  a.sel = sel;
  a.sel_off = sel_off;
  a.At = At;
  a.b = b;
  a.Sp = L.Sp;
  a.scale = (T)(1.0 / std::sqrt((double)N));
  const size_t lds_hi = sizeof(T) * (size_t)((int64_t)L.L << L.H);
  const unsigned lo_blocks = (unsigned)(N / MX_B1), hi_blocks = (unsigned)(MX_B1 / L.L);
  for (int64_t c0 = 0; c0 <= R; c0 += L.C) {
    const bool vals = c0 == R;
    const int64_t nc = vals ? 1 : std::min<int64_t>(L.C, R - c0);
    a.c0 = c0;
    a.values = vals ? 1 : 0;
    hipLaunchKernelGGL(k_mix_lo<T>, dim3(lo_blocks, (unsigned)(vals ? 1 : nc / a.r3)), dim3(MX_THREADS), 0,
                       S(stream), a);
    check_launch("k_mix_lo");
    hipLaunchKernelGGL(k_mix_hi<T>, dim3(hi_blocks, (unsigned)nc), dim3(MX_THREADS), lds_hi, S(stream), a);
    check_launch("k_mix_hi");
    if (!vals && c0 + L.C > R) c0 = R - L.C;   // next: the value column
  }
  if (L.Sp > nsamp) {
    const int64_t cnt = (R + 1) * (L.Sp - nsamp);
    hipLaunchKernelGGL(k_zero_tail<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, S(stream), At, b, R, nsamp,
                       L.Sp);
    check_launch("k_zero_tail");
  }
  // step 5: normal equations of the sampled mixed rows (the rows alone when G and h are NULL)
  if (G || h) dense_normal_equations(dtype, At, b, R, L.Sp, G, h, false, stream);
}

void mixed_rows(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z, const void* v,
                int64_t nsamp, uint64_t seed, void* ws, size_t ws_bytes, void* At, void* b, void* stream) {
  const MixLayout L = mix_layout(m, dtype, n, nsamp);
  mixed_normal_equations(m, dtype, n, x, y, z, v, nsamp, seed, ws, ws_bytes, nullptr, nullptr, stream);
  const size_t es = dtype == FST_F64 ? 8 : 4;
  if (At) copy_d2d(At, (char*)ws + L.At, es * (size_t)m->R() * (size_t)L.Sp, stream);
  if (b) copy_d2d(b, (char*)ws + L.b, es * (size_t)L.Sp, stream);
}

void mixed_normal_equations(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z,
                            const void* v, int64_t nsamp, uint64_t seed, void* ws, size_t ws_bytes, double* G,
                            double* h, void* stream) {
  const MixLayout L = mix_layout(m, dtype, n, nsamp);
  if (ws_bytes < L.total) fail(FST_E_NOMEM, "mixed rows: workspace too small");
  if (L.N > (int64_t(1) << MX_MAX_LOG2N)) fail(FST_E_UNSUPPORTED, "mixed rows: more than 2^23 points");
  if ((int64_t)m->R() * L.Sp >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "mixed rows: A^T too large");
  const DeviceModel& dm = device_model(m, dtype);
  if (dtype == FST_F64)
    mixed_normal_equations_t<double>(m, dm, n, x, y, z, v, nsamp, seed, ws, G, h, stream);
  else
    mixed_normal_equations_t<float>(m, dm, n, x, y, z, v, nsamp, seed, ws, G, h, stream);
}

// ------------------------------------------------------------------------------ leverage
// Leverage of sampled rows (Sec. 5): l_q = a_q^T (A^T A)^-1 a_q = ||y||^2 with L y = a_q, L the
// Cholesky factor of A^T A (fst_cholesky storage; a skipped column has L_jj = +inf, so y_j = 0).
// One wave per row: forward substitution, each step a wave-wide dot product over the solved
// entries, kept in LDS.
constexpr int LV_MAX_WAVES = 4;
constexpr size_t LV_LDS_BYTES = 65536;
__global__ __launch_bounds__(64 * LV_MAX_WAVES) void k_leverage(int64_t R, int64_t Sp, int64_t mrows,
                                                                const double* At, const double* L, double* out) {
  extern __shared__ double lv_y[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * waves + wave;
  if (q >= mrows) return;
  double* y = lv_y + (int64_t)wave * R;
  double ss = 0.0;
  for (int64_t j = 0; j < R; ++j) {
    const double* Lj = L + j * R;
    double part = 0.0;
    for (int64_t k = lane; k < j; k += 64) part += Lj[k] * y[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    const double yj = (At[j * Sp + q] - part) / Lj[j];
    if (lane == 0) y[j] = yj;
    ss += yj * yj;
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the LDS store is done before the next reads
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0) out[q] = ss;
}

void leverage(int64_t R, int64_t Sp, int64_t mrows, const double* At, const double* L, double* out, void* stream) {
  if (R < 1 || R > 8192 || mrows < 0 || Sp < mrows) fail(FST_E_INVAL, "leverage: need 1 <= R <= 8192, mrows <= Sp");
  if (mrows == 0) return;
  int waves = (int)(LV_LDS_BYTES / (sizeof(double) * (size_t)R));
  waves = waves > LV_MAX_WAVES ? LV_MAX_WAVES : waves;
  const int64_t blocks = (mrows + waves - 1) / waves;
  hipLaunchKernelGGL(k_leverage, dim3((unsigned)blocks), dim3(64 * waves), sizeof(double) * waves * (size_t)R,
                     S(stream), R, Sp, mrows, At, L, out);
  check_launch("k_leverage");
}

}  // namespace fst
