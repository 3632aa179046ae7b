// Split 16-bit Gram of the precision form for gfx950: the normal equations of Algorithm 2
// step 5 (eq. (6)), G = A^T A, formed on 16-bit MFMA from design rows split into NT 16-bit
// terms, A = A_0 + A_1 + ... + A_{NT-1}, each term the rounding of what the earlier ones left:
//
//   FP16 x 2  entries scaled by a power of two     G ~ (A_0 + A_1)^T (A_0 + A_1), 4 products
//   BF16 x 2                                       G ~ (A_0 + A_1)^T (A_0 + A_1), 4 products
//   BF16 x 3                                       G ~ sum over a + b <= 2 of A_a^T A_b, 6 products
//
// The two-term forms keep the whole square, so G is the Gram of the split rows (positive
// semidefinite); leaving out A_1^T A_1 would bias the diagonal by about 2^-24 of each entry,
// as large as the smallest eigenvalues of ill-conditioned systems, and slow the refinement
// that follows.  In the three-term form the products left out are below the FP32 rounding of
// the entries.  FP16 x 2 carries 22 significant bits, BF16 x 2 16 and BF16 x 3 24.
//
//   k_design_rows_split  A^T in NT planes, 16-bit, chunk-major: plane[(c R + j) 64 + k] holds
//                        row 64 c + k of design column j (64-row chunks of one column are
//                        contiguous, so a Gram tile's chunk is 128 runs of 128 bytes)
//   k_gram_split         lower-triangle 128 x 128 tiles, sixteen waves of 32 x 32 (2 x 2 MFMA
//                        16x16x32 blocks); KC rows of the tile's 256 design columns copied
//                        from HBM straight into double-buffered LDS; the leading product and
//                        the others summed in separate FP32 accumulators, folded into FP64
//                        every 512 rows (16 MFMA additions to the leading sum, as in the FP32
//                        Gram)
//
// Tiles are handed out in groups of GR x (32 / GR) (GR row blocks, 32 / GR column blocks), one
// group per XCD per round of 256 workgroups, so the 32 workgroups that share an XCD's L2 at a
// time read GR + 32 / GR blocks of design columns instead of up to 64 (12 for 4 x 8).  The
// group shape, and for the batched launch the choice between these groups and plain triangle
// order, is picked per shape by a small autotuner: every candidate computes the same G bit for
// bit (only the tile-to-workgroup order differs), so the first call of a shape times each
// candidate on the caller's data and keeps the fastest, in memory and, when the environment
// names a file in FST_TUNE_FILE, in that JSON object keyed by shape for later processes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

constexpr int SR_THREADS = 256, SR_VW = 8;
constexpr int64_t SR_SUPER = 4;

struct SplitRowsArgs {
  const float* U;       // [sum r][M] factor values of the sampled rows (feature-major)
  void* plane[3];       // NT planes, chunk-major, R x Sp entries each
  int64_t M, Sp, R;
  int32_t r1, r2, r3;
  float scale;          // power of two applied to every entry (FP16 range), 1 for BF16
};

// entry ((u1 u2) scale) u3 formed in FP32; term t is the rounding of e - (A_0 + .. + A_{t-1})
// (each subtraction exact in FP32); 8 consecutive rows per thread, one 16-byte store per term
// and design column; rows M .. Sp-1 are zero.  With the FP16 scale (entries up to 2^15) the
// second FP16 term is a normal number for every entry above 2^-3, i.e. within 18 binades of
// the largest; below that it is subnormal (absolute precision 2^-24, kept by the MFMA).
template <typename H, int NT>
__global__ __launch_bounds__(SR_THREADS) void k_design_rows_split(SplitRowsArgs a, int64_t sb0) {
  typedef H HV __attribute__((ext_vector_type(8)));
  typedef float F4 __attribute__((ext_vector_type(4)));
  const int64_t P = (int64_t)a.r1 * a.r2, nb = (a.Sp + SR_THREADS * SR_VW - 1) / (SR_THREADS * SR_VW);
  const int64_t sb = sb0 + (int64_t)blockIdx.x / (P * SR_SUPER), rem = (int64_t)blockIdx.x % (P * SR_SUPER);
  const int64_t w = min(SR_SUPER, nb - sb * SR_SUPER);
  if (w <= 0) return;
  const int64_t pr = rem / w, cb = sb * SR_SUPER + rem % w;
  if (pr >= P) return;
  const int64_t q = (cb * SR_THREADS + threadIdx.x) * SR_VW;
  if (q >= a.Sp) return;
  const int j1 = (int)(pr / a.r2), j2 = (int)(pr - (int64_t)j1 * a.r2);
  const float* U1 = a.U + (int64_t)j1 * a.M;
  const float* U2 = a.U + (int64_t)(a.r1 + j2) * a.M;
  const float* U3 = a.U + (int64_t)(a.r1 + a.r2) * a.M;
  const bool vec = q + SR_VW <= a.M && a.M % 4 == 0;
  float p12[SR_VW];
  if (vec) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const F4 x = *reinterpret_cast<const F4*>(U1 + q + 4 * h), y = *reinterpret_cast<const F4*>(U2 + q + 4 * h);
#pragma unroll
      for (int e = 0; e < 4; ++e) p12[4 * h + e] = x[e] * y[e] * a.scale;
    }
  } else {
#pragma unroll
    for (int e = 0; e < SR_VW; ++e) {
      const int64_t c = min(q + e, a.M - 1);
      p12[e] = q + e < a.M ? U1[c] * U2[c] * a.scale : 0.0f;
    }
  }
  // chunk-major offset of (column pr r3, row q); q is a multiple of 8, so the 8 rows share a chunk
  const int64_t base = ((q >> 6) * a.R + pr * a.r3) * 64 + (q & 63);
  for (int j3 = 0; j3 < a.r3; ++j3) {
    const float* u3 = U3 + (int64_t)j3 * a.M;
    float e[SR_VW];
    if (vec) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const F4 z = *reinterpret_cast<const F4*>(u3 + q + 4 * h);
#pragma unroll
        for (int i = 0; i < 4; ++i) e[4 * h + i] = p12[4 * h + i] * z[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < SR_VW; ++i) e[i] = p12[i] * u3[min(q + i, a.M - 1)];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      HV hv;
#pragma unroll
      for (int i = 0; i < SR_VW; ++i) {
        hv[i] = (H)e[i];
        e[i] -= (float)hv[i];
      }
      *reinterpret_cast<HV*>(reinterpret_cast<H*>(a.plane[t]) + base + (int64_t)j3 * 64) = hv;
    }
  }
}

constexpr int SG_TILE = 128, SG_LK = 64;

struct SplitGramArgs {
  const void* plane0;     // NT planes, chunk-major (SG_LK rows per chunk), R x Sp entries each,
  int64_t plane_stride;   // plane t at plane0 + t plane_stride entries
  double* G;              // R x R, lower triangle written
  int64_t R, Sp;
  int32_t nt;             // tiles per side
  int32_t fold;           // chunks between folds of the FP32 sums into FP64
  double unscale;         // 1 / scale^2
  int32_t accumulate;
};

// The products t_a^T t_b summed for each split: (a, b) and the FP32 accumulator they go to.
// Accumulator 0 holds the leading product alone; accumulator 1 the products that are 2^-8 or
// less of it (their own rounding does not matter); both are folded into FP64.  A product left
// out must be a cross term of random sign: a left-out square t_a^T t_a is positive
// semidefinite and would shift the Gram systematically (at 2^-24 of the diagonal for FP16
// terms, comparable to the smallest eigenvalue of a Gram with condition number 1e7-1e8).
struct SchemeF16x2 {      // FP16, two terms: the whole square of the two-term representation
  typedef _Float16 H;
  static constexpr int NT = 2, N = 4, NACC = 2, KC = 64;
  static constexpr int a[4] = {0, 0, 1, 1}, b[4] = {0, 1, 0, 1}, c[4] = {0, 1, 1, 1};
};
struct SchemeBF16x2 {     // BF16, two terms: the whole square
  typedef __bf16 H;
  static constexpr int NT = 2, N = 4, NACC = 2, KC = 64;
  static constexpr int a[4] = {0, 0, 1, 1}, b[4] = {0, 1, 0, 1}, c[4] = {0, 1, 1, 1};
};
struct SchemeBF16x3 {     // BF16, three terms: products of order <= 2 (order-3 cross terms left out)
  typedef __bf16 H;
  static constexpr int NT = 3, N = 6, NACC = 2, KC = 32;
  static constexpr int a[6] = {0, 0, 1, 0, 1, 2}, b[6] = {0, 1, 0, 2, 1, 0}, c[6] = {0, 1, 1, 1, 1, 1};
};

// LDS layout of one staged chunk: [term][256 rows][KC entries] without padding; the 16-byte
// piece p of row r sits at position p ^ swizzle(r), so that the 16 rows a lane group reads
// at one piece position fall in distinct banks (for 32 and for 64 banks of 4 bytes).
template <int PPR> __device__ __forceinline__ int split_swizzle(int r);
template <> __device__ __forceinline__ int split_swizzle<8>(int r) { return (r ^ (r >> 3)) & 7; }
template <> __device__ __forceinline__ int split_swizzle<4>(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

constexpr int SG_THREADS = 1024;   // sixteen waves of 32 x 32 (2 x 2 MFMA blocks of 16 x 16)

// One workgroup per lower-triangle tile.  Each chunk of KC rows of the tile's 256 design
// columns (its row block, then its column block) is copied from HBM straight into LDS by
// global_load_lds (1 KB per wave instruction, no register staging), one chunk ahead of the
// MFMAs, into two buffers that are separate arrays (so the compiler can tell the buffer
// being filled from the one being read and does not wait for the copy before reading).
// Rows past R are copied from row R - 1 (real memory); their products land only in entries
// that are never written.
// One 128 x 128 tile (rows r0.., columns c0..) of G = A^T A from the split planes.
struct SplitTile {
  const void* plane0;
  int64_t plane_stride;
  double* G;
  int64_t R, Sp, r0, c0;
  int32_t fold, accumulate;
  double unscale;
};

template <class SC>
__device__ __forceinline__ void split_tile(const SplitTile& a,
                                           typename SC::H (*bufA)[2 * SG_TILE][SC::KC],
                                           typename SC::H (*bufB)[2 * SG_TILE][SC::KC]) {
  typedef typename SC::H H;
  typedef typename Mfma16<H>::V8 V8;
  constexpr int NT = SC::NT, KC = SC::KC, NACC = SC::NACC;
  constexpr int PPR = KC / 8;                  // 16-byte pieces per row
  constexpr int RPI = 64 / PPR;                // rows per 1 KB copy instruction
  constexpr int INS = NT * 256 / RPI / 16;     // copy instructions per wave per chunk
  static_assert(INS * RPI * 16 == NT * 256, "a chunk must split evenly over the waves");
  static_assert(SG_LK % KC == 0 && KC % 32 == 0, "a chunk must be whole MFMA steps inside a layout chunk");
  const int64_t r0 = a.r0, c0 = a.c0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wrow = (wave >> 2) * 32, wcol = (wave & 3) * 32, li = lane & 15, g = lane >> 4;
  const bool active = c0 + wcol <= r0 + wrow + 31;

  // copy instruction i of this wave: term t, rows RPI q .. RPI q + RPI - 1 of the staged 256;
  // lane l brings piece (l % PPR) ^ swizzle(row) of row RPI q + l / PPR
  int64_t src[INS];    // entry offsets within a layout chunk
#pragma unroll
  for (int i = 0; i < INS; ++i) {
    const int blk = wave * INS + i, q = blk % (256 / RPI);
    const int rl = RPI * q + lane / PPR;
    const int pc = (lane % PPR) ^ split_swizzle<PPR>(rl);
    int64_t gr = rl < SG_TILE ? r0 + rl : c0 + (rl - SG_TILE);
    gr = gr < a.R ? gr : a.R - 1;
    src[i] = gr * SG_LK + pc * 8;
  }
  auto copy = [&](H (*buf)[2 * SG_TILE][KC], int64_t ch) {
    const int64_t base = (ch * KC / SG_LK) * a.R * SG_LK + (ch * KC) % SG_LK;
#pragma unroll
    for (int i = 0; i < INS; ++i) {
      const int blk = wave * INS + i, t = blk / (256 / RPI), q = blk % (256 / RPI);
      const H* p = reinterpret_cast<const H*>(a.plane0) + t * a.plane_stride + base + src[i];
      __builtin_amdgcn_global_load_lds((const void*)p, (__attribute__((address_space(3))) void*)&buf[t][RPI * q][0],
                                       16, 0, 0);
    }
  };

  floatx4 acc[NACC][2][2];
  double dacc[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int c = 0; c < NACC; ++c) acc[c][x][y] = floatx4{0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[x][y][v] = 0.0;
    }
  auto fold = [&]() {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int c = 0; c < NACC; ++c) {
#pragma unroll
          for (int v = 0; v < 4; ++v) dacc[x][y][v] += (double)acc[c][x][y][v];
          acc[c][x][y] = floatx4{0, 0, 0, 0};
        }
  };
  auto compute = [&](H (*buf)[2 * SG_TILE][KC]) {
#pragma unroll
    for (int ks = 0; ks < KC / 32; ++ks) {
      const int pc = ks * 4 + g;
      V8 av[NT][2], bv[NT][2];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int ra = wrow + x * 16 + li, rb = SG_TILE + wcol + x * 16 + li;
          av[t][x] = *reinterpret_cast<const V8*>(&buf[t][ra][(pc ^ split_swizzle<PPR>(ra)) * 8]);
          bv[t][x] = *reinterpret_cast<const V8*>(&buf[t][rb][(pc ^ split_swizzle<PPR>(rb)) * 8]);
        }
#pragma unroll
      for (int pp = 0; pp < SC::N; ++pp)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[SC::c[pp]][x][y] = Mfma16<H>::mfma(av[SC::a[pp]][x], bv[SC::b[pp]][y], acc[SC::c[pp]][x][y]);
    }
  };

  const int64_t nch = a.Sp / KC;
  int since = 0;
  auto step = [&](H (*cur)[2 * SG_TILE][KC], H (*nxt)[2 * SG_TILE][KC], int64_t ch) {
    if (ch + 1 < nch) copy(nxt, ch + 1);
    if (active) {
      compute(cur);
      if (++since == a.fold) {
        fold();
        since = 0;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);   // this wave's copies of the next chunk have landed
    __syncthreads();                 // everyone's, and nobody reads `cur` any more
  };
  copy(bufA, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t ch = 0; ch < nch; ch += 2) {
    step(bufA, bufB, ch);
    if (ch + 1 < nch) step(bufB, bufA, ch + 1);
  }
  if (!active) return;
  fold();
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + wrow + x * 16 + MfmaAcc<float>::row(g, v);
        const int64_t col = c0 + wcol + y * 16 + li;
        if (row < a.R && col <= row) {
          const double val = dacc[x][y][v] * a.unscale;
          a.G[row * a.R + col] = a.accumulate ? a.G[row * a.R + col] + val : val;
        }
      }
}


// Workgroup slot `local` (counted from a multiple of 256) -> lower-triangle tile (bi, bj) of an
// nt x nt tile grid in GR x (32 / GR) groups: round local / 256, XCD local % 8, slot
// (local % 256) / 8 of the group's 32.  False for slots past the triangle.
__device__ __forceinline__ bool group_tile(int64_t local, int64_t nt, int GR, int64_t& bi, int64_t& bj) {
  const int GC = 32 / GR;
  int64_t rest = (local >> 8) * 8 + (local & 7);
  const int slot = (int)((local & 255) >> 3);
  int64_t BI = 0;
  for (;; ++BI) {
    if (GR * BI >= nt) return false;
    const int64_t ngr = min(GR * BI + GR - 1, nt - 1) / GC + 1;   // groups in group row BI
    if (rest < ngr) break;
    rest -= ngr;
  }
  bi = GR * BI + slot / GC;
  bj = GC * rest + slot % GC;
  return bi < nt && bj <= bi;
}
// workgroup slots of that order: 256 per round of eight groups
static int64_t group_slots(int64_t nt, int GR) {
  const int GC = 32 / GR;
  int64_t groups = 0;
  for (int64_t BI = 0; GR * BI < nt; ++BI) groups += std::min(GR * BI + GR - 1, nt - 1) / GC + 1;
  return (groups + 7) / 8 * 256;
}

template <class SC, int GR>
__global__ __launch_bounds__(SG_THREADS) void k_gram_split(SplitGramArgs a) {
  __shared__ __align__(16) typename SC::H bufA[SC::NT][2 * SG_TILE][SC::KC];
  __shared__ __align__(16) typename SC::H bufB[SC::NT][2 * SG_TILE][SC::KC];
  int64_t bi, bj;
  if (!group_tile(blockIdx.x, a.nt, GR, bi, bj)) return;
  SplitTile t;
  t.plane0 = a.plane0;
  t.plane_stride = a.plane_stride;
  t.G = a.G;
  t.R = a.R;
  t.Sp = a.Sp;
  t.r0 = bi * SG_TILE;
  t.c0 = bj * SG_TILE;
  t.fold = a.fold;
  t.accumulate = a.accumulate;
  t.unscale = a.unscale;
  split_tile<SC>(t, bufA, bufB);
}

struct SplitVar {
  const void* plane0;
  int64_t plane_stride;
  double* G;
  int64_t R, Sp, tile0;
  double unscale;
};

// GR = 0: each variable's tiles in triangle order; GR > 0: in the groups above, each variable's
// slots starting at a multiple of 256 (tile0), so the slot's XCD is that of the workgroup
template <class SC, int GR>
__global__ __launch_bounds__(SG_THREADS) void k_gram_split_batched(const SplitVar* __restrict__ vars, int nvars,
                                                                   int32_t fold) {
  __shared__ __align__(16) typename SC::H bufA[SC::NT][2 * SG_TILE][SC::KC];
  __shared__ __align__(16) typename SC::H bufB[SC::NT][2 * SG_TILE][SC::KC];
  const int64_t tt = blockIdx.x;
  int lo = 0, hi = nvars - 1;   // last variable with tile0 <= tt
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (vars[mid].tile0 <= tt) lo = mid; else hi = mid - 1;
  }
  const SplitVar& v = vars[lo];
  int64_t bi, bj;
  if (GR == 0) {
    tri_tile(tt - v.tile0, bi, bj);
  } else {
    const int64_t nt = (v.R + SG_TILE - 1) / SG_TILE;
    if (!group_tile(tt - v.tile0, nt, GR, bi, bj)) return;
  }
  SplitTile t;
  t.plane0 = v.plane0;
  t.plane_stride = v.plane_stride;
  t.G = v.G;
  t.R = v.R;
  t.Sp = v.Sp;
  t.r0 = bi * SG_TILE;
  t.c0 = bj * SG_TILE;
  t.fold = fold;
  t.accumulate = 0;
  t.unscale = v.unscale;
  split_tile<SC>(t, bufA, bufB);
}

// ------------------------------------------------------------------------------ tile-order autotuner
// Candidates: single Gram, groups of 2 x 16, 4 x 8, 8 x 4 (index 0, 1, 2); batched Gram, triangle
// order or groups of 4 x 8, 8 x 4 (index 0, 1, 2).  Untimed calls (under graph capture, or
// accumulating into G) take 8 x 4, the fastest on a 13824-column Gram of 200k rows.  Keys: kind,
// precision, tile-grid size (log2 buckets for the batched launch), padded row count bucket,
// architecture.
static const int kSingleGR[3] = {2, 4, 8};
static const int kBatchedGR[3] = {0, 4, 8};
constexpr int kDefaultGR = 2;   // index of 8 x 4 in both tables
struct SplitTuner {
  std::mutex mu;
  bool loaded = false;
  std::string path;   // the file the choices were loaded from ("" for none)
  std::map<std::string, int> best;
};
static SplitTuner& tuner() {
  static SplitTuner t;
  return t;
}
static const char* tune_file() {
  const char* f = std::getenv("FST_TUNE_FILE");
  return (f && *f) ? f : nullptr;
}
// the file is a flat JSON object {"key": index, ...} written by tuner_store
static void tuner_load_locked(SplitTuner& t) {
  const char* path = tune_file();
  const std::string cur = path ? path : "";
  if (t.loaded && cur == t.path) return;
  // first use, or FST_TUNE_FILE names another file now: start from that file's choices
  t.loaded = true;
  t.path = cur;
  t.best.clear();
  if (!path) return;
  FILE* f = std::fopen(path, "rb");
  if (!f) return;
  std::string txt;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, got);
  std::fclose(f);
  size_t pos = 0;
  for (;;) {
    const size_t k0 = txt.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = txt.find('"', k0 + 1);
    if (k1 == std::string::npos) break;
    const size_t colon = txt.find(':', k1);
    if (colon == std::string::npos) break;
    char* end = nullptr;
    const long val = std::strtol(txt.c_str() + colon + 1, &end, 10);
    if (end == txt.c_str() + colon + 1) break;
    t.best[txt.substr(k0 + 1, k1 - k0 - 1)] = (int)val;
    pos = (size_t)(end - txt.c_str());
  }
}
static void tuner_save_locked(const SplitTuner& t) {
  const char* path = tune_file();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  std::fputs("{\n", f);
  size_t i = 0;
  for (const auto& kv : t.best)
    std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < t.best.size() ? "," : "");
  std::fputs("}\n", f);
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}
static int tuner_lookup(const std::string& key) {
  SplitTuner& t = tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  tuner_load_locked(t);
  auto it = t.best.find(key);
  return it == t.best.end() ? -1 : it->second;
}
static void tuner_store(const std::string& key, int v) {
  SplitTuner& t = tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  tuner_load_locked(t);
  t.best[key] = v;
  tuner_save_locked(t);
}
static std::string arch_name() {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, current_device()) != hipSuccess) return "gfx";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}
static int log2_bucket(int64_t x) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= x) ++b;
  return b;
}
// may the tuner time candidates on this stream (not while a graph is being captured)
static bool can_time(void* stream) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(S(stream), &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusNone;
}
// runs candidate `run(i)` for i < n once each, timed with events on the stream; returns the fastest
template <class F>
static int time_candidates(int n, F run, void* stream) {
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "hipEventCreate");
  check_hip(hipEventCreate(&e1), "hipEventCreate");
  int best = 0;
  float best_ms = 0.0f;
  for (int i = 0; i < n; ++i) {
    check_hip(hipEventRecord(e0, S(stream)), "hipEventRecord");
    run(i);
    check_hip(hipEventRecord(e1, S(stream)), "hipEventRecord");
    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.0f;
    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (i == 0 || ms < best_ms) {
      best = i;
      best_ms = ms;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return best;
}

static std::string split_key(int batched, int gram_prec, int64_t tiles_or_nt, int64_t Sp) {
  return std::string(batched ? "split_batched" : "split") + ":" + std::to_string(gram_prec) + ":" +
         (batched ? "tiles2^" + std::to_string(log2_bucket(tiles_or_nt)) : "nt" + std::to_string(tiles_or_nt)) +
         ":rows2^" + std::to_string(log2_bucket(Sp)) + ":" + arch_name();
}

int split_terms(int gram_prec) {
  switch (gram_prec) {
    case FST_GRAM_F16X2: return 2;
    case FST_GRAM_BF16X2: return 2;
    case FST_GRAM_BF16X3: return 3;
    default: return 0;
  }
}

int64_t split_rows_padded(int64_t mrows) { return (mrows + SG_LK - 1) / SG_LK * SG_LK; }

size_t split_rows_bytes(const fst_model* m, int gram_prec, int64_t mrows) {
  const int nt = split_terms(gram_prec);
  return (size_t)nt * align_up(2 * (size_t)m->R() * (size_t)split_rows_padded(mrows));
}

// FP16 terms: every entry scaled into [-2^15, 2^15] (the per-mode maxima give a power of two
// that brings the entries into [-1, 1]); products of two terms stay below 2^30 and the sums of
// one fold interval below 2^40, far inside FP32.
constexpr float kSplitF16Headroom = 32768.0f;

// the row planes of one variable (FP16: scaled by `scale`) into `rows`
static void split_rows(const fst_model* m, int gram_prec, int64_t mrows, const float* U, void* rows, float scale,
                       void* plane_out[3], void* stream) {
  const int NT = split_terms(gram_prec);
  const int64_t R = m->R(), Sp = split_rows_padded(mrows);
  const size_t pb = align_up(2 * (size_t)R * (size_t)Sp);
  SplitRowsArgs ra;
  ra.U = U;
  for (int t = 0; t < 3; ++t) ra.plane[t] = plane_out[t] = t < NT ? (char*)rows + t * pb : nullptr;
  ra.M = mrows;
  ra.Sp = Sp;
  ra.R = R;
  ra.r1 = m->rank[0];
  ra.r2 = m->rank[1];
  ra.r3 = m->rank[2];
  ra.scale = scale;
  const int64_t P = (int64_t)ra.r1 * ra.r2, nb = (Sp + SR_THREADS * SR_VW - 1) / (SR_THREADS * SR_VW);
  const int64_t nsb = (nb + SR_SUPER - 1) / SR_SUPER, per = std::max<int64_t>(1, (int64_t(1) << 30) / (P * SR_SUPER));
  for (int64_t sb0 = 0; sb0 < nsb; sb0 += per) {
    const dim3 grid((unsigned)(std::min(per, nsb - sb0) * P * SR_SUPER));
    if (gram_prec == FST_GRAM_F16X2)
      hipLaunchKernelGGL((k_design_rows_split<_Float16, 2>), grid, dim3(SR_THREADS), 0, S(stream), ra, sb0);
    else if (gram_prec == FST_GRAM_BF16X2)
      hipLaunchKernelGGL((k_design_rows_split<__bf16, 2>), grid, dim3(SR_THREADS), 0, S(stream), ra, sb0);
    else
      hipLaunchKernelGGL((k_design_rows_split<__bf16, 3>), grid, dim3(SR_THREADS), 0, S(stream), ra, sb0);
    check_launch("k_design_rows_split");
  }
}

static void check_split(const fst_model* m, int gram_prec, int64_t mrows) {
  if (split_terms(gram_prec) == 0) fail(FST_E_INVAL, "split Gram: not a split precision");
  if (m->d != 3 || mrows < 1) fail(FST_E_INVAL, "split Gram: 3-way model and mrows >= 1 needed");
  if (m->R() * split_rows_padded(mrows) >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "split Gram: A^T too large");
  if (m->R() * SG_LK >= (int64_t(1) << 31)) fail(FST_E_UNSUPPORTED, "split Gram: R too large");
}

static float split_scale(const fst_model* m, int gram_prec, int64_t mrows, const float* U, void* scratch,
                         void* stream) {
  return gram_prec == FST_GRAM_F16X2 ? f16_row_scale(m, mrows, U, scratch, stream) * kSplitF16Headroom : 1.0f;
}

void gram_split(const fst_model* m, int gram_prec, int64_t mrows, const float* U, double* G, void* rows,
                size_t rows_bytes, void* scratch, void* stream) {
  check_split(m, gram_prec, mrows);
  if (rows_bytes < split_rows_bytes(m, gram_prec, mrows)) fail(FST_E_NOMEM, "split Gram: row planes do not fit");
  const float scale = split_scale(m, gram_prec, mrows, U, scratch, stream);
  void* plane[3];
  split_rows(m, gram_prec, mrows, U, rows, scale, plane, stream);
  gram_split_rows(gram_prec, plane, m->R(), split_rows_padded(mrows), G, 1.0 / ((double)scale * (double)scale),
                  false, stream);
}

template <class SC>
static void launch_split_batched(const SplitVar* vars, int nvars, int64_t slots, int order, void* stream) {
  const dim3 grid((unsigned)slots), block(SG_THREADS);
  const int32_t fold = 512 / SC::KC;
  if (kBatchedGR[order] == 0)
    hipLaunchKernelGGL((k_gram_split_batched<SC, 0>), grid, block, 0, S(stream), vars, nvars, fold);
  else if (kBatchedGR[order] == 4)
    hipLaunchKernelGGL((k_gram_split_batched<SC, 4>), grid, block, 0, S(stream), vars, nvars, fold);
  else
    hipLaunchKernelGGL((k_gram_split_batched<SC, 8>), grid, block, 0, S(stream), vars, nvars, fold);
  check_launch("k_gram_split_batched");
}
static void launch_split_batched_prec(int gram_prec, const SplitVar* vars, int nvars, int64_t slots, int order,
                                      void* stream) {
  if (gram_prec == FST_GRAM_F16X2)
    launch_split_batched<SchemeF16x2>(vars, nvars, slots, order, stream);
  else if (gram_prec == FST_GRAM_BF16X2)
    launch_split_batched<SchemeBF16x2>(vars, nvars, slots, order, stream);
  else
    launch_split_batched<SchemeBF16x3>(vars, nvars, slots, order, stream);
}

size_t gram_split_batched_min_bytes(const std::vector<const fst_model*>& models, int gram_prec, int64_t mrows) {
  size_t mx = 0;
  for (const fst_model* m : models) mx = std::max(mx, split_rows_bytes(m, gram_prec, mrows));
  return 4096 + align_up(sizeof(SplitVar) * models.size()) + mx;
}

// Gram matrices of several variables: row planes of as many variables as fit in the
// workspace (largest R first), then one launch over all their tiles; repeated until every
// variable is done.  ws: 4096 bytes of scratch, the variable table, then the planes.
void gram_split_batched(const std::vector<const fst_model*>& models, const std::vector<const void*>& U,
                        int64_t mrows, const std::vector<double*>& G, int gram_prec, void* ws, size_t ws_bytes,
                        void* stream) {
  const size_t nv = models.size();
  for (const fst_model* m : models) check_split(m, gram_prec, mrows);
  if (ws_bytes < gram_split_batched_min_bytes(models, gram_prec, mrows))
    fail(FST_E_NOMEM, "batched split Gram: workspace too small");
  const size_t tab = align_up(sizeof(SplitVar) * nv);
  SplitVar* d_vars = (SplitVar*)((char*)ws + 4096);
  char* planes = (char*)ws + 4096 + tab;
  const size_t budget = ws_bytes - 4096 - tab;
  std::vector<size_t> order(nv);
  for (size_t i = 0; i < nv; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return models[a]->R() > models[b]->R(); });
  const int64_t Sp = split_rows_padded(mrows);
  size_t i0 = 0;
  while (i0 < nv) {
    std::vector<SplitVar> vars;
    size_t used = 0;
    int64_t tiles = 0;
    size_t i = i0;
    for (; i < nv; ++i) {
      const fst_model* m = models[order[i]];
      const size_t need = split_rows_bytes(m, gram_prec, mrows);
      if (used + need > budget) break;
      const float scale = split_scale(m, gram_prec, mrows, (const float*)U[order[i]], ws, stream);
      void* plane[3];
      split_rows(m, gram_prec, mrows, (const float*)U[order[i]], planes + used, scale, plane, stream);
      SplitVar v;
      v.plane0 = plane[0];
      v.plane_stride = (int64_t)(((char*)plane[1] - (char*)plane[0]) / 2);
      v.G = G[order[i]];
      v.R = m->R();
      v.Sp = Sp;
      v.tile0 = 0;
      v.unscale = 1.0 / ((double)scale * (double)scale);
      const int64_t nt = (v.R + SG_TILE - 1) / SG_TILE;
      tiles += nt * (nt + 1) / 2;
      vars.push_back(v);
      used += need;
    }
    // the variables' first workgroup slots for tile order `o` (group orders start each variable
    // at a multiple of 256), uploaded; returns the launch size
    auto table = [&](int o) {
      int64_t slots = 0;
      for (SplitVar& v : vars) {
        const int64_t nt = (v.R + SG_TILE - 1) / SG_TILE;
        v.tile0 = slots;
        slots += kBatchedGR[o] == 0 ? nt * (nt + 1) / 2 : group_slots(nt, kBatchedGR[o]);
      }
      if (slots >= (int64_t(1) << 31)) fail(FST_E_UNSUPPORTED, "batched split Gram: too many tiles");
      copy_h2d(d_vars, vars.data(), sizeof(SplitVar) * vars.size(), stream);
      return slots;
    };
    auto run = [&](int o) {
      const int64_t slots = table(o);
      launch_split_batched_prec(gram_prec, d_vars, (int)vars.size(), slots, o, stream);
    };
    const std::string key = split_key(1, gram_prec, tiles, Sp);
    const int known = tuner_lookup(key);
    if (known >= 0 && known < 3) {
      run(known);
    } else if (can_time(stream)) {
      // every candidate writes the same G bit for bit, so the last one timed leaves the result
      tuner_store(key, time_candidates(3, run, stream));
    } else {
      run(kDefaultGR);
    }
    stream_sync(stream);   // the planes and the table are reused by the next group
    i0 = i;
  }
}

template <class SC>
static void launch_split_single(int GR, dim3 grid, const SplitGramArgs& ga, void* stream) {
  if (GR == 2)
    hipLaunchKernelGGL((k_gram_split<SC, 2>), grid, dim3(SG_THREADS), 0, S(stream), ga);
  else if (GR == 4)
    hipLaunchKernelGGL((k_gram_split<SC, 4>), grid, dim3(SG_THREADS), 0, S(stream), ga);
  else
    hipLaunchKernelGGL((k_gram_split<SC, 8>), grid, dim3(SG_THREADS), 0, S(stream), ga);
}

void gram_split_rows(int gram_prec, void* const* plane, int64_t R, int64_t Sp, double* G, double unscale,
                     bool accumulate, void* stream) {
  const int NT = split_terms(gram_prec);
  if (NT == 0) fail(FST_E_INVAL, "split Gram: not a split precision");
  if (Sp < SG_LK || Sp % SG_LK != 0) fail(FST_E_INVAL, "split Gram: row count must be a multiple of 64");
  SplitGramArgs ga;
  ga.plane0 = plane[0];
  ga.plane_stride = (int64_t)(((char*)plane[1] - (char*)plane[0]) / 2);
  for (int t = 1; t < NT; ++t)
    if ((char*)plane[t] - (char*)plane[0] != (ptrdiff_t)(2 * t * ga.plane_stride))
      fail(FST_E_INVAL, "split Gram: planes must be equally spaced");
  ga.G = G;
  ga.R = R;
  ga.Sp = Sp;
  const int64_t nt = (R + SG_TILE - 1) / SG_TILE;
  if (nt > (int64_t(1) << 20) || R * SG_LK >= (int64_t(1) << 31)) fail(FST_E_UNSUPPORTED, "split Gram: R too large");
  ga.nt = (int32_t)nt;
  ga.unscale = unscale;
  ga.accumulate = accumulate ? 1 : 0;
  // FP32 sums over 512 rows (16 MFMA accumulations into the leading sum) before each fold
  ga.fold = 512 / (NT == 3 ? SchemeBF16x3::KC : SchemeF16x2::KC);
  auto run = [&](int c) {
    const int GR = kSingleGR[c];
    const int64_t slots = group_slots(nt, GR);
    if (slots >= (int64_t(1) << 31)) fail(FST_E_UNSUPPORTED, "split Gram: too many tiles");
    const dim3 grid((unsigned)slots);
    if (gram_prec == FST_GRAM_F16X2) launch_split_single<SchemeF16x2>(GR, grid, ga, stream);
    else if (gram_prec == FST_GRAM_BF16X2) launch_split_single<SchemeBF16x2>(GR, grid, ga, stream);
    else launch_split_single<SchemeBF16x3>(GR, grid, ga, stream);
  };
  const std::string key = split_key(0, gram_prec, nt, Sp);
  const int known = tuner_lookup(key);
  if (known >= 0 && known < 3) {
    run(known);
  } else if (!accumulate && can_time(stream)) {
    // every candidate writes the same G bit for bit, so the last one timed leaves the result
    tuner_store(key, time_candidates(3, run, stream));
  } else {
    run(kDefaultGR);
  }
  check_launch("k_gram_split");
}

}  // namespace fst
