// Learned residual corrector: g(xi) = W3 s(W2 s(W1 xi + b1) + b2) + b3, s(z) = z / (1 + e^-z),
// layers 3 -> 64 -> 64 -> 1, trained by Adam on the mean squared error against the scaled
// residual of the functional Tucker model.  BF16 operands with FP32 accumulation for the
// 64 x 64 layer (forward and the input gradient of the backward pass) on MFMA 16x16x32;
// FP32 master weights; weight-gradient reductions over the batch in FP32.
//
// Work mapping (forward): one wave per tile of 16 points; lane l owns point l % 16 and the
// hidden units 8 (l / 16) .. +7 and 32 + 8 (l / 16) .. +7, which is exactly the B-operand
// layout of MFMA 16x16x32 (lane l: B[8 (l / 16) + j][l % 16]), so layer 1 feeds the MFMA
// from registers.  The MFMA result lane l holds z2[16 ob + 4 (l / 16) + v][point l % 16].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fst_internal.h"
#include "fst_mlp.h"

namespace fst {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

static inline hipStream_t Sm(void* s) { return reinterpret_cast<hipStream_t>(s); }
static void check_launch_m(const char* what) { check_hip(hipGetLastError(), what); }

__device__ inline float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigm(z); }
__device__ inline float silu_d(float z) {
  float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// SplitMix64 output number k of the stream started at `state`, bounded to [0, n)
__device__ inline int64_t counter_draw(uint64_t state, uint64_t k, uint64_t n) {
  uint64_t z = state + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (int64_t)__umul64hi(z, n);
}

constexpr int H = kMlpHidden;
constexpr int PTS = 64;           // points per workgroup (4 waves x 16)
constexpr int RS = kMlpParams + 1; // partial record: gradients + loss

template <typename TIn>
struct MlpTrainArgs {
  const TIn *x, *y, *z;
  const float* target;     // scaled residual at every training point
  const int32_t* idx;      // explicit batch rows, or null (counter draws)
  int64_t n;               // training points
  int32_t B;               // batch size
  int64_t step;
  uint64_t rng_state;
  const float* P;          // FP32 master parameters
  const __bf16* W2b;       // [o][i]
  const __bf16* W2Tb;      // [i][o]
  float lo[3], scale[3];
  float* partial;          // [gridDim.x][RS]
};

// F32: the 64 x 64 layer in FP32 on the VALU from the FP32 master weights, activations kept in
// FP32 (the reference mode of the kernel, for checking the gradients against an FP64 oracle
// without the BF16 roundings); otherwise BF16 operands on MFMA as described above.
template <typename TIn, bool F32>
__global__ __launch_bounds__(256) void k_mlp_fwdbwd(MlpTrainArgs<TIn> a) {
  __shared__ float sP[kMlpParams];
  __shared__ __align__(16) __bf16 sW2[H][H + 8];
  __shared__ __align__(16) __bf16 sW2T[H][H + 8];
  __shared__ float sa1[PTS][H + 1], sa2[PTS][H + 1], sdz2[PTS][H + 1], sdz1[PTS][H + 1];
  __shared__ float sxi[PTS][3], sdy[PTS], sd2[PTS];
  for (int j = threadIdx.x; j < kMlpParams; j += blockDim.x) sP[j] = a.P[j];
  for (int j = threadIdx.x; j < H * H; j += blockDim.x) {
    sW2[j / H][j % H] = a.W2b[j];
    sW2T[j / H][j % H] = a.W2Tb[j];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
  const int p = w * 16 + li;
  const int64_t bpos = (int64_t)blockIdx.x * PTS + p;
  const bool valid = bpos < a.B;
  float xi[3] = {0.f, 0.f, 0.f}, t = 0.f;
  if (valid) {
    int64_t i = a.idx ? (int64_t)a.idx[bpos] : counter_draw(a.rng_state, (uint64_t)(a.step * a.B + bpos), (uint64_t)a.n);
    xi[0] = ((float)a.x[i] - a.lo[0]) * a.scale[0] - 1.0f;
    xi[1] = ((float)a.y[i] - a.lo[1]) * a.scale[1] - 1.0f;
    xi[2] = ((float)a.z[i] - a.lo[2]) * a.scale[2] - 1.0f;
    t = a.target[i];
  }
  if (g == 0) {
    sxi[p][0] = xi[0];
    sxi[p][1] = xi[1];
    sxi[p][2] = xi[2];
  }
  __syncthreads();
  const float* W1 = sP + kOffW1;
  const float* b1 = sP + kOffB1;
  const float* b2 = sP + kOffB2;
  const float* W3 = sP + kOffW3;
  // layer 1 into the MFMA B operand (two K blocks of 32 hidden units)
  bf16x8 B0, B1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      int h = kb * 32 + g * 8 + j;
      float z1 = W1[h * 3 + 0] * xi[0] + W1[h * 3 + 1] * xi[1] + W1[h * 3 + 2] * xi[2] + b1[h];
      if (F32) {
        sa1[p][h] = silu(z1);
      } else {
        __bf16 hb = (__bf16)silu(z1);
        if (kb == 0) B0[j] = hb; else B1[j] = hb;
        sa1[p][h] = (float)hb;
      }
    }
  }
  if (F32) __syncthreads();   // every hidden value of the point before layer 2 reads them
  const float* W2f = sP + kOffW2;   // [o][i], FP32 master weights
  // layer 2 (MFMA, or FP32 on the VALU), then the output layer
  float s2d[4][4];
  float ypart = 0.f;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    floatx4 acc = floatx4{0, 0, 0, 0};
    if (F32) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = ob * 16 + 4 * g + v;
        float s = 0.f;
        for (int i = 0; i < H; ++i) s += W2f[o * H + i] * sa1[p][i];
        acc[v] = s;
      }
    } else {
      bf16x8 A0 = *reinterpret_cast<const bf16x8*>(&sW2[ob * 16 + li][g * 8]);
      bf16x8 A1 = *reinterpret_cast<const bf16x8*>(&sW2[ob * 16 + li][32 + g * 8]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B1, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int o = ob * 16 + 4 * g + v;
      float z2 = acc[v] + b2[o];
      float a2 = silu(z2);
      s2d[ob][v] = silu_d(z2);
      ypart += W3[o] * a2;
      sa2[p][o] = a2;
    }
  }
  ypart += __shfl_xor(ypart, 16, 64);
  ypart += __shfl_xor(ypart, 32, 64);
  const float yv = ypart + sP[kOffB3];
  const float d = valid ? yv - t : 0.f;
  const float dy = valid ? 2.0f * d / (float)a.B : 0.f;
  if (g == 0) {
    sdy[p] = dy;
    sd2[p] = d * d;
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int o = ob * 16 + 4 * g + v;
      sdz2[p][o] = dy * W3[o] * s2d[ob][v];
    }
  __syncthreads();
  // input gradient of layer 2 (MFMA, or FP32 on the VALU): da1[i][p] = sum_o W2[o][i] dz2[o][p]
  bf16x8 D0, D1;
  if (!F32) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      D0[j] = (__bf16)sdz2[p][g * 8 + j];
      D1[j] = (__bf16)sdz2[p][32 + g * 8 + j];
    }
  }
#pragma unroll
  for (int ib = 0; ib < 4; ++ib) {
    floatx4 acc = floatx4{0, 0, 0, 0};
    if (F32) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ib * 16 + 4 * g + v;
        float s = 0.f;
        for (int o = 0; o < H; ++o) s += W2f[o * H + i] * sdz2[p][o];
        acc[v] = s;
      }
    } else {
      bf16x8 A0 = *reinterpret_cast<const bf16x8*>(&sW2T[ib * 16 + li][g * 8]);
      bf16x8 A1 = *reinterpret_cast<const bf16x8*>(&sW2T[ib * 16 + li][32 + g * 8]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, D0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, D1, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int h = ib * 16 + 4 * g + v;
      float z1 = W1[h * 3 + 0] * xi[0] + W1[h * 3 + 1] * xi[1] + W1[h * 3 + 2] * xi[2] + b1[h];
      sdz1[p][h] = valid ? acc[v] * silu_d(z1) : 0.f;
    }
  }
  __syncthreads();
  // weight gradients: sums over this workgroup's points, one output per thread at a time
  float* out = a.partial + (int64_t)blockIdx.x * RS;
  for (int j = threadIdx.x; j < RS; j += blockDim.x) {
    float s = 0.f;
    if (j < kOffB1) {
      int h = j / 3, k = j % 3;
      for (int q = 0; q < PTS; ++q) s += sdz1[q][h] * sxi[q][k];
    } else if (j < kOffW2) {
      int h = j - kOffB1;
      for (int q = 0; q < PTS; ++q) s += sdz1[q][h];
    } else if (j < kOffB2) {
      int o = (j - kOffW2) / H, i = (j - kOffW2) % H;
      for (int q = 0; q < PTS; ++q) s += sdz2[q][o] * sa1[q][i];
    } else if (j < kOffW3) {
      int o = j - kOffB2;
      for (int q = 0; q < PTS; ++q) s += sdz2[q][o];
    } else if (j < kOffB3) {
      int o = j - kOffW3;
      for (int q = 0; q < PTS; ++q) s += sdy[q] * sa2[q][o];
    } else if (j == kOffB3) {
      for (int q = 0; q < PTS; ++q) s += sdy[q];
    } else {
      for (int q = 0; q < PTS; ++q) s += sd2[q];
    }
    out[j] = s;
  }
}

// gradient = fixed-order sum of the workgroup partials; optional Adam update of the FP32
// master weights (bias-corrected moments) and refresh of the BF16 copies of W2
struct AdamArgs {
  const float* partial;
  int32_t nwg;
  float* P;
  float* m;
  float* v;
  __bf16* W2b;
  __bf16* W2Tb;
  float* grad_out;     // may be null
  float* loss_out;     // may be null (one float)
  int32_t update;
  float lr, beta1, beta2, eps, c1, c2;   // c1 = 1 - beta1^t, c2 = 1 - beta2^t
};
__global__ __launch_bounds__(256) void k_mlp_adam(AdamArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > kMlpParams) return;
  float gsum = 0.f;
  for (int w = 0; w < a.nwg; ++w) gsum += a.partial[(int64_t)w * RS + j];
  if (j == kMlpParams) {
    if (a.loss_out) *a.loss_out = gsum / 1.0f;
    if (a.grad_out) a.grad_out[j] = gsum;
    return;
  }
  if (a.grad_out) a.grad_out[j] = gsum;
  if (!a.update) return;
  float mj = a.beta1 * a.m[j] + (1.f - a.beta1) * gsum;
  float vj = a.beta2 * a.v[j] + (1.f - a.beta2) * gsum * gsum;
  a.m[j] = mj;
  a.v[j] = vj;
  float pj = a.P[j] - a.lr * (mj / a.c1) / (sqrtf(vj / a.c2) + a.eps);
  a.P[j] = pj;
  if (j >= kOffW2 && j < kOffB2) {
    int o = (j - kOffW2) / H, i = (j - kOffW2) % H;
    a.W2b[o * H + i] = (__bf16)pj;
    a.W2Tb[i * H + o] = (__bf16)pj;
  }
}

// inference: out[q] += out_scale * g(xi_q), wave per tile of 16 points, grid-stride
template <typename TIn>
struct MlpApplyArgs {
  const TIn *x, *y, *z;
  TIn* out;
  int64_t n;
  const float* P;       // parameters as stored (BF16-rounded values in FP32)
  const __bf16* W2b;
  float lo[3], scale[3];
  float out_scale;
};
template <typename TIn>
__global__ __launch_bounds__(256) void k_mlp_apply(MlpApplyArgs<TIn> a) {
  __shared__ float sP[kMlpParams];
  __shared__ __align__(16) __bf16 sW2[H][H + 8];
  for (int j = threadIdx.x; j < kMlpParams; j += blockDim.x) sP[j] = a.P[j];
  for (int j = threadIdx.x; j < H * H; j += blockDim.x) sW2[j / H][j % H] = a.W2b[j];
  __syncthreads();
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const float* W1 = sP + kOffW1;
  const float* b1 = sP + kOffB1;
  const float* b2 = sP + kOffB2;
  const float* W3 = sP + kOffW3;
  const int64_t ntiles = (a.n + 15) / 16;
  const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t tile = wave_id; tile < ntiles; tile += nwaves) {
    const int64_t q = tile * 16 + li;
    const bool valid = q < a.n;
    const int64_t qq = valid ? q : 0;
    float xi[3];
    xi[0] = ((float)a.x[qq] - a.lo[0]) * a.scale[0] - 1.0f;
    xi[1] = ((float)a.y[qq] - a.lo[1]) * a.scale[1] - 1.0f;
    xi[2] = ((float)a.z[qq] - a.lo[2]) * a.scale[2] - 1.0f;
    bf16x8 B0, B1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int h0 = g * 8 + j, h1 = 32 + g * 8 + j;
      float z0 = W1[h0 * 3 + 0] * xi[0] + W1[h0 * 3 + 1] * xi[1] + W1[h0 * 3 + 2] * xi[2] + b1[h0];
      float z1 = W1[h1 * 3 + 0] * xi[0] + W1[h1 * 3 + 1] * xi[1] + W1[h1 * 3 + 2] * xi[2] + b1[h1];
      B0[j] = (__bf16)silu(z0);
      B1[j] = (__bf16)silu(z1);
    }
    float ypart = 0.f;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      bf16x8 A0 = *reinterpret_cast<const bf16x8*>(&sW2[ob * 16 + li][g * 8]);
      bf16x8 A1 = *reinterpret_cast<const bf16x8*>(&sW2[ob * 16 + li][32 + g * 8]);
      floatx4 acc = floatx4{0, 0, 0, 0};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B1, acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int o = ob * 16 + 4 * g + v;
        ypart += W3[o] * silu(acc[v] + b2[o]);
      }
    }
    ypart += __shfl_xor(ypart, 16, 64);
    ypart += __shfl_xor(ypart, 32, 64);
    if (valid && g == 0) a.out[q] = (TIn)((float)a.out[q] + a.out_scale * (ypart + sP[kOffB3]));
  }
}

// ------------------------------------------------------------------------------ host side
struct CorrectorDevice {
  float* P = nullptr;      // master (training) or stored (inference) parameters
  __bf16* W2b = nullptr;
  __bf16* W2Tb = nullptr;
};

static void upload_params(const std::vector<float>& P, CorrectorDevice& d, void* stream) {
  if (!d.P) {
    d.P = (float*)device_alloc(sizeof(float) * kMlpParams);
    d.W2b = (__bf16*)device_alloc(sizeof(__bf16) * H * H);
    d.W2Tb = (__bf16*)device_alloc(sizeof(__bf16) * H * H);
  }
  std::vector<__bf16> w(H * H), wt(H * H);
  for (int o = 0; o < H; ++o)
    for (int i = 0; i < H; ++i) {
      __bf16 b = (__bf16)P[kOffW2 + o * H + i];
      w[o * H + i] = b;
      wt[i * H + o] = b;
    }
  copy_h2d(d.P, P.data(), sizeof(float) * kMlpParams, stream);
  copy_h2d(d.W2b, w.data(), sizeof(__bf16) * H * H, stream);
  copy_h2d(d.W2Tb, wt.data(), sizeof(__bf16) * H * H, stream);
  stream_sync(stream);
}

static void free_device(CorrectorDevice& d) {
  device_free(d.P);
  device_free(d.W2b);
  device_free(d.W2Tb);
  d = CorrectorDevice();
}

// Xavier-uniform initial weights from a SplitMix64 stream (state seed * 256 + 4), zero biases
std::vector<float> mlp_init_params(uint64_t seed) {
  std::vector<float> P(kMlpParams, 0.0f);
  uint64_t st = seed * 256ull + 4ull;
  auto uni = [&](double bound) {
    uint64_t r = splitmix64_next(st);
    double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);   // [0, 1) with 53 bits
    return (float)((2.0 * u - 1.0) * bound);
  };
  const double bw1 = std::sqrt(6.0 / (3 + H)), bw2 = std::sqrt(6.0 / (H + H)), bw3 = std::sqrt(6.0 / (H + 1));
  for (int j = 0; j < H * 3; ++j) P[kOffW1 + j] = uni(bw1);
  for (int j = 0; j < H * H; ++j) P[kOffW2 + j] = uni(bw2);
  for (int j = 0; j < H; ++j) P[kOffW3 + j] = uni(bw3);
  return P;
}

size_t mlp_train_workspace_bytes(int32_t batch) {
  const int nwg = (batch + PTS - 1) / PTS;
  return align_up(sizeof(float) * (size_t)nwg * RS) + 3 * align_up(sizeof(float) * kMlpParams) +
         2 * align_up(sizeof(__bf16) * H * H) + align_up(sizeof(float) * RS) + align_up(sizeof(int32_t) * (size_t)batch);
}

template <typename TIn>
static void fill_map(const double lo[3], const double hi[3], float flo[3], float fsc[3]) {
  for (int k = 0; k < 3; ++k) {
    flo[k] = (float)lo[k];
    fsc[k] = (float)(2.0 / (hi[k] - lo[k]));
  }
}

// One or more Adam steps; with steps == 0 and grad_out set it only evaluates the gradient of
// the batch given by idx (or the counter draw of step `first_step`).
template <typename TIn>
static void train_t(const double lo[3], const double hi[3], int64_t n, const void* x, const void* y,
                    const void* z, const float* target, const int32_t* idx, int32_t batch, int64_t first_step,
                    int64_t steps, uint64_t seed, const MlpAdam& opt, std::vector<float>& P, float* grad_out_dev,
                    std::vector<float>* losses, void* ws, size_t ws_bytes, void* stream) {
  if (ws_bytes < mlp_train_workspace_bytes(batch)) fail(FST_E_NOMEM, "corrector: workspace too small");
  const bool f32 = opt.fp32;
  const int nwg = (batch + PTS - 1) / PTS;
  char* base = (char*)ws;
  float* partial = (float*)base;
  base += align_up(sizeof(float) * (size_t)nwg * RS);
  float* dP = (float*)base;
  base += align_up(sizeof(float) * kMlpParams);
  float* dm = (float*)base;
  base += align_up(sizeof(float) * kMlpParams);
  float* dv = (float*)base;
  base += align_up(sizeof(float) * kMlpParams);
  __bf16* dW2 = (__bf16*)base;
  base += align_up(sizeof(__bf16) * H * H);
  __bf16* dW2T = (__bf16*)base;
  base += align_up(sizeof(__bf16) * H * H);
  float* dloss = (float*)base;
  CorrectorDevice d;
  d.P = dP;
  d.W2b = dW2;
  d.W2Tb = dW2T;
  upload_params(P, d, stream);
  std::vector<float> zero(kMlpParams, 0.0f);
  copy_h2d(dm, zero.data(), sizeof(float) * kMlpParams, stream);
  copy_h2d(dv, zero.data(), sizeof(float) * kMlpParams, stream);

  MlpTrainArgs<TIn> ta;
  ta.x = (const TIn*)x;
  ta.y = (const TIn*)y;
  ta.z = (const TIn*)z;
  ta.target = target;
  ta.idx = idx;
  ta.n = n;
  ta.B = batch;
  ta.rng_state = seed * 256ull + 3ull;
  ta.P = dP;
  ta.W2b = dW2;
  ta.W2Tb = dW2T;
  fill_map<TIn>(lo, hi, ta.lo, ta.scale);
  ta.partial = partial;
  AdamArgs aa;
  aa.partial = partial;
  aa.nwg = nwg;
  aa.P = dP;
  aa.m = dm;
  aa.v = dv;
  aa.W2b = dW2;
  aa.W2Tb = dW2T;
  aa.lr = (float)opt.lr;
  aa.beta1 = (float)opt.beta1;
  aa.beta2 = (float)opt.beta2;
  aa.eps = (float)opt.eps;
  const int64_t nsteps = steps > 0 ? steps : 1;
  std::vector<float> lossbuf;
  if (losses) losses->clear();
  for (int64_t s = 0; s < nsteps; ++s) {
    ta.step = first_step + s;
    if (f32)
      hipLaunchKernelGGL((k_mlp_fwdbwd<TIn, true>), dim3((unsigned)nwg), dim3(256), 0, Sm(stream), ta);
    else
      hipLaunchKernelGGL((k_mlp_fwdbwd<TIn, false>), dim3((unsigned)nwg), dim3(256), 0, Sm(stream), ta);
    check_launch_m("k_mlp_fwdbwd");
    aa.update = steps > 0 ? 1 : 0;
    aa.grad_out = steps > 0 ? nullptr : grad_out_dev;
    aa.loss_out = dloss;
    const double t = (double)(first_step + s + 1);
    aa.c1 = (float)(1.0 - std::pow(opt.beta1, t));
    aa.c2 = (float)(1.0 - std::pow(opt.beta2, t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, Sm(stream), aa);
    check_launch_m("k_mlp_adam");
    if (losses && (s % 50 == 0 || s + 1 == nsteps)) {
      float l;
      copy_d2h(&l, dloss, sizeof(float), stream);
      losses->push_back(l / (float)batch);
    }
  }
  copy_d2h(P.data(), dP, sizeof(float) * kMlpParams, stream);
}

void mlp_train(int dtype, const double lo[3], const double hi[3], int64_t n, const void* x, const void* y,
               const void* z, const float* target, const int32_t* idx, int32_t batch, int64_t first_step,
               int64_t steps, uint64_t seed, const MlpAdam& opt, std::vector<float>& P, float* grad_out_dev,
               std::vector<float>* losses, void* ws, size_t ws_bytes, void* stream) {
  if (dtype == FST_F64)
    train_t<double>(lo, hi, n, x, y, z, target, idx, batch, first_step, steps, seed, opt, P, grad_out_dev, losses,
                    ws, ws_bytes, stream);
  else
    train_t<float>(lo, hi, n, x, y, z, target, idx, batch, first_step, steps, seed, opt, P, grad_out_dev, losses,
                   ws, ws_bytes, stream);
}

void mlp_apply(int dtype, const double lo[3], const double hi[3], const std::vector<float>& stored,
               float out_scale, int64_t n, const void* x, const void* y, const void* z, void* out,
               CorrectorDeviceCache& cache, void* stream) {
  if (n <= 0) return;
  if (!cache.P) {
    CorrectorDevice d;
    upload_params(stored, d, stream);
    cache.P = d.P;
    cache.W2b = d.W2b;
    cache.W2Tb = d.W2Tb;
  }
  int64_t ntiles = (n + 15) / 16;
  unsigned blocks = (unsigned)std::min<int64_t>((ntiles + 3) / 4, 256 * 16);
  if (dtype == FST_F64) {
    MlpApplyArgs<double> a;
    a.x = (const double*)x;
    a.y = (const double*)y;
    a.z = (const double*)z;
    a.out = (double*)out;
    a.n = n;
    a.P = cache.P;
    a.W2b = (const __bf16*)cache.W2b;
    fill_map<double>(lo, hi, a.lo, a.scale);
    a.out_scale = out_scale;
    hipLaunchKernelGGL((k_mlp_apply<double>), dim3(blocks), dim3(256), 0, Sm(stream), a);
  } else {
    MlpApplyArgs<float> a;
    a.x = (const float*)x;
    a.y = (const float*)y;
    a.z = (const float*)z;
    a.out = (float*)out;
    a.n = n;
    a.P = cache.P;
    a.W2b = (const __bf16*)cache.W2b;
    fill_map<float>(lo, hi, a.lo, a.scale);
    a.out_scale = out_scale;
    hipLaunchKernelGGL((k_mlp_apply<float>), dim3(blocks), dim3(256), 0, Sm(stream), a);
  }
  check_launch_m("k_mlp_apply");
}

void free_corrector_cache(CorrectorDeviceCache& c) {
  device_free(c.P);
  device_free(c.W2b);
  device_free(c.W2Tb);
  c = CorrectorDeviceCache();
}

}  // namespace fst
