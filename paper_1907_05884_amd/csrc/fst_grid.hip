// Structured-grid and slice preview of a model (Sec. 6, fast visualisation) for gfx950.
//
// On a tensor grid gx x gy x gz the model of eq. (1) is the multilinear product
//   out = alpha x_1 U1 x_2 U2 x_3 U3,   U_k[i][j] = sum_m C_k[m][j] phi_m(xi_k(g_k[i]))  (eq. (2)),
// so the factor functions are evaluated once per grid line (k_factor_eval over the three
// axes, padded to a common length) and the grid follows from three mode products, done in
// the order mode 3, 2, 1 so that the output comes out in C order (i3 fastest):
//   T1[j1 j2][i3]   = sum_j3 alpha[j1 j2][j3] U3[i3][j3]          (r1 r2 x n3)
//   T2[j1][i2][i3]  = sum_j2 U2[i2][j2] T1[j1 j2][i3]              (r1 x n2 x n3)
//   out[i1][i2 i3]  = sum_j1 U1[i1][j1] T2[j1][i2 i3]              (n1 x n2 n3)
// The last product costs 2 r1 flop per grid point, against 2 R for evaluating eq. (1) point
// by point, and is bound by writing the grid to HBM.  A 2-D slice is a grid with one
// coordinate count equal to 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "fst_device.h"
#include "fst_internal.h"

namespace fst {

// Axis coordinates padded to a common length (the last coordinate repeated) so that one
// factor-evaluation launch covers the three axes.
template <typename T>
__global__ void k_grid_axes(const T* gx, int64_t n1, const T* gy, int64_t n2, const T* gz, int64_t n3,
                            int64_t nmax, T* px, T* py, T* pz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nmax) return;
  px[t] = gx[t < n1 ? t : n1 - 1];
  py[t] = gy[t < n2 ? t : n2 - 1];
  pz[t] = gz[t < n3 ? t : n3 - 1];
}

// O[b][i][c] = sum_{k < K} A[i][k] B[b][k][c] for i < n, c < C, b < gridDim.z, with
// arbitrary strides for A, c contiguous in B and O.  One thread per column c (VEC: per four
// columns) holds the K values B[b][k][c] in registers; the workgroup stages MP_ROWS rows of A
// in LDS (zero beyond K) and writes MP_ROWS output rows, each a coalesced run of 256 (VEC:
// 1024) columns.  The sum over k runs in a fixed order.  B rows k >= K are read clamped to row
// K - 1 (finite values that meet a zero in A), so every load is unconditional.  VEC (FP32,
// 16-byte aligned rows) writes 16 bytes per lane with non-temporal stores: the last product
// streams the whole grid to HBM, and per-lane 4-byte stores leave the store path, not HBM,
// as the limit.
constexpr int MP_ROWS = 32, MP_THREADS = 256;
template <typename T>
struct ModeArgs {
  const T* A;
  int64_t sa_i, sa_k;
  const T* B;
  int64_t sb_b, sb_k;
  T* O;
  int64_t so_b, so_i;
  int64_t n, C;
  int32_t K;
};

typedef float mp_float4 __attribute__((ext_vector_type(4)));
template <typename T, int KP, bool VEC>
__global__ __launch_bounds__(MP_THREADS) void k_mode_product(ModeArgs<T> a) {
  __shared__ T sA[MP_ROWS][KP];
  const int64_t b = blockIdx.z, i0 = (int64_t)blockIdx.y * MP_ROWS;
  const int nr = (int)std::min<int64_t>(MP_ROWS, a.n - i0);
  for (int e = threadIdx.x; e < MP_ROWS * KP; e += MP_THREADS) {
    const int r = e / KP, k = e % KP;
    sA[r][k] = (r < nr && k < a.K) ? a.A[(i0 + r) * a.sa_i + k * a.sa_k] : T(0);
  }
  __syncthreads();
  if constexpr (VEC) {
    const int64_t c = 4 * ((int64_t)blockIdx.x * MP_THREADS + threadIdx.x);   // C % 4 == 0
    if (c >= a.C) return;
    const float* Bp = a.B + b * a.sb_b + c;
    mp_float4 bv[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) bv[k] = *reinterpret_cast<const mp_float4*>(Bp + (int64_t)(k < a.K ? k : a.K - 1) * a.sb_k);
    float* Op = a.O + b * a.so_b + i0 * a.so_i + c;
    for (int r = 0; r < nr; ++r) {
      mp_float4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < KP; ++k) acc += sA[r][k] * bv[k];
      __builtin_nontemporal_store(acc, reinterpret_cast<mp_float4*>(Op + r * a.so_i));
    }
  } else {
    const int64_t c = (int64_t)blockIdx.x * MP_THREADS + threadIdx.x;
    if (c >= a.C) return;
    const T* Bp = a.B + b * a.sb_b + c;
    T bv[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) bv[k] = Bp[(int64_t)(k < a.K ? k : a.K - 1) * a.sb_k];
    T* Op = a.O + b * a.so_b + i0 * a.so_i + c;
    for (int r = 0; r < nr; ++r) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < KP; ++k) acc += sA[r][k] * bv[k];
      Op[r * a.so_i] = acc;
    }
  }
}

template <typename T, int KP>
static void mp_launch(const ModeArgs<T>& a, int64_t batch, void* stream) {
  const int64_t gy = (a.n + MP_ROWS - 1) / MP_ROWS;
  const auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const bool vec = sizeof(T) == 4 && a.C % 4 == 0 && a.sb_b % 4 == 0 && a.sb_k % 4 == 0 && a.so_b % 4 == 0 &&
                   a.so_i % 4 == 0 && aligned(a.B) && aligned(a.O);
  const int64_t per_block = vec ? 4 * MP_THREADS : MP_THREADS;
  const dim3 g((unsigned)((a.C + per_block - 1) / per_block), (unsigned)gy, (unsigned)batch);
  if constexpr (sizeof(T) == 4) {
    if (vec) {
      hipLaunchKernelGGL((k_mode_product<T, KP, true>), g, dim3(MP_THREADS), 0, S(stream), a);
      return;
    }
  }
  hipLaunchKernelGGL((k_mode_product<T, KP, false>), g, dim3(MP_THREADS), 0, S(stream), a);
}

template <typename T>
static void mode_product(const ModeArgs<T>& a, int64_t batch, void* stream) {
  if (a.n <= 0 || a.C <= 0 || batch <= 0) return;
  if (a.K < 1 || a.K > kMaxRank) fail(FST_E_INVAL, "mode product: contraction length out of range");
  const int64_t gy = (a.n + MP_ROWS - 1) / MP_ROWS;
  if (gy > 65535 || batch > 65535 || (a.C + MP_THREADS - 1) / MP_THREADS > 0x7fffffff)
    fail(FST_E_UNSUPPORTED, "mode product: grid too large");
  const int kp = (a.K + 7) / 8 * 8;
  switch (kp) {
    case 8: mp_launch<T, 8>(a, batch, stream); break;
    case 16: mp_launch<T, 16>(a, batch, stream); break;
    case 24: mp_launch<T, 24>(a, batch, stream); break;
    default: mp_launch<T, 32>(a, batch, stream); break;
  }
  check_launch("k_mode_product");
}

struct GridLayout {
  int64_t nmax, axes, U, T1, T2, total;   // byte offsets in the workspace
};
static GridLayout grid_layout(const fst_model* m, int dtype, int64_t n1, int64_t n2, int64_t n3) {
  const size_t es = dtype == FST_F64 ? 8 : 4;
  const int64_t r1 = m->rank[0], r2 = m->rank[1], r3 = m->rank[2];
  GridLayout L;
  L.nmax = std::max({n1, n2, n3});
  L.axes = 0;
  L.U = (int64_t)align_up(3 * es * (size_t)L.nmax);
  L.T1 = L.U + (int64_t)align_up(es * (size_t)(r1 + r2 + r3) * (size_t)L.nmax);
  L.T2 = L.T1 + (int64_t)align_up(es * (size_t)(r1 * r2) * (size_t)n3);
  L.total = L.T2 + (int64_t)align_up(es * (size_t)r1 * (size_t)n2 * (size_t)n3);
  return L;
}

size_t eval_grid_workspace_bytes(const fst_model* m, int dtype, int64_t n1, int64_t n2, int64_t n3) {
  return (size_t)grid_layout(m, dtype, n1, n2, n3).total;
}

template <typename T>
static void eval_grid_t(const fst_model* m, const DeviceModel& dm, const void* gx, int64_t n1, const void* gy,
                        int64_t n2, const void* gz, int64_t n3, void* out, void* ws, void* stream) {
  const int dtype = sizeof(T) == 8 ? FST_F64 : FST_F32;
  const GridLayout L = grid_layout(m, dtype, n1, n2, n3);
  char* w = (char*)ws;
  T* px = (T*)(w + L.axes);
  T* py = px + L.nmax;
  T* pz = py + L.nmax;
  T* U = (T*)(w + L.U);
  T* T1 = (T*)(w + L.T1);
  T* T2 = (T*)(w + L.T2);
  const int64_t r1 = m->rank[0], r2 = m->rank[1], r3 = m->rank[2], nm = L.nmax;
  hipLaunchKernelGGL(k_grid_axes<T>, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, S(stream), (const T*)gx, n1,
                     (const T*)gy, n2, (const T*)gz, n3, nm, px, py, pz);
  check_launch("k_grid_axes");
  // U[(o_k + j) nmax + i]: factor functions of mode k at the i-th coordinate of axis k
  launch_factor_eval(m, dm, dtype, nm, px, py, pz, nullptr, nullptr, nm, U, nullptr, stream);
  const T* U1 = U;
  const T* U2 = U + r1 * nm;
  const T* U3 = U + (r1 + r2) * nm;
  ModeArgs<T> a;
  // T1[j12][i3] = sum_j3 alpha[j12][j3] U3[j3][i3]
  a.A = (const T*)dm.core; a.sa_i = r3; a.sa_k = 1;
  a.B = U3; a.sb_b = 0; a.sb_k = nm;
  a.O = T1; a.so_b = 0; a.so_i = n3;
  a.n = r1 * r2; a.C = n3; a.K = (int32_t)r3;
  mode_product(a, 1, stream);
  // T2[j1][i2][i3] = sum_j2 U2[j2][i2] T1[j1 r2 + j2][i3]
  a.A = U2; a.sa_i = 1; a.sa_k = nm;
  a.B = T1; a.sb_b = r2 * n3; a.sb_k = n3;
  a.O = T2; a.so_b = n2 * n3; a.so_i = n3;
  a.n = n2; a.C = n3; a.K = (int32_t)r2;
  mode_product(a, r1, stream);
  // out[i1][i2 i3] = sum_j1 U1[j1][i1] T2[j1][i2 i3]
  a.A = U1; a.sa_i = 1; a.sa_k = nm;
  a.B = T2; a.sb_b = 0; a.sb_k = n2 * n3;
  a.O = (T*)out; a.so_b = 0; a.so_i = n2 * n3;
  a.n = n1; a.C = n2 * n3; a.K = (int32_t)r1;
  mode_product(a, 1, stream);
}

void eval_grid(const fst_model* m, const DeviceModel& dm, int dtype, const void* gx, int64_t n1, const void* gy,
               int64_t n2, const void* gz, int64_t n3, void* out, void* ws, void* stream) {
  if (dtype == FST_F64)
    eval_grid_t<double>(m, dm, gx, n1, gy, n2, gz, n3, out, ws, stream);
  else
    eval_grid_t<float>(m, dm, gx, n1, gy, n2, gz, n3, out, ws, stream);
}

}  // namespace fst
