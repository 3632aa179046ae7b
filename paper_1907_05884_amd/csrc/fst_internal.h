// Internal declarations shared by the host C++ files and the HIP kernel file.
#pragma once

#include <cstddef>
#include <cstdint>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fst.h"

namespace fst {

constexpr int kMaxRank = 32;     // r_k limit of this version
constexpr int kMaxBasis = 32;    // n_k = p_k + 1 limit of this version
constexpr int kMaxModes = 4;     // d = 3 (the 3-way calls) or 4 (the d-way calls)
constexpr int kMaxWaveDegree = 7;   // q of a wavelet space W_{s,q}
constexpr int kMaxDetail = 128;     // (q + 1)(2^s - 1) detail functions per mode at most
constexpr int kWaveTable = 2 * (kMaxWaveDegree + 1) * (kMaxWaveDegree + 1);   // mother wavelets per mode

// Error carried from deep inside the library to the C ABI boundary, where it becomes a
// status code plus a thread-local message.
struct Error : std::runtime_error {
  fst_status code;
  Error(fst_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};
[[noreturn]] void fail(fst_status code, const std::string& msg);
void set_last_error(const std::string& msg);

// Device copy of a model for one (device, dtype): coefficient matrices padded to
// kMaxBasis x kMaxRank per mode (kMaxModes slots, unused modes zero), and the core in C order.
struct DeviceModel {
  void* coefs = nullptr;   // kMaxModes * kMaxBasis * kMaxRank elements of the dtype
  // FP32 models without wavelets: the factor functions in the Chebyshev basis (same layout,
  // D[i][j] = sum_m L[m][i] C[m][j] for phi_m = sum_i L[m][i] T_i, formed in FP64)
  void* cheb = nullptr;
  // each mode's scale exponent xc of cheb: the stored values are D 2^xc, the largest |D| of
  // the mode brought to [2^14, 2^15) (xc clamped to [-20, 26])
  int32_t cheb_xc[kMaxModes] = {0, 0, 0, 0};
  void* detail = nullptr;  // models with wavelets: kMaxModes * kMaxDetail * kMaxRank detail coefficients
  void* wave = nullptr;    // models with wavelets: kMaxModes * kWaveTable mother-wavelet coefficients
  void* core = nullptr;    // R elements of the dtype
  void* core64 = nullptr;  // R doubles (for refinement), only for dtype FP64 copy
};

}  // namespace fst

namespace fst {
// How the core of a refit was solved: Gram precision after the precision ladder (-1 for
// models not produced by a refit), core entries skipped as numerically dependent,
// refinement steps taken and the final ||A^T (v - A alpha)|| / ||A^T v|| (NaN if none).
struct SolveInfo {
  int32_t gram_prec = -1;
  int64_t dropped = 0;
  int32_t refine_steps = 0;
  double rel_residual = std::numeric_limits<double>::quiet_NaN();
};
}  // namespace fst

struct fst_model {
  int32_t d = 3;                  // modes; entries k >= d of the arrays below are unused
  double lo[4] = {0, 0, 0, 0}, hi[4] = {1, 1, 1, 1};
  int32_t rank[4] = {1, 1, 1, 1}, degree[4] = {0, 0, 0, 0};
  // wavelet space W_{s,q} held beside P_p in mode k (s = wlevel[k] > 0, q = wdegree[k] <= p)
  int32_t wlevel[4] = {0, 0, 0, 0}, wdegree[4] = {0, 0, 0, 0};
  std::vector<double> core;      // r1 .. rd, C order
  std::vector<double> coef[4];   // rows(k) x r_k row-major: phi_0..phi_p, then the detail functions
  fst::SolveInfo fit;             // how the core was solved (models from a refit)
  // lazily uploaded device copies, keyed by (device ordinal, dtype)
  mutable std::mutex mu;
  mutable std::map<std::pair<int, int>, fst::DeviceModel> dev;
  ~fst_model();
  int64_t R() const {
    int64_t r = 1;
    for (int k = 0; k < d; ++k) r *= rank[k];
    return r;
  }
  int sum_r() const {
    int s = 0;
    for (int k = 0; k < d; ++k) s += rank[k];
    return s;
  }
  int details(int k) const { return wlevel[k] > 0 ? (wdegree[k] + 1) * ((1 << wlevel[k]) - 1) : 0; }
  int rows(int k) const { return degree[k] + 1 + details(k); }
  bool has_wavelets() const {
    for (int k = 0; k < d; ++k)
      if (wlevel[k] > 0) return true;
    return false;
  }
};

namespace fst {

// ---------------------------------------------------------------- host steps (fst_host.cpp)
uint64_t splitmix64_next(uint64_t& state);
void sample_indices(uint64_t seed, int stream, int64_t n, int64_t m, int64_t* out);
void idw_grid(const double* xi, const double* v, int64_t K, const int32_t grid[3], int k,
              double power, int n_threads, double* out);
void idw_knn(const double* xi, int64_t K, const int32_t grid[3], int k, double power, int n_threads,
             std::vector<int64_t>& nbr, std::vector<double>& wgt, std::vector<int32_t>& count);
void idw_apply(const std::vector<int64_t>& nbr, const std::vector<double>& wgt, const std::vector<int32_t>& count,
               int k, const double* v, int n_threads, double* out);
void sthosvd(const double* T, const int32_t dims[3], const int32_t rank[3], int n_threads,
             double* core, double* const W[3], double* const sigma[3]);
void sthosvd_eps(const double* T, const int32_t dims[3], double eps, const int32_t max_rank[3], int n_threads,
                 int32_t rank_out[3], double* core, double* const W[3], double* const sigma[3]);
// the same for D = 3 or 4 modes (xi: K x D; dims, rank, grid: D entries)
void idw_knn_d(const double* xi, int64_t K, int D, const int32_t* grid, int k, double power, int n_threads,
               std::vector<int64_t>& nbr, std::vector<double>& wgt, std::vector<int32_t>& count);
void idw_grid_d(const double* xi, const double* v, int64_t K, int D, const int32_t* grid, int k, double power,
                int n_threads, double* out);
void sthosvd_d(const double* T, int D, const int32_t* dims, const int32_t* rank, int n_threads, double* core,
               double* const* W, double* const* sigma);
void sthosvd_eps_d(const double* T, int D, const int32_t* dims, double eps, const int32_t* max_rank, int n_threads,
                   int32_t* rank_out, double* core, double* const* W, double* const* sigma);
void sparse_fit(const double* W, int I, int r, int p, double* C);
void sparse_fit_lars(const double* W, int I, int r, int p, double* C);
// wavelet space W_{s,q}: mother wavelets H[(m * 2 + half) * (q + 1) + n], the number of detail
// functions, their values at t (order (l, c, m)), and the per-column choice between P_p and
// W_{s,q} (C: (p + 1 + detail_count) x r)
void mother_wavelets_host(int q, double* H);
int detail_count(int s, int q);
void detail_values_host(double t, int s, int q, const double* H, double* out);
void sparse_fit_choice(const double* W, int I, int r, int p, int s, int q, int solver, double* C);
// the sparse fit of one factor matrix with the chosen solver (FST_SOLVER_*), and with the
// choice against W_{s,q} when s > 0
inline void sparse_fit_with(int solver, const double* W, int I, int r, int p, double* C, int s = 0, int q = 0) {
  if (s > 0)
    sparse_fit_choice(W, I, r, p, s, q, solver, C);
  else if (solver == FST_SOLVER_LARS)
    sparse_fit_lars(W, I, r, p, C);
  else
    sparse_fit(W, I, r, p, C);
}
void legendre_orthonormal_host(double t, int p, double* phi);
int hardware_threads(int requested);

// ---------------------------------------------------------------- model (fst_model.cpp)
fst_model* model_new(const double lo[3], const double hi[3], const int32_t rank[3],
                     const int32_t degree[3]);
fst_model* model_new_d(int d, const double* lo, const double* hi, const int32_t* rank, const int32_t* degree,
                       const int32_t* wlevel = nullptr, const int32_t* wdegree = nullptr);
fst_model* copy_with_core(const fst_model* m, const std::vector<double>& core);
void check_model(const fst_model* m);    // any d
void check_model3(const fst_model* m);   // the 3-way calls: d = 3 only
const DeviceModel& device_model(const fst_model* m, int dtype);   // uploads on first use

// ---------------------------------------------------------------- GPU launchers (fst_kernels.hip)
int current_device();
void check_hip(int err, const char* what);
void launch_factor_eval(const fst_model* m, const DeviceModel& dm, int dtype, int64_t n,
                        const void* x, const void* y, const void* z, const void* v,
                        const int32_t* idx, int64_t mrows, void* U, void* vs, void* stream);
// the same for a model of any d: coords holds m->d coordinate arrays
// FP32 Legendre models (d = 3 or 4): eq. (2) with the contraction on MFMA
bool factor_eval_mfma_applies(const fst_model* m, int64_t mrows);
void launch_factor_eval_mfma(const fst_model* m, const DeviceModel& dm, const void* const* coords, const void* v,
                             const int32_t* idx, int64_t mrows, void* U, void* vs, void* stream);
void launch_factor_eval_d(const fst_model* m, const DeviceModel& dm, int dtype, const void* const* coords,
                          const void* v, const int32_t* idx, int64_t mrows, void* U, void* vs, void* stream);
size_t gram_workspace_bytes(const fst_model* m, int64_t mrows);
// returns the Gram precision used: gram_prec, or FST_GRAM_F32 for a split precision whose row
// planes do not fit in the workspace
int launch_gram(const fst_model* m, int dtype, int64_t mrows, const void* U, const void* vs,
                int gram_prec, double* G, double* h, void* ws, size_t ws_bytes, void* stream);
// workspace beyond gram_workspace_bytes that lets launch_gram take its dense route at gram_prec
size_t gram_route_bytes(const fst_model* m, int dtype, int gram_prec, int64_t mrows);
// free device memory of the current device (bytes)
size_t device_free_bytes();
size_t cholesky_workspace_bytes(int64_t R);
// returns 0 on success, else the 1-based index of the failing pivot
// FP64 Cholesky in place; returns the first breakdown pivot (1-based) or 0.  A pivot breaks
// down when it is not above R 2^-52 times its original diagonal.  With drop_tol > 0, a pivot
// not above max(R 2^-52, drop_tol) times its original diagonal marks a column (numerically)
// dependent on the earlier ones: it is skipped (L_jj = +inf, so its solution entry is zero)
// and counted in *dropped instead of being reported.  shift > 0 factors G + shift diag(G)
// (thresholds stay relative to the unshifted diagonal).
int64_t cholesky(int64_t R, double* G, void* ws, size_t ws_bytes, void* stream, double drop_tol = 0.0,
                 int64_t* dropped = nullptr, double shift = 0.0);

// the same factorisation (drop_tol 0) with its scratch in the library's file-scope device
// array instead of a workspace (fst_linalg.hip); R <= FST_CHOLESKY_NOALLOC_MAX_R
int64_t cholesky_static_scratch(int64_t R, double* G, void* stream, double shift);
// 1 for every column a semidefinite factorisation skipped (ws: R doubles of scratch)
std::vector<uint8_t> dropped_mask(const double* L, int64_t R, void* ws, void* stream);
void cholesky_solve(int64_t R, const double* L, const double* b, double* x, void* stream);
void launch_eval(const fst_model* m, const DeviceModel& dm, int dtype, int64_t n,
                 const void* x, const void* y, const void* z, const int32_t* idx,
                 const void* v, void* out, void* stream);
// FP32 reconstruction with the core contraction on MFMA (fst_eval_mfma.hip): 3-way Legendre
// models whose core fits the kernel's LDS layout; out = f, or v[idx] - f with residual
bool eval_mfma_applies(const fst_model* m);
void launch_eval_mfma(const fst_model* m, const DeviceModel& dm, int64_t n, const float* x, const float* y,
                      const float* z, const int32_t* idx, const float* v, float* out, bool residual, void* stream);
size_t residual_workspace_bytes(const fst_model* m, int64_t mrows);
void residual(const fst_model* m, int dtype, int64_t n, const void* x, const void* y,
              const void* z, const void* v, const int32_t* idx, int64_t mrows,
              const double* alpha, double* r, void* ws, size_t ws_bytes, void* stream);
void launch_gram_batched(const std::vector<const fst_model*>& models, const std::vector<const void*>& U,
                         const std::vector<int64_t>& mrows, const std::vector<double*>& G, int prec, void* ws,
                         void* stream);
size_t eval_error_workspace_bytes(int dtype, int64_t n);
// mixed least-squares rows (Algorithm 2 steps 2-4): normal equations of S sampled rows of
// F D W and F D u into G (lower triangle) and h
int64_t mixed_length(int64_t n);
// the S sampled mixed rows themselves: A^T (R x Sp, Sp = S rounded up to 64, zero past S) and b
void mixed_rows(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z, const void* v,
                int64_t nsamp, uint64_t seed, void* ws, size_t ws_bytes, void* At, void* b, void* stream);
// leverage of the rows of A^T (R x Sp, FP64) given the Cholesky factor L of A^T A
void leverage(int64_t R, int64_t Sp, int64_t mrows, const double* At, const double* L, double* out, void* stream);
size_t mixed_workspace_bytes(const fst_model* m, int dtype, int64_t n, int64_t nsamp);
void mixed_normal_equations(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z,
                            const void* v, int64_t nsamp, uint64_t seed, void* ws, size_t ws_bytes, double* G,
                            double* h, void* stream);
// G = A^T A (lower triangle, FP64) and h = A^T b from materialised rows: At is R x Sp (row j of
// A^T contiguous), b is Sp long, Sp a multiple of GD_SP_MULTIPLE with rows past the data zero;
// in the point dtype (FP32: FP32 MFMA folded into FP64; FP64: FP64 MFMA).  accumulate adds to
// G and h instead of overwriting them; G or h may be NULL to skip that product.
constexpr int64_t GD_SP_MULTIPLE = 64;
// the dense route of the Gram: A^T of mrows rows (factor values U as k_factor_eval writes them)
// materialised `chunk` rows at a time in At (dense_rows_bytes(chunk) bytes), then k_gram_dense
// (G = A^T A, lower triangle, accumulated over the chunks)
size_t dense_rows_bytes(const fst_model* m, int dtype, int64_t chunk);
void dense_gram_from_rows(const fst_model* m, int dtype, int64_t mrows, const void* U, double* G, void* At,
                          int64_t chunk, void* stream);
// the dense route of the 16-bit Gram (3-way, FP32 factor values): A^T rounded to BF16 or scaled
// FP16 (R x Sp 16-bit entries, Sp a multiple of GD16_SP_MULTIPLE), then G = sums x unscale
constexpr int64_t GD16_SP_MULTIPLE = 128;
void design_rows16(const fst_model* m, int gram_prec, int64_t mrows, const float* U, int64_t Sp, void* At, float scale,
                   void* stream);
void dense_gram16(int gram_prec, const void* At, int64_t R, int64_t Sp, double* G, double unscale, void* stream);
// power of two that brings every 16-bit design-row entry u1 u2 u3 into [-1, 1] (ws: 16 bytes)
float f16_row_scale(const fst_model* m, int64_t mrows, const float* U, void* ws, void* stream);
// split 16-bit Gram (fst_gram16.hip): terms per entry of a split precision (0 for the others),
// padded row count and bytes of the row planes, and G = A^T A from FP32 factor values U
// (planes written to `rows`; scratch: 16 bytes for the FP16 scale) or from planes already written
int split_terms(int gram_prec);
int64_t split_rows_padded(int64_t mrows);
size_t split_rows_bytes(const fst_model* m, int gram_prec, int64_t mrows);
void gram_split(const fst_model* m, int gram_prec, int64_t mrows, const float* U, double* G, void* rows,
                size_t rows_bytes, void* scratch, void* stream);
void gram_split_rows(int gram_prec, void* const* plane, int64_t R, int64_t Sp, double* G, double unscale,
                     bool accumulate, void* stream);
// Gram matrices of several variables (same mrows) from their FP32 factor values, in as few
// launches as the workspace allows (at least gram_split_batched_min_bytes)
size_t gram_split_batched_min_bytes(const std::vector<const fst_model*>& models, int gram_prec, int64_t mrows);
void gram_split_batched(const std::vector<const fst_model*>& models, const std::vector<const void*>& U,
                        int64_t mrows, const std::vector<double*>& G, int gram_prec, void* ws, size_t ws_bytes,
                        void* stream);
// A^T (R x Sp) and b (Sp, may be NULL) of mrows rows given by their factor values and values
void design_rows(const fst_model* m, int dtype, int64_t mrows, const void* U, const void* vs, int64_t Sp, void* At,
                 void* b, void* stream);
void dense_normal_equations(int dtype, const void* At, const void* b, int64_t R, int64_t Sp, double* G, double* h,
                            bool accumulate, void* stream);
// d-way form (fst_dway.hip): normal equations of M sampled rows (idx) of a d = 3 or 4 model
// from materialised row chunks, and the reconstruction for any d (d = 3: launch_eval)
size_t dway_workspace_bytes(const fst_model* m, int dtype, int64_t M);
void dway_normal_equations(const fst_model* m, int dtype, const void* const* coords, const void* v,
                           const int32_t* idx, int64_t M, void* ws, size_t ws_bytes, double* G, double* h,
                           void* stream);
void launch_eval_d(const fst_model* m, const DeviceModel& dm, int dtype, int64_t n, const void* const* coords,
                   void* out, void* stream);
int device_cu_count();
// reconstruction of a model with wavelet factors (d = 3 or 4): arithmetic in dtype, points and
// values in in_dtype; idx (may be NULL) selects the points; residual: out = v - f in dtype
void launch_eval_wave(const fst_model* m, const DeviceModel& dm, int dtype, int in_dtype, int64_t n,
                      const void* const* coords, const int32_t* idx, const void* v, void* out, bool residual,
                      void* stream);
// out_host[(D + 1) t + k] = coordinate k of point idx_host[t] (k < D), then its value, in FP64
void gather_points_d(int dtype, int64_t K, const int64_t* idx_host, int D, const void* const* coords, const void* v,
                     double* out_host, void* ws, size_t ws_bytes, void* stream);
size_t gather_workspace_bytes(int64_t K, int D);
size_t eval_grid_workspace_bytes(const fst_model* m, int dtype, int64_t n1, int64_t n2, int64_t n3);
void eval_grid(const fst_model* m, const DeviceModel& dm, int dtype, const void* gx, int64_t n1, const void* gy,
               int64_t n2, const void* gz, int64_t n3, void* out, void* ws, void* stream);
void eval_error(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z,
                const void* v, void* ws, size_t ws_bytes, void* stream, double out[2]);
size_t solve_scratch_bytes(const fst_model* m, int64_t M);
// Cholesky + solve + refinement of one sampled system with the precision ladder (fst_api.cpp).
// On entry G holds the Gram at gram_prec and h = A^T v from the rows U, vs.
// Gsave (may be NULL): room for a copy of G (R x R doubles), used with a split gram_prec to
// factor the same Gram again with dependent columns skipped before climbing to FP64 rows.
SolveInfo solve_core(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z,
                     const void* v, const int32_t* idx, int64_t M, const void* U, const void* vs, int gram_prec,
                     int refine, double* G, double* h, double* alpha, void* scr, size_t scr_bytes, void* stream,
                     double* Gsave = nullptr);
size_t gram_f64_rows_workspace_bytes(const fst_model* m, int64_t mrows);
void gram_from_f64_rows(const fst_model* m, int dtype, int64_t n, const void* x, const void* y,
                        const void* z, const void* v, const int32_t* idx, int64_t mrows, double* G,
                        double* h, void* ws, size_t ws_bytes, void* stream);
void* eval_graph_create(const std::vector<const fst_model*>& models, int dtype, int64_t n, const void* x,
                        const void* y, const void* z, const std::vector<void*>& outs);
void eval_graph_launch(void* graph, void* stream);
void eval_graph_free(void* graph);
void gather_points(int dtype, int64_t K, const int64_t* idx_host, const void* x,
                   const void* y, const void* z, const void* v, double* out_host, void* ws,
                   size_t ws_bytes, void* stream);
void device_axpy(int64_t n, double a, const double* x, double* y, void* stream);
void stream_sync(void* stream);
void set_device(int dev);
void* stream_create();            // a non-blocking stream of default priority on the current device
void stream_destroy(void* stream);
void* device_alloc(size_t bytes);
void device_free(void* p);
void copy_h2d(void* dst, const void* src, size_t bytes, void* stream);
void copy_d2h(void* dst, const void* src, size_t bytes, void* stream);
void copy_d2d(void* dst, const void* src, size_t bytes, void* stream);

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace fst
