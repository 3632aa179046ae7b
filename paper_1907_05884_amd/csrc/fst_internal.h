// Internal declarations shared by the host C++ files and the HIP kernel file.
#pragma once

#include <cstddef>
#include <cstdint>
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

// Error carried from deep inside the library to the C ABI boundary, where it becomes a
// status code plus a thread-local message.
struct Error : std::runtime_error {
  fst_status code;
  Error(fst_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};
[[noreturn]] void fail(fst_status code, const std::string& msg);
void set_last_error(const std::string& msg);

// Device copy of a model for one (device, dtype): coefficient matrices padded to
// kMaxBasis x kMaxRank per mode, and the core in C order.
struct DeviceModel {
  void* coefs = nullptr;   // 3 * kMaxBasis * kMaxRank elements of the dtype
  void* core = nullptr;    // R elements of the dtype
  void* core64 = nullptr;  // R doubles (for refinement), only for dtype FP64 copy
};

}  // namespace fst

struct fst_model {
  double lo[3], hi[3];
  int32_t rank[3], degree[3];
  std::vector<double> core;      // r1 r2 r3, C order
  std::vector<double> coef[3];   // (p_k + 1) x r_k row-major
  // lazily uploaded device copies, keyed by (device ordinal, dtype)
  mutable std::mutex mu;
  mutable std::map<std::pair<int, int>, fst::DeviceModel> dev;
  ~fst_model();
  int64_t R() const { return (int64_t)rank[0] * rank[1] * rank[2]; }
  int sum_r() const { return rank[0] + rank[1] + rank[2]; }
};

namespace fst {

// ---------------------------------------------------------------- host steps (fst_host.cpp)
uint64_t splitmix64_next(uint64_t& state);
void sample_indices(uint64_t seed, int stream, int64_t n, int64_t m, int64_t* out);
void idw_grid(const double* xi, const double* v, int64_t K, const int32_t grid[3], int k,
              double power, int n_threads, double* out);
void sthosvd(const double* T, const int32_t dims[3], const int32_t rank[3], int n_threads,
             double* core, double* const W[3], double* const sigma[3]);
void sparse_fit(const double* W, int I, int r, int p, double* C);
void legendre_orthonormal_host(double t, int p, double* phi);
int hardware_threads(int requested);

// ---------------------------------------------------------------- model (fst_model.cpp)
fst_model* model_new(const double lo[3], const double hi[3], const int32_t rank[3],
                     const int32_t degree[3]);
void check_model(const fst_model* m);
const DeviceModel& device_model(const fst_model* m, int dtype);   // uploads on first use

// ---------------------------------------------------------------- GPU launchers (fst_kernels.hip)
int current_device();
void check_hip(int err, const char* what);
void launch_factor_eval(const fst_model* m, const DeviceModel& dm, int dtype, int64_t n,
                        const void* x, const void* y, const void* z, const void* v,
                        const int32_t* idx, int64_t mrows, void* U, void* vs, void* stream);
size_t gram_workspace_bytes(const fst_model* m, int64_t mrows);
void launch_gram(const fst_model* m, int dtype, int64_t mrows, const void* U, const void* vs,
                 int gram_prec, double* G, double* h, void* ws, size_t ws_bytes, void* stream);
size_t cholesky_workspace_bytes(int64_t R);
// returns 0 on success, else the 1-based index of the failing pivot
int64_t cholesky(int64_t R, double* G, void* ws, size_t ws_bytes, void* stream);
void cholesky_solve(int64_t R, const double* L, const double* b, double* x, void* stream);
void launch_eval(const fst_model* m, const DeviceModel& dm, int dtype, int64_t n,
                 const void* x, const void* y, const void* z, const int32_t* idx,
                 const void* v, void* out, void* stream);
size_t residual_workspace_bytes(const fst_model* m, int64_t mrows);
void residual(const fst_model* m, int dtype, int64_t n, const void* x, const void* y,
              const void* z, const void* v, const int32_t* idx, int64_t mrows,
              const double* alpha, double* r, void* ws, size_t ws_bytes, void* stream);
void gather_points(int dtype, int64_t K, const int64_t* idx_host, const void* x,
                   const void* y, const void* z, const void* v, double* out_host, void* ws,
                   size_t ws_bytes, void* stream);
void device_axpy(int64_t n, double a, const double* x, double* y, void* stream);
void stream_sync(void* stream);
void* device_alloc(size_t bytes);
void device_free(void* p);
void copy_h2d(void* dst, const void* src, size_t bytes, void* stream);
void copy_d2h(void* dst, const void* src, size_t bytes, void* stream);
void copy_d2d(void* dst, const void* src, size_t bytes, void* stream);

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace fst
