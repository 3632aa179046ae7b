// Internal declarations of the residual corrector (3 -> 64 -> 64 -> 1 SiLU network).
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "fst_internal.h"

namespace fst {

constexpr int kMlpHidden = 64;
// flat parameter order: W1 (64 x 3) | b1 (64) | W2 (64 x 64, [out][in]) | b2 (64) | W3 (64) | b3
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 256, kOffB2 = 4352, kOffW3 = 4416, kOffB3 = 4480;
constexpr int kMlpParams = 4481;

struct MlpAdam {
  double lr = 1e-3, beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
  bool fp32 = false;   // the 64 x 64 layer in FP32 (reference mode) instead of BF16 MFMA
};

struct CorrectorDeviceCache {
  float* P = nullptr;
  void* W2b = nullptr;
  void* W2Tb = nullptr;
};

std::vector<float> mlp_init_params(uint64_t seed);
size_t mlp_train_workspace_bytes(int32_t batch);
void mlp_train(int dtype, const double lo[3], const double hi[3], int64_t n, const void* x, const void* y,
               const void* z, const float* target, const int32_t* idx, int32_t batch, int64_t first_step,
               int64_t steps, uint64_t seed, const MlpAdam& opt, std::vector<float>& P, float* grad_out_dev,
               std::vector<float>* losses, void* ws, size_t ws_bytes, void* stream);
void mlp_apply(int dtype, const double lo[3], const double hi[3], const std::vector<float>& stored,
               float out_scale, int64_t n, const void* x, const void* y, const void* z, void* out,
               CorrectorDeviceCache& cache, void* stream);
void free_corrector_cache(CorrectorDeviceCache& c);
// values v - u~(x) at all n points (FP64 arithmetic for FP64 data, FP32 otherwise)
void launch_residual_values(const fst_model* m, int dtype, int64_t n, const void* x, const void* y,
                            const void* z, const void* v, void* out, void* stream);

}  // namespace fst

struct fst_corrector {
  double lo[3], hi[3];
  std::vector<float> P;      // stored parameters: BF16-rounded values, FP32 container
  float out_scale = 1.0f;    // the network predicts residual / out_scale
  std::vector<float> losses; // training loss, sampled every 50 steps
  mutable std::mutex mu;
  mutable std::map<int, fst::CorrectorDeviceCache> dev;
  ~fst_corrector() {
    for (auto& kv : dev) fst::free_corrector_cache(kv.second);
  }
};
