// C ABI of the learned residual corrector: training on the functional Tucker residual,
// inference added to the reconstruction, gradient evaluation for parity checks.
#include <cmath>
#include <cstring>

#include "fst_mlp.h"

namespace {

void check_train_params(const fst_train_params* tp) {
  if (!tp) fst::fail(FST_E_INVAL, "null training parameters");
  if (tp->struct_size != sizeof(fst_train_params)) fst::fail(FST_E_INVAL, "fst_train_params.struct_size mismatch");
  if (tp->steps < 0 || tp->steps > 10000000) fst::fail(FST_E_INVAL, "steps out of range");
  if (tp->batch < 1 || tp->batch > (1 << 22)) fst::fail(FST_E_INVAL, "batch out of range");
  if (!(tp->lr > 0 && tp->beta1 >= 0 && tp->beta1 < 1 && tp->beta2 >= 0 && tp->beta2 < 1 && tp->eps > 0))
    fst::fail(FST_E_INVAL, "bad Adam hyper-parameters");
}

// BF16 rounding (round to nearest even) of an FP32 value, kept in an FP32 container
float round_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return f;
  uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7fffu + lsb) & 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

fst::CorrectorDeviceCache& cache_of(const fst_corrector* c) {
  int d = fst::current_device();
  std::lock_guard<std::mutex> lk(c->mu);
  return c->dev[d];
}

fst::MlpAdam adam_of(const fst_train_params* tp) {
  fst::MlpAdam a;
  a.lr = tp->lr;
  a.beta1 = tp->beta1;
  a.beta2 = tp->beta2;
  a.eps = tp->eps;
  return a;
}

}  // namespace

#define FST_TRY try {
#define FST_CATCH                                   \
  }                                                 \
  catch (const fst::Error& e) {                     \
    fst::set_last_error(e.what());                  \
    return e.code;                                  \
  }                                                 \
  catch (const std::bad_alloc&) {                   \
    fst::set_last_error("host allocation failed");  \
    return FST_E_NOMEM;                             \
  }                                                 \
  catch (const std::exception& e) {                 \
    fst::set_last_error(e.what());                  \
    return FST_E_INVAL;                             \
  }

extern "C" {

void fst_train_params_default(fst_train_params* tp) {
  if (!tp) return;
  std::memset(tp, 0, sizeof(*tp));
  tp->struct_size = sizeof(fst_train_params);
  tp->steps = 2000;
  tp->batch = 8192;
  tp->lr = 1e-3;
  tp->beta1 = 0.9;
  tp->beta2 = 0.999;
  tp->eps = 1e-8;
  tp->seed = 1;
  tp->init_params = nullptr;
}

size_t fst_corrector_workspace_bytes(const fst_train_params* tp, int64_t n) {
  try {
    check_train_params(tp);
    return fst::mlp_train_workspace_bytes(tp->batch) + 2 * fst::align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1));
  } catch (const std::exception& e) {
    fst::set_last_error(e.what());
    return 0;
  }
}

fst_status fst_corrector_train(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                               const void* z, const void* v, const fst_train_params* tp, void* ws,
                               size_t ws_bytes, void* stream, fst_corrector** out) {
  FST_TRY
  fst::set_last_error("");
  fst::check_model3(m);
  check_train_params(tp);
  if (dtype != FST_F64 && dtype != FST_F32) fst::fail(FST_E_INVAL, "bad dtype");
  if (n < 2 || n >= (int64_t(1) << 31)) fst::fail(FST_E_INVAL, "need 2 <= n < 2^31 training points");
  if (!x || !y || !z || !v || !out || !ws) fst::fail(FST_E_INVAL, "null argument");
  if (ws_bytes < fst_corrector_workspace_bytes(tp, n)) fst::fail(FST_E_NOMEM, "corrector: workspace too small");
  const size_t es = dtype == FST_F64 ? sizeof(double) : sizeof(float);
  char* base = (char*)ws;
  void* d_res = base;                                       // residual v - u~(x) in the data type
  float* d_target = (float*)(base + fst::align_up(sizeof(double) * (size_t)n));
  void* d_train = base + 2 * fst::align_up(sizeof(double) * (size_t)n);
  // residual of the functional Tucker model at every training point
  fst::launch_residual_values(m, dtype, n, x, y, z, v, d_res, stream);
  std::vector<double> e((size_t)n);
  if (dtype == FST_F64) {
    fst::copy_d2h(e.data(), d_res, es * (size_t)n, stream);
  } else {
    std::vector<float> ef((size_t)n);
    fst::copy_d2h(ef.data(), d_res, es * (size_t)n, stream);
    for (int64_t i = 0; i < n; ++i) e[(size_t)i] = ef[(size_t)i];
  }
  double mean = 0.0, sq = 0.0;
  for (double t : e) {
    if (!std::isfinite(t)) fst::fail(FST_E_INVAL, "non-finite residual (coordinates or values)");
    mean += t;
  }
  mean /= (double)n;
  for (double t : e) sq += (t - mean) * (t - mean);
  double sd = std::sqrt(sq / (double)n);
  if (!(sd > 0)) sd = 1.0;
  std::vector<float> target((size_t)n);
  for (int64_t i = 0; i < n; ++i) target[(size_t)i] = (float)(e[(size_t)i] / sd);
  if (tp->init_params)
    for (int j = 0; j < fst::kMlpParams; ++j)
      if (!std::isfinite(tp->init_params[j])) fst::fail(FST_E_INVAL, "non-finite initial parameter");
  fst::copy_h2d(d_target, target.data(), sizeof(float) * (size_t)n, stream);
  std::unique_ptr<fst_corrector> c(new fst_corrector());
  for (int k = 0; k < 3; ++k) {
    c->lo[k] = m->lo[k];
    c->hi[k] = m->hi[k];
  }
  c->out_scale = (float)sd;
  std::vector<float> P = tp->init_params ? std::vector<float>(tp->init_params, tp->init_params + fst::kMlpParams)
                                         : fst::mlp_init_params(tp->seed);
  fst::mlp_train(dtype, m->lo, m->hi, n, x, y, z, d_target, nullptr, tp->batch, 0, tp->steps, tp->seed,
                 adam_of(tp), P, nullptr, &c->losses, d_train, ws_bytes - (size_t)((char*)d_train - base), stream);
  c->P.resize(P.size());
  for (size_t j = 0; j < P.size(); ++j) c->P[j] = round_bf16(P[j]);
  *out = c.release();
  return FST_OK;
  FST_CATCH
}

fst_status fst_corrector_from_params(const double lo[3], const double hi[3], const float* params, float out_scale,
                                     fst_corrector** out) {
  FST_TRY
  fst::set_last_error("");
  if (!lo || !hi || !params || !out) fst::fail(FST_E_INVAL, "null argument");
  std::unique_ptr<fst_corrector> c(new fst_corrector());
  for (int k = 0; k < 3; ++k) {
    if (!(std::isfinite(lo[k]) && std::isfinite(hi[k]) && hi[k] > lo[k])) fst::fail(FST_E_INVAL, "bad box");
    c->lo[k] = lo[k];
    c->hi[k] = hi[k];
  }
  c->P.assign(params, params + fst::kMlpParams);
  for (float t : c->P)
    if (!std::isfinite(t)) fst::fail(FST_E_INVAL, "non-finite parameter");
  c->out_scale = out_scale;
  *out = c.release();
  return FST_OK;
  FST_CATCH
}

fst_status fst_corrector_params(const fst_corrector* c, float* params_out, float* out_scale) {
  FST_TRY
  fst::set_last_error("");
  if (!c) fst::fail(FST_E_INVAL, "null corrector");
  if (params_out) std::memcpy(params_out, c->P.data(), sizeof(float) * c->P.size());
  if (out_scale) *out_scale = c->out_scale;
  return FST_OK;
  FST_CATCH
}

fst_status fst_corrector_losses(const fst_corrector* c, float* out, int32_t* count) {
  FST_TRY
  fst::set_last_error("");
  if (!c || !count) fst::fail(FST_E_INVAL, "null argument");
  if (out) std::memcpy(out, c->losses.data(), sizeof(float) * std::min<size_t>(c->losses.size(), (size_t)*count));
  *count = (int32_t)c->losses.size();
  return FST_OK;
  FST_CATCH
}

void fst_corrector_free(fst_corrector* c) { delete c; }

int64_t fst_corrector_stored_bytes(const fst_corrector* c) {
  if (!c) return -1;
  return 2 * (int64_t)fst::kMlpParams + 4;
}

fst_status fst_corrector_apply(const fst_corrector* c, int32_t dtype, int64_t n, const void* x, const void* y,
                               const void* z, void* out, void* stream) {
  FST_TRY
  fst::set_last_error("");
  if (!c) fst::fail(FST_E_INVAL, "null corrector");
  if (dtype != FST_F64 && dtype != FST_F32) fst::fail(FST_E_INVAL, "bad dtype");
  if (n < 0 || n >= (int64_t(1) << 31)) fst::fail(FST_E_INVAL, "bad n");
  if (n == 0) return FST_OK;
  if (!x || !y || !z || !out) fst::fail(FST_E_INVAL, "null argument");
  fst::mlp_apply(dtype, c->lo, c->hi, c->P, c->out_scale, n, x, y, z, out, cache_of(c), stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_eval_corrected(const fst_model* m, const fst_corrector* c, int32_t dtype, int64_t n, const void* x,
                              const void* y, const void* z, void* out, void* stream) {
  fst_status st = fst_eval(m, dtype, n, x, y, z, out, stream);
  if (st != FST_OK || !c) return st;
  return fst_corrector_apply(c, dtype, n, x, y, z, out, stream);
}

static fst_status mlp_grad_impl(const fst_corrector* c, int32_t dtype, int64_t n, const void* x, const void* y,
                                const void* z, const float* target, const int32_t* idx, int32_t batch,
                                float* grad_out, void* ws, size_t ws_bytes, void* stream, bool fp32) {
  FST_TRY
  fst::set_last_error("");
  if (!c) fst::fail(FST_E_INVAL, "null corrector");
  if (dtype != FST_F64 && dtype != FST_F32) fst::fail(FST_E_INVAL, "bad dtype");
  if (batch < 1 || n < 1) fst::fail(FST_E_INVAL, "bad sizes");
  if (!x || !y || !z || !target || !idx || !grad_out || !ws) fst::fail(FST_E_INVAL, "null argument");
  std::vector<float> P = c->P;
  fst::MlpAdam opt;
  opt.fp32 = fp32;
  fst::mlp_train(dtype, c->lo, c->hi, n, x, y, z, target, idx, batch, 0, 0, 0, opt, P, grad_out, nullptr, ws,
                 ws_bytes, stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_mlp_grad(const fst_corrector* c, int32_t dtype, int64_t n, const void* x, const void* y, const void* z,
                        const float* target, const int32_t* idx, int32_t batch, float* grad_out, void* ws,
                        size_t ws_bytes, void* stream) {
  return mlp_grad_impl(c, dtype, n, x, y, z, target, idx, batch, grad_out, ws, ws_bytes, stream, false);
}

fst_status fst_mlp_grad_fp32(const fst_corrector* c, int32_t dtype, int64_t n, const void* x, const void* y,
                             const void* z, const float* target, const int32_t* idx, int32_t batch,
                             float* grad_out, void* ws, size_t ws_bytes, void* stream) {
  return mlp_grad_impl(c, dtype, n, x, y, z, target, idx, batch, grad_out, ws, ws_bytes, stream, true);
}

size_t fst_mlp_grad_workspace_bytes(int32_t batch) { return fst::mlp_train_workspace_bytes(batch); }

}  // extern "C"
