// Batched form: many field variables on one shared point set.  Algorithm 1 runs per variable
// on host threads (the nearest-neighbour search of the interpolation is shared, since every
// variable uses the same subset); Algorithm 2 runs on the GPU with the Gram of every variable
// in one persistent launch; reconstructions of all variables can be replayed as one graph.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>

#include "fst_internal.h"

namespace {

struct DeviceBuffer {
  void* p = nullptr;
  explicit DeviceBuffer(size_t bytes) : p(fst::device_alloc(bytes)) {}
  ~DeviceBuffer() { fst::device_free(p); }
  DeviceBuffer(const DeviceBuffer&) = delete;
  DeviceBuffer& operator=(const DeviceBuffer&) = delete;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct fst_graph {
  void* g = nullptr;
  ~fst_graph() { fst::eval_graph_free(g); }
};

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

fst_status fst_fit_batched(const fst_fit_params* base, int32_t V, const int32_t* ranks, const int32_t* degrees,
                           int64_t n, const void* x, const void* y, const void* z, const void* const* values,
                           void* stream, fst_model** out, int32_t* gram_prec_used, double* timings) {
  FST_TRY
  fst::set_last_error("");
  if (!base || !ranks || !degrees || !values || !out || !x || !y || !z) fst::fail(FST_E_INVAL, "null argument");
  if (V < 1 || V > 4096) fst::fail(FST_E_INVAL, "V must be in [1, 4096]");
  if (base->struct_size == sizeof(fst_fit_params) && base->eps != 0.0)
    fst::fail(FST_E_UNSUPPORTED, "the batched form takes fixed ranks (eps must be 0)");
  if (base->struct_size == sizeof(fst_fit_params) && base->wavelet_level != 0)
    fst::fail(FST_E_UNSUPPORTED, "the batched form fits Legendre factors only (wavelet_level must be 0)");
  // every variable must form a valid problem on its own
  std::vector<fst_fit_params> pv((size_t)V, *base);
  for (int v = 0; v < V; ++v) {
    for (int k = 0; k < 3; ++k) {
      pv[(size_t)v].rank[k] = ranks[3 * v + k];
      pv[(size_t)v].degree[k] = degrees[3 * v + k];
    }
    if (!values[v]) fst::fail(FST_E_INVAL, "null value array");
    size_t need = fst_fit_workspace_bytes(&pv[(size_t)v], n);
    if (need == 0) throw fst::Error(FST_E_INVAL, std::string("variable ") + std::to_string(v) + ": " + fst_last_error());
  }
  const double t0 = now_s();
  // Algorithm 1 step 1: one shared subset (stream 1 of the base seed)
  const int64_t K = llround(base->interp_fraction * (double)n);
  std::vector<int64_t> sub((size_t)K);
  fst::sample_indices(base->seed, FST_STREAM_INTERP, n, K, sub.data());
  std::vector<double> xi((size_t)K * 3);
  std::vector<std::vector<double>> vals((size_t)V, std::vector<double>((size_t)K));
  {
    DeviceBuffer gws(fst::align_up(sizeof(int32_t) * (size_t)K) + sizeof(double) * 4 * (size_t)K);
    std::vector<double> xyzv((size_t)K * 4);
    for (int v = 0; v < V; ++v) {
      fst::gather_points(base->dtype, K, sub.data(), x, y, z, values[v], xyzv.data(), gws.p,
                         fst::align_up(sizeof(int32_t) * (size_t)K) + sizeof(double) * 4 * (size_t)K, stream);
      for (int64_t i = 0; i < K; ++i) {
        if (v == 0)
          for (int k = 0; k < 3; ++k) {
            double c = xyzv[(size_t)(4 * i + k)];
            if (!std::isfinite(c)) fst::fail(FST_E_INVAL, "non-finite coordinate in the interpolation subset");
            xi[(size_t)(3 * i + k)] = 2.0 * (c - base->lo[k]) / (base->hi[k] - base->lo[k]) - 1.0;
          }
        double t = xyzv[(size_t)(4 * i + 3)];
        if (!std::isfinite(t)) fst::fail(FST_E_INVAL, "non-finite value in the interpolation subset");
        vals[(size_t)v][(size_t)i] = t;
      }
    }
  }
  // shared nearest neighbours, then per-variable interpolation, ST-HOSVD and sparse fits
  std::vector<int64_t> nbr;
  std::vector<double> wgt;
  std::vector<int32_t> cnt;
  const int kk = (int)std::min<int64_t>(std::max(base->idw_k, 1), K);
  fst::idw_knn(xi.data(), K, base->grid, kk, base->idw_power, base->n_threads, nbr, wgt, cnt);
  std::vector<std::unique_ptr<fst_model>> m0((size_t)V);
  {
    std::atomic<int> next(0);
    std::vector<std::string> errs((size_t)V);
    const int nth = std::min(fst::hardware_threads(base->n_threads), V);
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&] {
        for (int v = next++; v < V; v = next++) {
          try {
            const fst_fit_params& p = pv[(size_t)v];
            const int64_t nodes = (int64_t)p.grid[0] * p.grid[1] * p.grid[2];
            std::vector<double> T((size_t)nodes);
            fst::idw_apply(nbr, wgt, cnt, kk, vals[(size_t)v].data(), 1, T.data());
            std::unique_ptr<fst_model> m(fst::model_new(p.lo, p.hi, p.rank, p.degree));
            std::vector<double> W[3];
            double* Wp[3];
            for (int k = 0; k < 3; ++k) {
              W[k].assign((size_t)p.grid[k] * p.rank[k], 0.0);
              Wp[k] = W[k].data();
            }
            fst::sthosvd(T.data(), p.grid, p.rank, 1, m->core.data(), Wp, nullptr);
            for (int k = 0; k < 3; ++k)
              fst::sparse_fit_with(p.sparse_solver, W[k].data(), p.grid[k], p.rank[k], p.degree[k],
                                   m->coef[k].data());
            m0[(size_t)v] = std::move(m);
          } catch (const std::exception& e) {
            errs[(size_t)v] = e.what();
          }
        }
      });
    for (auto& t : th) t.join();
    for (int v = 0; v < V; ++v)
      if (!errs[(size_t)v].empty()) fst::fail(FST_E_INVAL, "variable " + std::to_string(v) + ": " + errs[(size_t)v]);
  }
  const double t1 = now_s();
  // Algorithm 2 on the GPU: rows of every variable (seed + v, stream 2), then all Gram
  // matrices in one persistent launch, then per-variable solves
  const int dtype = base->dtype;
  const size_t es = dtype == FST_F64 ? sizeof(double) : sizeof(float);
  const int64_t M = base->n_samples;
  // the sampled rows of every variable (seed + v, stream 2), drawn on host threads
  std::vector<std::vector<int32_t>> rows((size_t)V);
  {
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    const int nth = std::min(fst::hardware_threads(base->n_threads), V);
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&] {
        try {
          std::vector<int64_t> idx((size_t)M);
          for (int v = next++; v < V; v = next++) {
            fst::sample_indices(base->seed + (uint64_t)v, FST_STREAM_LS, n, M, idx.data());
            rows[(size_t)v].assign(idx.begin(), idx.end());
          }
        } catch (...) {
          next = V;   // the missing rows are reported below
        }
      });
    for (auto& t : th) t.join();
    for (int v = 0; v < V; ++v)
      if ((int64_t)rows[(size_t)v].size() != M) fst::fail(FST_E_NOMEM, "sampling the least-squares rows failed");
  }
  std::vector<std::unique_ptr<DeviceBuffer>> bU, bvs, bidx, bG, bh, ba;
  std::vector<const fst_model*> mods;
  std::vector<const void*> Up;
  std::vector<int64_t> Ms;
  std::vector<double*> Gp;
  size_t scr_need = 0;
  for (int v = 0; v < V; ++v) {
    const fst_model* m = m0[(size_t)v].get();
    const int64_t R = m->R();
    bU.emplace_back(new DeviceBuffer(es * (size_t)m->sum_r() * (size_t)M));
    bvs.emplace_back(new DeviceBuffer(es * (size_t)M));
    bidx.emplace_back(new DeviceBuffer(sizeof(int32_t) * (size_t)M));
    bG.emplace_back(new DeviceBuffer(sizeof(double) * (size_t)R * (size_t)R));
    bh.emplace_back(new DeviceBuffer(sizeof(double) * (size_t)R));
    ba.emplace_back(new DeviceBuffer(sizeof(double) * (size_t)R));
    scr_need = std::max(scr_need, fst::solve_scratch_bytes(m, M));
    fst::copy_h2d(bidx.back()->p, rows[(size_t)v].data(), sizeof(int32_t) * (size_t)M, stream);
    const fst::DeviceModel& dm = fst::device_model(m, dtype);
    fst::launch_factor_eval(m, dm, dtype, n, x, y, z, values[v], (const int32_t*)bidx.back()->p, M, bU.back()->p,
                            bvs.back()->p, stream);
    mods.push_back(m);
    Up.push_back(bU.back()->p);
    Ms.push_back(M);
    Gp.push_back((double*)bG.back()->p);
  }
  DeviceBuffer scr(scr_need);
  fst::stream_sync(stream);
  const double t2 = now_s();
  if (fst::split_terms(base->gram_prec) > 0) {
    // split 16-bit rows: the row planes of as many variables as the workspace holds, then one
    // launch over all their tiles (the workspace takes what the device can spare, at least
    // the planes of the largest variable)
    size_t all = 0, largest = 0;
    for (const fst_model* m : mods) {
      all += fst::split_rows_bytes(m, base->gram_prec, M);
      largest = std::max(largest, fst::split_rows_bytes(m, base->gram_prec, M));
    }
    const size_t lo = fst::gram_split_batched_min_bytes(mods, base->gram_prec, M);
    size_t want = lo - largest + all;   // every variable's planes at once
    const size_t spare = fst::device_free_bytes();
    if (spare < want + (size_t(8) << 30)) want = std::max(lo, spare > (size_t(8) << 30) ? spare - (size_t(8) << 30) : 0);
    DeviceBuffer pws(want);
    fst::gram_split_batched(mods, Up, M, Gp, base->gram_prec, pws.p, want, stream);
  } else {
    fst::launch_gram_batched(mods, Up, Ms, Gp, base->gram_prec, scr.p, stream);
  }
  fst::stream_sync(stream);
  const double t3 = now_s();
  for (int v = 0; v < V; ++v)
    fst::launch_gram(mods[(size_t)v], dtype, M, Up[(size_t)v], bvs[(size_t)v]->p, base->gram_prec, nullptr,
                     (double*)bh[(size_t)v]->p, scr.p, scr_need, stream);
  fst::stream_sync(stream);
  const double t3b = now_s();
  // Cholesky, solve and refinement of every variable, with the precision ladder (a Gram that
  // breaks down, or whose refinement stops above its tolerance, is formed again from more
  // precise rows).  Variables run concurrently on a few streams of their own, largest R first,
  // so that the latency-bound factorisations of the small systems overlap.
  std::vector<fst::SolveInfo> infos((size_t)V);
  {
    std::vector<int> order((size_t)V);
    for (int v = 0; v < V; ++v) order[(size_t)v] = v;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mods[(size_t)a]->R() > mods[(size_t)b]->R(); });
    const int nst = std::min(V, 4);
    const int dev = fst::current_device();
    std::atomic<int> next(0);
    std::vector<std::string> errs((size_t)V);
    std::vector<fst_status> codes((size_t)V, FST_OK);
    std::vector<std::unique_ptr<DeviceBuffer>> scratch, gsave;
    int64_t maxR = 0;
    for (const fst_model* m : mods) maxR = std::max<int64_t>(maxR, m->R());
    const bool split = fst::split_terms(base->gram_prec) > 0;
    for (int t = 0; t < nst; ++t) {
      scratch.emplace_back(new DeviceBuffer(scr_need));
      if (split) gsave.emplace_back(new DeviceBuffer(sizeof(double) * (size_t)maxR * (size_t)maxR));
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nst; ++t)
      th.emplace_back([&, t] {
        void* st = nullptr;
        try {
          fst::set_device(dev);
          st = fst::stream_create();
        } catch (const fst::Error& e) {
          for (int k = next++; k < V; k = next++) {
            errs[(size_t)order[(size_t)k]] = e.what();
            codes[(size_t)order[(size_t)k]] = e.code;
          }
          return;
        }
        for (int k = next++; k < V; k = next++) {
          const int v = order[(size_t)k];
          const fst_model* m = mods[(size_t)v];
          const int64_t R = m->R();
          double* alpha = (double*)ba[(size_t)v]->p;
          try {
            infos[(size_t)v] = fst::solve_core(m, dtype, n, x, y, z, values[v], (const int32_t*)bidx[(size_t)v]->p,
                                               M, Up[(size_t)v], bvs[(size_t)v]->p, base->gram_prec,
                                               base->refine_steps, Gp[(size_t)v], (double*)bh[(size_t)v]->p, alpha,
                                               scratch[(size_t)t]->p, scr_need, st,
                                               split ? (double*)gsave[(size_t)t]->p : nullptr);
            std::vector<double> core((size_t)R);
            fst::copy_d2h(core.data(), alpha, sizeof(double) * (size_t)R, st);
            for (double c : core)
              if (!std::isfinite(c)) fst::fail(FST_E_NOT_SPD, "non-finite core");
            m0[(size_t)v]->core = core;
          } catch (const fst::Error& e) {
            errs[(size_t)v] = e.what();
            codes[(size_t)v] = e.code;
          } catch (const std::exception& e) {
            errs[(size_t)v] = e.what();
            codes[(size_t)v] = FST_E_INVAL;
          }
        }
        fst::stream_sync(st);
        fst::stream_destroy(st);
      });
    for (auto& t : th) t.join();
    for (int v = 0; v < V; ++v)
      if (codes[(size_t)v] != FST_OK)
        throw fst::Error(codes[(size_t)v], "variable " + std::to_string(v) + ": " + errs[(size_t)v]);
  }
  const double t4 = now_s();
  for (int v = 0; v < V; ++v) {
    // the device copies uploaded with the refit-time core are stale: rebuild the objects
    const fst_model* m = m0[(size_t)v].get();
    fst_model* fresh = fst::model_new(m->lo, m->hi, m->rank, m->degree);
    fresh->core = m->core;
    for (int k = 0; k < 3; ++k) fresh->coef[k] = m->coef[k];
    fresh->fit = infos[(size_t)v];
    out[v] = fresh;
  }
  if (gram_prec_used)
    for (int v = 0; v < V; ++v) gram_prec_used[v] = infos[(size_t)v].gram_prec;
  if (timings) {
    timings[0] = t1 - t0;   // host steps
    timings[1] = t2 - t1;   // row generation (sampling, upload, factor values)
    timings[2] = t3 - t2;   // batched Gram
    timings[3] = t3b - t3;  // A^T v
    timings[4] = t4 - t3b;  // Cholesky, solves, refinement
  }
  return FST_OK;
  FST_CATCH
}

fst_status fst_eval_batched(const fst_model* const* models, int32_t V, int32_t dtype, int64_t n, const void* x,
                            const void* y, const void* z, void* const* outs, void* stream) {
  FST_TRY
  fst::set_last_error("");
  if (!models || !outs || V < 1) fst::fail(FST_E_INVAL, "bad arguments");
  for (int v = 0; v < V; ++v) {
    fst_status st = fst_eval(models[v], dtype, n, x, y, z, outs[v], stream);
    if (st != FST_OK) return st;
  }
  return FST_OK;
  FST_CATCH
}

fst_status fst_eval_graph_create(const fst_model* const* models, int32_t V, int32_t dtype, int64_t n, const void* x,
                                 const void* y, const void* z, void* const* outs, fst_graph** out) {
  FST_TRY
  fst::set_last_error("");
  if (!models || !outs || !out || V < 1 || !x || !y || !z) fst::fail(FST_E_INVAL, "bad arguments");
  if (dtype != FST_F64 && dtype != FST_F32) fst::fail(FST_E_INVAL, "bad dtype");
  if (n < 1 || n >= (int64_t(1) << 31)) fst::fail(FST_E_INVAL, "bad n");
  std::vector<const fst_model*> ms(models, models + V);
  std::vector<void*> os(outs, outs + V);
  for (int v = 0; v < V; ++v) {
    if (!os[(size_t)v]) fst::fail(FST_E_INVAL, "null model or output");
    fst::check_model3(ms[(size_t)v]);
  }
  std::unique_ptr<fst_graph> g(new fst_graph());
  g->g = fst::eval_graph_create(ms, dtype, n, x, y, z, os);
  *out = g.release();
  return FST_OK;
  FST_CATCH
}

fst_status fst_graph_launch(const fst_graph* g, void* stream) {
  FST_TRY
  fst::set_last_error("");
  if (!g) fst::fail(FST_E_INVAL, "null graph");
  fst::eval_graph_launch(g->g, stream);
  return FST_OK;
  FST_CATCH
}

void fst_graph_free(fst_graph* g) { delete g; }

}  // extern "C"
