// C ABI entry points: argument validation, error reporting, and the orchestration of
// Algorithm 1 (host steps) and Algorithm 2 (GPU refit of the core).
#include <cmath>
#include <limits>
#include <cstring>
#include <new>

#include "fst_internal.h"

namespace fst {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
[[noreturn]] void fail(fst_status code, const std::string& msg) { throw Error(code, msg); }

// Owns a device workspace when the caller passes none.
struct Workspace {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = false;
  Workspace(void* user, size_t user_bytes, size_t need) {
    if (user) {
      if (user_bytes < need)
        fail(FST_E_NOMEM, "workspace too small: " + std::to_string(user_bytes) + " < " + std::to_string(need));
      p = user;
      bytes = user_bytes;
    } else {
      p = device_alloc(need);
      bytes = need;
      owned = true;
    }
  }
  ~Workspace() {
    if (owned) device_free(p);
  }
};

static void check_dtype(int dtype) {
  if (dtype != FST_F64 && dtype != FST_F32) fail(FST_E_INVAL, "dtype must be FST_F64 or FST_F32");
}
static void check_prec(int dtype, int gram_prec) {
  if (dtype == FST_F64 && gram_prec != FST_GRAM_F64) fail(FST_E_INVAL, "FP64 points need gram_prec FST_GRAM_F64");
  if (dtype == FST_F32 && gram_prec != FST_GRAM_F32 && gram_prec != FST_GRAM_BF16 && gram_prec != FST_GRAM_F16 &&
      split_terms(gram_prec) == 0)
    fail(FST_E_INVAL, "FP32 points need gram_prec FST_GRAM_F32, BF16, F16, F16X2, BF16X3 or BF16X2");
}
static size_t dsize(int dtype) { return dtype == FST_F64 ? sizeof(double) : sizeof(float); }

static void check_wavelet_params(int s, int q, const int32_t* degree, int D) {
  if (s == 0) return;
  if (s < 0 || s > 7) fail(FST_E_INVAL, "wavelet_level must be in [0, 7]");
  for (int k = 0; k < D; ++k)
    if (q < 0 || q > std::min(degree[k], kMaxWaveDegree))
      fail(FST_E_INVAL, "wavelet_degree must be in [0, min(degree, 7)]");
  if (detail_count(s, q) > kMaxDetail) fail(FST_E_INVAL, "wavelet space too large: (q + 1)(2^s - 1) > 128");
}

static int D_OF(const fst_fit_params*) { return 3; }
static int D_OF(const fst_fit_params_d* p) { return p->d; }

static void validate_params(const fst_fit_params* p, int64_t n) {
  if (!p) fail(FST_E_INVAL, "null parameters");
  if (p->struct_size != sizeof(fst_fit_params)) fail(FST_E_INVAL, "fst_fit_params.struct_size mismatch");
  check_dtype(p->dtype);
  check_prec(p->dtype, p->gram_prec);
  if (n < 1 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 1 <= n < 2^31 points");
  for (int k = 0; k < 3; ++k) {
    if (!(std::isfinite(p->lo[k]) && std::isfinite(p->hi[k]) && p->hi[k] > p->lo[k]))
      fail(FST_E_INVAL, "need finite lo < hi in every mode");
    if (p->grid[k] < 3 || p->grid[k] > 4096) fail(FST_E_INVAL, "grid sizes must be in [3, 4096]");
    if (p->rank[k] < 1 || p->rank[k] > p->grid[k]) fail(FST_E_INVAL, "need 1 <= rank <= grid size");
    if (p->rank[k] > kMaxRank) fail(FST_E_UNSUPPORTED, "rank above 32 is not supported");
    if (p->degree[k] < 0) fail(FST_E_INVAL, "degree must be >= 0");
    if (p->degree[k] + 1 > kMaxBasis) fail(FST_E_UNSUPPORTED, "degree above 31 is not supported");
  }
  for (int k = 0; k < 3; ++k)
    if ((int64_t)p->rank[k] > (int64_t)p->rank[(k + 1) % 3] * p->rank[(k + 2) % 3])
      fail(FST_E_INVAL, "each rank must not exceed the product of the other two");
  for (int k = 0; k < 3; ++k)
    if (p->rank[k] > p->degree[k] + 1)
      fail(FST_E_INVAL, "each rank must not exceed degree + 1 (more factor functions than basis functions "
                        "makes the core least-squares problem singular)");
  if ((int64_t)p->grid[0] * p->grid[1] * p->grid[2] > (int64_t(1) << 28)) fail(FST_E_INVAL, "grid too large");
  if (!(p->interp_fraction > 0.0 && p->interp_fraction <= 1.0)) fail(FST_E_INVAL, "interp_fraction must be in (0, 1]");
  if (p->idw_k < 1 || p->idw_k > 64) fail(FST_E_INVAL, "idw_k must be in [1, 64]");
  if (!(p->idw_power > 0.0 && std::isfinite(p->idw_power))) fail(FST_E_INVAL, "idw_power must be positive");
  const int64_t R = (int64_t)p->rank[0] * p->rank[1] * p->rank[2];
  if (p->n_samples <= R || p->n_samples > n)
    fail(FST_E_INVAL, "Algorithm 2 needs r1 r2 r3 < n_samples <= n (more sampled rows than core entries)");
  if (llround(p->interp_fraction * (double)n) < 1) fail(FST_E_INVAL, "interpolation subset is empty");
  if (p->refine_steps < 0 || p->refine_steps > 100) fail(FST_E_INVAL, "refine_steps must be in [0, 100]");
  if (!(p->eps >= 0.0 && p->eps < 1.0)) fail(FST_E_INVAL, "eps must be in [0, 1)");
  if (p->sparse_solver != FST_SOLVER_OMP && p->sparse_solver != FST_SOLVER_LARS)
    fail(FST_E_INVAL, "sparse_solver must be FST_SOLVER_OMP or FST_SOLVER_LARS");
  check_wavelet_params(p->wavelet_level, p->wavelet_degree, p->degree, D_OF(p));
}

// --------------------------------------------------------------------------- refit layout
struct RefitLayout {
  size_t idx, U, vs, G, h, alpha, scratch, total;
};
static RefitLayout refit_layout(int64_t R, int sr, int64_t M, int dtype, int refine, size_t scratch_need) {
  RefitLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.idx = take(sizeof(int32_t) * (size_t)M);
  L.U = take(dsize(dtype) * (size_t)sr * (size_t)M);
  L.vs = take(dsize(dtype) * (size_t)M);
  L.G = take(sizeof(double) * (size_t)R * (size_t)R);
  L.h = take(sizeof(double) * (size_t)R);
  L.alpha = take(sizeof(double) * (size_t)R);
  L.scratch = take(scratch_need);
  L.total = off;
  return L;
}
static size_t refit_scratch(const fst_model* m, int64_t M, int refine) {
  (void)refine;
  return std::max(gram_workspace_bytes(m, M), solve_scratch_bytes(m, M));
}

// --------------------------------------------------------------------------- solve + ladder

size_t solve_scratch_bytes(const fst_model* m, int64_t M) {
  const size_t r8 = align_up(sizeof(double) * (size_t)m->R());
  size_t s = std::max(gram_workspace_bytes(m, M), cholesky_workspace_bytes(m->R()));
  s = std::max(s, residual_workspace_bytes(m, M) + 2 * r8);
  return std::max(s, gram_f64_rows_workspace_bytes(m, M));
}

// Euclidean norm of a device vector over the entries not masked out (mask may be empty)
static double device_norm(const double* d, int64_t R, const std::vector<uint8_t>& skip, void* stream) {
  std::vector<double> t((size_t)R);
  copy_d2h(t.data(), d, sizeof(double) * (size_t)R, stream);
  double s = 0.0;
  for (int64_t j = 0; j < R; ++j)
    if (skip.empty() || !skip[(size_t)j]) s += t[(size_t)j] * t[(size_t)j];
  return std::sqrt(s);
}

// Relative pivot below which the FP64 step of the ladder treats a column as dependent on the
// earlier ones: sqrt(2^-52).  The squared sine of the column's angle to the span of the
// earlier columns is resolved by FP64 normal equations only well above 2^-52; kept
// columns closer to that span would give core entries with large, cancelling values.
constexpr double kDropTol = 1.4901161193847656e-08;
// A refinement that stops making progress, or ends its steps, above this relative residual
// ||A^T (v - A alpha)|| / ||A^T v|| means the factor is too inaccurate for the problem, and the
// ladder climbs.
constexpr double kStallTol = 1e-8;

// Iterative refinement (Algorithm 2 step 5 solved through the factored normal equations,
// corrected with residuals r = A^T (v_S - A alpha) formed from FP64 rows).  Every step must
// reduce ||r||; a step that does not is undone.  After `steps` steps a residual still above
// kStallTol gets more steps while each step at least halves it (up to 4 steps in all per
// step asked for).  Returns 1 when the factor is too inaccurate for refinement to reach
// kStallTol (the residual grew by more than a factor 2, stalled above kStallTol, or the extra
// steps ran out), else 0.
static int refine_loop(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z,
                       const void* v, const int32_t* idx, int64_t M, const double* L, double* alpha, int steps,
                       double hnorm, const std::vector<uint8_t>& skip, void* scr, size_t scr_bytes, void* stream,
                       SolveInfo& info) {
  const int64_t R = m->R();
  const size_t r8 = align_up(sizeof(double) * (size_t)R);
  double* r = (double*)scr;
  double* prev_alpha = (double*)((char*)scr + r8);
  char* rest = (char*)scr + 2 * r8;
  const size_t rest_bytes = scr_bytes - 2 * r8;
  double prev = std::numeric_limits<double>::infinity();
  const int max_steps = 4 * steps;
  for (int s = 0; s <= max_steps; ++s) {
    residual(m, dtype, n, x, y, z, v, idx, M, alpha, r, rest, rest_bytes, stream);
    const double nr = device_norm(r, R, skip, stream);
    if (!(nr < prev)) {
      info.rel_residual = nr / hnorm;
      if (s == 0) return 1;   // non-finite residual of the first solution
      copy_d2d(alpha, prev_alpha, sizeof(double) * (size_t)R, stream);
      info.refine_steps = s - 1;
      info.rel_residual = prev / hnorm;
      return (nr > 2.0 * prev || info.rel_residual > kStallTol) ? 1 : 0;
    }
    info.rel_residual = nr / hnorm;
    if (nr == 0.0) return 0;
    if (s >= steps) {
      // the steps asked for are spent: done at kStallTol, else go on only while converging
      if (info.rel_residual <= kStallTol) return 0;
      if (s == max_steps || nr > 0.5 * prev) return 1;
    }
    prev = nr;
    copy_d2d(prev_alpha, alpha, sizeof(double) * (size_t)R, stream);
    cholesky_solve(R, L, r, r, stream);
    device_axpy(R, 1.0, r, alpha, stream);
    info.refine_steps = s + 1;
  }
  return 0;
}

// Relative pivot below which a factorisation of a split 16-bit Gram (FP32-class entries,
// about 1e-7 of the diagonal) treats a column as dependent on the earlier ones: 2^-16, well
// above the rounding of the entries, so that a dropped column is within an angle of 4e-3 of
// the span of the kept ones.
constexpr double kSplitDropTol = 1.52587890625e-05;

SolveInfo solve_core(const fst_model* m, int dtype, int64_t n, const void* x, const void* y, const void* z,
                     const void* v, const int32_t* idx, int64_t M, const void* U, const void* vs, int gram_prec,
                     int refine, double* G, double* h, double* alpha, void* scr, size_t scr_bytes, void* stream,
                     double* Gsave) {
  if (scr_bytes < solve_scratch_bytes(m, M)) fail(FST_E_NOMEM, "solve: scratch too small");
  const int64_t R = m->R();
  const std::vector<uint8_t> none;
  if (!std::isfinite(device_norm(h, R, none, stream)))
    fail(FST_E_INVAL, "non-finite coordinates or values among the sampled rows");
  SolveInfo info;
  int level = gram_prec;
  bool semidefinite = false;   // FP64 rows, strict factorisation already broke down
  // split 16-bit Gram kept in Gsave: when its strict factorisation or refinement fails, it is
  // factored again with dependent columns (relative pivot below kSplitDropTol) skipped
  // before the ladder goes to FP64 rows
  const bool can_resplit = Gsave && split_terms(gram_prec) > 0;
  bool split_semidefinite = false;
  if (can_resplit) copy_d2d(Gsave, G, sizeof(double) * (size_t)R * (size_t)R, stream);
  auto resplit = [&]() {
    split_semidefinite = true;
    copy_d2d(G, Gsave, sizeof(double) * (size_t)R * (size_t)R, stream);
  };
  auto reform = [&](int prec) {
    if (prec == FST_GRAM_F32)
      launch_gram(m, dtype, M, U, vs, FST_GRAM_F32, G, nullptr, scr, scr_bytes, stream);
    else if (dtype == FST_F32)
      gram_from_f64_rows(m, dtype, n, x, y, z, v, idx, M, G, h, scr, scr_bytes, stream);
    else
      launch_gram(m, dtype, M, U, vs, FST_GRAM_F64, G, nullptr, scr, scr_bytes, stream);
  };
  for (;;) {
    int64_t dropped = 0;
    const double tol = semidefinite ? kDropTol : (split_semidefinite ? kSplitDropTol : 0.0);
    const int64_t piv = cholesky(R, G, scr, scr_bytes, stream, tol, &dropped);
    if (piv != 0) {
      if (semidefinite)
        fail(FST_E_NOT_SPD, "Cholesky breakdown at pivot " + std::to_string(piv) +
                                ": non-finite entries in the sampled Gram matrix");
      if (can_resplit && !split_semidefinite) {
        resplit();
        continue;
      }
      // precision ladder: 16-bit -> FP32 rows -> FP64 rows (G and h) -> FP64 rows with
      // dependent columns skipped; split 16-bit rows are FP32-class and go to FP64 rows
      if (split_terms(level) > 0) {
        level = FST_GRAM_F64;
      } else if (level == FST_GRAM_BF16 || level == FST_GRAM_F16) {
        level = FST_GRAM_F32;
      } else if (level == FST_GRAM_F32) {
        level = FST_GRAM_F64;
      } else {
        semidefinite = true;
      }
      reform(level);
      continue;
    }
    info.gram_prec = level;
    info.dropped = dropped;
    info.refine_steps = 0;
    info.rel_residual = std::numeric_limits<double>::quiet_NaN();
    cholesky_solve(R, G, h, alpha, stream);
    if (refine <= 0) break;
    const std::vector<uint8_t> skip = dropped > 0 ? dropped_mask(G, R, scr, stream) : none;
    const double hnorm = device_norm(h, R, skip, stream);
    if (!(hnorm > 0.0)) break;
    const int climb = refine_loop(m, dtype, n, x, y, z, v, idx, M, G, alpha, refine, hnorm, skip, scr, scr_bytes,
                                  stream, info);
    if (!climb || level == FST_GRAM_F64) break;
    if (can_resplit && !split_semidefinite) {
      resplit();
      continue;
    }
    level = (level == FST_GRAM_BF16 || level == FST_GRAM_F16) ? FST_GRAM_F32 : FST_GRAM_F64;
    reform(level);
  }
  return info;
}
// the same bound without a model object (for fst_fit_workspace_bytes)
static size_t refit_bytes_for(const int32_t rank[3], const int32_t degree[3], int64_t M, int dtype, int refine) {
  double lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
  std::unique_ptr<fst_model> tmp(model_new(lo, hi, rank, degree));
  return refit_layout(tmp->R(), tmp->sum_r(), M, dtype, refine, refit_scratch(tmp.get(), M, refine)).total;
}

// Algorithm 2 with mixing: workspace = G, h, alpha, Cholesky scratch, then the mixed rows
struct MixedRefitLayout {
  size_t G, h, alpha, chol, mix, total;
};
static MixedRefitLayout mixed_refit_layout(const fst_model* m, int dtype, int64_t n, int64_t M) {
  const int64_t R = m->R();
  MixedRefitLayout L;
  size_t off = 0;
  L.G = off;
  off += align_up(sizeof(double) * (size_t)R * (size_t)R);
  L.h = off;
  off += align_up(sizeof(double) * (size_t)R);
  L.alpha = off;
  off += align_up(sizeof(double) * (size_t)R);
  L.chol = off;
  off += align_up(cholesky_workspace_bytes(R));
  L.mix = off;
  off += mixed_workspace_bytes(m, dtype, n, M);
  L.total = off;
  return L;
}

static fst_model* refit_mixed_impl(const fst_model* m, int dtype, int64_t n, const void* x, const void* y,
                                   const void* z, const void* v, int64_t M, uint64_t seed, void* ws_user,
                                   size_t ws_bytes, void* stream) {
  check_model3(m);
  check_dtype(dtype);
  const int64_t R = m->R();
  if (n < 1 || n > (int64_t(1) << 23)) fail(FST_E_INVAL, "the mixed refit needs 1 <= n <= 2^23 points");
  if (M <= R || M > mixed_length(n)) fail(FST_E_INVAL, "the mixed refit needs r1 r2 r3 < n_samples <= N");
  for (int k = 0; k < 3; ++k)
    if (m->rank[k] > m->degree[k] + 1) fail(FST_E_INVAL, "Algorithm 2 needs rank <= degree + 1 in every mode");
  if (!x || !y || !z || !v) fail(FST_E_INVAL, "null point or value array");
  const MixedRefitLayout L = mixed_refit_layout(m, dtype, n, M);
  Workspace ws(ws_user, ws_bytes, L.total);
  char* base = (char*)ws.p;
  double* d_G = (double*)(base + L.G);
  double* d_h = (double*)(base + L.h);
  double* d_alpha = (double*)(base + L.alpha);
  mixed_normal_equations(m, dtype, n, x, y, z, v, M, seed, base + L.mix, ws.bytes - L.mix, d_G, d_h, stream);
  const int64_t piv = cholesky(R, d_G, base + L.chol, cholesky_workspace_bytes(R), stream);
  if (piv != 0)
    fail(FST_E_NOT_SPD, "mixed refit: Cholesky breakdown at pivot " + std::to_string(piv) +
                            " (numerically rank-deficient sampled rows)");
  cholesky_solve(R, d_G, d_h, d_alpha, stream);
  std::vector<double> alpha((size_t)R);
  copy_d2h(alpha.data(), d_alpha, sizeof(double) * (size_t)R, stream);
  for (double t : alpha)
    if (!std::isfinite(t)) fail(FST_E_NOT_SPD, "mixed refit produced non-finite core values");
  fst_model* out = copy_with_core(m, alpha);
  out->fit.gram_prec = dtype == FST_F64 ? FST_GRAM_F64 : FST_GRAM_F32;
  out->fit.refine_steps = 0;
  return out;
}

static fst_model* refit_impl(const fst_model* m, int dtype, int64_t n, const void* x, const void* y,
                             const void* z, const void* v, int64_t M, uint64_t seed, int gram_prec,
                             int refine, void* ws_user, size_t ws_bytes, void* stream) {
  check_model3(m);
  check_dtype(dtype);
  check_prec(dtype, gram_prec);
  const int64_t R = m->R();
  if (n < 1 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 1 <= n < 2^31 points");
  if (M <= R || M > n) fail(FST_E_INVAL, "Algorithm 2 needs r1 r2 r3 < n_samples <= n");
  for (int k = 0; k < 3; ++k)
    if (m->rank[k] > m->degree[k] + 1)
      fail(FST_E_INVAL, "Algorithm 2 needs rank <= degree + 1 in every mode (otherwise the design rows are "
                        "linearly dependent)");
  if (!x || !y || !z || !v) fail(FST_E_INVAL, "null point or value array");
  if (refine < 0 || refine > 100) fail(FST_E_INVAL, "refine_steps must be in [0, 100]");
  const RefitLayout L = refit_layout(R, m->sum_r(), M, dtype, refine, refit_scratch(m, M, refine));
  // without a caller workspace the library allocates one, with room for the dense route of
  // the Gram (rows materialised) when the device has that much free memory to spare
  size_t want = L.total;
  if (!ws_user) {
    const size_t route = gram_route_bytes(m, dtype, gram_prec, M);
    if (device_free_bytes() >= L.total + route + (size_t(2) << 30)) want = L.total + route;
  }
  Workspace ws(ws_user, ws_user ? ws_bytes : want, want);
  char* base = (char*)ws.p;
  int32_t* d_idx = (int32_t*)(base + L.idx);
  void* d_U = base + L.U;
  void* d_vs = base + L.vs;
  double* d_G = (double*)(base + L.G);
  double* d_h = (double*)(base + L.h);
  double* d_alpha = (double*)(base + L.alpha);
  void* d_scr = base + L.scratch;
  const size_t scr_bytes = ws.bytes - L.scratch;

  // Algorithm 2 step 4: M rows drawn uniformly without replacement (stream 2), sorted
  std::vector<int64_t> idx((size_t)M);
  sample_indices(seed, FST_STREAM_LS, n, M, idx.data());
  std::vector<int32_t> idx32((size_t)M);
  for (int64_t i = 0; i < M; ++i) idx32[(size_t)i] = (int32_t)idx[(size_t)i];
  copy_h2d(d_idx, idx32.data(), sizeof(int32_t) * (size_t)M, stream);

  // step 1 at the sampled rows (factor functions), then the normal equations of step 5
  const DeviceModel& dm = device_model(m, dtype);
  launch_factor_eval(m, dm, dtype, n, x, y, z, v, d_idx, M, d_U, d_vs, stream);
  const int used = launch_gram(m, dtype, M, d_U, d_vs, gram_prec, d_G, d_h, d_scr, scr_bytes, stream);
  // a split Gram leaves its row planes' room free: a copy of G goes there (after the solve's scratch)
  double* Gsave = nullptr;
  const size_t gbytes = align_up(sizeof(double) * (size_t)R * (size_t)R), sneed = align_up(solve_scratch_bytes(m, M));
  if (split_terms(used) > 0 && scr_bytes >= sneed + gbytes) Gsave = (double*)((char*)d_scr + sneed);
  const SolveInfo si = solve_core(m, dtype, n, x, y, z, v, d_idx, M, d_U, d_vs, used, refine, d_G, d_h,
                                  d_alpha, d_scr, sneed < scr_bytes && Gsave ? sneed : scr_bytes, stream, Gsave);
  std::vector<double> alpha((size_t)R);
  copy_d2h(alpha.data(), d_alpha, sizeof(double) * (size_t)R, stream);
  for (double t : alpha)
    if (!std::isfinite(t)) fail(FST_E_NOT_SPD, "solve produced non-finite core values");
  fst_model* out = copy_with_core(m, alpha);
  out->fit = si;
  return out;
}

// Algorithm 1 from the gathered interpolation subset (host FP64, K x 4: x, y, z, v).
static fst_model* compress_from_subset(const fst_fit_params* p, const std::vector<double>& sub, int64_t K) {
  std::vector<double> xi((size_t)K * 3), v((size_t)K);
  for (int64_t i = 0; i < K; ++i) {
    for (int k = 0; k < 3; ++k) {
      double c = sub[(size_t)(4 * i + k)];
      if (!std::isfinite(c)) fail(FST_E_INVAL, "non-finite coordinate in the interpolation subset");
      xi[(size_t)(3 * i + k)] = 2.0 * (c - p->lo[k]) / (p->hi[k] - p->lo[k]) - 1.0;
    }
    v[(size_t)i] = sub[(size_t)(4 * i + 3)];
    if (!std::isfinite(v[(size_t)i])) fail(FST_E_INVAL, "non-finite value in the interpolation subset");
  }
  const int64_t nodes = (int64_t)p->grid[0] * p->grid[1] * p->grid[2];
  std::vector<double> T((size_t)nodes);
  idw_grid(xi.data(), v.data(), K, p->grid, p->idw_k, p->idw_power, p->n_threads, T.data());
  int32_t rank[3] = {p->rank[0], p->rank[1], p->rank[2]};
  std::vector<double> W[3];
  double* Wp[3];
  for (int k = 0; k < 3; ++k) {
    W[k].assign((size_t)p->grid[k] * p->rank[k], 0.0);
    Wp[k] = W[k].data();
  }
  std::vector<double> core((size_t)rank[0] * rank[1] * rank[2]);
  if (p->eps > 0.0) {
    // ranks from the precision, capped by rank[] (valid ranks by validation); a rank above
    // the product of the other two would only add dependent design columns, so such ranks
    // are lowered and the decomposition is taken again at the final ranks
    int32_t r[3];
    sthosvd_eps(T.data(), p->grid, p->eps, p->rank, p->n_threads, r, core.data(), Wp, nullptr);
    bool lowered = false;
    for (int pass = 0; pass < 3; ++pass)
      for (int k = 0; k < 3; ++k) {
        const int32_t lim = r[(k + 1) % 3] * r[(k + 2) % 3];
        if (r[k] > lim) {
          r[k] = lim;
          lowered = true;
        }
      }
    for (int k = 0; k < 3; ++k) rank[k] = r[k];
    if (lowered) sthosvd(T.data(), p->grid, rank, p->n_threads, core.data(), Wp, nullptr);
  } else {
    sthosvd(T.data(), p->grid, rank, p->n_threads, core.data(), Wp, nullptr);
  }
  const int32_t wl[3] = {p->wavelet_level, p->wavelet_level, p->wavelet_level};
  const int32_t wd[3] = {p->wavelet_degree, p->wavelet_degree, p->wavelet_degree};
  std::unique_ptr<fst_model> m(model_new_d(3, p->lo, p->hi, rank, p->degree, wl, wd));
  std::copy(core.begin(), core.begin() + (size_t)rank[0] * rank[1] * rank[2], m->core.begin());
  for (int k = 0; k < 3; ++k)
    sparse_fit_with(p->sparse_solver, W[k].data(), p->grid[k], rank[k], p->degree[k], m->coef[k].data(),
                    p->wavelet_level, p->wavelet_degree);
  return m.release();
}

// ---------------------------------------------------------------- d-way refit (d = 3 or 4)
// Algorithm 2 from materialised row chunks: workspace = sampled indices, G, h, alpha,
// Cholesky scratch, then the rows
struct DwayRefitLayout {
  size_t idx, G, h, alpha, chol, rows, total;
};
static DwayRefitLayout dway_refit_layout(const fst_model* m, int dtype, int64_t M) {
  const int64_t R = m->R();
  DwayRefitLayout L;
  size_t off = 0;
  L.idx = off;
  off += align_up(sizeof(int32_t) * (size_t)M);
  L.G = off;
  off += align_up(sizeof(double) * (size_t)R * (size_t)R);
  L.h = off;
  off += align_up(sizeof(double) * (size_t)R);
  L.alpha = off;
  off += align_up(sizeof(double) * (size_t)R);
  L.chol = off;
  off += align_up(cholesky_workspace_bytes(R));
  L.rows = off;
  off += dway_workspace_bytes(m, dtype, M);
  L.total = off;
  return L;
}

static void validate_params_d(const fst_fit_params_d* p, int64_t n) {
  if (!p) fail(FST_E_INVAL, "null parameters");
  if (p->struct_size != sizeof(fst_fit_params_d)) fail(FST_E_INVAL, "fst_fit_params_d.struct_size mismatch");
  check_dtype(p->dtype);
  if (p->d != 3 && p->d != 4) fail(FST_E_UNSUPPORTED, "only d = 3 and d = 4 are supported");
  const int D = p->d;
  if (n < 1 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 1 <= n < 2^31 points");
  int64_t nodes = 1, R = 1;
  for (int k = 0; k < D; ++k) {
    if (!(std::isfinite(p->lo[k]) && std::isfinite(p->hi[k]) && p->hi[k] > p->lo[k]))
      fail(FST_E_INVAL, "need finite lo < hi in every mode");
    if (p->grid[k] < 3 || p->grid[k] > 4096) fail(FST_E_INVAL, "grid sizes must be in [3, 4096]");
    if (p->rank[k] < 1 || p->rank[k] > p->grid[k]) fail(FST_E_INVAL, "need 1 <= rank <= grid size");
    if (p->rank[k] > kMaxRank) fail(FST_E_UNSUPPORTED, "rank above 32 is not supported");
    if (p->degree[k] < 0) fail(FST_E_INVAL, "degree must be >= 0");
    if (p->degree[k] + 1 > kMaxBasis) fail(FST_E_UNSUPPORTED, "degree above 31 is not supported");
    if (p->rank[k] > p->degree[k] + 1)
      fail(FST_E_INVAL, "each rank must not exceed degree + 1 (more factor functions than basis functions "
                        "makes the core least-squares problem singular)");
    nodes *= p->grid[k];
    R *= p->rank[k];
  }
  for (int k = 0; k < D; ++k) {
    int64_t other = 1;
    for (int l = 0; l < D; ++l)
      if (l != k) other *= p->rank[l];
    if (p->rank[k] > other) fail(FST_E_INVAL, "each rank must not exceed the product of the others");
  }
  if (nodes > (int64_t(1) << 28)) fail(FST_E_INVAL, "grid too large");
  if (!(p->interp_fraction > 0.0 && p->interp_fraction <= 1.0)) fail(FST_E_INVAL, "interp_fraction must be in (0, 1]");
  if (p->idw_k < 1 || p->idw_k > 64) fail(FST_E_INVAL, "idw_k must be in [1, 64]");
  if (!(p->idw_power > 0.0 && std::isfinite(p->idw_power))) fail(FST_E_INVAL, "idw_power must be positive");
  if (p->n_samples <= R || p->n_samples > n)
    fail(FST_E_INVAL, "Algorithm 2 needs r1 .. rd < n_samples <= n (more sampled rows than core entries)");
  if (llround(p->interp_fraction * (double)n) < 1) fail(FST_E_INVAL, "interpolation subset is empty");
  if (!(p->eps >= 0.0 && p->eps < 1.0)) fail(FST_E_INVAL, "eps must be in [0, 1)");
  if (p->sparse_solver != FST_SOLVER_OMP && p->sparse_solver != FST_SOLVER_LARS)
    fail(FST_E_INVAL, "sparse_solver must be FST_SOLVER_OMP or FST_SOLVER_LARS");
  check_wavelet_params(p->wavelet_level, p->wavelet_degree, p->degree, D_OF(p));
}

// Algorithm 1 for D modes from the gathered subset (host FP64, K x (D + 1): coordinates, value)
static fst_model* compress_from_subset_d(const fst_fit_params_d* p, const std::vector<double>& sub, int64_t K) {
  const int D = p->d;
  std::vector<double> xi((size_t)K * D), v((size_t)K);
  for (int64_t i = 0; i < K; ++i) {
    for (int k = 0; k < D; ++k) {
      const double c = sub[(size_t)((D + 1) * i + k)];
      if (!std::isfinite(c)) fail(FST_E_INVAL, "non-finite coordinate in the interpolation subset");
      xi[(size_t)(D * i + k)] = 2.0 * (c - p->lo[k]) / (p->hi[k] - p->lo[k]) - 1.0;
    }
    v[(size_t)i] = sub[(size_t)((D + 1) * i + D)];
    if (!std::isfinite(v[(size_t)i])) fail(FST_E_INVAL, "non-finite value in the interpolation subset");
  }
  int64_t nodes = 1;
  for (int k = 0; k < D; ++k) nodes *= p->grid[k];
  std::vector<double> T((size_t)nodes);
  idw_grid_d(xi.data(), v.data(), K, D, p->grid, p->idw_k, p->idw_power, p->n_threads, T.data());
  int32_t rank[kMaxModes];
  std::vector<double> W[kMaxModes];
  double* Wp[kMaxModes];
  int64_t Rcap = 1;
  for (int k = 0; k < D; ++k) {
    rank[k] = p->rank[k];
    W[k].assign((size_t)p->grid[k] * p->rank[k], 0.0);
    Wp[k] = W[k].data();
    Rcap *= p->rank[k];
  }
  std::vector<double> core((size_t)Rcap);
  if (p->eps > 0.0) {
    // ranks from the precision, capped by rank[]; a rank above the product of the others
    // would only add dependent design columns, so such ranks are lowered and the
    // decomposition is taken again at the final ranks
    int32_t r[kMaxModes];
    sthosvd_eps_d(T.data(), D, p->grid, p->eps, p->rank, p->n_threads, r, core.data(), Wp, nullptr);
    bool lowered = false;
    for (int pass = 0; pass < D; ++pass)
      for (int k = 0; k < D; ++k) {
        int64_t lim = 1;
        for (int l = 0; l < D; ++l)
          if (l != k) lim *= r[l];
        if (r[k] > lim) {
          r[k] = (int32_t)lim;
          lowered = true;
        }
      }
    for (int k = 0; k < D; ++k) rank[k] = r[k];
    if (lowered) sthosvd_d(T.data(), D, p->grid, rank, p->n_threads, core.data(), Wp, nullptr);
  } else {
    sthosvd_d(T.data(), D, p->grid, rank, p->n_threads, core.data(), Wp, nullptr);
  }
  const int32_t wl[4] = {p->wavelet_level, p->wavelet_level, p->wavelet_level, p->wavelet_level};
  const int32_t wd[4] = {p->wavelet_degree, p->wavelet_degree, p->wavelet_degree, p->wavelet_degree};
  std::unique_ptr<fst_model> m(model_new_d(D, p->lo, p->hi, rank, p->degree, wl, wd));
  std::copy(core.begin(), core.begin() + (size_t)m->R(), m->core.begin());
  for (int k = 0; k < D; ++k)
    sparse_fit_with(p->sparse_solver, W[k].data(), p->grid[k], rank[k], p->degree[k], m->coef[k].data(),
                    p->wavelet_level, p->wavelet_degree);
  return m.release();
}

static void check_coords(const fst_model* m, const void* const* coords) {
  if (!coords) fail(FST_E_INVAL, "null coordinate list");
  for (int k = 0; k < m->d; ++k)
    if (!coords[k]) fail(FST_E_INVAL, "null coordinate array");
}

static fst_model* refit_d_impl(const fst_model* m, int dtype, int64_t n, const void* const* coords, const void* v,
                               int64_t M, uint64_t seed, void* ws_user, size_t ws_bytes, void* stream) {
  check_model(m);
  check_dtype(dtype);
  const int64_t R = m->R();
  if (n < 1 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 1 <= n < 2^31 points");
  if (M <= R || M > n) fail(FST_E_INVAL, "Algorithm 2 needs r1 .. rd < n_samples <= n");
  for (int k = 0; k < m->d; ++k)
    if (m->rank[k] > m->degree[k] + 1) fail(FST_E_INVAL, "Algorithm 2 needs rank <= degree + 1 in every mode");
  check_coords(m, coords);
  if (!v) fail(FST_E_INVAL, "null value array");
  const DwayRefitLayout L = dway_refit_layout(m, dtype, M);
  Workspace ws(ws_user, ws_bytes, L.total);
  char* base = (char*)ws.p;
  int32_t* d_idx = (int32_t*)(base + L.idx);
  double* d_G = (double*)(base + L.G);
  double* d_h = (double*)(base + L.h);
  double* d_alpha = (double*)(base + L.alpha);
  // step 4: M rows drawn uniformly without replacement (stream 2), sorted
  std::vector<int64_t> idx((size_t)M);
  sample_indices(seed, FST_STREAM_LS, n, M, idx.data());
  std::vector<int32_t> idx32((size_t)M);
  for (int64_t i = 0; i < M; ++i) idx32[(size_t)i] = (int32_t)idx[(size_t)i];
  copy_h2d(d_idx, idx32.data(), sizeof(int32_t) * (size_t)M, stream);
  // steps 1 and 5
  dway_normal_equations(m, dtype, coords, v, d_idx, M, base + L.rows, ws.bytes - L.rows, d_G, d_h, stream);
  const int64_t piv = cholesky(R, d_G, base + L.chol, cholesky_workspace_bytes(R), stream);
  if (piv != 0)
    fail(FST_E_NOT_SPD, "d-way refit: Cholesky breakdown at pivot " + std::to_string(piv) +
                            " (numerically rank-deficient sampled rows)");
  cholesky_solve(R, d_G, d_h, d_alpha, stream);
  std::vector<double> alpha((size_t)R);
  copy_d2h(alpha.data(), d_alpha, sizeof(double) * (size_t)R, stream);
  for (double t : alpha)
    if (!std::isfinite(t)) fail(FST_E_NOT_SPD, "d-way refit produced non-finite core values");
  fst_model* out = copy_with_core(m, alpha);
  out->fit.gram_prec = dtype == FST_F64 ? FST_GRAM_F64 : FST_GRAM_F32;
  out->fit.refine_steps = 0;
  return out;
}

}  // namespace fst

using namespace fst;

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

// size queries return 0 (with the message in fst_last_error) instead of a status
#define FST_SIZE_TRY try {
#define FST_SIZE_CATCH                              \
  }                                                 \
  catch (const std::exception& e) {                 \
    fst::set_last_error(e.what());                  \
    return 0;                                       \
  }

extern "C" {

const char* fst_last_error(void) { return fst::g_last_error.c_str(); }
const char* fst_version(void) { return "fst-mi355x 0.1.0 (gfx950)"; }

void fst_fit_params_default(fst_fit_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(fst_fit_params);
  p->dtype = FST_F64;
  for (int k = 0; k < 3; ++k) {
    p->lo[k] = -1.0;
    p->hi[k] = 1.0;
    p->grid[k] = 32;
    p->rank[k] = 8;
    p->degree[k] = 15;
  }
  p->interp_fraction = 0.10;
  p->idw_k = 8;
  p->idw_power = 2.0;
  p->n_samples = 2000;
  p->seed = 1;
  p->gram_prec = FST_GRAM_F64;
  p->eps = 0.0;
  p->refine_steps = 0;
  p->n_threads = 0;
}

size_t fst_fit_workspace_bytes(const fst_fit_params* p, int64_t n) {
  try {
    validate_params(p, n);
    int64_t K = llround(p->interp_fraction * (double)n);
    size_t gather = align_up(sizeof(int32_t) * (size_t)K) + sizeof(double) * 4 * (size_t)K;
    size_t refit = refit_bytes_for(p->rank, p->degree, p->n_samples, p->dtype, p->refine_steps);
    return std::max(gather, refit);
  } catch (const std::exception& e) {
    fst::set_last_error(e.what());
    return 0;
  }
}

fst_status fst_compress_host(const fst_fit_params* p, int64_t n, const void* x, const void* y,
                             const void* z, const void* v, fst_model** out) {
  FST_TRY
  set_last_error("");
  validate_params(p, n);
  if (!x || !y || !z || !v || !out) fail(FST_E_INVAL, "null argument");
  const int64_t K = llround(p->interp_fraction * (double)n);
  std::vector<int64_t> sub((size_t)K);
  sample_indices(p->seed, FST_STREAM_INTERP, n, K, sub.data());
  std::vector<double> xyzv((size_t)K * 4);
  for (int64_t t = 0; t < K; ++t) {
    int64_t i = sub[(size_t)t];
    if (p->dtype == FST_F64) {
      xyzv[(size_t)(4 * t + 0)] = ((const double*)x)[i];
      xyzv[(size_t)(4 * t + 1)] = ((const double*)y)[i];
      xyzv[(size_t)(4 * t + 2)] = ((const double*)z)[i];
      xyzv[(size_t)(4 * t + 3)] = ((const double*)v)[i];
    } else {
      xyzv[(size_t)(4 * t + 0)] = ((const float*)x)[i];
      xyzv[(size_t)(4 * t + 1)] = ((const float*)y)[i];
      xyzv[(size_t)(4 * t + 2)] = ((const float*)z)[i];
      xyzv[(size_t)(4 * t + 3)] = ((const float*)v)[i];
    }
  }
  *out = compress_from_subset(p, xyzv, K);
  return FST_OK;
  FST_CATCH
}

fst_status fst_fit(const fst_fit_params* p, int64_t n, const void* x, const void* y, const void* z,
                   const void* v, void* ws, size_t ws_bytes, void* stream, fst_model** out) {
  FST_TRY
  set_last_error("");
  validate_params(p, n);
  if (!x || !y || !z || !v || !out) fail(FST_E_INVAL, "null argument");
  const int64_t K = llround(p->interp_fraction * (double)n);
  const size_t need = fst_fit_workspace_bytes(p, n);
  // without a caller workspace, this one holds the gathered subset only and the refit
  // allocates its own (with room for the dense Gram route when memory allows)
  const size_t gather = align_up(sizeof(int32_t) * (size_t)K) + sizeof(double) * 4 * (size_t)K;
  Workspace w(ws, ws_bytes, ws ? need : gather);
  // Algorithm 1 step 1: a random subset (stream 1) is gathered on the device and copied out
  std::vector<int64_t> sub((size_t)K);
  sample_indices(p->seed, FST_STREAM_INTERP, n, K, sub.data());
  std::vector<double> xyzv((size_t)K * 4);
  gather_points(p->dtype, K, sub.data(), x, y, z, v, xyzv.data(), w.p, w.bytes, stream);
  std::unique_ptr<fst_model> m0(compress_from_subset(p, xyzv, K));
  // Algorithm 2 on the device
  *out = refit_impl(m0.get(), p->dtype, n, x, y, z, v, p->n_samples, p->seed, p->gram_prec,
                    p->refine_steps, ws ? w.p : nullptr, ws ? w.bytes : 0, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_refit_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n_samples,
                                 int32_t refine_steps) {
  try {
    check_model3(m);
    check_dtype(dtype);
    if (n_samples < 1 || refine_steps < 0) fail(FST_E_INVAL, "bad sizes");
    return refit_layout(m->R(), m->sum_r(), n_samples, dtype, refine_steps,
                        refit_scratch(m, n_samples, refine_steps)).total;
  } catch (const std::exception& e) {
    fst::set_last_error(e.what());
    return 0;
  }
}

fst_status fst_refit_core(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                          const void* z, const void* v, int64_t n_samples, uint64_t seed,
                          int32_t gram_prec, int32_t refine_steps, void* ws, size_t ws_bytes,
                          void* stream, fst_model** out) {
  FST_TRY
  set_last_error("");
  if (!out) fail(FST_E_INVAL, "null output");
  *out = refit_impl(m, dtype, n, x, y, z, v, n_samples, seed, gram_prec, refine_steps, ws, ws_bytes, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_solve_core_workspace_bytes(const fst_model* m, int64_t mrows, int32_t gram_prec) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || mrows < 1) return 0;
  const int64_t R = m->R();
  size_t bytes = align_up(solve_scratch_bytes(m, mrows));
  if (split_terms(gram_prec) > 0) bytes += align_up(sizeof(double) * (size_t)R * (size_t)R);
  return bytes;
  FST_SIZE_CATCH
}

fst_status fst_solve_core(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                          const void* z, const void* v, const int32_t* idx, int64_t mrows, const void* U,
                          const void* vs, int32_t gram_prec, int32_t refine_steps, double* G, double* h,
                          double* alpha, int32_t* gram_prec_used, int64_t* dropped, int32_t* steps_kept,
                          double* rel_residual, void* ws, size_t ws_bytes, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  check_prec(dtype, gram_prec);
  const int64_t R = m->R();
  if (n < 1 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 1 <= n < 2^31 points");
  if (mrows <= R || mrows > n) fail(FST_E_INVAL, "Algorithm 2 needs r1 r2 r3 < mrows <= n");
  if (refine_steps < 0 || refine_steps > 100) fail(FST_E_INVAL, "refine_steps must be in [0, 100]");
  if (!x || !y || !z || !v || !idx || !U || !vs || !G || !h || !alpha || !ws)
    fail(FST_E_INVAL, "null argument");
  const size_t sneed = align_up(solve_scratch_bytes(m, mrows));
  const size_t need = fst_solve_core_workspace_bytes(m, mrows, gram_prec);
  if (ws_bytes < need) fail(FST_E_NOMEM, "solve: workspace smaller than fst_solve_core_workspace_bytes");
  double* Gsave = split_terms(gram_prec) > 0 ? (double*)((char*)ws + sneed) : nullptr;
  const SolveInfo si = solve_core(m, dtype, n, x, y, z, v, idx, mrows, U, vs, gram_prec, refine_steps, G, h, alpha,
                                  ws, sneed, stream, Gsave);
  if (gram_prec_used) *gram_prec_used = si.gram_prec;
  if (dropped) *dropped = si.dropped;
  if (steps_kept) *steps_kept = si.refine_steps;
  if (rel_residual) *rel_residual = si.rel_residual;
  return FST_OK;
  FST_CATCH
}

fst_status fst_eval(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                    const void* z, void* out, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  if (n < 0 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 0 <= n < 2^31 points");
  if (n == 0) return FST_OK;
  if (!x || !y || !z || !out) fail(FST_E_INVAL, "null point or output array");
  const DeviceModel& dm = device_model(m, dtype);
  launch_eval(m, dm, dtype, n, x, y, z, nullptr, nullptr, out, stream);
  return FST_OK;
  FST_CATCH
}

static void check_grid_counts(int64_t n1, int64_t n2, int64_t n3) {
  const int64_t lim = (int64_t(1) << 31) - 1;
  if (n1 < 1 || n2 < 1 || n3 < 1 || n1 > lim || n2 > lim || n3 > lim)
    fail(FST_E_INVAL, "grid counts must be in [1, 2^31 - 1]");
  if (n1 > 65535LL * 32 || n2 > 65535LL * 32) fail(FST_E_UNSUPPORTED, "more than 65535 x 32 lines along one axis");
}

size_t fst_eval_grid_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n1, int64_t n2, int64_t n3) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || (dtype != FST_F64 && dtype != FST_F32) || n1 < 1 || n2 < 1 || n3 < 1) return 0;
  return eval_grid_workspace_bytes(m, dtype, n1, n2, n3);
  FST_SIZE_CATCH
}

fst_status fst_eval_grid(const fst_model* m, int32_t dtype, const void* gx, int64_t n1, const void* gy, int64_t n2,
                         const void* gz, int64_t n3, void* out, void* ws, size_t ws_bytes, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  check_grid_counts(n1, n2, n3);
  if (!gx || !gy || !gz || !out) fail(FST_E_INVAL, "null coordinate or output array");
  const size_t need = eval_grid_workspace_bytes(m, dtype, n1, n2, n3);
  const DeviceModel& dm = device_model(m, dtype);
  if (ws) {
    if (ws_bytes < need) fail(FST_E_NOMEM, "eval_grid: workspace too small");
    eval_grid(m, dm, dtype, gx, n1, gy, n2, gz, n3, out, ws, stream);
  } else {
    void* own = device_alloc(need);
    try {
      eval_grid(m, dm, dtype, gx, n1, gy, n2, gz, n3, out, own, stream);
      stream_sync(stream);
    } catch (...) {
      device_free(own);
      throw;
    }
    device_free(own);
  }
  return FST_OK;
  FST_CATCH
}

size_t fst_refit_core_mixed_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n, int64_t n_samples) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || (dtype != FST_F64 && dtype != FST_F32) || n < 1 || n > (int64_t(1) << 23) || n_samples < 1)
    return 0;
  return mixed_refit_layout(m, dtype, n, n_samples).total;
  FST_SIZE_CATCH
}

fst_status fst_refit_core_mixed(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                                const void* z, const void* v, int64_t n_samples, uint64_t seed, void* ws,
                                size_t ws_bytes, void* stream, fst_model** out) {
  FST_TRY
  set_last_error("");
  if (!out) fail(FST_E_INVAL, "null output");
  *out = refit_mixed_impl(m, dtype, n, x, y, z, v, n_samples, seed, ws, ws_bytes, stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_mixed_rows(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                          const void* z, const void* v, int64_t n_samples, uint64_t seed, void* At, void* b,
                          void* ws, size_t ws_bytes, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  if (n < 1 || n > (int64_t(1) << 23)) fail(FST_E_INVAL, "mixed rows: need 1 <= n <= 2^23 points");
  if (n_samples < 1 || n_samples > mixed_length(n)) fail(FST_E_INVAL, "mixed rows: need 1 <= n_samples <= N");
  if (!x || !y || !z || !v || !At || !ws) fail(FST_E_INVAL, "null argument");
  const size_t need = mixed_workspace_bytes(m, dtype, n, n_samples);
  if (ws_bytes < need) fail(FST_E_NOMEM, "mixed rows: workspace too small");
  mixed_rows(m, dtype, n, x, y, z, v, n_samples, seed, ws, ws_bytes, At, b, stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_leverage(int64_t R, int64_t Sp, int64_t mrows, const double* At, const double* L, double* out,
                        void* stream) {
  FST_TRY
  set_last_error("");
  if (!At || !L || (!out && mrows > 0)) fail(FST_E_INVAL, "null argument");
  leverage(R, Sp, mrows, At, L, out, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_eval_error_workspace_bytes(int32_t dtype, int64_t n) {
  FST_SIZE_TRY
  if ((dtype != FST_F64 && dtype != FST_F32) || n < 0) return 0;
  return eval_error_workspace_bytes(dtype, n);
  FST_SIZE_CATCH
}

fst_status fst_eval_error(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                          const void* z, const void* v, void* ws, size_t ws_bytes, void* stream,
                          double* sums_out) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  if (n < 1 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 1 <= n < 2^31 points");
  if (!x || !y || !z || !v || !sums_out) fail(FST_E_INVAL, "null argument");
  Workspace w(ws, ws_bytes, eval_error_workspace_bytes(dtype, n));
  eval_error(m, dtype, n, x, y, z, v, w.p, w.bytes, stream, sums_out);
  return FST_OK;
  FST_CATCH
}

fst_status fst_factor_eval(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                           const void* z, const void* v, const int32_t* idx, int64_t mrows, void* U,
                           void* vs, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  if (n < 0 || mrows < 0 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "bad sizes");
  if (!idx && mrows > n) fail(FST_E_INVAL, "mrows > n without an index array");
  if (mrows == 0) return FST_OK;
  if (!x || !y || !z || !U) fail(FST_E_INVAL, "null argument");
  if (vs && !v) fail(FST_E_INVAL, "vs requested without values");
  const DeviceModel& dm = device_model(m, dtype);
  launch_factor_eval(m, dm, dtype, n, x, y, z, v, idx, mrows, U, vs, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_gram_workspace_bytes(const fst_model* m, int64_t mrows) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || mrows < 0) return 0;
  return gram_workspace_bytes(m, mrows);
  FST_SIZE_CATCH
}

size_t fst_gram_dense_workspace_bytes(const fst_model* m, int32_t dtype, int64_t mrows) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || mrows < 1 || (dtype != FST_F64 && dtype != FST_F32)) return 0;
  const int64_t all = (mrows + GD_SP_MULTIPLE - 1) / GD_SP_MULTIPLE * GD_SP_MULTIPLE;
  return gram_workspace_bytes(m, mrows) + dense_rows_bytes(m, dtype, all);
  FST_SIZE_CATCH
}

size_t fst_gram_split_workspace_bytes(const fst_model* m, int32_t gram_prec, int64_t mrows) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || mrows < 1 || split_terms(gram_prec) == 0) return 0;
  return gram_workspace_bytes(m, mrows) + split_rows_bytes(m, gram_prec, mrows);
  FST_SIZE_CATCH
}

fst_status fst_gram(const fst_model* m, int32_t dtype, int64_t mrows, const void* U, const void* vs,
                    int32_t gram_prec, double* G, double* h, void* ws, size_t ws_bytes, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  check_prec(dtype, gram_prec);
  if (mrows < 1) fail(FST_E_INVAL, "need mrows >= 1");
  if (!U || (!G && !h)) fail(FST_E_INVAL, "null argument");
  if (h && !vs) fail(FST_E_INVAL, "h requested without vs");
  if ((h || gram_prec == FST_GRAM_F16 || split_terms(gram_prec) > 0) && !ws)
    fail(FST_E_INVAL, "h, FP16 rows and split rows need a workspace");
  const int used = launch_gram(m, dtype, mrows, U, vs, gram_prec, G, h, ws, ws ? ws_bytes : 0, stream);
  if (G && used != gram_prec)
    fail(FST_E_NOMEM, "the split rows of this precision need fst_gram_split_workspace_bytes of workspace");
  return FST_OK;
  FST_CATCH
}

fst_status fst_design_rows(const fst_model* m, int32_t dtype, int64_t mrows, const void* U, const void* vs,
                           int64_t Sp, void* At, void* b, void* stream) {
  FST_TRY
  set_last_error("");
  if (!m) fail(FST_E_INVAL, "null model");
  check_dtype(dtype);
  if (!U || !At) fail(FST_E_INVAL, "null argument");
  design_rows(m, dtype, mrows, U, vs, Sp, At, b, stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_gram_rows(int32_t dtype, int64_t R, int64_t Sp, const void* At, const void* b, double* G, double* h,
                         int32_t accumulate, void* stream) {
  FST_TRY
  set_last_error("");
  check_dtype(dtype);
  if (R < 1 || Sp < GD_SP_MULTIPLE || Sp % GD_SP_MULTIPLE != 0)
    fail(FST_E_INVAL, "need R >= 1 and Sp a positive multiple of 64");
  if (R * Sp >= (int64_t(1) << 40)) fail(FST_E_UNSUPPORTED, "A^T too large");
  if (!At || (!G && !h)) fail(FST_E_INVAL, "null argument");
  if (h && !b) fail(FST_E_INVAL, "h requested without b");
  dense_normal_equations(dtype, At, b, R, Sp, G, h, accumulate != 0, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_cholesky_workspace_bytes(int64_t R) { return cholesky_workspace_bytes(R); }

fst_status fst_cholesky(int64_t R, double* G, double shift, int64_t* info, void* ws, size_t ws_bytes,
                        void* stream) {
  FST_TRY
  set_last_error("");
  if (info) *info = 0;
  if (R < 1 || !G || !ws) fail(FST_E_INVAL, "bad arguments");
  if (!(shift >= 0.0 && shift < 1.0)) fail(FST_E_INVAL, "shift must be in [0, 1)");
  int64_t piv = cholesky(R, G, ws, ws_bytes, stream, 0.0, nullptr, shift);
  if (info) *info = piv;
  if (piv != 0) fail(FST_E_NOT_SPD, "Cholesky breakdown at pivot " + std::to_string(piv));
  return FST_OK;
  FST_CATCH
}

fst_status fst_cholesky_noalloc(int64_t R, double* G, double shift, int64_t* info, void* stream) {
  FST_TRY
  set_last_error("");
  if (info) *info = 0;
  if (R < 1 || !G) fail(FST_E_INVAL, "bad arguments");
  if (!(shift >= 0.0 && shift < 1.0)) fail(FST_E_INVAL, "shift must be in [0, 1)");
  const int64_t piv = cholesky_static_scratch(R, G, stream, shift);
  if (info) *info = piv;
  if (piv != 0) fail(FST_E_NOT_SPD, "Cholesky breakdown at pivot " + std::to_string(piv));
  return FST_OK;
  FST_CATCH
}

fst_status fst_cholesky_solve(int64_t R, const double* L, const double* b, double* x, void* stream) {
  FST_TRY
  set_last_error("");
  if (R < 1 || !L || !b || !x) fail(FST_E_INVAL, "bad arguments");
  cholesky_solve(R, L, b, x, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_residual_workspace_bytes(const fst_model* m, int64_t mrows) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || mrows < 0) return 0;
  return residual_workspace_bytes(m, mrows);
  FST_SIZE_CATCH
}

fst_status fst_residual(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                        const void* z, const void* v, const int32_t* idx, int64_t mrows,
                        const double* alpha, double* r, void* ws, size_t ws_bytes, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  if (mrows < 1 || n < 1) fail(FST_E_INVAL, "bad sizes");
  if (!x || !y || !z || !v || !idx || !alpha || !r || !ws) fail(FST_E_INVAL, "null argument");
  residual(m, dtype, n, x, y, z, v, idx, mrows, alpha, r, ws, ws_bytes, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_refine_workspace_bytes(const fst_model* m, int64_t mrows) {
  FST_SIZE_TRY
  if (!m || m->d != 3 || mrows < 0) return 0;
  return align_up(sizeof(double) * (size_t)m->R()) + residual_workspace_bytes(m, mrows);
  FST_SIZE_CATCH
}

fst_status fst_refine_step(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                           const void* z, const void* v, const int32_t* idx, int64_t mrows, const double* L,
                           double* alpha, double* r_out, void* ws, size_t ws_bytes, void* stream) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  check_dtype(dtype);
  if (mrows < 1 || n < 1) fail(FST_E_INVAL, "bad sizes");
  if (!x || !y || !z || !v || !idx || !L || !alpha || !ws) fail(FST_E_INVAL, "null argument");
  if (ws_bytes < fst_refine_workspace_bytes(m, mrows)) fail(FST_E_NOMEM, "refine: workspace too small");
  double* d_r = (double*)ws;
  char* rest = (char*)ws + align_up(sizeof(double) * (size_t)m->R());
  residual(m, dtype, n, x, y, z, v, idx, mrows, alpha, d_r, rest, ws_bytes - (size_t)(rest - (char*)ws), stream);
  cholesky_solve(m->R(), L, d_r, d_r, stream);
  device_axpy(m->R(), 1.0, d_r, alpha, stream);
  if (r_out) copy_d2d(r_out, d_r, sizeof(double) * (size_t)m->R(), stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_sample_indices(uint64_t seed, int32_t stream, int64_t n, int64_t m, int64_t* out) {
  FST_TRY
  set_last_error("");
  if (!out && m > 0) fail(FST_E_INVAL, "null output");
  sample_indices(seed, stream, n, m, out);
  return FST_OK;
  FST_CATCH
}

fst_status fst_idw_grid(const double* xi, const double* v, int64_t K, const int32_t grid[3], int32_t k,
                        double power, int32_t n_threads, double* out) {
  FST_TRY
  set_last_error("");
  if (!xi || !v || !grid || !out) fail(FST_E_INVAL, "null argument");
  if (!(power > 0.0)) fail(FST_E_INVAL, "power must be positive");
  for (int64_t i = 0; i < 3 * K; ++i)
    if (!std::isfinite(xi[i])) fail(FST_E_INVAL, "non-finite coordinate");
  for (int64_t i = 0; i < K; ++i)
    if (!std::isfinite(v[i])) fail(FST_E_INVAL, "non-finite value");
  idw_grid(xi, v, K, grid, k, power, n_threads, out);
  return FST_OK;
  FST_CATCH
}

fst_status fst_sthosvd_eps(const double* T, const int32_t dims[3], double eps, const int32_t max_rank[3],
                           int32_t n_threads, int32_t rank_out[3], double* core, double* const W[3],
                           double* const sigma[3]) {
  FST_TRY
  set_last_error("");
  if (!T || !dims || !max_rank || !rank_out || !core || !W || !W[0] || !W[1] || !W[2]) fail(FST_E_INVAL, "null argument");
  sthosvd_eps(T, dims, eps, max_rank, n_threads, rank_out, core, W, sigma);
  return FST_OK;
  FST_CATCH
}

fst_status fst_sthosvd(const double* T, const int32_t dims[3], const int32_t rank[3], int32_t n_threads,
                       double* core, double* const W[3], double* const sigma[3]) {
  FST_TRY
  set_last_error("");
  if (!T || !dims || !rank || !core || !W || !W[0] || !W[1] || !W[2]) fail(FST_E_INVAL, "null argument");
  sthosvd(T, dims, rank, n_threads, core, W, sigma);
  return FST_OK;
  FST_CATCH
}

fst_status fst_sparse_fit(const double* W, int32_t I, int32_t r, int32_t p, double* C) {
  FST_TRY
  set_last_error("");
  if (!W || !C) fail(FST_E_INVAL, "null argument");
  sparse_fit(W, I, r, p, C);
  return FST_OK;
  FST_CATCH
}

fst_status fst_sparse_fit_lars(const double* W, int32_t I, int32_t r, int32_t p, double* C) {
  FST_TRY
  set_last_error("");
  if (!W || !C) fail(FST_E_INVAL, "null argument");
  sparse_fit_lars(W, I, r, p, C);
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_from_parts(const double lo[3], const double hi[3], const int32_t rank[3],
                                const int32_t degree[3], const double* core, const double* const coefs[3],
                                fst_model** out) {
  return fst_model_from_parts_d(3, lo, hi, rank, degree, core, coefs, out);
}

fst_status fst_model_from_parts_d(int32_t d, const double* lo, const double* hi, const int32_t* rank,
                                  const int32_t* degree, const double* core, const double* const* coefs,
                                  fst_model** out) {
  return fst_model_from_parts_wavelet(d, lo, hi, rank, degree, nullptr, nullptr, core, coefs, out);
}

fst_status fst_model_wavelets(const fst_model* m, int32_t* wlevel, int32_t* wdegree) {
  FST_TRY
  set_last_error("");
  check_model(m);
  for (int k = 0; k < m->d; ++k) {
    if (wlevel) wlevel[k] = m->wlevel[k];
    if (wdegree) wdegree[k] = m->wdegree[k];
  }
  return FST_OK;
  FST_CATCH
}

fst_status fst_sparse_fit_choice(const double* W, int32_t I, int32_t r, int32_t p, int32_t s, int32_t q,
                                 int32_t solver, double* C) {
  FST_TRY
  set_last_error("");
  if (!W || !C) fail(FST_E_INVAL, "null argument");
  if (solver != FST_SOLVER_OMP && solver != FST_SOLVER_LARS) fail(FST_E_INVAL, "unknown solver");
  sparse_fit_choice(W, I, r, p, s, q, solver, C);
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_from_parts_wavelet(int32_t d, const double* lo, const double* hi, const int32_t* rank,
                                        const int32_t* degree, const int32_t* wlevel, const int32_t* wdegree,
                                        const double* core, const double* const* coefs, fst_model** out) {
  FST_TRY
  set_last_error("");
  if (!lo || !hi || !rank || !degree || !core || !coefs || !out) fail(FST_E_INVAL, "null argument");
  if ((wlevel == nullptr) != (wdegree == nullptr)) fail(FST_E_INVAL, "wlevel and wdegree go together");
  std::unique_ptr<fst_model> m(model_new_d(d, lo, hi, rank, degree, wlevel, wdegree));
  for (size_t i = 0; i < m->core.size(); ++i) {
    if (!std::isfinite(core[i])) fail(FST_E_INVAL, "non-finite core entry");
    m->core[i] = core[i];
  }
  for (int k = 0; k < d; ++k) {
    if (!coefs[k]) fail(FST_E_INVAL, "null coefficient matrix");
    for (size_t i = 0; i < m->coef[k].size(); ++i) {
      if (!std::isfinite(coefs[k][i])) fail(FST_E_INVAL, "non-finite coefficient");
      m->coef[k][i] = coefs[k][i];
    }
  }
  *out = m.release();
  return FST_OK;
  FST_CATCH
}

void fst_model_free(fst_model* m) { delete m; }

fst_status fst_model_info(const fst_model* m, double* lo, double* hi, int32_t* rank, int32_t* degree,
                          int64_t* nnz) {
  FST_TRY
  set_last_error("");
  check_model3(m);
  for (int k = 0; k < 3; ++k) {
    if (lo) lo[k] = m->lo[k];
    if (hi) hi[k] = m->hi[k];
    if (rank) rank[k] = m->rank[k];
    if (degree) degree[k] = m->degree[k];
  }
  if (nnz) {
    int64_t c = 0;
    for (int k = 0; k < 3; ++k)
      for (double t : m->coef[k]) c += t != 0.0;
    *nnz = c;
  }
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_info_d(const fst_model* m, int32_t* d, double* lo, double* hi, int32_t* rank,
                            int32_t* degree, int64_t* nnz) {
  FST_TRY
  set_last_error("");
  check_model(m);
  if (d) *d = m->d;
  for (int k = 0; k < m->d; ++k) {
    if (lo) lo[k] = m->lo[k];
    if (hi) hi[k] = m->hi[k];
    if (rank) rank[k] = m->rank[k];
    if (degree) degree[k] = m->degree[k];
  }
  if (nnz) {
    int64_t c = 0;
    for (int k = 0; k < m->d; ++k)
      for (double t : m->coef[k]) c += t != 0.0;
    *nnz = c;
  }
  return FST_OK;
  FST_CATCH
}

void fst_fit_params_d_default(fst_fit_params_d* p, int32_t d) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(fst_fit_params_d);
  p->dtype = FST_F64;
  p->d = d;
  for (int k = 0; k < kMaxModes; ++k) {
    p->lo[k] = -1.0;
    p->hi[k] = 1.0;
    p->grid[k] = 16;
    p->rank[k] = 4;
    p->degree[k] = 15;
  }
  p->interp_fraction = 0.10;
  p->idw_k = 8;
  p->idw_power = 2.0;
  p->n_samples = 2000;
  p->seed = 1;
  p->eps = 0.0;
}

size_t fst_fit_d_workspace_bytes(const fst_fit_params_d* p, int64_t n) {
  try {
    validate_params_d(p, n);
    const int64_t K = llround(p->interp_fraction * (double)n);
    // the refit of a model with the largest ranks allowed (eps may choose smaller ones)
    std::unique_ptr<fst_model> cap(model_new_d(p->d, p->lo, p->hi, p->rank, p->degree));
    return std::max(gather_workspace_bytes(K, p->d), dway_refit_layout(cap.get(), p->dtype, p->n_samples).total);
  } catch (const std::exception& e) {
    fst::set_last_error(e.what());
    return 0;
  }
}

fst_status fst_compress_host_d(const fst_fit_params_d* p, int64_t n, const void* const* coords, const void* v,
                               fst_model** out) {
  FST_TRY
  set_last_error("");
  validate_params_d(p, n);
  if (!coords || !v || !out) fail(FST_E_INVAL, "null argument");
  const int D = p->d;
  for (int k = 0; k < D; ++k)
    if (!coords[k]) fail(FST_E_INVAL, "null coordinate array");
  const int64_t K = llround(p->interp_fraction * (double)n);
  std::vector<int64_t> sub((size_t)K);
  sample_indices(p->seed, FST_STREAM_INTERP, n, K, sub.data());
  std::vector<double> rows((size_t)K * (D + 1));
  for (int64_t t = 0; t < K; ++t) {
    const int64_t i = sub[(size_t)t];
    for (int k = 0; k <= D; ++k) {
      const void* src = k < D ? coords[k] : v;
      rows[(size_t)((D + 1) * t + k)] =
          p->dtype == FST_F64 ? ((const double*)src)[i] : (double)((const float*)src)[i];
    }
  }
  *out = compress_from_subset_d(p, rows, K);
  return FST_OK;
  FST_CATCH
}

fst_status fst_fit_d(const fst_fit_params_d* p, int64_t n, const void* const* coords, const void* v, void* ws,
                     size_t ws_bytes, void* stream, fst_model** out) {
  FST_TRY
  set_last_error("");
  validate_params_d(p, n);
  if (!coords || !v || !out) fail(FST_E_INVAL, "null argument");
  for (int k = 0; k < p->d; ++k)
    if (!coords[k]) fail(FST_E_INVAL, "null coordinate array");
  const int64_t K = llround(p->interp_fraction * (double)n);
  Workspace w(ws, ws_bytes, fst_fit_d_workspace_bytes(p, n));
  // Algorithm 1 step 1: a random subset (stream 1) is gathered on the device and copied out
  std::vector<int64_t> sub((size_t)K);
  sample_indices(p->seed, FST_STREAM_INTERP, n, K, sub.data());
  std::vector<double> rows((size_t)K * (p->d + 1));
  gather_points_d(p->dtype, K, sub.data(), p->d, coords, v, rows.data(), w.p, w.bytes, stream);
  std::unique_ptr<fst_model> m0(compress_from_subset_d(p, rows, K));
  // Algorithm 2 on the device
  *out = refit_d_impl(m0.get(), p->dtype, n, coords, v, p->n_samples, p->seed, w.p, w.bytes, stream);
  return FST_OK;
  FST_CATCH
}

size_t fst_refit_core_d_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n_samples) {
  FST_SIZE_TRY
  if (!m || (dtype != FST_F64 && dtype != FST_F32) || n_samples < 1) return 0;
  return dway_refit_layout(m, dtype, n_samples).total;
  FST_SIZE_CATCH
}

fst_status fst_refit_core_d(const fst_model* m, int32_t dtype, int64_t n, const void* const* coords, const void* v,
                            int64_t n_samples, uint64_t seed, void* ws, size_t ws_bytes, void* stream,
                            fst_model** out) {
  FST_TRY
  set_last_error("");
  if (!out) fail(FST_E_INVAL, "null output");
  *out = refit_d_impl(m, dtype, n, coords, v, n_samples, seed, ws, ws_bytes, stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_eval_d(const fst_model* m, int32_t dtype, int64_t n, const void* const* coords, void* out,
                      void* stream) {
  FST_TRY
  set_last_error("");
  check_model(m);
  check_dtype(dtype);
  if (n < 0 || n >= (int64_t(1) << 31)) fail(FST_E_INVAL, "need 0 <= n < 2^31 points");
  if (n == 0) return FST_OK;
  check_coords(m, coords);
  if (!out) fail(FST_E_INVAL, "null output array");
  const void* c4[kMaxModes] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < m->d; ++k) c4[k] = coords[k];
  const DeviceModel& dm = device_model(m, dtype);
  launch_eval_d(m, dm, dtype, n, c4, out, stream);
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_core(const fst_model* m, double* core_out) {
  FST_TRY
  set_last_error("");
  check_model(m);
  if (!core_out) fail(FST_E_INVAL, "null output");
  std::memcpy(core_out, m->core.data(), sizeof(double) * m->core.size());
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_coefs(const fst_model* m, int32_t k, double* C_out) {
  FST_TRY
  set_last_error("");
  check_model(m);
  if (k < 0 || k >= m->d || !C_out) fail(FST_E_INVAL, "bad mode or null output");
  std::memcpy(C_out, m->coef[k].data(), sizeof(double) * m->coef[k].size());
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_factor(const fst_model* m, int32_t k, int32_t* colptr, int32_t* rowidx, double* vals,
                            int64_t* nnz) {
  FST_TRY
  set_last_error("");
  check_model(m);
  if (k < 0 || k >= m->d) fail(FST_E_INVAL, "bad mode");
  const int rows = m->rows(k), r = m->rank[k];
  const std::vector<double>& C = m->coef[k];
  int64_t count = 0;
  for (int j = 0; j < r; ++j) {
    if (colptr) colptr[j] = (int32_t)count;
    for (int i = 0; i < rows; ++i) {
      const double c = C[(size_t)i * r + j];
      if (c == 0.0) continue;
      if (rowidx) rowidx[count] = i;
      if (vals) vals[count] = c;
      ++count;
    }
  }
  if (colptr) colptr[r] = (int32_t)count;
  if (nnz) *nnz = count;
  return FST_OK;
  FST_CATCH
}

fst_status fst_model_fit_info(const fst_model* m, int32_t* gram_prec_used, int64_t* dropped,
                              int32_t* refine_steps, double* rel_residual) {
  FST_TRY
  set_last_error("");
  check_model(m);
  if (gram_prec_used) *gram_prec_used = m->fit.gram_prec;
  if (dropped) *dropped = m->fit.dropped;
  if (refine_steps) *refine_steps = m->fit.refine_steps;
  if (rel_residual) *rel_residual = m->fit.rel_residual;
  return FST_OK;
  FST_CATCH
}

int64_t fst_model_paper_bytes(const fst_model* m) {
  if (!m) return -1;
  int64_t nnz = 0;
  for (int k = 0; k < m->d; ++k)
    for (double t : m->coef[k]) nnz += t != 0.0;
  return 8 * (m->R() + nnz);
}

}  // extern "C"
