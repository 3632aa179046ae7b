// Host steps of Algorithm 1 (Sec. 4): random subset draw, interpolation onto the equispaced
// grid, ST-HOSVD at fixed ranks, sparse Legendre fit of each singular vector.  These steps
// work on small objects (a grid of at most a few million nodes, factor vectors of a few
// hundred entries) and stay on host threads.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <thread>

#include "fst_internal.h"

namespace fst {

int hardware_threads(int requested) {
  if (requested > 0) return requested;
  unsigned h = std::thread::hardware_concurrency();
  return h == 0 ? 1 : (int)std::min(h, 64u);
}

template <class F>
static void parallel_for(int64_t n, int n_threads, F&& body) {
  n_threads = (int)std::max<int64_t>(1, std::min<int64_t>(n_threads, n));
  if (n_threads <= 1) {
    body(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + n_threads - 1) / n_threads;
  for (int t = 0; t < n_threads; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&body, a, b] { body(a, b); });
  }
  for (auto& t : th) t.join();
}

// ------------------------------------------------------------------------------ sampler
// SplitMix64 (Steele, Lea, Flood 2014): golden-ratio increment, then the 64-bit finaliser
// with constants 0xBF58476D1CE4E5B9 / 0x94D049BB133111EB and shifts 30, 27, 31.
uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Algorithm 2 samples rows uniformly; draws are without replacement, sorted, from a partial
// Fisher-Yates shuffle whose bounded draw in [0, k) is the high half of r * k.
void sample_indices(uint64_t seed, int stream, int64_t n, int64_t m, int64_t* out) {
  if (n < 0 || m < 0 || m > n) fail(FST_E_INVAL, "sample_indices: need 0 <= m <= n");
  if (n >= (int64_t(1) << 32)) fail(FST_E_UNSUPPORTED, "sample_indices: n must be < 2^32");
  uint64_t state = seed * 256ull + (uint64_t)stream;
  std::vector<int64_t> a((size_t)n);
  std::iota(a.begin(), a.end(), int64_t(0));
  for (int64_t i = 0; i < m; ++i) {
    uint64_t r = splitmix64_next(state);
    uint64_t span = (uint64_t)(n - i);
    int64_t j = i + (int64_t)(((unsigned __int128)r * span) >> 64);
    std::swap(a[(size_t)i], a[(size_t)j]);
  }
  std::sort(a.begin(), a.begin() + m);
  std::memcpy(out, a.data(), sizeof(int64_t) * (size_t)m);
}

// ------------------------------------------------------------------------------ IDW
// Exact k-nearest neighbours through a uniform bin grid over [-1,1]^D, searched in growing
// shells of cells until the k-th best distance is below the distance to any unsearched cell.
// Candidates are ordered by (squared distance, index): equal distances go to the lower index.
namespace {
struct Cand {
  double d2;
  int64_t idx;
  bool operator<(const Cand& o) const { return d2 < o.d2 || (d2 == o.d2 && idx < o.idx); }
};

struct BinGrid {
  int B = 1;
  double h = 2.0;
  std::vector<int64_t> start;   // B^D + 1
  std::vector<int64_t> order;   // point indices sorted by cell (stable, so ascending in a cell)
  int cell_of(double t) const {
    int c = (int)std::floor((t + 1.0) / h);
    return std::min(std::max(c, 0), B - 1);
  }
};
}  // namespace

// The k nearest subset points of every grid node (C order, last mode fastest), as (index,
// weight) pairs with weights d^-power; an exact hit is stored as a single neighbour with a
// negative weight.  xi: K x D reference coordinates, D = 3 or 4; the bins are D-dimensional
// cubes and the shells are searched with an odometer over the cells of each shell.
void idw_knn_d(const double* xi, int64_t K, int D, const int32_t* grid, int k, double power, int n_threads,
               std::vector<int64_t>& nbr, std::vector<double>& wgt, std::vector<int32_t>& count) {
  if (D < 1 || D > kMaxModes) fail(FST_E_INVAL, "idw_grid: need 1 <= d <= 4");
  if (K <= 0) fail(FST_E_INVAL, "idw_grid: no points");
  for (int d = 0; d < D; ++d)
    if (grid[d] < 2) fail(FST_E_INVAL, "idw_grid: grid sizes must be >= 2");
  if (k < 1) fail(FST_E_INVAL, "idw_grid: k must be >= 1");
  k = (int)std::min<int64_t>(k, K);
  BinGrid bg;
  const double per_bin = (double)K / 2.0;   // about two points per bin
  bg.B = std::max(1, (int)(D == 3 ? std::cbrt(per_bin) : D == 4 ? std::sqrt(std::sqrt(per_bin))
                                                              : std::pow(per_bin, 1.0 / D)));
  bg.B = std::min(bg.B, 256);
  bg.h = 2.0 / bg.B;
  const int B = bg.B;
  int64_t ncell = 1;
  for (int d = 0; d < D; ++d) ncell *= B;
  auto cell_index = [&](const int* c) {
    int64_t cc = 0;
    for (int d = 0; d < D; ++d) cc = cc * B + c[d];
    return cc;
  };
  std::vector<int64_t> cell((size_t)K);
  bg.start.assign((size_t)ncell + 1, 0);
  for (int64_t i = 0; i < K; ++i) {
    int c[kMaxModes];
    for (int d = 0; d < D; ++d) c[d] = bg.cell_of(xi[D * i + d]);
    const int64_t cc = cell_index(c);
    cell[(size_t)i] = cc;
    bg.start[(size_t)cc + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) bg.start[(size_t)c + 1] += bg.start[(size_t)c];
  bg.order.resize((size_t)K);
  {
    std::vector<int64_t> fill(bg.start.begin(), bg.start.end() - 1);
    for (int64_t i = 0; i < K; ++i) bg.order[(size_t)fill[(size_t)cell[(size_t)i]]++] = i;
  }
  int64_t nodes = 1;
  for (int d = 0; d < D; ++d) nodes *= grid[d];
  nbr.assign((size_t)(nodes * k), 0);
  wgt.assign((size_t)(nodes * k), 0.0);
  count.assign((size_t)nodes, 0);
  parallel_for(nodes, hardware_threads(n_threads), [&](int64_t a, int64_t b) {
    std::vector<Cand> best;
    best.reserve((size_t)k + 1);
    for (int64_t node = a; node < b; ++node) {
      double q[kMaxModes];
      int c[kMaxModes];
      int64_t rem = node;
      for (int d = D - 1; d >= 0; --d) {
        const int64_t id = rem % grid[d];
        rem /= grid[d];
        q[d] = -1.0 + 2.0 * id / (grid[d] - 1);
        c[d] = bg.cell_of(q[d]);
      }
      best.clear();
      for (int rho = 0;; ++rho) {
        int lo[kMaxModes], hi[kMaxModes], x[kMaxModes];
        for (int d = 0; d < D; ++d) {
          lo[d] = std::max(0, c[d] - rho);
          hi[d] = std::min(B - 1, c[d] + rho);
          x[d] = lo[d];
        }
        for (;;) {
          // only the shell at Chebyshev distance rho (inner cells were done before)
          int cheb = 0;
          for (int d = 0; d < D; ++d) cheb = std::max(cheb, std::abs(x[d] - c[d]));
          if (cheb == rho) {
            const int64_t cc = cell_index(x);
            for (int64_t s = bg.start[(size_t)cc]; s < bg.start[(size_t)cc + 1]; ++s) {
              const int64_t i = bg.order[(size_t)s];
              double d2 = 0.0;
              for (int d = 0; d < D; ++d) {
                const double t = xi[D * i + d] - q[d];
                d2 += t * t;
              }
              Cand cd{d2, i};
              if ((int)best.size() < k) {
                best.insert(std::upper_bound(best.begin(), best.end(), cd), cd);
              } else if (cd < best.back()) {
                best.pop_back();
                best.insert(std::upper_bound(best.begin(), best.end(), cd), cd);
              }
            }
          }
          int d = D - 1;   // next cell of the box lo..hi, last mode fastest
          while (d >= 0 && x[d] == hi[d]) {
            x[d] = lo[d];
            --d;
          }
          if (d < 0) break;
          ++x[d];
        }
        bool covers_all = true;
        double bound = std::numeric_limits<double>::infinity();
        for (int d = 0; d < D; ++d) {
          if (c[d] - rho > 0) {
            covers_all = false;
            bound = std::min(bound, q[d] - (-1.0 + (c[d] - rho) * bg.h));
          }
          if (c[d] + rho < B - 1) {
            covers_all = false;
            bound = std::min(bound, (-1.0 + (c[d] + rho + 1) * bg.h) - q[d]);
          }
        }
        if (covers_all) break;
        // Points in unsearched cells lie at least `bound` away (cells are clamped at the
        // domain edge, so points slightly outside [-1,1] sit in edge cells already searched).
        if ((int)best.size() == k && best.back().d2 < bound * bound) break;
      }
      int64_t* nb = &nbr[(size_t)(node * k)];
      double* wt = &wgt[(size_t)(node * k)];
      if (best.front().d2 == 0.0) {
        nb[0] = best.front().idx;
        wt[0] = -1.0;
        count[(size_t)node] = 1;
        continue;
      }
      for (size_t t = 0; t < best.size(); ++t) {
        nb[t] = best[t].idx;
        wt[t] = 1.0 / std::pow(std::sqrt(best[t].d2), power);
      }
      count[(size_t)node] = (int32_t)best.size();
    }
  });
}

void idw_knn(const double* xi, int64_t K, const int32_t grid[3], int k, double power, int n_threads,
             std::vector<int64_t>& nbr, std::vector<double>& wgt, std::vector<int32_t>& count) {
  idw_knn_d(xi, K, 3, grid, k, power, n_threads, nbr, wgt, count);
}

void idw_apply(const std::vector<int64_t>& nbr, const std::vector<double>& wgt, const std::vector<int32_t>& count,
               int k, const double* v, int n_threads, double* out) {
  const int64_t nodes = (int64_t)count.size();
  parallel_for(nodes, hardware_threads(n_threads), [&](int64_t a, int64_t b) {
    for (int64_t node = a; node < b; ++node) {
      const int64_t* nb = &nbr[(size_t)(node * k)];
      const double* wt = &wgt[(size_t)(node * k)];
      if (wt[0] < 0.0) {
        out[node] = v[nb[0]];
        continue;
      }
      double num = 0.0, den = 0.0;
      for (int t = 0; t < count[(size_t)node]; ++t) {
        num += wt[t] * v[nb[t]];
        den += wt[t];
      }
      out[node] = num / den;
    }
  });
}

void idw_grid_d(const double* xi, const double* v, int64_t K, int D, const int32_t* grid, int k, double power,
                int n_threads, double* out) {
  std::vector<int64_t> nbr;
  std::vector<double> wgt;
  std::vector<int32_t> count;
  k = (int)std::min<int64_t>(std::max(k, 1), std::max<int64_t>(K, 1));
  idw_knn_d(xi, K, D, grid, k, power, n_threads, nbr, wgt, count);
  idw_apply(nbr, wgt, count, k, v, n_threads, out);
}

void idw_grid(const double* xi, const double* v, int64_t K, const int32_t grid[3], int k,
              double power, int n_threads, double* out) {
  idw_grid_d(xi, v, K, 3, grid, k, power, n_threads, out);
}

// ------------------------------------------------------------------------------ ST-HOSVD
namespace {

// Householder QR of a column-major m x n matrix (m >= n); returns R (n x n, column-major,
// upper triangular) and keeps the reflectors in A so that Q can be applied afterwards.
struct HouseholderQR {
  int64_t m, n;
  std::vector<double> A;      // column-major m x n; reflectors below the diagonal
  std::vector<double> beta;   // 2 / (v^T v) per reflector, v = (1, A[j+1.., j])
  std::vector<double> diag;   // R diagonal
  void factor() {
    beta.assign((size_t)n, 0.0);
    diag.assign((size_t)n, 0.0);
    for (int64_t j = 0; j < n; ++j) {
      double* col = &A[(size_t)(j * m)];
      double norm2 = 0.0;
      for (int64_t i = j; i < m; ++i) norm2 += col[i] * col[i];
      double norm = std::sqrt(norm2);
      if (norm == 0.0) {
        beta[(size_t)j] = 0.0;
        diag[(size_t)j] = 0.0;
        continue;
      }
      double alpha = col[j] > 0 ? -norm : norm;   // R_jj
      double v0 = col[j] - alpha;
      // v = (v0, col[j+1..]) scaled so that v[0] = 1
      for (int64_t i = j + 1; i < m; ++i) col[i] /= v0;
      double vtv = 1.0;
      for (int64_t i = j + 1; i < m; ++i) vtv += col[i] * col[i];
      beta[(size_t)j] = 2.0 / vtv;
      diag[(size_t)j] = alpha;
      col[j] = alpha;
      for (int64_t c = j + 1; c < n; ++c) {
        double* cc = &A[(size_t)(c * m)];
        double s = cc[j];
        for (int64_t i = j + 1; i < m; ++i) s += col[i] * cc[i];
        s *= beta[(size_t)j];
        cc[j] -= s;
        for (int64_t i = j + 1; i < m; ++i) cc[i] -= s * col[i];
      }
    }
  }
  std::vector<double> R() const {
    std::vector<double> r((size_t)(n * n), 0.0);
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i <= c; ++i) r[(size_t)(c * n + i)] = A[(size_t)(c * m + i)];
    for (int64_t j = 0; j < n; ++j) r[(size_t)(j * n + j)] = diag[(size_t)j];
    return r;
  }
  // y (length m) <- Q y, where y holds an n-vector padded with zeros below
  void apply_Q(double* y) const {
    for (int64_t j = n - 1; j >= 0; --j) {
      if (beta[(size_t)j] == 0.0) continue;
      const double* col = &A[(size_t)(j * m)];
      double s = y[j];
      for (int64_t i = j + 1; i < m; ++i) s += col[i] * y[i];
      s *= beta[(size_t)j];
      y[j] -= s;
      for (int64_t i = j + 1; i < m; ++i) y[i] -= s * col[i];
    }
  }
};

// One-sided (Hestenes) Jacobi on a column-major n x n matrix B: rotates columns until they
// are mutually orthogonal, B V = W.  Returns V (column-major) and the column norms of W.
void hestenes(std::vector<double>& B, int64_t n, std::vector<double>& V, std::vector<double>& sig) {
  V.assign((size_t)(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i) V[(size_t)(i * n + i)] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int64_t i = 0; i < n - 1; ++i) {
      for (int64_t j = i + 1; j < n; ++j) {
        double* bi = &B[(size_t)(i * n)];
        double* bj = &B[(size_t)(j * n)];
        double a = 0, b = 0, g = 0;
        for (int64_t t = 0; t < n; ++t) {
          a += bi[t] * bi[t];
          b += bj[t] * bj[t];
          g += bi[t] * bj[t];
        }
        if (g == 0.0 || std::fabs(g) <= tol * std::sqrt(a * b)) continue;
        rotated = true;
        double zeta = (b - a) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int64_t r = 0; r < n; ++r) {
          double x = bi[r], y = bj[r];
          bi[r] = c * x - s * y;
          bj[r] = s * x + c * y;
        }
        double* vi = &V[(size_t)(i * n)];
        double* vj = &V[(size_t)(j * n)];
        for (int64_t r = 0; r < n; ++r) {
          double x = vi[r], y = vj[r];
          vi[r] = c * x - s * y;
          vj[r] = s * x + c * y;
        }
      }
    }
    if (!rotated) break;
  }
  sig.assign((size_t)n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    double s = 0;
    for (int64_t t = 0; t < n; ++t) s += B[(size_t)(i * n + t)] * B[(size_t)(i * n + t)];
    sig[(size_t)i] = std::sqrt(s);
  }
}

// Sizes of a C-order tensor with dims d (D modes) around mode k: A = prod_{l<k} d_l rows
// before it, Bs = prod_{l>k} d_l contiguous entries after it.
void around_mode(const int64_t* d, int D, int k, int64_t& A, int64_t& Bs) {
  A = 1;
  Bs = 1;
  for (int l = 0; l < k; ++l) A *= d[l];
  for (int l = k + 1; l < D; ++l) Bs *= d[l];
}

// Leading r left singular vectors (I x r, row-major, signs fixed) of the mode-k unfolding
// of Y with dims d (D modes); all singular values into sig_out (length min(I, L)).
void leading_left_singular(const std::vector<double>& Y, const int64_t* d, int D, int k, int r,
                           std::vector<double>& Wout, std::vector<double>& sig_out) {
  const int64_t I = d[k];
  int64_t A, Bs;
  around_mode(d, D, k, A, Bs);
  const int64_t L = A * Bs;
  // element (i, l) of the unfolding with l = a * Bs + b
  auto at = [&](int64_t i, int64_t l) {
    int64_t a = l / Bs, b = l % Bs;
    return Y[(size_t)((a * I + i) * Bs + b)];
  };
  std::vector<double> U((size_t)(I * I), 0.0);   // left singular vectors, column-major I x nsv
  std::vector<double> sig;
  int64_t nsv;
  if (L >= I) {
    // B = Y_(k)^T (L x I, column-major: column i is row i of the unfolding); B = QR;
    // Hestenes on R gives V = left singular vectors of Y_(k).
    HouseholderQR qr;
    qr.m = L;
    qr.n = I;
    qr.A.resize((size_t)(L * I));
    for (int64_t i = 0; i < I; ++i)
      for (int64_t l = 0; l < L; ++l) qr.A[(size_t)(i * L + l)] = at(i, l);
    qr.factor();
    std::vector<double> R = qr.R();
    std::vector<double> V;
    hestenes(R, I, V, sig);
    nsv = I;
    U = V;
  } else {
    // B = Y_(k) (I x L, column-major: column l is column l of the unfolding); B = QR;
    // Hestenes on R: R V = W, left singular vectors of Y_(k) are Q W / sigma.
    HouseholderQR qr;
    qr.m = I;
    qr.n = L;
    qr.A.resize((size_t)(I * L));
    for (int64_t l = 0; l < L; ++l)
      for (int64_t i = 0; i < I; ++i) qr.A[(size_t)(l * I + i)] = at(i, l);
    qr.factor();
    std::vector<double> R = qr.R();
    std::vector<double> V;
    hestenes(R, L, V, sig);   // R now holds W (columns)
    nsv = L;
    for (int64_t c = 0; c < L; ++c) {
      std::vector<double> y((size_t)I, 0.0);
      for (int64_t t = 0; t < L; ++t) y[(size_t)t] = sig[(size_t)c] > 0 ? R[(size_t)(c * L + t)] / sig[(size_t)c] : 0.0;
      qr.apply_Q(y.data());
      for (int64_t i = 0; i < I; ++i) U[(size_t)(c * I + i)] = y[(size_t)i];
    }
  }
  std::vector<int64_t> ord((size_t)nsv);
  std::iota(ord.begin(), ord.end(), int64_t(0));
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int64_t a, int64_t b) { return sig[(size_t)a] > sig[(size_t)b]; });
  sig_out.assign((size_t)nsv, 0.0);
  for (int64_t i = 0; i < nsv; ++i) sig_out[(size_t)i] = sig[(size_t)ord[(size_t)i]];
  Wout.assign((size_t)(I * r), 0.0);
  for (int j = 0; j < r; ++j) {
    const double* col = &U[(size_t)(ord[(size_t)j] * I)];
    int64_t imax = 0;
    for (int64_t i = 1; i < I; ++i)
      if (std::fabs(col[i]) > std::fabs(col[imax])) imax = i;
    double sgn = col[imax] < 0 ? -1.0 : 1.0;
    for (int64_t i = 0; i < I; ++i) Wout[(size_t)(i * r + j)] = sgn * col[i];
  }
}

// Y (dims d, D modes) <- Y x_k W^T with W (I_k x r) row-major; d[k] becomes r.
void mode_product_transposed(std::vector<double>& Y, int64_t* d, int D, int k, const std::vector<double>& W, int r) {
  const int64_t I = d[k];
  int64_t A, Bs;
  around_mode(d, D, k, A, Bs);
  std::vector<double> out((size_t)(A * r * Bs), 0.0);
  for (int64_t a = 0; a < A; ++a)
    for (int j = 0; j < r; ++j) {
      double* o = &out[(size_t)((a * r + j) * Bs)];
      for (int64_t i = 0; i < I; ++i) {
        double w = W[(size_t)(i * r + j)];
        const double* y = &Y[(size_t)((a * I + i) * Bs)];
        for (int64_t b = 0; b < Bs; ++b) o[b] += w * y[b];
      }
    }
  Y.swap(out);
  d[k] = r;
}

}  // namespace

void sthosvd_d(const double* T, int D, const int32_t* dims, const int32_t* rank, int n_threads, double* core,
               double* const* W, double* const* sigma) {
  (void)n_threads;
  if (D < 1 || D > kMaxModes) fail(FST_E_INVAL, "sthosvd: need 1 <= d <= 4");
  int64_t d[kMaxModes], total = 1;
  for (int k = 0; k < D; ++k) {
    d[k] = dims[k];
    if (d[k] < 1 || rank[k] < 1 || rank[k] > d[k]) fail(FST_E_INVAL, "sthosvd: need 1 <= r_k <= I_k");
    total *= d[k];
  }
  std::vector<double> Y(T, T + total);
  for (int k = 0; k < D; ++k) {
    int64_t L = 1;
    for (int l = 0; l < D; ++l)
      if (l != k) L *= d[l];
    if (rank[k] > L) fail(FST_E_INVAL, "sthosvd: r_k exceeds the product of the other sizes");
    std::vector<double> Wk, sig;
    leading_left_singular(Y, d, D, k, rank[k], Wk, sig);
    std::memcpy(W[k], Wk.data(), sizeof(double) * Wk.size());
    if (sigma && sigma[k]) {
      for (int64_t i = 0; i < dims[k]; ++i) sigma[k][i] = i < (int64_t)sig.size() ? sig[(size_t)i] : 0.0;
    }
    mode_product_transposed(Y, d, D, k, Wk, rank[k]);
  }
  std::memcpy(core, Y.data(), sizeof(double) * Y.size());
}

void sthosvd(const double* T, const int32_t dims[3], const int32_t rank[3], int n_threads,
             double* core, double* const W[3], double* const sigma[3]) {
  sthosvd_d(T, 3, dims, rank, n_threads, core, W, sigma);
}

// Ranks from a precision (Sec. 4.1, Table 1): the ST-HOSVD truncation rule that bounds the
// error, ||T - T~||_F^2 <= sum_k sum_{i > r_k} sigma_i^(k)2 <= eps^2 ||T||_F^2, spread evenly
// over the D modes: at step k, r_k is the smallest r with
// sum_{i > r} sigma_i^2 <= eps^2 ||T||_F^2 / D over the singular values of the current
// (already truncated) unfolding.  Ranks are capped at max_rank[k] (the bound then need not
// hold).  W[k] receives I_k x r_k row-major, core r1 .. rD.
void sthosvd_eps_d(const double* T, int D, const int32_t* dims, double eps, const int32_t* max_rank, int n_threads,
                   int32_t* rank_out, double* core, double* const* W, double* const* sigma) {
  (void)n_threads;
  if (D < 1 || D > kMaxModes) fail(FST_E_INVAL, "sthosvd_eps: need 1 <= d <= 4");
  if (!(eps > 0.0 && eps < 1.0)) fail(FST_E_INVAL, "sthosvd_eps: need 0 < eps < 1");
  int64_t d[kMaxModes], total = 1;
  for (int k = 0; k < D; ++k) {
    d[k] = dims[k];
    if (d[k] < 1 || max_rank[k] < 1) fail(FST_E_INVAL, "sthosvd_eps: need I_k >= 1 and max_rank_k >= 1");
    total *= d[k];
  }
  std::vector<double> Y(T, T + total);
  double norm2 = 0.0;
  for (int64_t i = 0; i < total; ++i) norm2 += T[i] * T[i];
  const double thr = eps * eps * norm2 / (double)D;
  for (int k = 0; k < D; ++k) {
    int64_t L = 1;
    for (int l = 0; l < D; ++l)
      if (l != k) L *= d[l];
    const int cap = (int)std::min<int64_t>({(int64_t)max_rank[k], d[k], L});
    std::vector<double> Wk, sig;
    leading_left_singular(Y, d, D, k, cap, Wk, sig);
    // tail[r] = sum_{i >= r} sigma_i^2 (0-based), summed from the smallest value up
    const int ns = (int)sig.size();
    std::vector<double> tail((size_t)ns + 1, 0.0);
    for (int i = ns - 1; i >= 0; --i) tail[(size_t)i] = tail[(size_t)i + 1] + sig[(size_t)i] * sig[(size_t)i];
    int r = 1;
    while (r < ns && tail[(size_t)r] > thr) ++r;
    r = std::min(r, cap);
    rank_out[k] = r;
    // the leading r of the cap columns (row-major I_k x cap -> I_k x r)
    for (int64_t i = 0; i < d[k]; ++i)
      for (int j = 0; j < r; ++j) W[k][(size_t)(i * r + j)] = Wk[(size_t)(i * cap + j)];
    if (sigma && sigma[k])
      for (int64_t i = 0; i < dims[k]; ++i) sigma[k][i] = i < (int64_t)sig.size() ? sig[(size_t)i] : 0.0;
    std::vector<double> Wr(W[k], W[k] + d[k] * r);
    mode_product_transposed(Y, d, D, k, Wr, r);
  }
  std::memcpy(core, Y.data(), sizeof(double) * Y.size());
}

void sthosvd_eps(const double* T, const int32_t dims[3], double eps, const int32_t max_rank[3], int n_threads,
                 int32_t rank_out[3], double* core, double* const W[3], double* const sigma[3]) {
  sthosvd_eps_d(T, 3, dims, eps, max_rank, n_threads, rank_out, core, W, sigma);
}

// ------------------------------------------------------------------------------ sparse fit
void legendre_orthonormal_host(double t, int p, double* phi) {
  // Bonnet recurrence (m+1) P_{m+1} = (2m+1) t P_m - m P_{m-1}, then phi_m = sqrt(2m+1) P_m
  double pm1 = 1.0, pm = t;
  phi[0] = 1.0;
  if (p >= 1) phi[1] = std::sqrt(3.0) * t;
  for (int m = 1; m < p; ++m) {
    double pn = ((2.0 * m + 1.0) * t * pm - m * pm1) / (m + 1.0);
    pm1 = pm;
    pm = pn;
    phi[m + 1] = std::sqrt(2.0 * (m + 1) + 1.0) * pn;
  }
}

namespace {
// Least squares on the selected columns by Householder QR; returns coefficients, residual
// and leverages h_ii (squared row norms of Phi_S R^-1).
void ls_select(const std::vector<double>& Phi, int I, int n, const std::vector<int>& S,
               const double* z, std::vector<double>& c, std::vector<double>& res,
               std::vector<double>& lev) {
  const int t = (int)S.size();
  HouseholderQR qr;
  qr.m = I;
  qr.n = t;
  qr.A.resize((size_t)I * t);
  for (int j = 0; j < t; ++j)
    for (int i = 0; i < I; ++i) qr.A[(size_t)j * I + i] = Phi[(size_t)i * n + S[(size_t)j]];
  qr.factor();
  std::vector<double> R = qr.R();   // column-major t x t
  // Q^T z: apply reflectors in forward order
  std::vector<double> y(z, z + I);
  for (int j = 0; j < t; ++j) {
    if (qr.beta[(size_t)j] == 0.0) continue;
    const double* col = &qr.A[(size_t)j * I];
    double s = y[(size_t)j];
    for (int i = j + 1; i < I; ++i) s += col[i] * y[(size_t)i];
    s *= qr.beta[(size_t)j];
    y[(size_t)j] -= s;
    for (int i = j + 1; i < I; ++i) y[(size_t)i] -= s * col[i];
  }
  c.assign((size_t)t, 0.0);
  for (int j = t - 1; j >= 0; --j) {
    double s = y[(size_t)j];
    for (int l = j + 1; l < t; ++l) s -= R[(size_t)l * t + j] * c[(size_t)l];
    c[(size_t)j] = s / R[(size_t)j * t + j];
  }
  res.assign((size_t)I, 0.0);
  lev.assign((size_t)I, 0.0);
  std::vector<double> w((size_t)t);
  for (int i = 0; i < I; ++i) {
    double f = 0.0;
    for (int j = 0; j < t; ++j) f += Phi[(size_t)i * n + S[(size_t)j]] * c[(size_t)j];
    res[(size_t)i] = z[i] - f;
    // solve R^T w = Phi_S[i, :]^T
    double h = 0.0;
    for (int j = 0; j < t; ++j) {
      double s = Phi[(size_t)i * n + S[(size_t)j]];
      for (int l = 0; l < j; ++l) s -= R[(size_t)j * t + l] * w[(size_t)l];
      w[(size_t)j] = s / R[(size_t)j * t + j];
      h += w[(size_t)j] * w[(size_t)j];
    }
    lev[(size_t)i] = h;
  }
}
}  // namespace

namespace {
// Lasso-modified least angle regression (Efron, Hastie, Johnstone, Tibshirani 2004) on the
// unit-norm columns X (I x n, row-major): the active set after every event of the path, in
// entry order.  Per step, with s the signs of the active correlations: G = (X_A S)^T (X_A S),
// A_A = (1^T G^-1 1)^(-1/2), w = A_A G^-1 1, u = X_A S w, a = X^T u; the path moves by the
// smaller of the first entry of an inactive column (correlation reaching C) and the first
// sign change of an active coefficient (Lasso modification: that column leaves).  Entry ties
// go to the lowest index; a column that has just left is not re-admitted in the next step;
// the path stops at max_active columns, when the correlations vanish, or at its end.
std::vector<std::vector<int>> lars_active_sets(const std::vector<double>& X, int I, int n, const double* z,
                                               int max_active) {
  std::vector<std::vector<int>> sets;
  std::vector<double> beta((size_t)n, 0.0), mu((size_t)I, 0.0), c((size_t)n), u((size_t)I), a((size_t)n);
  auto correlations = [&]() {
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int i = 0; i < I; ++i) t += X[(size_t)i * n + j] * (z[i] - mu[(size_t)i]);
      c[(size_t)j] = t;
    }
  };
  correlations();
  int j0 = 0;
  for (int j = 1; j < n; ++j)
    if (std::fabs(c[(size_t)j]) > std::fabs(c[(size_t)j0])) j0 = j;
  const double C0 = n > 0 ? std::fabs(c[(size_t)j0]) : 0.0;
  if (C0 == 0.0 || max_active < 1) return sets;
  std::vector<int> A{j0};
  sets.push_back(A);
  int barred = -1;
  for (int it = 0; it < 64 * n; ++it) {
    correlations();
    const int k = (int)A.size();
    double C = 0.0;
    std::vector<double> sg((size_t)k);
    for (int q = 0; q < k; ++q) {
      const double cq = c[(size_t)A[(size_t)q]];
      sg[(size_t)q] = cq > 0 ? 1.0 : (cq < 0 ? -1.0 : 0.0);
      C = std::max(C, std::fabs(cq));
    }
    if (C <= 1e-14 * C0) break;
    // G g1 = 1 by Cholesky (G is the Gram of linearly independent signed columns)
    std::vector<double> L((size_t)k * k, 0.0), g1((size_t)k, 1.0);
    for (int q = 0; q < k; ++q)
      for (int t = 0; t <= q; ++t) {
        double g = 0.0;
        for (int i = 0; i < I; ++i) g += X[(size_t)i * n + A[(size_t)q]] * X[(size_t)i * n + A[(size_t)t]];
        g *= sg[(size_t)q] * sg[(size_t)t];
        for (int l = 0; l < t; ++l) g -= L[(size_t)q * k + l] * L[(size_t)t * k + l];
        if (q == t) {
          if (!(g > 0.0)) return sets;   // numerically dependent active columns: end of the path
          L[(size_t)q * k + q] = std::sqrt(g);
        } else {
          L[(size_t)q * k + t] = g / L[(size_t)t * k + t];
        }
      }
    for (int q = 0; q < k; ++q) {
      double t = g1[(size_t)q];
      for (int l = 0; l < q; ++l) t -= L[(size_t)q * k + l] * g1[(size_t)l];
      g1[(size_t)q] = t / L[(size_t)q * k + q];
    }
    for (int q = k - 1; q >= 0; --q) {
      double t = g1[(size_t)q];
      for (int l = q + 1; l < k; ++l) t -= L[(size_t)l * k + q] * g1[(size_t)l];
      g1[(size_t)q] = t / L[(size_t)q * k + q];
    }
    double sum1 = 0.0;
    for (double t : g1) sum1 += t;
    const double AA = 1.0 / std::sqrt(sum1);
    std::vector<double> w((size_t)k);
    for (int q = 0; q < k; ++q) w[(size_t)q] = AA * g1[(size_t)q];
    for (int i = 0; i < I; ++i) {
      double t = 0.0;
      for (int q = 0; q < k; ++q) t += X[(size_t)i * n + A[(size_t)q]] * sg[(size_t)q] * w[(size_t)q];
      u[(size_t)i] = t;
    }
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int i = 0; i < I; ++i) t += X[(size_t)i * n + j] * u[(size_t)i];
      a[(size_t)j] = t;
    }
    double gamma_hat = C / AA;
    int j_hat = -1;
    for (int j = 0; j < n; ++j) {
      if (j == barred || std::find(A.begin(), A.end(), j) != A.end()) continue;
      const double num[2] = {C - c[(size_t)j], C + c[(size_t)j]}, den[2] = {AA - a[(size_t)j], AA + a[(size_t)j]};
      for (int e = 0; e < 2; ++e) {
        if (den[e] == 0.0) continue;
        const double g = num[e] / den[e];
        if (g > 0.0 && g < gamma_hat) {
          gamma_hat = g;
          j_hat = j;
        }
      }
    }
    double gamma_til = std::numeric_limits<double>::infinity();
    int k_til = -1;
    for (int q = 0; q < k; ++q) {
      const double d = sg[(size_t)q] * w[(size_t)q];
      if (d == 0.0) continue;
      const double g = -beta[(size_t)A[(size_t)q]] / d;
      if (g > 0.0 && g < gamma_til) {
        gamma_til = g;
        k_til = q;
      }
    }
    const bool drop = gamma_til < gamma_hat;
    const double gamma = drop ? gamma_til : gamma_hat;
    for (int i = 0; i < I; ++i) mu[(size_t)i] += gamma * u[(size_t)i];
    for (int q = 0; q < k; ++q) beta[(size_t)A[(size_t)q]] += gamma * sg[(size_t)q] * w[(size_t)q];
    barred = -1;
    if (drop) {
      const int j_out = A[(size_t)k_til];
      beta[(size_t)j_out] = 0.0;
      A.erase(A.begin() + k_til);
      barred = j_out;
      sets.push_back(A);
      continue;
    }
    if (j_hat < 0) {   // end of the path: every correlation reached zero
      sets.push_back(A);
      break;
    }
    if ((int)A.size() >= max_active) break;
    A.push_back(j_hat);
    sets.push_back(A);
  }
  return sets;
}
}  // namespace

namespace {
// One column's sparse fit: the support and least-squares coefficients of the path step with
// the smallest PRESS (first on ties), and that PRESS (infinite when nothing was fitted).
struct ColumnFit {
  std::vector<int> S;
  std::vector<double> c;
  double press = std::numeric_limits<double>::infinity();
};

// A basis sampled at the nodes: Phi (I x n row-major) and its unit-norm columns X
struct NodeBasis {
  int I = 0, n = 0;
  std::vector<double> Phi, X, colnorm;
};

NodeBasis node_basis(std::vector<double> Phi, int I, int n) {
  NodeBasis b;
  b.I = I;
  b.n = n;
  b.Phi = std::move(Phi);
  b.X.resize((size_t)I * n);
  b.colnorm.assign((size_t)n, 0.0);
  for (int m = 0; m < n; ++m) {
    double s2 = 0;
    for (int i = 0; i < I; ++i) s2 += b.Phi[(size_t)i * n + m] * b.Phi[(size_t)i * n + m];
    b.colnorm[(size_t)m] = std::sqrt(s2);
    for (int i = 0; i < I; ++i) b.X[(size_t)i * n + m] = b.Phi[(size_t)i * n + m] / b.colnorm[(size_t)m];
  }
  return b;
}

double press_of(const std::vector<double>& res, const std::vector<double>& lev, int I) {
  double pr = 0.0;
  for (int i = 0; i < I; ++i) {
    const double e = res[(size_t)i] / (1.0 - lev[(size_t)i]);
    pr += e * e;
  }
  pr /= I;
  return pr == pr ? pr : std::numeric_limits<double>::infinity();
}

// Orthogonal matching pursuit: the column of largest normalised correlation with the residual
// joins (lowest index on ties), least squares on the support, PRESS after every step.
ColumnFit omp_column(const NodeBasis& B, const double* z) {
  const int I = B.I, n = B.n;
  ColumnFit out;
  double zn = 0;
  for (int i = 0; i < I; ++i) zn += z[i] * z[i];
  zn = std::sqrt(zn);
  if (zn == 0.0) return out;
  std::vector<int> S;
  std::vector<std::vector<double>> coefs;
  std::vector<double> press, res, lev, c, rcur(z, z + I);
  const int tmax = std::min(n, I - 2);
  for (int t = 0; t < tmax; ++t) {
    int best = -1;
    double bscore = -1.0;
    for (int m = 0; m < n; ++m) {
      if (std::find(S.begin(), S.end(), m) != S.end()) continue;
      double s = 0;
      for (int i = 0; i < I; ++i) s += B.Phi[(size_t)i * n + m] * rcur[(size_t)i];
      const double score = std::fabs(s) / B.colnorm[(size_t)m];
      if (score > bscore) {
        bscore = score;
        best = m;
      }
    }
    S.push_back(best);
    ls_select(B.Phi, I, n, S, z, c, res, lev);
    press.push_back(press_of(res, lev, I));
    coefs.push_back(c);
    rcur = res;
    double rn = 0;
    for (double t2 : res) rn += t2 * t2;
    if (std::sqrt(rn) <= 1e-14 * zn) break;
  }
  if (press.empty()) return out;
  size_t tb = 0;
  for (size_t t = 1; t < press.size(); ++t)
    if (press[t] < press[tb]) tb = t;
  out.S.assign(S.begin(), S.begin() + (long)tb + 1);
  out.c = coefs[tb];
  out.press = press[tb];
  return out;
}

// Lasso-LARS path (lars_active_sets on the unit-norm columns), every active set refitted by
// least squares and scored by PRESS.
ColumnFit lars_column(const NodeBasis& B, const double* z) {
  const int I = B.I, n = B.n;
  ColumnFit out;
  double zn = 0;
  for (int i = 0; i < I; ++i) zn += z[i] * z[i];
  zn = std::sqrt(zn);
  if (zn == 0.0) return out;
  const std::vector<std::vector<int>> sets = lars_active_sets(B.X, I, n, z, std::min(n, I - 2));
  std::vector<std::vector<double>> coefs;
  std::vector<double> press, res, lev, c;
  for (const std::vector<int>& S : sets) {
    if (S.empty()) {
      press.push_back(std::numeric_limits<double>::infinity());
      coefs.emplace_back();
      continue;
    }
    ls_select(B.Phi, I, n, S, z, c, res, lev);
    press.push_back(press_of(res, lev, I));
    coefs.push_back(c);
    double rn = 0;
    for (double t2 : res) rn += t2 * t2;
    if (std::sqrt(rn) <= 1e-14 * zn) break;
  }
  if (press.empty()) return out;
  size_t tb = 0;
  for (size_t t = 1; t < press.size(); ++t)
    if (press[t] < press[tb]) tb = t;
  out.S = sets[tb];
  out.c = coefs[tb];
  out.press = press[tb];
  return out;
}

ColumnFit fit_column(int solver, const NodeBasis& B, const double* z) {
  return solver == FST_SOLVER_LARS ? lars_column(B, z) : omp_column(B, z);
}

std::vector<double> legendre_at_nodes(int I, int p) {
  std::vector<double> Phi((size_t)I * (p + 1));
  for (int i = 0; i < I; ++i) legendre_orthonormal_host(-1.0 + 2.0 * i / (I - 1), p, &Phi[(size_t)i * (p + 1)]);
  return Phi;
}

void fit_columns(int solver, const double* W, int I, int r, int p, double* C) {
  if (I < 3 || r < 1 || p < 0) fail(FST_E_INVAL, "sparse_fit: need I >= 3, r >= 1, p >= 0");
  const int n = p + 1;
  const NodeBasis B = node_basis(legendre_at_nodes(I, p), I, n);
  std::fill(C, C + (size_t)n * r, 0.0);
  std::vector<double> z((size_t)I);
  for (int j = 0; j < r; ++j) {
    for (int i = 0; i < I; ++i) z[(size_t)i] = W[(size_t)i * r + j];
    const ColumnFit f = fit_column(solver, B, z.data());
    for (size_t l = 0; l < f.S.size(); ++l) C[(size_t)f.S[l] * r + j] = f.c[l];
  }
}
}  // namespace

void sparse_fit(const double* W, int I, int r, int p, double* C) { fit_columns(FST_SOLVER_OMP, W, I, r, p, C); }
void sparse_fit_lars(const double* W, int I, int r, int p, double* C) { fit_columns(FST_SOLVER_LARS, W, I, r, p, C); }

// ------------------------------------------------------------------------------ wavelets
// Gauss-Legendre nodes and weights on [-1, 1] (weights sum to 2): Newton's method on P_n from
// the usual cosine first guesses, P_n and P_n' from Bonnet's recurrence.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign((size_t)n, 0.0);
  w.assign((size_t)n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double t = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 0 ? 1.0 : p1, pm = n == 0 ? 0.0 : p0;
      dp = n * (t * pn - pm) / (t * t - 1.0);
      const double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) <= 1e-16 * std::max(1.0, std::fabs(t))) break;
    }
    {   // derivative at the converged node
      double p0 = 1.0, p1 = t;
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
    }
    x[(size_t)i] = t;
    w[(size_t)i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Mother wavelets psi_0..psi_q of W_{s,q} on [-1, 1]: psi_m(x) = sqrt(2) sum_n H[m][half][n]
// phi_n(2x + 1) on [-1, 0) (half 0) or phi_n(2x - 1) on [0, 1] (half 1).  In the coordinates of
// the orthonormal half-cell functions sqrt(2) phi_n(2x -+ 1), psi_m is the unit vector
// orthogonal to phi_0..phi_{q+m} and to psi_{m+1}..psi_q (found from the top down as the last
// column of the Q factor of the constraint rows), signed so that its largest right-half
// coordinate is positive.
void mother_wavelets_host(int q, double* H) {
  if (q < 0 || q > kMaxWaveDegree) fail(FST_E_UNSUPPORTED, "wavelet degree out of range");
  const int nh = q + 1, dim = 2 * nh, nc = 2 * q + 1;
  std::vector<double> xg, wg;
  gauss_legendre(2 * q + 2, xg, wg);
  // M[i][half * nh + n] = <h_{half,n}, phi_i> under dt/2, i = 0..2q
  std::vector<double> M((size_t)nc * dim, 0.0), h((size_t)nh), g((size_t)2 * q + 1);
  for (int half = 0; half < 2; ++half)
    for (size_t k = 0; k < xg.size(); ++k) {
      const double x = (xg[k] + (half ? 1.0 : -1.0)) / 2.0;
      legendre_orthonormal_host(xg[k], q, h.data());
      legendre_orthonormal_host(x, 2 * q, g.data());
      for (int i = 0; i < nc; ++i)
        for (int n = 0; n < nh; ++n)
          M[(size_t)i * dim + half * nh + n] += 0.25 * wg[k] * g[(size_t)i] * std::sqrt(2.0) * h[(size_t)n];
    }
  std::vector<std::vector<double>> psi((size_t)nh);
  for (int m = q; m >= 0; --m) {
    HouseholderQR qr;   // of A^T, A = the 2q + 1 constraint rows
    qr.m = dim;
    qr.n = nc;
    qr.A.assign((size_t)dim * nc, 0.0);
    int row = 0;
    for (int i = 0; i <= q + m; ++i, ++row)
      for (int c = 0; c < dim; ++c) qr.A[(size_t)row * dim + c] = M[(size_t)i * dim + c];
    for (int k = m + 1; k <= q; ++k, ++row)
      for (int c = 0; c < dim; ++c) qr.A[(size_t)row * dim + c] = psi[(size_t)k][(size_t)c];
    qr.factor();
    std::vector<double> v((size_t)dim, 0.0);
    v[(size_t)dim - 1] = 1.0;
    qr.apply_Q(v.data());
    int jmax = nh;
    for (int c = nh + 1; c < dim; ++c)
      if (std::fabs(v[(size_t)c]) > std::fabs(v[(size_t)jmax])) jmax = c;
    double nrm = 0.0;
    for (double t : v) nrm += t * t;
    nrm = std::sqrt(nrm) * (v[(size_t)jmax] < 0 ? -1.0 : 1.0);
    for (double& t : v) t /= nrm;
    psi[(size_t)m] = v;
  }
  for (int m = 0; m < nh; ++m)
    for (int c = 0; c < dim; ++c) H[(size_t)m * dim + c] = psi[(size_t)m][(size_t)c];
}

int detail_count(int s, int q) { return s <= 0 ? 0 : (q + 1) * ((1 << s) - 1); }

// psi_{l,c,m}(t) for every level l < s, in the order (l, c, m), zero off the point's cells
void detail_values_host(double t, int s, int q, const double* H, double* out) {
  const int nh = q + 1;
  std::fill(out, out + detail_count(s, q), 0.0);
  std::vector<double> ph((size_t)nh);
  for (int l = 0; l < s; ++l) {
    const int ncell = 1 << l;
    const int c = (int)std::min<double>(std::max<double>(std::floor((t + 1.0) * ncell / 2.0), 0.0), ncell - 1);
    const double x = (t + 1.0) * ncell - 2.0 * c - 1.0;
    const int half = x >= 0.0 ? 1 : 0;
    legendre_orthonormal_host(half ? 2.0 * x - 1.0 : 2.0 * x + 1.0, q, ph.data());
    const double scale = std::sqrt(2.0) * std::pow(2.0, 0.5 * l);
    for (int m = 0; m < nh; ++m) {
      double v = 0.0;
      for (int n = 0; n < nh; ++n) v += H[(size_t)(m * 2 + half) * nh + n] * ph[(size_t)n];
      out[(size_t)nh * (ncell - 1 + c) + m] = scale * v;
    }
  }
}

// Algorithm 1 steps 5-6 with both spaces: every column is fitted in P_p (rows 0..p of the mode
// basis) and in W_{s,q} (rows 0..q and the detail rows), and the fit with the smaller
// leave-one-out error is kept (P_p on ties).  C: (p + 1 + detail_count) x r row-major.
void sparse_fit_choice(const double* W, int I, int r, int p, int s, int q, int solver, double* C) {
  if (I < 3 || r < 1 || p < 0) fail(FST_E_INVAL, "sparse_fit: need I >= 3, r >= 1, p >= 0");
  if (s < 1 || q < 0 || q > p || q > kMaxWaveDegree || detail_count(s, q) > kMaxDetail)
    fail(FST_E_INVAL, "wavelet space: need s >= 1, 0 <= q <= p, q <= 7 and (q + 1)(2^s - 1) <= 128");
  const int nd = detail_count(s, q), nrow = p + 1 + nd, nw = q + 1 + nd;
  std::vector<double> H((size_t)(q + 1) * 2 * (q + 1)), dv((size_t)nd);
  mother_wavelets_host(q, H.data());
  std::vector<double> PL = legendre_at_nodes(I, p), PW((size_t)I * nw);
  for (int i = 0; i < I; ++i) {
    const double t = -1.0 + 2.0 * i / (I - 1);
    for (int n = 0; n <= q; ++n) PW[(size_t)i * nw + n] = PL[(size_t)i * (p + 1) + n];
    detail_values_host(t, s, q, H.data(), dv.data());
    for (int e = 0; e < nd; ++e) PW[(size_t)i * nw + q + 1 + e] = dv[(size_t)e];
  }
  const NodeBasis BL = node_basis(PL, I, p + 1), BW = node_basis(PW, I, nw);
  std::fill(C, C + (size_t)nrow * r, 0.0);
  std::vector<double> z((size_t)I);
  for (int j = 0; j < r; ++j) {
    for (int i = 0; i < I; ++i) z[(size_t)i] = W[(size_t)i * r + j];
    const ColumnFit fl = fit_column(solver, BL, z.data()), fw = fit_column(solver, BW, z.data());
    if (fl.S.empty() && fw.S.empty()) continue;
    if (!fl.S.empty() && (fw.S.empty() || fl.press <= fw.press)) {
      for (size_t l = 0; l < fl.S.size(); ++l) C[(size_t)fl.S[l] * r + j] = fl.c[l];
    } else {
      for (size_t l = 0; l < fw.S.size(); ++l) {
        const int col = fw.S[l], rowi = col <= q ? col : p + 1 + (col - q - 1);
        C[(size_t)rowi * r + j] = fw.c[l];
      }
    }
  }
}

}  // namespace fst
