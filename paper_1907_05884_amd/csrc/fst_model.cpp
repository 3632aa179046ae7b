// The functional sparse Tucker model object (eq. (1)-(2)): validation, device copies and a
// versioned binary serialisation.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fst_internal.h"

fst_model::~fst_model() {
  for (auto& kv : dev) {
    fst::device_free(kv.second.coefs);
    fst::device_free(kv.second.cheb);
    fst::device_free(kv.second.core);
    fst::device_free(kv.second.core64);
    fst::device_free(kv.second.detail);
    fst::device_free(kv.second.wave);
  }
}

namespace fst {

fst_model* model_new(const double lo[3], const double hi[3], const int32_t rank[3],
                     const int32_t degree[3]) {
  return model_new_d(3, lo, hi, rank, degree);
}

fst_model* model_new_d(int d, const double* lo, const double* hi, const int32_t* rank, const int32_t* degree,
                       const int32_t* wlevel, const int32_t* wdegree) {
  if (d != 3 && d != 4) fail(FST_E_UNSUPPORTED, "model: only d = 3 and d = 4 are supported");
  if (wlevel)
    for (int k = 0; k < d; ++k) {
      if (wlevel[k] < 0 || wlevel[k] > 7) fail(FST_E_INVAL, "model: wavelet level must be in [0, 7]");
      if (wlevel[k] > 0 && (!wdegree || wdegree[k] < 0 || wdegree[k] > std::min(degree[k], kMaxWaveDegree) ||
                            detail_count(wlevel[k], wdegree[k]) > kMaxDetail))
        fail(FST_E_INVAL, "model: wavelet degree must be in [0, min(p, 7)] with (q + 1)(2^s - 1) <= 128");
    }
  for (int k = 0; k < d; ++k) {
    if (!(std::isfinite(lo[k]) && std::isfinite(hi[k]) && hi[k] > lo[k]))
      fail(FST_E_INVAL, "model: need finite lo < hi in every mode");
    if (rank[k] < 1) fail(FST_E_INVAL, "model: ranks must be >= 1");
    if (degree[k] < 0) fail(FST_E_INVAL, "model: degrees must be >= 0");
    if (rank[k] > kMaxRank) fail(FST_E_UNSUPPORTED, "model: rank above 32 is not supported");
    if (degree[k] + 1 > kMaxBasis) fail(FST_E_UNSUPPORTED, "model: degree above 31 is not supported");
  }
  fst_model* m = new fst_model();
  m->d = d;
  for (int k = 0; k < d; ++k) {
    m->lo[k] = lo[k];
    m->hi[k] = hi[k];
    m->rank[k] = rank[k];
    m->degree[k] = degree[k];
    m->wlevel[k] = wlevel ? wlevel[k] : 0;
    m->wdegree[k] = m->wlevel[k] > 0 ? wdegree[k] : 0;
    m->coef[k].assign((size_t)m->rows(k) * rank[k], 0.0);
  }
  m->core.assign((size_t)m->R(), 0.0);
  return m;
}

void check_model(const fst_model* m) {
  if (!m) fail(FST_E_INVAL, "null model");
}

void check_model3(const fst_model* m) {
  check_model(m);
  if (m->d != 3) fail(FST_E_INVAL, "this call takes a 3-way model; 4-way models go through the d-way calls");
}

fst_model* copy_with_core(const fst_model* m, const std::vector<double>& core) {
  fst_model* out = model_new_d(m->d, m->lo, m->hi, m->rank, m->degree, m->wlevel, m->wdegree);
  for (int k = 0; k < m->d; ++k) out->coef[k] = m->coef[k];
  out->core = core;
  return out;
}

template <class T>
static void pack_model(const fst_model* m, std::vector<T>& coefs, std::vector<T>& core, std::vector<T>& detail,
                       std::vector<T>& wave) {
  coefs.assign((size_t)kMaxModes * kMaxBasis * kMaxRank, T(0));
  for (int k = 0; k < m->d; ++k) {
    const int n = m->degree[k] + 1, r = m->rank[k];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < r; ++j)
        coefs[(size_t)(k * kMaxBasis + i) * kMaxRank + j] = (T)m->coef[k][(size_t)i * r + j];
  }
  core.resize(m->core.size());
  for (size_t i = 0; i < core.size(); ++i) core[i] = (T)m->core[i];
  detail.clear();
  wave.clear();
  if (!m->has_wavelets()) return;
  detail.assign((size_t)kMaxModes * kMaxDetail * kMaxRank, T(0));
  wave.assign((size_t)kMaxModes * kWaveTable, T(0));
  for (int k = 0; k < m->d; ++k) {
    if (m->wlevel[k] == 0) continue;
    const int n = m->degree[k] + 1, r = m->rank[k], q = m->wdegree[k];
    for (int e = 0; e < m->details(k); ++e)
      for (int j = 0; j < r; ++j)
        detail[(size_t)(k * kMaxDetail + e) * kMaxRank + j] = (T)m->coef[k][(size_t)(n + e) * r + j];
    // mother wavelets in a fixed stride: [m][half][n] with kMaxWaveDegree + 1 entries per index
    std::vector<double> H((size_t)2 * (q + 1) * (q + 1));
    mother_wavelets_host(q, H.data());
    for (int mm = 0; mm <= q; ++mm)
      for (int half = 0; half < 2; ++half)
        for (int nn = 0; nn <= q; ++nn)
          wave[(size_t)k * kWaveTable + (size_t)((mm * 2 + half) * (kMaxWaveDegree + 1) + nn)] =
              (T)H[(size_t)(mm * 2 + half) * (q + 1) + nn];
  }
}

// The factor functions of eq. (2) in the Chebyshev basis: phi_m = sqrt(2m+1) P_m =
// sum_i L[m][i] T_i, with P_m = sum_i a[m][i] T_i from (m+1) P_{m+1} = (2m+1) t P_m - m P_{m-1}
// and t T_0 = T_1, t T_i = (T_{i+1} + T_{i-1}) / 2; the coefficients of mode k become
// D[i][j] = sum_m L[m][i] C[m][j] (FP64, rounded once to FP32).  The row sums of L are
// phi_m(1) = sqrt(2m+1) with all entries >= 0, so sum_i |D[i][j]| <= sum_m sqrt(2m+1) |C[m][j]|.
// Each mode is then scaled by 2^xc[k] (exact), its largest |D| to [2^14, 2^15), for the FP16
// operands of the factor kernel.
static void pack_chebyshev(const fst_model* m, std::vector<float>& cheb, int32_t* xc) {
  double a[kMaxBasis][kMaxBasis] = {};
  a[0][0] = 1.0;
  a[1][1] = 1.0;
  for (int n = 1; n + 1 < kMaxBasis; ++n) {
    double tp[kMaxBasis + 1] = {};   // t P_n
    tp[1] += a[n][0];
    for (int i = 1; i <= n; ++i) {
      tp[i + 1] += 0.5 * a[n][i];
      tp[i - 1] += 0.5 * a[n][i];
    }
    for (int i = 0; i <= n + 1; ++i) a[n + 1][i] = ((2.0 * n + 1.0) * tp[i] - n * a[n - 1][i]) / (n + 1.0);
  }
  cheb.assign((size_t)kMaxModes * kMaxBasis * kMaxRank, 0.0f);
  for (int k = 0; k < m->d; ++k) {
    const int n = m->degree[k] + 1, r = m->rank[k];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < r; ++j) {
        double sum = 0.0;
        for (int mm = i; mm < n; mm += 2) sum += std::sqrt(2.0 * mm + 1.0) * a[mm][i] * m->coef[k][(size_t)mm * r + j];
        cheb[(size_t)(k * kMaxBasis + i) * kMaxRank + j] = (float)sum;
      }
    float mx = 0.0f;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < r; ++j) mx = std::max(mx, std::fabs(cheb[(size_t)(k * kMaxBasis + i) * kMaxRank + j]));
    int e = 0;
    std::frexp(mx, &e);
    xc[k] = std::max(-20, std::min(26, 15 - e));
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < r; ++j) {
        float& c = cheb[(size_t)(k * kMaxBasis + i) * kMaxRank + j];
        c = std::ldexp(c, xc[k]);
      }
  }
}

template <class T>
static void upload(void*& dst, const std::vector<T>& v) {
  if (v.empty()) return;
  dst = device_alloc(v.size() * sizeof(T));
  copy_h2d(dst, v.data(), v.size() * sizeof(T), nullptr);
}

const DeviceModel& device_model(const fst_model* m, int dtype) {
  int dev = current_device();
  std::lock_guard<std::mutex> lk(m->mu);
  auto key = std::make_pair(dev, dtype);
  auto it = m->dev.find(key);
  if (it != m->dev.end()) return it->second;
  DeviceModel dm;
  if (dtype == FST_F64) {
    std::vector<double> c, a, dt, wv;
    pack_model(m, c, a, dt, wv);
    upload(dm.coefs, c);
    upload(dm.core, a);
    upload(dm.detail, dt);
    upload(dm.wave, wv);
  } else {
    std::vector<float> c, a, dt, wv;
    pack_model(m, c, a, dt, wv);
    upload(dm.coefs, c);
    upload(dm.core, a);
    upload(dm.detail, dt);
    upload(dm.wave, wv);
    if (!m->has_wavelets()) {
      std::vector<float> ch;
      pack_chebyshev(m, ch, dm.cheb_xc);
      upload(dm.cheb, ch);
    }
  }
  stream_sync(nullptr);
  return m->dev.emplace(key, dm).first->second;
}

}  // namespace fst

// ------------------------------------------------------------------------------ serialisation
// Layout (little endian):
//   "FSTM" | u32 version (1, or 2 with wavelets) | u32 d (3 or 4) | f64 lo[d] | f64 hi[d]
//   | i32 rank[d] | i32 degree[d] | version 2: i32 wlevel[d], i32 wdegree[d]
//   | f64 core[R] | per mode: i32 nnz, i32 colptr[r+1], u8 row[nnz], f64 val[nnz]
//   | u64 FNV-1a checksum of all preceding bytes
namespace {
struct Writer {
  std::vector<unsigned char> b;
  template <class T> void put(const T& v) {
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
    b.insert(b.end(), p, p + sizeof(T));
  }
};
struct Reader {
  const unsigned char* p;
  size_t n, off = 0;
  template <class T> T get() {
    if (off + sizeof(T) > n) fst::fail(FST_E_FORMAT, "model buffer is truncated");
    T v;
    std::memcpy(&v, p + off, sizeof(T));
    off += sizeof(T);
    return v;
  }
};
uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}
std::vector<unsigned char> serialise(const fst_model* m) {
  Writer w;
  w.b.insert(w.b.end(), {'F', 'S', 'T', 'M'});
  const bool wav = m->has_wavelets();
  w.put<uint32_t>(wav ? 2 : 1);
  w.put<uint32_t>((uint32_t)m->d);
  for (int k = 0; k < m->d; ++k) w.put<double>(m->lo[k]);
  for (int k = 0; k < m->d; ++k) w.put<double>(m->hi[k]);
  for (int k = 0; k < m->d; ++k) w.put<int32_t>(m->rank[k]);
  for (int k = 0; k < m->d; ++k) w.put<int32_t>(m->degree[k]);
  if (wav) {
    for (int k = 0; k < m->d; ++k) w.put<int32_t>(m->wlevel[k]);
    for (int k = 0; k < m->d; ++k) w.put<int32_t>(m->wdegree[k]);
  }
  for (double c : m->core) w.put<double>(c);
  for (int k = 0; k < m->d; ++k) {
    const int n = m->rows(k), r = m->rank[k];
    std::vector<int32_t> colptr(1, 0);
    std::vector<uint8_t> rows;
    std::vector<double> vals;
    for (int j = 0; j < r; ++j) {
      for (int i = 0; i < n; ++i) {
        double v = m->coef[k][(size_t)i * r + j];
        if (v != 0.0) {
          rows.push_back((uint8_t)i);
          vals.push_back(v);
        }
      }
      colptr.push_back((int32_t)rows.size());
    }
    w.put<int32_t>((int32_t)rows.size());
    for (int32_t c : colptr) w.put<int32_t>(c);
    for (uint8_t rr : rows) w.put<uint8_t>(rr);
    for (double v : vals) w.put<double>(v);
  }
  w.put<uint64_t>(fnv1a(w.b.data(), w.b.size()));
  return w.b;
}
}  // namespace

extern "C" {

fst_status fst_model_save(const fst_model* m, void* buf, size_t* nbytes) {
  try {
    fst::check_model(m);
    if (!nbytes) fst::fail(FST_E_INVAL, "nbytes is null");
    std::vector<unsigned char> b = serialise(m);
    if (!buf) {
      *nbytes = b.size();
      return FST_OK;
    }
    if (*nbytes < b.size()) fst::fail(FST_E_INVAL, "buffer too small for the model");
    std::memcpy(buf, b.data(), b.size());
    *nbytes = b.size();
    return FST_OK;
  } catch (const fst::Error& e) {
    fst::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    fst::set_last_error(e.what());
    return FST_E_NOMEM;
  }
}

fst_status fst_model_load(const void* buf, size_t nbytes, fst_model** out) {
  fst_model* m = nullptr;
  try {
    if (!buf || !out) fst::fail(FST_E_INVAL, "null argument");
    const unsigned char* p = static_cast<const unsigned char*>(buf);
    if (nbytes < 4 + 8 || std::memcmp(p, "FSTM", 4) != 0) fst::fail(FST_E_FORMAT, "not a model buffer");
    if (nbytes < 8 + 4) fst::fail(FST_E_FORMAT, "model buffer is truncated");
    uint64_t stored;
    Reader r{p, nbytes, 4};
    uint32_t version = r.get<uint32_t>();
    uint32_t d = r.get<uint32_t>();
    if (version != 1 && version != 2) fst::fail(FST_E_FORMAT, "unknown model version");
    if (d != 3 && d != 4) fst::fail(FST_E_UNSUPPORTED, "only d = 3 and d = 4 models are supported");
    double lo[4], hi[4];
    int32_t rank[4], degree[4];
    for (uint32_t k = 0; k < d; ++k) lo[k] = r.get<double>();
    for (uint32_t k = 0; k < d; ++k) hi[k] = r.get<double>();
    for (uint32_t k = 0; k < d; ++k) rank[k] = r.get<int32_t>();
    for (uint32_t k = 0; k < d; ++k) degree[k] = r.get<int32_t>();
    for (uint32_t k = 0; k < d; ++k)
      if (rank[k] < 1 || rank[k] > fst::kMaxRank || degree[k] < 0 || degree[k] + 1 > fst::kMaxBasis)
        fst::fail(FST_E_FORMAT, "model header out of range");
    int32_t wl[4] = {0, 0, 0, 0}, wd[4] = {0, 0, 0, 0};
    if (version == 2) {
      for (uint32_t k = 0; k < d; ++k) wl[k] = r.get<int32_t>();
      for (uint32_t k = 0; k < d; ++k) wd[k] = r.get<int32_t>();
    }
    try {
      m = fst::model_new_d((int)d, lo, hi, rank, degree, wl, wd);
    } catch (const fst::Error&) {
      fst::fail(FST_E_FORMAT, "model header out of range");
    }
    if (r.n - r.off < sizeof(double) * m->core.size()) fst::fail(FST_E_FORMAT, "model buffer is truncated");
    for (auto& c : m->core) c = r.get<double>();
    for (uint32_t k = 0; k < d; ++k) {
      const int n = m->rows((int)k), rk = rank[k];
      int32_t nnz = r.get<int32_t>();
      if (nnz < 0 || nnz > n * rk) fst::fail(FST_E_FORMAT, "bad coefficient count");
      std::vector<int32_t> colptr((size_t)rk + 1);
      for (auto& c : colptr) c = r.get<int32_t>();
      if (colptr[0] != 0 || colptr[(size_t)rk] != nnz) fst::fail(FST_E_FORMAT, "bad column pointers");
      for (int j = 0; j < rk; ++j)
        if (colptr[(size_t)j + 1] < colptr[(size_t)j]) fst::fail(FST_E_FORMAT, "bad column pointers");
      std::vector<uint8_t> rows((size_t)nnz);
      for (auto& x : rows) x = r.get<uint8_t>();
      for (int j = 0; j < rk; ++j)
        for (int32_t s = colptr[(size_t)j]; s < colptr[(size_t)j + 1]; ++s) {
          if (rows[(size_t)s] >= n) fst::fail(FST_E_FORMAT, "coefficient row out of range");
          m->coef[k][(size_t)rows[(size_t)s] * rk + j] = 0.0;  // placeholder, value below
        }
      std::vector<double> vals((size_t)nnz);
      for (auto& x : vals) x = r.get<double>();
      for (int j = 0; j < rk; ++j)
        for (int32_t s = colptr[(size_t)j]; s < colptr[(size_t)j + 1]; ++s)
          m->coef[k][(size_t)rows[(size_t)s] * rk + j] = vals[(size_t)s];
    }
    size_t body = r.off;
    stored = r.get<uint64_t>();
    if (stored != fnv1a(p, body)) fst::fail(FST_E_FORMAT, "model checksum mismatch");
    *out = m;
    return FST_OK;
  } catch (const fst::Error& e) {
    delete m;
    fst::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    delete m;
    fst::set_last_error(e.what());
    return FST_E_NOMEM;
  }
}

}  // extern "C"
