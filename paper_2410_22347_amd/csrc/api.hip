// C ABI of the library: argument validation, handle lifetime and the
// sequencing of the device stages.  No exception crosses this boundary.
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>

#include "common.hpp"

namespace gv {

static thread_local std::string g_err;
static std::atomic<uint64_t> g_handle_gen{0};
uint64_t next_handle_gen() { return ++g_handle_gen; }
static thread_local int g_splits = 0, g_qpw = 0, g_cap = 0;
void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
int tuned_splits() { return g_splits; }
int tuned_qpw() { return g_qpw; }
int tuned_cap() { return g_cap; }
static thread_local int g_optimism = 0;
int tuned_optimism() { return g_optimism; }

// forced allocation failure (gv_debug_fail_alloc): the allocation that finds
// the count at 0 fails; -1 is off
static std::atomic<long> g_fail_alloc{-1};
bool take_forced_alloc_failure() {
  long v = g_fail_alloc.load();
  while (v >= 0) {
    if (g_fail_alloc.compare_exchange_weak(v, v - 1)) return v == 0;
  }
  return false;
}
void set_tuning(int splits, int qpw, int cap) {
  g_splits = splits;
  g_qpw = qpw;
  g_cap = cap;
}

namespace {
struct ProfRec {
  hipEvent_t a, b;
  int kind;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
hipEvent_t g_prof_open[2] = {nullptr, nullptr};
bool g_prof_on = false;
}  // namespace

bool profiling() { return g_prof_on; }

// set while gv_search_batched captures a graph, or while a call that must not
// allocate runs: no profiling events then
static thread_local bool g_capturing = false;
static thread_local bool g_no_events = false;
bool capturing_batch() { return g_capturing || g_no_events; }
void suppress_profile_events(bool on) { g_no_events = on; }

void profile_mark(hipStream_t st, int kind, bool begin) {
  if (!g_prof_on || capturing_batch()) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, st);
  if (begin) {
    if (g_prof_open[kind]) (void)hipEventDestroy(g_prof_open[kind]);
    g_prof_open[kind] = e;
  } else if (g_prof_open[kind]) {
    g_prof.push_back({g_prof_open[kind], e, kind});
    g_prof_open[kind] = nullptr;
  } else {
    (void)hipEventDestroy(e);
  }
}

namespace {

__global__ void k_nonfinite_f32(const float* __restrict__ p, int64_t count, int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (bad) atomicOr(flag, 1);
}

bool finite_host(const double* p, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename F>
gv_status guarded(F f) {
  try {
    clear_error();
    return f();
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GV_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GV_EDEVICE;
  } catch (...) {
    set_error("unknown failure");
    return GV_EDEVICE;
  }
}

bool valid(const gv_index* x) { return x && x->magic == kIndexMagic; }

}  // namespace

bool valid_model(const gv_model* m) { return m && m->magic == kModelMagic; }

gv_status alloc_model(int C, int d, int D, gv_model** out) {
  gv_model* m = new gv_model();
  m->magic = kModelMagic;
  m->gen = next_handle_gen();
  m->C = C;
  m->d = d;
  m->D = D;
  m->mu = m->A = m->B = nullptr;
  m->fitted = false;
  m->iters = 0;
  if (hipGetDevice(&m->device) != hipSuccess) m->device = 0;
  hipError_t e1 = dev_malloc(&m->mu, sizeof(double) * C * D);
  hipError_t e2 = dev_malloc(&m->A, sizeof(double) * C * d * D);
  hipError_t e3 = dev_malloc(&m->B, sizeof(double) * C * d * D);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    gv_model_destroy(m);
    set_error("device allocation of the model failed");
    return GV_ENOMEM;
  }
  *out = m;
  return GV_OK;
}

namespace {
bool valid(const gv_model* m) { return valid_model(m); }
}  // namespace

gv_status check_finite_f32(const float* p, int64_t count, hipStream_t st, bool* finite) {
  int* flag = nullptr;
  GV_HIP(dev_malloc_async((void**)&flag, sizeof(int), st));
  GV_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  if (count > 0) {
    int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_nonfinite_f32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, flag);
    GV_HIP(hipGetLastError());
  }
  int h = 0;
  GV_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  GV_HIP(hipFreeAsync(flag, st));
  GV_HIP(hipStreamSynchronize(st));
  *finite = (h == 0);
  return GV_OK;
}

}  // namespace gv

using namespace gv;

extern "C" {

const char* gv_status_string(gv_status s) {
  switch (s) {
    case GV_OK: return "ok";
    case GV_EINVAL: return "invalid argument";
    case GV_ENOMEM: return "out of memory";
    case GV_EDEVICE: return "device error";
    case GV_ENOTFIT: return "invalid or missing handle";
    case GV_ENONFINITE: return "non-finite input";
    case GV_EUNSUPPORTED: return "unsupported";
    case GV_ENOCONV: return "eigensolver did not converge";
  }
  return "unknown status";
}

const char* gv_last_error(void) { return g_err.c_str(); }

gv_status gv_fit(const float* X_learn, int64_t n_learn, const float* Q_learn, int64_t m_learn, int32_t D, int32_t d,
                 int32_t C, uint64_t seed, const gv_fit_opts* opts, void* stream, gv_model** out) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(out != nullptr, "gv_fit: out is NULL");
    *out = nullptr;
    GV_REQUIRE(X_learn && Q_learn, "gv_fit: NULL input");
    GV_REQUIRE(D >= 1 && d >= 1 && d <= D, "gv_fit: need 1 <= d <= D");
    GV_REQUIRE(C >= 1 && C <= 255, "gv_fit: need 1 <= C <= 255");
    GV_REQUIRE(n_learn >= C && m_learn >= 1, "gv_fit: need n_learn >= C and m_learn >= 1");
    GV_REQUIRE(n_learn <= 0x7fffffffLL, "gv_fit: n_learn too large");
    if (opts && opts->init_centroids) {
      if (!finite_host(opts->init_centroids, (size_t)C * D)) return GV_ENONFINITE;
    }
    hipStream_t st = (hipStream_t)stream;
    bool f1 = false, f2 = false;
    GV_TRY(check_finite_f32(X_learn, n_learn * D, st, &f1));
    GV_TRY(check_finite_f32(Q_learn, m_learn * D, st, &f2));
    if (!f1 || !f2) {
      set_error("gv_fit: NaN or Inf in the learn data");
      return GV_ENONFINITE;
    }
    gv_model* m = nullptr;
    GV_TRY(alloc_model(C, d, D, &m));
    gv_status s = fit_impl(X_learn, n_learn, Q_learn, m_learn, D, d, C, seed, opts, st, m);
    if (s != GV_OK) {
      gv_model_destroy(m);
      return s;
    }
    *out = m;
    return GV_OK;
  });
}

gv_status gv_model_import(const double* mu, const double* A, const double* B, int32_t C, int32_t d, int32_t D,
                          gv_model** out) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(out != nullptr, "gv_model_import: out is NULL");
    *out = nullptr;
    GV_REQUIRE(mu && A && B, "gv_model_import: NULL input");
    GV_REQUIRE(D >= 1 && d >= 1 && d <= D && C >= 1 && C <= 255, "gv_model_import: bad shape");
    if (!finite_host(mu, (size_t)C * D) || !finite_host(A, (size_t)C * d * D) || !finite_host(B, (size_t)C * d * D))
      return GV_ENONFINITE;
    gv_model* m = nullptr;
    GV_TRY(alloc_model(C, d, D, &m));
    hipError_t e = hipMemcpy(m->mu, mu, sizeof(double) * C * D, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->A, A, sizeof(double) * C * d * D, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->B, B, sizeof(double) * C * d * D, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      gv_model_destroy(m);
      set_error(std::string("gv_model_import: ") + hipGetErrorString(e));
      return GV_EDEVICE;
    }
    *out = m;
    return GV_OK;
  });
}

gv_status gv_model_shape(const gv_model* m, int32_t* C, int32_t* d, int32_t* D) {
  if (!valid(m)) return GV_ENOTFIT;
  if (C) *C = m->C;
  if (d) *d = m->d;
  if (D) *D = m->D;
  return GV_OK;
}

gv_status gv_model_export(const gv_model* m, double* mu, double* A, double* B) {
  return guarded([&]() -> gv_status {
    if (!valid(m)) return GV_ENOTFIT;
    const size_t cdD = (size_t)m->C * m->d * m->D;
    if (mu) GV_HIP(hipMemcpy(mu, m->mu, sizeof(double) * m->C * m->D, hipMemcpyDeviceToHost));
    if (A) GV_HIP(hipMemcpy(A, m->A, sizeof(double) * cdD, hipMemcpyDeviceToHost));
    if (B) GV_HIP(hipMemcpy(B, m->B, sizeof(double) * cdD, hipMemcpyDeviceToHost));
    return GV_OK;
  });
}

gv_status gv_model_stats(const gv_model* m, double* KQ, double* KX, double* lam_Q, double* lam_c, int64_t* counts,
                         uint8_t* fallback, int32_t* iters) {
  if (!valid(m)) return GV_ENOTFIT;
  if (!m->fitted) return GV_EUNSUPPORTED;
  if (KQ) std::memcpy(KQ, m->KQ.data(), sizeof(double) * m->KQ.size());
  if (KX) std::memcpy(KX, m->KX.data(), sizeof(double) * m->KX.size());
  if (lam_Q) std::memcpy(lam_Q, m->lamQ.data(), sizeof(double) * m->lamQ.size());
  if (lam_c) std::memcpy(lam_c, m->lamc.data(), sizeof(double) * m->lamc.size());
  if (counts) std::memcpy(counts, m->counts.data(), sizeof(int64_t) * m->counts.size());
  if (fallback) std::memcpy(fallback, m->fallback.data(), m->fallback.size());
  if (iters) *iters = m->iters;
  return GV_OK;
}

void gv_model_destroy(gv_model* m) {
  if (!m || m->magic != kModelMagic) return;
  m->magic = 0;
  if (m->mu) (void)hipFree(m->mu);
  if (m->A) (void)hipFree(m->A);
  if (m->B) (void)hipFree(m->B);
  delete m;
}

gv_status gv_encode(const gv_model* model, const float* X, int64_t n, gv_format fmt, int32_t copy_X, void* stream,
                    gv_index** out) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(out != nullptr, "gv_encode: out is NULL");
    *out = nullptr;
    if (!valid(model)) return GV_ENOTFIT;
    GV_REQUIRE(X != nullptr, "gv_encode: X is NULL");
    GV_REQUIRE(n >= 1 && n <= 0x7fffffffLL, "gv_encode: need 1 <= n < 2^31");
    GV_REQUIRE(fmt >= GV_FP32 && fmt <= GV_FP8_E4M3, "gv_encode: unknown format");
    GV_REQUIRE(copy_X >= 0 && copy_X <= 2, "gv_encode: copy_X must be 0, 1 or 2");
    hipStream_t st = (hipStream_t)stream;
    bool fin = false;
    GV_TRY(check_finite_f32(X, n * model->D, st, &fin));
    if (!fin) {
      set_error("gv_encode: NaN or Inf in X");
      return GV_ENONFINITE;
    }
    int dev = 0;
    GV_HIP(hipGetDevice(&dev));
    gv_index* x = new gv_index();
    x->device = dev;
    x->magic = kIndexMagic;
    x->gen = next_handle_gen();
    x->C = model->C;
    x->d = model->d;
    x->dp = pad_dim(model->d);
    x->D = model->D;
    x->fmt = fmt;
    x->n = n;
    x->n_rows = n;
    x->tags = nullptr;
    x->offsets = nullptr;
    x->seg_end = nullptr;
    x->ids = nullptr;
    x->pos = nullptr;
    x->xlow = nullptr;
    x->scale = nullptr;
    x->X = nullptr;
    x->own_X = copy_X == 1;
    auto fail = [&](gv_status s) {
      gv_index_destroy(x);
      return s;
    };
    x->n_pad = 0;
    if (dev_malloc(&x->tags, n) != hipSuccess || dev_malloc(&x->offsets, sizeof(int64_t) * (x->C + 1)) != hipSuccess ||
        dev_malloc(&x->seg_end, sizeof(int64_t) * x->C) != hipSuccess ||
        dev_malloc(&x->scale, sizeof(float) * x->C) != hipSuccess) {
      set_error("gv_encode: device allocation failed");
      return fail(GV_ENOMEM);
    }
    if (x->own_X) {
      float* copy = nullptr;
      if (dev_malloc(&copy, sizeof(float) * n * x->D) != hipSuccess) {
        set_error("gv_encode: device allocation of the X copy failed");
        return fail(GV_ENOMEM);
      }
      x->X = copy;
      if (hipMemcpyAsync(copy, X, sizeof(float) * n * x->D, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(GV_EDEVICE);
    } else {
      x->X = copy_X == 0 ? X : nullptr;  // 2: no full-dimension vectors kept
    }
    gv_status s = encode_impl(model, X, n, fmt, st, x);
    if (s != GV_OK) return fail(s);
    *out = x;
    return GV_OK;
  });
}

gv_status gv_index_reproject(const gv_model* old_model, const gv_model* new_model, const gv_index* in,
                             const uint8_t* keep, const float* X_new, int64_t n_new, gv_format fmt, void* stream,
                             gv_index** out) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(out != nullptr, "gv_index_reproject: out is NULL");
    *out = nullptr;
    if (!valid(old_model) || !valid(new_model) || !valid(in)) return GV_ENOTFIT;
    const int C = new_model->C, D = new_model->D;
    GV_REQUIRE(old_model->C == C && old_model->D == D && in->C == C && in->D == D,
               "gv_index_reproject: models and index differ in C or D");
    GV_REQUIRE(old_model->d == D && new_model->d == D && in->d == D,
               "gv_index_reproject: the models and the index must keep all D coordinates (d = D)");
    GV_REQUIRE(fmt >= GV_FP32 && fmt <= GV_FP8_E4M3, "gv_index_reproject: unknown format");
    GV_REQUIRE(n_new >= 0 && (n_new == 0 || X_new != nullptr), "gv_index_reproject: NULL new vectors");
    GV_REQUIRE(in->n + n_new <= 0x7fffffffLL, "gv_index_reproject: id space beyond 2^31");
    int dev = 0;
    GV_HIP(hipGetDevice(&dev));
    GV_REQUIRE(in->device == dev, "gv_index_reproject: the index lives on another device");
    {  // the landmarks must be the same: kept vectors keep their clusters
      std::vector<double> mu0((size_t)C * D), mu1((size_t)C * D);
      GV_HIP(hipMemcpy(mu0.data(), old_model->mu, sizeof(double) * mu0.size(), hipMemcpyDeviceToHost));
      GV_HIP(hipMemcpy(mu1.data(), new_model->mu, sizeof(double) * mu1.size(), hipMemcpyDeviceToHost));
      GV_REQUIRE(std::memcmp(mu0.data(), mu1.data(), sizeof(double) * mu0.size()) == 0,
                 "gv_index_reproject: the models' landmarks differ (refit with the landmarks kept)");
    }
    hipStream_t st = (hipStream_t)stream;
    if (n_new > 0) {
      bool fin = false;
      GV_TRY(check_finite_f32(X_new, n_new * D, st, &fin));
      if (!fin) {
        set_error("gv_index_reproject: NaN or Inf in the new vectors");
        return GV_ENONFINITE;
      }
    }
    gv_index* x = new gv_index();
    x->device = dev;
    x->magic = kIndexMagic;
    x->gen = next_handle_gen();
    x->C = C;
    x->d = D;
    x->dp = pad_dim(D);
    x->D = D;
    x->fmt = fmt;
    x->n = in->n + n_new;
    x->n_rows = 0;
    x->tags = nullptr;
    x->offsets = nullptr;
    x->seg_end = nullptr;
    x->ids = nullptr;
    x->pos = nullptr;
    x->xlow = nullptr;
    x->scale = nullptr;
    x->X = nullptr;  // no full-dimension vectors: searches rerank from the stored ones
    x->own_X = false;
    x->n_pad = 0;
    auto fail = [&](gv_status s) {
      gv_index_destroy(x);
      return s;
    };
    if (dev_malloc(&x->tags, std::max<int64_t>(x->n, 1)) != hipSuccess ||
        dev_malloc(&x->offsets, sizeof(int64_t) * (C + 1)) != hipSuccess ||
        dev_malloc(&x->seg_end, sizeof(int64_t) * C) != hipSuccess ||
        dev_malloc(&x->scale, sizeof(float) * C) != hipSuccess) {
      set_error("gv_index_reproject: device allocation failed");
      return fail(GV_ENOMEM);
    }
    gv_status s = reproject_impl(old_model, new_model, in, keep, X_new, n_new, fmt, st, x);
    if (s != GV_OK) return fail(s);
    if (x->n_rows < 1) {
      set_error("gv_index_reproject: no vectors left");
      return fail(GV_EINVAL);
    }
    *out = x;
    return GV_OK;
  });
}

gv_status gv_index_rows(const gv_index* x, int64_t* rows) {
  if (!valid(x)) return GV_ENOTFIT;
  if (rows) *rows = x->n_rows;
  return GV_OK;
}

gv_status gv_index_shape(const gv_index* x, int64_t* n, int32_t* C, int32_t* d, int32_t* d_pad, int32_t* fmt) {
  if (!valid(x)) return GV_ENOTFIT;
  if (n) *n = x->n;
  if (C) *C = x->C;
  if (d) *d = x->d;
  if (d_pad) *d_pad = x->dp;
  if (fmt) *fmt = x->fmt;
  return GV_OK;
}

gv_status gv_index_export(const gv_index* x, uint8_t* tags, int64_t* offsets, int32_t* ids, void* xlow, float* scale) {
  return guarded([&]() -> gv_status {
    if (!valid(x)) return GV_ENOTFIT;
    // the device keeps padded segments and operand tiles; the export is dense and row-major
    std::vector<int64_t> roff(x->C + 1, 0);
    for (int c = 0; c < x->C; ++c) roff[c + 1] = roff[c] + x->h_counts[c];
    if (tags) GV_HIP(hipMemcpy(tags, x->tags, x->n, hipMemcpyDeviceToHost));
    if (offsets) std::memcpy(offsets, roff.data(), sizeof(int64_t) * (x->C + 1));
    if (ids) {
      std::vector<int32_t> pid(x->n_pad);
      GV_HIP(hipMemcpy(pid.data(), x->ids, sizeof(int32_t) * x->n_pad, hipMemcpyDeviceToHost));
      for (int c = 0; c < x->C; ++c)
        for (int64_t i = 0; i < x->h_counts[c]; ++i) ids[roff[c] + i] = pid[x->h_offsets[c] + i];
    }
    if (xlow) {
      const int eb = fmt_bytes(x->fmt), km = fmt_km(x->fmt), epl = fmt_epl(x->fmt);
      std::vector<uint8_t> tiles((size_t)x->n_pad * x->dp * eb);
      GV_HIP(hipMemcpy(tiles.data(), x->xlow, tiles.size(), hipMemcpyDeviceToHost));
      uint8_t* out = (uint8_t*)xlow;
      for (int c = 0; c < x->C; ++c)
        for (int64_t i = 0; i < x->h_counts[c]; ++i)
          for (int j = 0; j < x->dp; ++j)
            std::memcpy(out + ((roff[c] + i) * x->dp + j) * eb,
                        tiles.data() + tiled_offset(x->h_offsets[c] + i, j, x->dp, km, epl) * eb, eb);
    }
    if (scale) GV_HIP(hipMemcpy(scale, x->scale, sizeof(float) * x->C, hipMemcpyDeviceToHost));
    return GV_OK;
  });
}

void gv_index_destroy(gv_index* x) {
  if (!x || x->magic != kIndexMagic) return;
  x->magic = 0;
  if (x->tags) (void)hipFree(x->tags);
  if (x->offsets) (void)hipFree(x->offsets);
  if (x->seg_end) (void)hipFree(x->seg_end);
  if (x->ids) (void)hipFree(x->ids);
  if (x->pos) (void)hipFree(x->pos);
  if (x->xlow) (void)hipFree(x->xlow);
  if (x->scale) (void)hipFree(x->scale);
  if (x->own_X && x->X) (void)hipFree((void*)x->X);
  delete x;
}

}  // extern "C"

namespace gv {
gv_status check_search_args(const gv_index* idx, int64_t m, int32_t k, int32_t kappa) {
  GV_REQUIRE(m >= 0, "search: m < 0");
  GV_REQUIRE(kappa >= 1 && kappa <= kMaxKappa, "search: need 1 <= kappa <= 1024");
  GV_REQUIRE(k >= 1 && k <= kappa, "search: need 1 <= k <= kappa");
  GV_REQUIRE(kappa <= idx->n_rows, "search: need kappa <= stored vectors");
  return GV_OK;
}
}  // namespace gv

extern "C" {

gv_status gv_project(const gv_model* model, gv_format fmt, const float* Q, int64_t m, float* qc, float* t, void* qhat,
                     void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(model)) return GV_ENOTFIT;
    GV_REQUIRE(m >= 0, "gv_project: m < 0");
    GV_REQUIRE(fmt >= GV_FP32 && fmt <= GV_FP8_E4M3, "gv_project: unknown format");
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && t && qhat, "gv_project: NULL argument");
    return project_impl(model, fmt, Q, m, qc, t, qhat, (hipStream_t)stream);
  });
}

gv_status gv_tags(const gv_model* model, const float* X, int64_t n, uint8_t* tags, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(model)) return GV_ENOTFIT;
    GV_REQUIRE(n >= 0, "gv_tags: n < 0");
    if (n == 0) return GV_OK;
    GV_REQUIRE(X && tags, "gv_tags: NULL argument");
    return tags_impl(model, X, n, tags, (hipStream_t)stream);
  });
}

gv_status gv_moments(const float* V, int64_t n, int32_t D, const uint8_t* tags, int32_t C, double* K, void* stream) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(n >= 0 && D >= 1 && C >= 1 && C <= 256, "gv_moments: bad sizes");
    GV_REQUIRE(tags || C == 1 || n == 0, "gv_moments: C must be 1 without tags");
    GV_REQUIRE(K && (V || n == 0), "gv_moments: NULL argument");
    return moments_impl(V, n, D, tags, C, K, (hipStream_t)stream);
  });
}

gv_status gv_moments_update(const float* V, int64_t n, int32_t D, const uint8_t* tags, int32_t C, int32_t sign,
                            double* K, void* stream) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(n >= 0 && D >= 1 && C >= 1 && C <= 256, "gv_moments_update: bad sizes");
    GV_REQUIRE(sign == 1 || sign == -1, "gv_moments_update: sign must be +1 or -1");
    GV_REQUIRE(tags || C == 1 || n == 0, "gv_moments_update: C must be 1 without tags");
    GV_REQUIRE(K && (V || n == 0), "gv_moments_update: NULL argument");
    return moments_impl(V, n, D, tags, C, K, (hipStream_t)stream, sign);
  });
}

gv_status gv_fit_from_stats(const double* mu, const double* KQ, double m_q, const double* KX, const int64_t* counts,
                            int32_t C, int32_t d, int32_t D, void* stream, gv_model** out) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(out != nullptr, "gv_fit_from_stats: out is NULL");
    *out = nullptr;
    GV_REQUIRE(mu && KQ && KX && counts, "gv_fit_from_stats: NULL input");
    GV_REQUIRE(D >= 1 && d >= 1 && d <= D, "gv_fit_from_stats: need 1 <= d <= D");
    GV_REQUIRE(C >= 1 && C <= 255, "gv_fit_from_stats: need 1 <= C <= 255");
    GV_REQUIRE(m_q > 0.0 && std::isfinite(m_q), "gv_fit_from_stats: m_q must be positive and finite");
    if (!finite_host(mu, (size_t)C * D)) return GV_ENONFINITE;
    for (int c = 0; c < C; ++c) GV_REQUIRE(counts[c] >= 0, "gv_fit_from_stats: negative count");
    gv_model* m = nullptr;
    GV_TRY(alloc_model(C, d, D, &m));
    gv_status s = fit_from_stats_impl(mu, KQ, m_q, KX, counts, (hipStream_t)stream, m);
    if (s != GV_OK) {
      gv_model_destroy(m);
      return s;
    }
    *out = m;
    return GV_OK;
  });
}

gv_status gv_loss_grad(int32_t C, int32_t d, int32_t D, const float* A, const float* B, const double* KQ,
                       const double* KX, double n_pairs, double* loss, float* dA, float* dB, void* stream) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(C >= 1 && C <= 65535 && d >= 1 && d <= D && D >= 1, "gv_loss_grad: bad sizes (need 1 <= d <= D)");
    GV_REQUIRE(A && B && KQ && KX && loss, "gv_loss_grad: NULL argument");
    GV_REQUIRE(n_pairs > 0.0 && std::isfinite(n_pairs), "gv_loss_grad: n_pairs must be positive and finite");
    return loss_grad_impl(C, d, D, A, B, KQ, KX, n_pairs, loss, dA, dB, (hipStream_t)stream);
  });
}

gv_status gv_score_topk(const gv_index* index, const void* qhat, const float* t, int64_t m, int32_t kappa,
                        int32_t* cand_ids, float* cand_scores, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(index)) return GV_ENOTFIT;
    GV_TRY(check_search_args(index, m, 1, kappa));
    if (m == 0) return GV_OK;
    GV_REQUIRE(qhat && t && cand_ids && cand_scores, "gv_score_topk: NULL argument");
    return score_topk_impl(index, qhat, t, m, kappa, cand_ids, cand_scores, (hipStream_t)stream);
  });
}

gv_status gv_rerank(const gv_index* index, const float* Q, int64_t m, const int32_t* cand_ids, int32_t kappa, int32_t k,
                    int32_t* out_ids, float* out_scores, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(index)) return GV_ENOTFIT;
    GV_TRY(check_search_args(index, m, k, kappa));
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && cand_ids && out_ids, "gv_rerank: NULL argument");
    GV_REQUIRE(index->X != nullptr, "gv_rerank: the index keeps no full-dimension vectors (use gv_rerank_stored)");
    return rerank_impl(index, Q, m, cand_ids, kappa, k, out_ids, out_scores, (hipStream_t)stream);
  });
}

gv_status gv_search(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int32_t k, int32_t kappa,
                    int32_t* out_ids, float* out_scores, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(model) || !valid(index)) return GV_ENOTFIT;
    GV_REQUIRE(model->C == index->C && model->d == index->d && model->D == index->D,
               "gv_search: model and index shapes differ");
    GV_TRY(check_search_args(index, m, k, kappa));
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && out_ids, "gv_search: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    keep_pool(index->device);
    SearchPlan plan;
    GV_TRY(search_plan(model, index, m, kappa, &plan));
    void* ws = nullptr;
    GV_HIP(dev_malloc_async(&ws, plan.bytes, st));
    const gv_status s = search_run(model, index, Q, m, k, kappa, out_ids, out_scores, plan, ws, st);
    (void)hipFreeAsync(ws, st);
    return s;
  });
}

gv_status gv_search_lazy(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int32_t k,
                         int32_t kappa, int32_t* out_ids, float* out_scores, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(model) || !valid(index)) return GV_ENOTFIT;
    GV_REQUIRE(model->C == index->C && model->d == index->d && model->D == index->D,
               "gv_search_lazy: model and index shapes differ");
    GV_TRY(check_search_args(index, m, k, kappa));
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && out_ids, "gv_search_lazy: NULL argument");
    return search_lazy_impl(model, index, Q, m, k, kappa, out_ids, out_scores, (hipStream_t)stream);
  });
}

// ---------------------------------------------------------------------------- Euclidean adaptation
gv_status gv_augment(const float* V, int64_t n, int32_t D, int32_t kind, float* out, void* stream) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(n >= 0 && D >= 1, "gv_augment: need n >= 0 and D >= 1");
    GV_REQUIRE(kind == GV_AUG_DATABASE || kind == GV_AUG_QUERY, "gv_augment: unknown kind");
    if (n == 0) return GV_OK;
    GV_REQUIRE(V && out, "gv_augment: NULL argument");
    GV_REQUIRE((const void*)V != (const void*)out, "gv_augment: out must not alias V");
    return augment_impl(V, n, D, kind == GV_AUG_DATABASE, out, (hipStream_t)stream);
  });
}

// ---------------------------------------------------------------------------- flexible d (Section 3.3)
static gv_status check_d_search(const gv_model* model, int32_t d_search) {
  GV_REQUIRE(d_search >= 1 && d_search <= model->d, "d_search must lie in [1, d]");
  GV_REQUIRE(pad_dim(d_search) <= 256, "the scan reads at most 256 leading coordinates (padded)");
  return GV_OK;
}

gv_status gv_project_flex(const gv_model* model, gv_format fmt, const float* Q, int64_t m, int32_t d_search, float* qc,
                          float* t, void* qhat, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(model)) return GV_ENOTFIT;
    GV_REQUIRE(m >= 0, "gv_project_flex: m < 0");
    GV_REQUIRE(fmt >= GV_FP32 && fmt <= GV_FP8_E4M3, "gv_project_flex: unknown format");
    GV_TRY(check_d_search(model, d_search));
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && t && qhat, "gv_project_flex: NULL argument");
    return project_impl(model, fmt, Q, m, qc, t, qhat, (hipStream_t)stream, d_search);
  });
}

gv_status gv_score_topk_flex(const gv_index* index, const void* qhat, const float* t, int64_t m, int32_t d_search,
                             int32_t kappa, int32_t* cand_ids, float* cand_scores, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(index)) return GV_ENOTFIT;
    GV_TRY(check_search_args(index, m, 1, kappa));
    GV_REQUIRE(d_search >= 1 && d_search <= index->d, "gv_score_topk_flex: d_search must lie in [1, d]");
    if (m == 0) return GV_OK;
    GV_REQUIRE(qhat && t && cand_ids && cand_scores, "gv_score_topk_flex: NULL argument");
    return score_topk_impl(index, qhat, t, m, kappa, cand_ids, cand_scores, (hipStream_t)stream, d_search);
  });
}

gv_status gv_rerank_stored(const gv_index* index, const float* qc, int64_t m, const int32_t* cand_ids, int32_t kappa,
                           int32_t k, int32_t* out_ids, float* out_scores, void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(index)) return GV_ENOTFIT;
    GV_TRY(check_search_args(index, m, k, kappa));
    if (m == 0) return GV_OK;
    GV_REQUIRE(qc && cand_ids && out_ids, "gv_rerank_stored: NULL argument");
    return rerank_stored_impl(index, qc, m, cand_ids, kappa, k, out_ids, out_scores, (hipStream_t)stream);
  });
}

gv_status gv_search_flex(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int32_t k,
                         int32_t kappa, int32_t d_search, int32_t rerank, int32_t* out_ids, float* out_scores,
                         void* stream) {
  return guarded([&]() -> gv_status {
    if (!valid(model) || !valid(index)) return GV_ENOTFIT;
    GV_REQUIRE(model->C == index->C && model->d == index->d && model->D == index->D,
               "gv_search_flex: model and index shapes differ");
    GV_TRY(check_search_args(index, m, k, kappa));
    GV_TRY(check_d_search(model, d_search));
    GV_REQUIRE(rerank == GV_RERANK_FULL || rerank == GV_RERANK_STORED, "gv_search_flex: unknown rerank source");
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && out_ids, "gv_search_flex: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    keep_pool(index->device);
    SearchPlan plan;
    GV_TRY(search_plan(model, index, m, kappa, &plan, d_search, rerank == GV_RERANK_STORED));
    void* ws = nullptr;
    GV_HIP(dev_malloc_async(&ws, plan.bytes, st));
    const gv_status s = search_run(model, index, Q, m, k, kappa, out_ids, out_scores, plan, ws, st);
    (void)hipFreeAsync(ws, st);
    return s;
  });
}

// ---------------------------------------------------------------------------- batched search
namespace {

// One captured batch: the graph of every collection's search, its workspace,
// and the arguments it was captured with (a replay needs the same ones).
struct BatchGraph {
  std::vector<uintptr_t> key;
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  int device = -1;
};
std::mutex g_batch_mu;
BatchGraph g_batch;
int64_t g_batch_captures = 0, g_batch_replays = 0;
constexpr int kBatchStreams = 4;
hipStream_t g_side[64][kBatchStreams] = {};
hipStream_t g_origin[64] = {};  // captures start here (the caller's stream may be the legacy default stream)
hipEvent_t g_fork[64] = {}, g_join[64][kBatchStreams] = {};
void release_batch(BatchGraph& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(b.ws);
  }
  b = BatchGraph{};
}

gv_status side_streams(int dev) {
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range");
    return GV_EDEVICE;
  }
  if (g_fork[dev]) return GV_OK;
  for (int j = 0; j < kBatchStreams; ++j) {
    GV_HIP(hipStreamCreateWithFlags(&g_side[dev][j], hipStreamNonBlocking));
    GV_HIP(hipEventCreateWithFlags(&g_join[dev][j], hipEventDisableTiming));
  }
  GV_HIP(hipStreamCreateWithFlags(&g_origin[dev], hipStreamNonBlocking));
  GV_HIP(hipEventCreateWithFlags(&g_fork[dev], hipEventDisableTiming));
  return GV_OK;
}

}  // namespace

gv_status gv_search_batched(int32_t n_coll, const gv_model* const* models, const gv_index* const* indexes,
                            const float* const* Q, const int64_t* m, int32_t k, int32_t kappa,
                            int32_t* const* out_ids, float* const* out_scores, void* stream) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(n_coll >= 0, "gv_search_batched: n_coll < 0");
    if (n_coll == 0) return GV_OK;
    GV_REQUIRE(models && indexes && Q && m && out_ids, "gv_search_batched: NULL argument");
    int dev = 0;
    GV_HIP(hipGetDevice(&dev));
    std::vector<BatchEntry> ent;
    // every search keeps a workspace of its own: its lists live from its
    // cascade levels, through the shared full-scan launches, to its final select
    std::vector<uintptr_t> key{(uintptr_t)n_coll, (uintptr_t)k, (uintptr_t)kappa, (uintptr_t)stream, (uintptr_t)dev,
                               (uintptr_t)tuned_splits(), (uintptr_t)tuned_qpw(), (uintptr_t)tuned_cap(), (uintptr_t)tuned_optimism(),
                               (uintptr_t)tuning_table_version()};
    size_t ws_bytes = 0;
    for (int i = 0; i < n_coll; ++i) {
      const gv_model* md = models[i];
      const gv_index* ix = indexes[i];
      if (!valid(md) || !valid(ix)) return GV_ENOTFIT;
      GV_REQUIRE(md->C == ix->C && md->d == ix->d && md->D == ix->D, "gv_search_batched: model and index shapes differ");
      GV_REQUIRE(ix->device == dev, "gv_search_batched: index on another device");
      GV_TRY(check_search_args(ix, m[i], k, kappa));
      GV_REQUIRE(m[i] == 0 || (Q[i] && out_ids[i]), "gv_search_batched: NULL query or output");
      if (m[i] > 0) {
        BatchEntry b{md, ix, Q[i], m[i], out_ids[i], out_scores ? out_scores[i] : nullptr, SearchPlan{}, nullptr};
        GV_TRY(search_plan(md, ix, m[i], kappa, &b.plan, 0, false, kListBudget));
        b.ws = (uint8_t*)(uintptr_t)ws_bytes;  // offset until the workspace exists
        ws_bytes += (b.plan.bytes + 255) / 256 * 256;
        ent.push_back(b);
      }
      // handles enter the key by generation: a handle freed and another created at
      // the same address must not replay a graph that holds the old one's buffers
      for (uintptr_t v : {(uintptr_t)md->gen, (uintptr_t)ix->gen, (uintptr_t)Q[i], (uintptr_t)m[i],
                          (uintptr_t)out_ids[i], (uintptr_t)(out_scores ? out_scores[i] : nullptr)})
        key.push_back(v);
    }
    if (ent.empty()) return GV_OK;
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (g_batch.exec && g_batch.key == key) {  // same batch as last time: replay
      GV_HIP(hipGraphLaunch(g_batch.exec, st));
      ++g_batch_replays;
      return GV_OK;
    }
    release_batch(g_batch);
    GV_TRY(side_streams(dev));
    int n_cu = 0;
    GV_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t qbytes = batched_queue_bytes((int)ent.size());
    void* ws = nullptr;
    GV_HIP(dev_malloc(&ws, ws_bytes + qbytes));
    for (BatchEntry& b : ent) b.ws = (uint8_t*)ws + (uintptr_t)b.ws;
    uint8_t* qmem = (uint8_t*)ws + ws_bytes;
    // capture: projections and cascades as branches, the full scans of all
    // searches as persistent queue launches, the selects and reranks as branches
    gv_status s = GV_OK;
    hipGraph_t graph = nullptr;
    hipStream_t org = g_origin[dev];
    if (hipStreamBeginCapture(org, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipFree(ws);
      set_error("gv_search_batched: stream capture failed to start");
      return GV_EDEVICE;
    }
    g_capturing = true;
    std::vector<uint8_t> upload;
    s = batched_run(ent, k, kappa, org, g_side[dev], kBatchStreams, g_fork[dev], g_join[dev], qmem, qbytes, n_cu,
                    &upload);
    g_capturing = false;
    const hipError_t ec = hipStreamEndCapture(org, &graph);
    if (s == GV_OK && ec != hipSuccess) {
      set_error(std::string("gv_search_batched: capture failed: ") + hipGetErrorString(ec));
      s = GV_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    if (s == GV_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      set_error("gv_search_batched: graph instantiation failed");
      s = GV_EDEVICE;
    }
    // the queue launches' arguments and piece offsets: written once, read by every replay
    if (s == GV_OK && !upload.empty() && hipMemcpy(qmem, upload.data(), upload.size(), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("gv_search_batched: upload of the queue arguments failed");
      s = GV_EDEVICE;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (s != GV_OK) {
      if (exec) (void)hipGraphExecDestroy(exec);
      (void)hipFree(ws);
      return s;
    }
    g_batch.key = std::move(key);
    g_batch.exec = exec;
    g_batch.ws = ws;
    g_batch.device = dev;
    ++g_batch_captures;
    GV_HIP(hipGraphLaunch(exec, st));
    return GV_OK;
  });
}

void gv_batch_release(void) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  release_batch(g_batch);
}

void gv_batch_counts(int64_t* captures, int64_t* replays) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (captures) *captures = g_batch_captures;
  if (replays) *replays = g_batch_replays;
}

gv_status gv_scan_plan(int64_t n, int64_t n_pad, int32_t C, gv_format fmt, int32_t d, int32_t d_search, int64_t m,
                       int32_t kappa, gv_scan_level* levels, int32_t max_levels, int32_t* n_levels, int64_t* list_keys,
                       int64_t* scratch_bytes) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(n >= 1 && C >= 1 && C <= 255 && n_pad >= n && n_pad <= n + 31LL * C && n_pad % 32 == 0,
               "gv_scan_plan: need n >= 1, 1 <= C <= 255, n <= n_pad <= n + 31 C, n_pad a multiple of 32");
    GV_REQUIRE(fmt >= GV_FP32 && fmt <= GV_FP8_E4M3, "gv_scan_plan: unknown format");
    GV_REQUIRE(d >= 1 && d_search >= 0 && d_search <= d, "gv_scan_plan: need d >= 1 and 0 <= d_search <= d");
    GV_REQUIRE(m >= 1 && kappa >= 1 && kappa <= kMaxKappa && kappa <= n, "gv_scan_plan: need m >= 1, 1 <= kappa <= min(n, 1024)");
    GV_REQUIRE(max_levels >= 0, "gv_scan_plan: max_levels < 0");
    int nl = 0;
    GV_TRY(scan_plan_describe(n, n_pad, C, fmt, d, d_search, m, kappa, levels, max_levels, &nl, list_keys,
                              scratch_bytes));
    if (n_levels) *n_levels = nl;
    return GV_OK;
  });
}

gv_status gv_debug_fail_alloc(int32_t after) {
  clear_error();
  if (after < -1) {
    set_error("gv_debug_fail_alloc: after must be -1 or non-negative");
    return GV_EINVAL;
  }
  g_fail_alloc = after;
  return GV_OK;
}

int32_t gv_debug_allocs_pending(void) { return (int32_t)std::max(-1L, g_fail_alloc.load()); }

gv_status gv_search_optimism(int32_t rank) {
  clear_error();
  if (rank < -1) {
    set_error("gv_search_optimism: rank must be -1, 0 or positive");
    return GV_EINVAL;
  }
  g_optimism = rank;
  return GV_OK;
}

gv_status gv_search_tuning(int32_t splits, int32_t qpw, int32_t cap) {
  if (splits < 0 || splits > 4096) return GV_EINVAL;
  if (qpw != 0 && qpw != 32 && qpw != 64 && qpw != 128) return GV_EINVAL;
  if (cap != 0 && (cap < 64 || cap > 2048)) return GV_EINVAL;
  g_splits = splits;
  g_qpw = qpw;
  g_cap = cap;
  return GV_OK;
}

int32_t gv_padded_dim(int32_t d) { return d >= 1 ? pad_dim(d) : 0; }

gv_status gv_profile_enable(int32_t on) {
  g_prof_on = on != 0;
  return GV_OK;
}

gv_status gv_profile_read(double* ms_score, int64_t* n_score, double* ms_merge, int64_t* n_merge) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms[2] = {0.0, 0.0};
  int64_t cnt[2] = {0, 0};
  gv_status st = GV_OK;
  for (auto& r : g_prof) {
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) st = GV_EDEVICE;
    ms[r.kind] += t;
    cnt[r.kind] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  if (ms_score) *ms_score = ms[0];
  if (n_score) *n_score = cnt[0];
  if (ms_merge) *ms_merge = ms[1];
  if (n_merge) *n_merge = cnt[1];
  return st;
}

gv_status gv_host_eigh(int32_t n, const double* A, double* lam, double* Vt) {
  return guarded([&]() -> gv_status {
    GV_REQUIRE(n >= 1 && A && lam && Vt, "gv_host_eigh: bad arguments");
    std::vector<double> a(A, A + (size_t)n * n), l, v;
    const bool ok = eigh_desc(n, a, l, v);
    std::memcpy(lam, l.data(), sizeof(double) * n);
    std::memcpy(Vt, v.data(), sizeof(double) * (size_t)n * n);
    if (!ok) {
      set_error("gv_host_eigh: the QR steps did not converge within the step budget");
      return GV_ENOCONV;
    }
    return GV_OK;
  });
}

gv_status gv_eig_step_limit(int32_t max_steps) {
  if (max_steps < 0) return GV_EINVAL;
  set_eig_step_limit(max_steps);
  return GV_OK;
}

}  // extern "C"
