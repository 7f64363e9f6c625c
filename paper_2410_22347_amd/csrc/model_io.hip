// Model files: everything a fit produces -- landmarks, projections and, for
// fitted models, the FP64 statistics and the sphering factors they came from --
// written as one little-endian binary file and read back into a new handle.
//
// Layout (all integers and reals little-endian, no padding):
//   char     magic[8] = "GLEANVEC"
//   uint32   version  = 1
//   uint32   flags    (bit 0: statistics present)
//   int32    C, d, D, iters
//   float64  mu[C*D], A[C*d*D], B[C*d*D]
//   if statistics:
//     float64  KQ[D*D] (mean of q q^T), KX[C*D*D] (per-cluster sums),
//              lam_Q[D], lam_c[C*D], W[D*D], W+[D*D], P[C*d*D]
//     int64    counts[C]
//     uint8    fallback[C]
//   uint64   FNV-1a (64-bit) of every preceding byte
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

namespace gv {
namespace {

constexpr char kFileMagic[8] = {'G', 'L', 'E', 'A', 'N', 'V', 'E', 'C'};
constexpr uint32_t kFileVersion = 1;
constexpr uint32_t kHasStats = 1;

uint64_t fnv1a(const uint8_t* p, size_t n) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

struct Header {
  uint32_t version, flags;
  int32_t C, d, D, iters;
};

// bytes of the file for a header (checksum included)
size_t file_bytes(const Header& h) {
  const size_t C = h.C, d = h.d, D = h.D;
  size_t n = 8 + 4 * 2 + 4 * 4;
  n += 8 * (C * D + 2 * C * d * D);
  if (h.flags & kHasStats) n += 8 * (D * D + C * D * D + D + C * D + 2 * D * D + C * d * D) + 8 * C + C;
  return n + 8;
}

struct Writer {
  std::vector<uint8_t> buf;
  template <typename T>
  void put(const T* p, size_t count) {
    const uint8_t* b = (const uint8_t*)p;
    buf.insert(buf.end(), b, b + sizeof(T) * count);
  }
  template <typename T>
  void one(T v) { put(&v, 1); }
};

struct Reader {
  const uint8_t* p;
  size_t n, at = 0;
  template <typename T>
  void get(T* dst, size_t count) {
    std::memcpy(dst, p + at, sizeof(T) * count);
    at += sizeof(T) * count;
  }
  template <typename T>
  T one() {
    T v;
    get(&v, 1);
    return v;
  }
};

gv_status read_file(const char* path, std::vector<uint8_t>* out) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    set_error(std::string("model file: cannot open ") + path);
    return GV_EINVAL;
  }
  std::fseek(f, 0, SEEK_END);
  const long len = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  if (len < 0) {
    std::fclose(f);
    set_error("model file: cannot size the file");
    return GV_EINVAL;
  }
  out->resize((size_t)len);
  const size_t got = len > 0 ? std::fread(out->data(), 1, (size_t)len, f) : 0;
  std::fclose(f);
  if (got != (size_t)len) {
    set_error("model file: short read");
    return GV_EINVAL;
  }
  return GV_OK;
}

// checks magic, version, shape, size and checksum; fills the header
gv_status parse_header(const std::vector<uint8_t>& b, Header* h) {
  if (b.size() < 8 + 24 + 8 || std::memcmp(b.data(), kFileMagic, 8) != 0) {
    set_error("model file: not a model file (magic)");
    return GV_EINVAL;
  }
  Reader r{b.data(), b.size(), 8};
  h->version = r.one<uint32_t>();
  h->flags = r.one<uint32_t>();
  h->C = r.one<int32_t>();
  h->d = r.one<int32_t>();
  h->D = r.one<int32_t>();
  h->iters = r.one<int32_t>();
  if (h->version != kFileVersion) {
    set_error("model file: unsupported version " + std::to_string(h->version));
    return GV_EUNSUPPORTED;
  }
  if ((h->flags & ~kHasStats) != 0 || h->C < 1 || h->C > 255 || h->D < 1 || h->D > (1 << 16) || h->d < 1 ||
      h->d > h->D) {
    set_error("model file: invalid header");
    return GV_EINVAL;
  }
  if (file_bytes(*h) != b.size()) {
    set_error("model file: size does not match the header (truncated or corrupt)");
    return GV_EINVAL;
  }
  uint64_t sum;
  std::memcpy(&sum, b.data() + b.size() - 8, 8);
  if (sum != fnv1a(b.data(), b.size() - 8)) {
    set_error("model file: checksum mismatch (corrupt file)");
    return GV_EINVAL;
  }
  return GV_OK;
}

template <typename F>
gv_status guarded_io(F f) {
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

}  // namespace
}  // namespace gv

using namespace gv;

extern "C" {

gv_status gv_model_save(const gv_model* m, const char* path) {
  return guarded_io([&]() -> gv_status {
    if (!valid_model(m)) return GV_ENOTFIT;
    GV_REQUIRE(path != nullptr, "gv_model_save: path is NULL");
    const size_t C = m->C, d = m->d, D = m->D, DD = D * D;
    const bool stats = m->fitted;
    Header h{kFileVersion, stats ? kHasStats : 0u, m->C, m->d, m->D, m->iters};
    Writer w;
    w.buf.reserve(file_bytes(h));
    w.put(kFileMagic, 8);
    w.one(h.version);
    w.one(h.flags);
    w.one(h.C);
    w.one(h.d);
    w.one(h.D);
    w.one(h.iters);
    std::vector<double> mu(C * D), A(C * d * D), B(C * d * D);
    GV_HIP(hipMemcpy(mu.data(), m->mu, sizeof(double) * mu.size(), hipMemcpyDeviceToHost));
    GV_HIP(hipMemcpy(A.data(), m->A, sizeof(double) * A.size(), hipMemcpyDeviceToHost));
    GV_HIP(hipMemcpy(B.data(), m->B, sizeof(double) * B.size(), hipMemcpyDeviceToHost));
    w.put(mu.data(), mu.size());
    w.put(A.data(), A.size());
    w.put(B.data(), B.size());
    if (stats) {
      if (m->KQ.size() != DD || m->KX.size() != C * DD || m->lamQ.size() != D || m->lamc.size() != C * D ||
          m->W.size() != DD || m->Wp.size() != DD || m->P.size() != C * d * D || m->counts.size() != C ||
          m->fallback.size() != C) {
        set_error("gv_model_save: the model's statistics are incomplete");
        return GV_EDEVICE;
      }
      w.put(m->KQ.data(), DD);
      w.put(m->KX.data(), C * DD);
      w.put(m->lamQ.data(), D);
      w.put(m->lamc.data(), C * D);
      w.put(m->W.data(), DD);
      w.put(m->Wp.data(), DD);
      w.put(m->P.data(), C * d * D);
      w.put(m->counts.data(), C);
      w.put(m->fallback.data(), C);
    }
    w.one(fnv1a(w.buf.data(), w.buf.size()));
    FILE* f = std::fopen(path, "wb");
    if (!f) {
      set_error(std::string("gv_model_save: cannot open ") + path);
      return GV_EINVAL;
    }
    const size_t put = std::fwrite(w.buf.data(), 1, w.buf.size(), f);
    const int closed = std::fclose(f);
    if (put != w.buf.size() || closed != 0) {
      set_error("gv_model_save: write failed");
      return GV_EDEVICE;
    }
    return GV_OK;
  });
}

gv_status gv_model_file_info(const char* path, int32_t* C, int32_t* d, int32_t* D, int32_t* has_stats) {
  return guarded_io([&]() -> gv_status {
    GV_REQUIRE(path != nullptr, "gv_model_file_info: path is NULL");
    std::vector<uint8_t> b;
    GV_TRY(read_file(path, &b));
    Header h;
    GV_TRY(parse_header(b, &h));
    if (C) *C = h.C;
    if (d) *d = h.d;
    if (D) *D = h.D;
    if (has_stats) *has_stats = (h.flags & kHasStats) ? 1 : 0;
    return GV_OK;
  });
}

gv_status gv_model_load(const char* path, gv_model** out) {
  return guarded_io([&]() -> gv_status {
    GV_REQUIRE(out != nullptr, "gv_model_load: out is NULL");
    *out = nullptr;
    GV_REQUIRE(path != nullptr, "gv_model_load: path is NULL");
    std::vector<uint8_t> b;
    GV_TRY(read_file(path, &b));
    Header h;
    GV_TRY(parse_header(b, &h));
    const size_t C = h.C, d = h.d, D = h.D, DD = D * D;
    Reader r{b.data(), b.size(), 8 + 24};
    std::vector<double> mu(C * D), A(C * d * D), B(C * d * D);
    r.get(mu.data(), mu.size());
    r.get(A.data(), A.size());
    r.get(B.data(), B.size());
    gv_model* m = nullptr;
    GV_TRY(alloc_model(h.C, h.d, h.D, &m));
    auto fail = [&](gv_status s) {
      gv_model_destroy(m);
      return s;
    };
    hipError_t e = hipMemcpy(m->mu, mu.data(), sizeof(double) * mu.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->A, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->B, B.data(), sizeof(double) * B.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_error(std::string("gv_model_load: ") + hipGetErrorString(e));
      return fail(GV_EDEVICE);
    }
    m->iters = h.iters;
    if (h.flags & kHasStats) {
      m->KQ.resize(DD);
      m->KX.resize(C * DD);
      m->lamQ.resize(D);
      m->lamc.resize(C * D);
      m->W.resize(DD);
      m->Wp.resize(DD);
      m->P.resize(C * d * D);
      m->counts.resize(C);
      m->fallback.resize(C);
      r.get(m->KQ.data(), DD);
      r.get(m->KX.data(), C * DD);
      r.get(m->lamQ.data(), D);
      r.get(m->lamc.data(), C * D);
      r.get(m->W.data(), DD);
      r.get(m->Wp.data(), DD);
      r.get(m->P.data(), C * d * D);
      r.get(m->counts.data(), C);
      r.get(m->fallback.data(), C);
      m->fitted = true;
    }
    *out = m;
    return GV_OK;
  });
}

gv_status gv_model_sphering(const gv_model* m, double* W, double* Wp, double* P) {
  if (!valid_model(m)) return GV_ENOTFIT;
  if (!m->fitted || m->W.empty()) return GV_EUNSUPPORTED;
  if (W) std::memcpy(W, m->W.data(), sizeof(double) * m->W.size());
  if (Wp) std::memcpy(Wp, m->Wp.data(), sizeof(double) * m->Wp.size());
  if (P) std::memcpy(P, m->P.data(), sizeof(double) * m->P.size());
  return GV_OK;
}

}  // extern "C"
