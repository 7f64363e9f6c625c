// Autotuner of the scan's launch shape.  The scan's results do not depend on
// its launch shape (row ranges per query block, queries per wavefront, list
// capacity), only its speed does.  The tuner times a small set of candidate
// shapes on a caller's index and queries and keeps the fastest per shape
// class -- (storage format, padded reduced length, batch class, size class) --
// in a process-wide table that every later search of that class uses, unless
// the thread sets explicit overrides (gv_search_tuning).  The table can be
// written to and read from a text file.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace gv {
namespace {

// batch classes: 1, 2..32, 33..64, 65..256, 257..1024, 1025..4096, larger
int m_class(int64_t m) {
  if (m <= 1) return 0;
  if (m <= 32) return 1;
  if (m <= 64) return 2;
  if (m <= 256) return 3;
  if (m <= 1024) return 4;
  if (m <= 4096) return 5;
  return 6;
}
// size classes: floor(log2(stored rows))
int n_class(int64_t n) {
  int c = 0;
  while (n > 1) {
    n >>= 1;
    ++c;
  }
  return c;
}

using Key = std::tuple<int, int, int, int>;  // fmt, d_pad, batch class, size class
struct Entry {
  Tuning t;
  double ms;
};
std::mutex g_mu;
std::map<Key, Entry> g_table;
uint64_t g_version = 0;
thread_local bool g_bypass = false;  // set while the tuner times its candidates

}  // namespace

bool tuning_table_lookup(int fmt, int dp, int64_t m, int64_t n_rows, Tuning* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(Key{fmt, dp, m_class(m), n_class(n_rows)});
  if (it == g_table.end()) return false;
  *t = it->second.t;
  return true;
}

void tuning_table_store(int fmt, int dp, int64_t m, int64_t n_rows, const Tuning& t, double ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[Key{fmt, dp, m_class(m), n_class(n_rows)}] = Entry{t, ms};
  ++g_version;
}

uint64_t tuning_table_version() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_version;
}

Tuning effective_tuning(int fmt, int dp, int64_t m, int64_t n_rows) {
  Tuning t;
  t.splits = tuned_splits();
  t.qpw = tuned_qpw();
  t.cap = tuned_cap();
  if (t.splits || t.qpw || t.cap || g_bypass) return t;  // the thread's explicit overrides
  Tuning tab;
  if (tuning_table_lookup(fmt, dp, m, n_rows, &tab)) return tab;
  return t;
}

}  // namespace gv

using namespace gv;

extern "C" {

gv_status gv_autotune(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int32_t k,
                      int32_t kappa, int32_t reps, gv_tune_result* out, void* stream) {
  try {
    clear_error();
    if (!valid_model(model) || !index || index->magic != kIndexMagic) return GV_ENOTFIT;
    GV_REQUIRE(model->C == index->C && model->d == index->d && model->D == index->D,
               "gv_autotune: model and index shapes differ");
    GV_TRY(check_search_args(index, m, k, kappa));
    GV_REQUIRE(m >= 1 && Q != nullptr, "gv_autotune: need m >= 1 queries");
    GV_REQUIRE(reps >= 1 && reps <= 1000, "gv_autotune: need 1 <= reps <= 1000");
    GV_REQUIRE(index->X != nullptr, "gv_autotune: the index must keep X (the tuned search reranks from it)");
    hipStream_t st = (hipStream_t)stream;
    // candidates: the automatic shape, and row ranges, queries per wavefront
    // and list capacities around it
    std::vector<Tuning> cand;
    cand.push_back(Tuning{});
    for (int qpw : {32, 64, 128})
      for (int splits : {0, 16, 64, 256, 1024}) cand.push_back(Tuning{splits, qpw, 0});
    for (int cap : {768, 1024}) cand.push_back(Tuning{0, 0, cap});
    const int s0 = tuned_splits(), q0 = tuned_qpw(), c0 = tuned_cap();
    TempBuf<int32_t> ibuf(st);
    TempBuf<float> sbuf(st);
    GV_HIP(ibuf.alloc(sizeof(int32_t) * m * k));
    GV_HIP(sbuf.alloc(sizeof(float) * m * k));
    int32_t* ids = ibuf.p;
    float* sc = sbuf.p;
    hipEvent_t e0, e1;
    GV_HIP(hipEventCreate(&e0));
    GV_HIP(hipEventCreate(&e1));
    double best = INFINITY, base_ms = INFINITY;
    Tuning best_t{};
    int tried = 0;
    gv_status s = GV_OK;
    g_bypass = true;  // candidates run with exactly their own overrides, not the table's
    for (const Tuning& t : cand) {
      // a candidate that cannot hold the lists (kappa too large for its shapes) is skipped
      set_tuning(t.splits, t.qpw, t.cap);
      SearchPlan plan;
      if (search_plan(model, index, m, kappa, &plan) != GV_OK) continue;
      void* ws = nullptr;
      if (dev_malloc(&ws, plan.bytes) != hipSuccess) continue;
      gv_status r = search_run(model, index, Q, m, k, kappa, ids, sc, plan, ws, st);  // warm-up
      if (r == GV_OK && hipEventRecord(e0, st) == hipSuccess) {
        for (int i = 0; i < reps && r == GV_OK; ++i) r = search_run(model, index, Q, m, k, kappa, ids, sc, plan, ws, st);
        if (r == GV_OK && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
          float ms = 0.0f;
          if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
            const double per = ms / reps;
            ++tried;
            if (tried == 1) base_ms = per;
            if (per < best) {
              best = per;
              best_t = t;
            }
          }
        }
      }
      (void)hipStreamSynchronize(st);
      (void)hipFree(ws);
      if (r != GV_OK && r != GV_EUNSUPPORTED && r != GV_EINVAL) {
        s = r;
        break;
      }
    }
    g_bypass = false;
    set_tuning(s0, q0, c0);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    GV_TRY(s);
    if (tried == 0) {
      set_error("gv_autotune: no candidate launch shape could run this search");
      return GV_EUNSUPPORTED;
    }
    const int dp = pad_dim(index->d);
    tuning_table_store(index->fmt, dp, m, index->n_rows, best_t, best);
    if (out) {
      out->splits = best_t.splits;
      out->qpw = best_t.qpw;
      out->cap = best_t.cap;
      out->ms = best;
      out->ms_automatic = base_ms;
      out->candidates = tried;
    }
    return GV_OK;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GV_EDEVICE;
  } catch (...) {
    set_error("unknown failure");
    return GV_EDEVICE;
  }
}

gv_status gv_tuning_table_save(const char* path) {
  if (!path) return GV_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) {
    set_error(std::string("gv_tuning_table_save: cannot open ") + path);
    return GV_EINVAL;
  }
  std::fprintf(f, "# fmt d_pad batch_class size_class splits qpw cap ms\n");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_table)
      std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", std::get<0>(kv.first), std::get<1>(kv.first),
                   std::get<2>(kv.first), std::get<3>(kv.first), kv.second.t.splits, kv.second.t.qpw,
                   kv.second.t.cap, kv.second.ms);
  }
  return std::fclose(f) == 0 ? GV_OK : GV_EDEVICE;
}

gv_status gv_tuning_table_load(const char* path) {
  if (!path) return GV_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) {
    set_error(std::string("gv_tuning_table_load: cannot open ") + path);
    return GV_EINVAL;
  }
  std::map<Key, Entry> tab;
  char line[256];
  gv_status s = GV_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int fmt, dp, mc, nc, sp, qpw, cap;
    double ms;
    if (std::sscanf(line, "%d %d %d %d %d %d %d %lf", &fmt, &dp, &mc, &nc, &sp, &qpw, &cap, &ms) != 8 || fmt < 0 ||
        fmt > 3 || dp < 1 || mc < 0 || mc > 6 || nc < 0 || nc > 62 || sp < 0 || sp > 4096 ||
        (qpw != 0 && qpw != 32 && qpw != 64 && qpw != 128) || (cap != 0 && (cap < 64 || cap > 2048))) {
      set_error("gv_tuning_table_load: malformed line");
      s = GV_EINVAL;
      break;
    }
    tab[Key{fmt, dp, mc, nc}] = Entry{Tuning{sp, qpw, cap}, ms};
  }
  std::fclose(f);
  GV_TRY(s);
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : tab) g_table[kv.first] = kv.second;
  ++g_version;
  return GV_OK;
}

gv_status gv_tuning_lookup(int32_t fmt, int32_t d_pad, int64_t m, int64_t n_rows, int32_t* splits, int32_t* qpw,
                           int32_t* cap) {
  Tuning t;
  if (!tuning_table_lookup(fmt, d_pad, m, n_rows, &t)) return GV_EUNSUPPORTED;
  if (splits) *splits = t.splits;
  if (qpw) *qpw = t.qpw;
  if (cap) *cap = t.cap;
  return GV_OK;
}

void gv_tuning_table_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  ++g_version;
}

}  // extern "C"
