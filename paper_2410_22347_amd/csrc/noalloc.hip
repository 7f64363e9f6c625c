// gv_search_noalloc: gv_search for callers that cannot allocate device memory
// (code under graph capture, tight serving loops).  The search scratch -- the
// S1 views and scales, the candidate lists, list lengths, cascade seeds and
// dense sample, the candidates -- lives in one file-scope device array instead
// of the stream-ordered pool.  Every device that runs the library holds its own
// copy of the array until the process ends; calls on one device share it.
#include <algorithm>
#include <mutex>

#include "common.hpp"

namespace gv {
namespace {

// the scratch of one allocation-free search, at most this many bytes
constexpr size_t kNoAllocScratch = 64ull << 20;

static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

// the address of this device's copy of `scratch`, looked up once per device
// with that device current (the array's name in host code is not a device
// address)
gv_status scratch_of(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("gv_search_noalloc: device index out of range");
    return GV_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error(std::string("gv_search_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return GV_EDEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GV_OK;
}

}  // namespace
}  // namespace gv

using namespace gv;

extern "C" {

int64_t gv_search_noalloc_capacity(void) { return (int64_t)kNoAllocScratch; }

gv_status gv_search_noalloc(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int32_t k,
                            int32_t kappa, int32_t* out_ids, float* out_scores, void* stream) {
  try {
    clear_error();
    if (!valid_model(model) || !index || index->magic != kIndexMagic) return GV_ENOTFIT;
    GV_REQUIRE(model->C == index->C && model->d == index->d && model->D == index->D,
               "gv_search_noalloc: model and index shapes differ");
    GV_TRY(check_search_args(index, m, k, kappa));
    if (m == 0) return GV_OK;
    GV_REQUIRE(Q && out_ids, "gv_search_noalloc: NULL argument");
    GV_REQUIRE(index->X != nullptr, "gv_search_noalloc: the index keeps no full-dimension vectors");
    int dev = 0;
    GV_HIP(hipGetDevice(&dev));
    GV_REQUIRE(index->device == dev, "gv_search_noalloc: the index lives on another device");
    // The launch shape changes only the speed, never the result: when the usual
    // plan needs more scratch than the array, take shorter candidate lists and,
    // if that is not enough, fewer row ranges per query block.
    // The overrides stay in force until the search has been issued (it plans its
    // launches again from them, and checks that the plan is the one sized here).
    struct Restore {
      int s, q, c;
      ~Restore() { set_tuning(s, q, c); }
    } restore{tuned_splits(), tuned_qpw(), tuned_cap()};
    SearchPlan plan;
    GV_TRY(search_plan(model, index, m, kappa, &plan));
    if (plan.bytes > kNoAllocScratch) {
      const int cap = std::max(512, min_list_cap(kappa));
      set_tuning(restore.s, restore.q, cap);
      GV_TRY(search_plan(model, index, m, kappa, &plan));
      if (plan.bytes > kNoAllocScratch) {
        // the lists take m * R * cap * 8 bytes; leave a quarter for the rest
        const int64_t R = (int64_t)(kNoAllocScratch / 4 * 3) / (m * (int64_t)cap * 8) / 8 * 8;
        if (R >= 8) {
          set_tuning((int)std::min<int64_t>(R - 4, 4096), restore.q, cap);
          GV_TRY(search_plan(model, index, m, kappa, &plan));
        }
      }
    }
    if (plan.bytes > kNoAllocScratch) {
      set_error("gv_search_noalloc: this search needs " + std::to_string(plan.bytes) +
                " bytes of scratch, more than the " + std::to_string(kNoAllocScratch) +
                " of the allocation-free path (use gv_search or a smaller batch)");
      return GV_EINVAL;
    }
    void* ws = nullptr;
    GV_TRY(scratch_of(dev, &ws));
    // no profiling events: creating them is an allocation
    suppress_profile_events(true);
    const gv_status s = search_run(model, index, Q, m, k, kappa, out_ids, out_scores, plan, ws, (hipStream_t)stream);
    suppress_profile_events(false);
    return s;
  } catch (const std::exception& e) {
    suppress_profile_events(false);
    set_error(e.what());
    return GV_EDEVICE;
  } catch (...) {
    suppress_profile_events(false);
    set_error("unknown failure");
    return GV_EDEVICE;
  }
}

}  // extern "C"
