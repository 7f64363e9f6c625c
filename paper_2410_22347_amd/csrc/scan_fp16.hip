// Instantiation of the scoring kernel for fp16 storage.
#include "search_kernels.hpp"

namespace gv {

template <int FMT, int MODE>
gv_status dispatch_scan(int dp, const scan::Shape& sh, const scan::ScoreArgs& args, hipStream_t st) {
  return scan::dispatch_ks<FMT, MODE>(dp, sh, args, st);
}

template gv_status dispatch_scan<GV_FP16, scan::kFilter>(int, const scan::Shape&, const scan::ScoreArgs&, hipStream_t);
template gv_status dispatch_scan<GV_FP16, scan::kDense>(int, const scan::Shape&, const scan::ScoreArgs&, hipStream_t);

template <>
gv_status dispatch_scan_queue<GV_FP16>(int dp, const scan::Shape& sh, int grid, const scan::ScoreArgs* args,
                                 const int64_t* off, int ncoll, int* head, hipStream_t st) {
  return scan::dispatch_queue_ks<GV_FP16>(dp, sh, grid, args, off, ncoll, head, st);
}

template <int MODE>
gv_status dispatch_scan_lazy(const scan::Shape& sh, const scan::ScoreArgs& args, hipStream_t st) {
  scan::launch_lazy<MODE>(sh, args, st);
  GV_HIP(hipGetLastError());
  return GV_OK;
}
template gv_status dispatch_scan_lazy<scan::kFilter>(const scan::Shape&, const scan::ScoreArgs&, hipStream_t);
template gv_status dispatch_scan_lazy<scan::kDense>(const scan::Shape&, const scan::ScoreArgs&, hipStream_t);

}  // namespace gv
