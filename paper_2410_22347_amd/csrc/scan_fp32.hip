// Instantiation of the scoring kernel for fp32 storage.
#include "search_kernels.hpp"

namespace gv {

template <int FMT, int MODE>
gv_status dispatch_scan(int dp, const scan::Shape& sh, const scan::ScoreArgs& args, hipStream_t st) {
  return scan::dispatch_ks<FMT, MODE>(dp, sh, args, st);
}

template gv_status dispatch_scan<GV_FP32, scan::kFilter>(int, const scan::Shape&, const scan::ScoreArgs&, hipStream_t);
template gv_status dispatch_scan<GV_FP32, scan::kDense>(int, const scan::Shape&, const scan::ScoreArgs&, hipStream_t);

template <>
gv_status dispatch_scan_queue<GV_FP32>(int dp, const scan::Shape& sh, int grid, const scan::ScoreArgs* args,
                                 const int64_t* off, int ncoll, int* head, hipStream_t st) {
  return scan::dispatch_queue_ks<GV_FP32>(dp, sh, grid, args, off, ncoll, head, st);
}

}  // namespace gv
