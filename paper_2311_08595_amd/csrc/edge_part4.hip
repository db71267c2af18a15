// Instantiates the per-bucket edge kernels for series windows W = 51..54
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part4(EdgeTables& t) {
  fill_range<double, 51, 54>(t.small64);
  fill_run_range<51, 54>(t.run64);
  fill_range<float, 51, 54>(t.small32);
}
}  // namespace sttsv
