// Instantiates the per-bucket edge kernels for series windows W = 55..57
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part5(EdgeTables& t) {
  fill_range<double, 55, 57>(t.small64);
  fill_run_range<55, 57>(t.run64);
  fill_range<float, 55, 57>(t.small32);
}
}  // namespace sttsv
