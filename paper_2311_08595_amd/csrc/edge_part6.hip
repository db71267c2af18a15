// Instantiates the per-bucket edge kernels for series windows W = 58..60
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part6(EdgeTables& t) {
  fill_range<double, 58, 60>(t.small64);
  fill_run_range<58, 60>(t.run64);
  fill_range<float, 58, 60>(t.small32);
}
}  // namespace sttsv
