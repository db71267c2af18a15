// Instantiates the per-bucket edge kernels for series windows W = 46..50
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part3(EdgeTables& t) {
  fill_range<double, 46, 50>(t.small64);
  fill_run_range<46, 50>(t.run64);
  fill_range<float, 46, 50>(t.small32);
}
}  // namespace sttsv
