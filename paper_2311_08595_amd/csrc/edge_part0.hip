// Instantiates the per-bucket edge kernels for series windows W = 1..31
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part0(EdgeTables& t) {
  fill_range<double, 1, 31>(t.small64);
  fill_run_range<1, 31>(t.run64);
  fill_range<float, 1, 31>(t.small32);
}
}  // namespace sttsv
