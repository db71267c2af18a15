// Instantiates the per-bucket edge kernels for series windows W = 32..39
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part1(EdgeTables& t) {
  fill_range<double, 32, 39>(t.small64);
  fill_run_range<32, 39>(t.run64);
  fill_range<float, 32, 39>(t.small32);
}
}  // namespace sttsv
