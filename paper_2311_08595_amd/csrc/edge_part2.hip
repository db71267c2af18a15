// Instantiates the per-bucket edge kernels for series windows W = 40..45
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part2(EdgeTables& t) {
  fill_range<double, 40, 45>(t.small64);
  fill_run_range<40, 45>(t.run64);
  fill_range<float, 40, 45>(t.small32);
}
}  // namespace sttsv
