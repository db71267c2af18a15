// Instantiates the per-bucket edge kernels for series windows W = 61..63
// (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part7(EdgeTables& t) {
  fill_range<double, 61, 63>(t.small64);
  fill_run_range<61, 63>(t.run64);
  fill_range<float, 61, 63>(t.small32);
}
}  // namespace sttsv
