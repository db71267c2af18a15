// Instantiates the edge kernels for series windows W = 51..54 (FP64 and FP32).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part4(EdgeTables& t) {
  fill_range<double, 51, 54>(t.f64);
  fill_range<float, 51, 54>(t.f32);
}
}  // namespace sttsv
