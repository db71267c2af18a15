// Instantiates the edge kernels for series windows W = 1..31 (FP64 and FP32).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_part0(EdgeTables& t) {
  fill_range<double, 1, 31>(t.f64);
  fill_range<float, 1, 31>(t.f32);
}
}  // namespace sttsv
