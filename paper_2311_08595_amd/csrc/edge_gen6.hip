// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 49..56 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen6(EdgeTables& t) {
  t.gen64[6] = &launch_generic<double, 49, 56>;
  t.gen32[6] = &launch_generic<float, 49, 56>;
}
}  // namespace sttsv
