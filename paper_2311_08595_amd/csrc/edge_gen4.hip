// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 33..40 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen4(EdgeTables& t) {
  t.gen64[4] = &launch_generic<double, 33, 40>;
  t.gen32[4] = &launch_generic<float, 33, 40>;
}
}  // namespace sttsv
