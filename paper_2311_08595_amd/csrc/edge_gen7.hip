// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 57..63 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen7(EdgeTables& t) {
  t.gen64[7] = &launch_generic<double, 57, 63>;
  t.gen32[7] = &launch_generic<float, 57, 63>;
}
}  // namespace sttsv
