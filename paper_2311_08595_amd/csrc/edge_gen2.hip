// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 17..24 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen2(EdgeTables& t) {
  t.gen64[2] = &launch_generic<double, 17, 24>;
  t.gen32[2] = &launch_generic<float, 17, 24>;
}
}  // namespace sttsv
