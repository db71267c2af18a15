// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 1..8 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen0(EdgeTables& t) {
  t.gen64[0] = &launch_generic<double, 1, 8>;
  t.gen32[0] = &launch_generic<float, 1, 8>;
}
}  // namespace sttsv
