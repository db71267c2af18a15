// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 9..16 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen1(EdgeTables& t) {
  t.gen64[1] = &launch_generic<double, 9, 16>;
  t.gen32[1] = &launch_generic<float, 9, 16>;
}
}  // namespace sttsv
