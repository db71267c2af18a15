// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 25..32 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen3(EdgeTables& t) {
  t.gen64[3] = &launch_generic<double, 25, 32>;
  t.gen32[3] = &launch_generic<float, 25, 32>;
}
}  // namespace sttsv
