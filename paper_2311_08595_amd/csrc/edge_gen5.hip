// Instantiates the fused generic edge kernel (runtime edge size) for series
// windows W = 41..48 (FP64 and FP32 series).
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_gen5(EdgeTables& t) {
  t.gen64[5] = &launch_generic<double, 41, 48>;
  t.gen32[5] = &launch_generic<float, 41, 48>;
}
}  // namespace sttsv
