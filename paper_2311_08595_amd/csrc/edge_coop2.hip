// Instantiates the fused lane-group edge kernel for FP32 series, windows 1..32.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_coop2(EdgeTables& t) {
  t.coop32[0] = &launch_coop<float, 1, 8>;
  t.coop32[1] = &launch_coop<float, 9, 16>;
  t.coop32[2] = &launch_coop<float, 17, 24>;
  t.coop32[3] = &launch_coop<float, 25, 32>;
}
}  // namespace sttsv
