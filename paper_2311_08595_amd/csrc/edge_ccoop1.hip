// Instantiates the compact FP32-apply variants of the fused lane-group edge
// kernel for series windows W = 33..63.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_ccoop1(EdgeTables& t) {
  t.coop32c[4] = &launch_coop<float, 33, 40, true>;
  t.coop32c[5] = &launch_coop<float, 41, 48, true>;
  t.coop32c[6] = &launch_coop<float, 49, 56, true>;
  t.coop32c[7] = &launch_coop<float, 57, 63, true>;
}
}  // namespace sttsv
