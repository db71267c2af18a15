// Instantiates the fused lane-group edge kernel for FP32 series, windows 33..63.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_coop3(EdgeTables& t) {
  t.coop32[4] = &launch_coop<float, 33, 40>;
  t.coop32[5] = &launch_coop<float, 41, 48>;
  t.coop32[6] = &launch_coop<float, 49, 56>;
  t.coop32[7] = &launch_coop<float, 57, 63>;
}
}  // namespace sttsv
