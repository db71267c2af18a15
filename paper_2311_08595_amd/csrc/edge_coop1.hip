// Instantiates the fused lane-group edge kernel for FP64 series, windows 25..48.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_coop1(EdgeTables& t) {
  t.coop64[3] = &launch_coop<double, 25, 32>;
  t.coop64[4] = &launch_coop<double, 33, 40>;
  t.coop64[5] = &launch_coop<double, 41, 48>;
}
}  // namespace sttsv
