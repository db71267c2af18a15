// Instantiates the fused lane-group edge kernel for FP64 series, windows 1..24.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_coop0(EdgeTables& t) {
  t.coop64[0] = &launch_coop<double, 1, 8>;
  t.coop64[1] = &launch_coop<double, 9, 16>;
  t.coop64[2] = &launch_coop<double, 17, 24>;
}
}  // namespace sttsv
