// The Monte-Carlo cell scan instances with the directions drawn on the device from the seed (vg_philox.h) and the
// nodes in scan order: one instance set of the
// kernels in vg_cell_scan.h, in a translation unit of its own so that the
// sets compile in parallel.
#include "vg_cell_scan.h"

namespace vg {

hipError_t launch_cells_gen_sorted(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s) {
  return launch_cells_set<true, true>(a, bf16, rw, grid, s);
}

}  // namespace vg
