// The Monte-Carlo cell scan with the directions drawn on the device from the
// seed (vg_philox.h): the GEN instances of the kernels in vg_cell_scan.h, in
// a translation unit of their own so that they compile in parallel with the
// directions-as-input ones.
#include "vg_cell_scan.h"

namespace vg {

hipError_t launch_cells_gen(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s) {
  if (bf16) {
    switch (rw) {
      case 1024: return launch_kq_g<4, 8, true>(a, s, grid);
      case 512: return launch_kq_g<2, 8, true>(a, s, grid);
      case 256: return launch_kq_g<2, 4, true>(a, s, grid);
      case 128: return launch_kq_g<1, 4, true>(a, s, grid);
      default: return launch_kq_g<1, 2, true>(a, s, grid);
    }
  }
  switch (rw) {
    case 1024: return launch_kp_g<4, 8, true>(a, s, grid);
    case 512: return launch_kp_g<2, 8, true>(a, s, grid);
    case 256: return launch_kp_g<2, 4, true>(a, s, grid);
    case 128: return launch_kp_g<1, 4, true>(a, s, grid);
    default: return launch_kp_g<1, 2, true>(a, s, grid);
  }
}

}  // namespace vg
