// Launchers of the Monte-Carlo cell scan (kernels in vg_cell_scan.h): the
// dispatch over tile shapes and instance sets, and the instances that read
// the directions from memory with the nodes in index order (also the
// candidate-list scans).  The other instance sets -- directions drawn on the
// device, nodes in scan order -- are compiled in translation units of their
// own (vg_cell_scan_sorted.hip, vg_cell_scan_gen.hip,
// vg_cell_scan_gen_sorted.hip) so that they build in parallel.
#include "vg_cell_scan.h"

namespace vg {

hipError_t launch_cells_read_index(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s) {
  return launch_cells_set<false, false>(a, bf16, rw, grid, s);
}

int cell_scan_rays_per_wg(int R) {
  if (R >= 1024) return 1024;
  if (R >= 512) return 512;
  if (R >= 256) return 256;
  if (R >= 128) return 128;
  return 64;
}

hipError_t launch_cell_scan_rw(const CellScanArgs &a0, bool bf16, int rw, int64_t n_cells, hipStream_t s) {
  CellScanArgs a = a0;
  if (rw != 64 && rw != 128 && rw != 256 && rw != 512 && rw != 1024) return hipErrorInvalidValue;
  a.wg_per_cell = (a.R + rw - 1) / rw;
  const int64_t grid64 = n_cells * a.wg_per_cell;
  if (grid64 <= 0) return hipSuccess;
  if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
  const int grid = (int)grid64;
  const bool sorted = a.xs != nullptr;
  if (a.dirs) return sorted ? launch_cells_read_sorted(a, bf16, rw, grid, s) : launch_cells_read_index(a, bf16, rw, grid, s);
  return sorted ? launch_cells_gen_sorted(a, bf16, rw, grid, s) : launch_cells_gen_index(a, bf16, rw, grid, s);
}

hipError_t launch_cell_scan_fp32(const CellScanArgs &a, hipStream_t s) {
  return launch_cell_scan_rw(a, false, cell_scan_rays_per_wg(a.R), a.n, s);
}

hipError_t launch_cell_scan_bf16x3(const CellScanArgs &a, hipStream_t s) {
  return launch_cell_scan_rw(a, true, cell_scan_rays_per_wg(a.R), a.n, s);
}

}  // namespace vg
