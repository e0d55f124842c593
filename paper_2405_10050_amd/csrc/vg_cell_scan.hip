// Launchers of the Monte-Carlo cell scan (kernels in vg_cell_scan.h), the
// directions-as-input instances; the instances that draw the directions on
// the device are compiled separately (vg_cell_scan_gen.hip).
#include "vg_cell_scan.h"

namespace vg {
namespace {
template <int C, int WAVES>
hipError_t launch_kq(const CellScanArgs &a, hipStream_t s, int grid) {
  return a.dirs ? launch_kq_g<C, WAVES, false>(a, s, grid) : launch_cells_gen(a, true, C * WAVES * 32, grid, s);
}

template <int C, int WAVES>
hipError_t launch_kp(const CellScanArgs &a, hipStream_t s, int grid) {
  return a.dirs ? launch_kp_g<C, WAVES, false>(a, s, grid) : launch_cells_gen(a, false, C * WAVES * 32, grid, s);
}

}  // namespace

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
  if (bf16) {
    switch (rw) {
      case 1024: return launch_kq<4, 8>(a, s, grid);
      case 512: return launch_kq<2, 8>(a, s, grid);
      case 256: return launch_kq<2, 4>(a, s, grid);
      case 128: return launch_kq<1, 4>(a, s, grid);
      default: return launch_kq<1, 2>(a, s, grid);
    }
  }
  switch (rw) {
    case 1024: return launch_kp<4, 8>(a, s, grid);
    case 512: return launch_kp<2, 8>(a, s, grid);
    case 256: return launch_kp<2, 4>(a, s, grid);
    case 128: return launch_kp<1, 4>(a, s, grid);
    default: return launch_kp<1, 2>(a, s, grid);
  }
}

hipError_t launch_cell_scan_fp32(const CellScanArgs &a, hipStream_t s) {
  return launch_cell_scan_rw(a, false, cell_scan_rays_per_wg(a.R), a.n, s);
}

hipError_t launch_cell_scan_bf16x3(const CellScanArgs &a, hipStream_t s) {
  return launch_cell_scan_rw(a, true, cell_scan_rays_per_wg(a.R), a.n, s);
}

}  // namespace vg
