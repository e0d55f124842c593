// Fixed device scratch of vg_raycast_cells_noalloc, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The array below lives in the library's code object: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device by noalloc_attach
// (called from vg_create with that device current) and kept in `g_ptr`.
// Calls on one GPU share the array: calls that overlap on that GPU race.
#include <mutex>

#include "vg_internal.h"

namespace vg {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_attach(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = p;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace vg
