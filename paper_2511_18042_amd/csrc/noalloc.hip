// Entry point that allocates nothing: lg_metrics_from_coords with its [9][N] scratch of
// inner coordinate derivatives in a file-scope device array instead of a hipMalloc'd
// buffer (for callers under graph capture or in loops that must not allocate).
//
// The array is a module global: every GPU the library runs on holds its own copy from the
// time the code object is loaded until the process ends.  Host code never passes the
// array's name to a kernel (in host code it is a stand-in, not a device address); the
// device address is looked up once per device with hipGetSymbolAddress, with that device
// current, and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lgbr.h"
#include "lgbr_kernels.h"

static constexpr long long SCRATCH_NODES = LG_NOALLOC_MAX_NODES;   // padded grid nodes the scratch covers

static __device__ __align__(256) double scratch[9 * SCRATCH_NODES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of the scratch (looked up on first use).
lg_status scratch_ptr(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return LG_EHIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LG_EHIP;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return LG_OK;
}

}  // namespace

extern "C" {

lg_status lg_metrics_from_coords_noalloc(const lg_grid* grid, const double* coords, double* node_metrics,
                                         void* stream) {
  if (!grid || !coords || !node_metrics) return LG_EINVAL;
  if (grid->ndim < 1 || grid->ndim > 3 || grid->ng != lg::NG) return LG_EINVAL;
  int N[3];
  long long total = 1;
  for (int d = 0; d < 3; ++d) {
    if (d >= grid->ndim && grid->n[d] != 1) return LG_EINVAL;
    if (d < grid->ndim && grid->n[d] < 5) return LG_EINVAL;
    N[d] = grid->n[d] + (d < grid->ndim ? 2 * lg::NG : 0);
    total *= N[d];
  }
  if (total > SCRATCH_NODES) return LG_EUNSUPPORTED;
  double* s9 = nullptr;
  const lg_status st = scratch_ptr(&s9);
  if (st != LG_OK) return st;
  // the inner kernel writes all 9 x total scratch entries before the outer one reads them,
  // so nothing needs clearing between calls
  lg::launch_metrics(grid->ndim, N, coords, s9, node_metrics, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? LG_OK : LG_EHIP;
}

}  // extern "C"
