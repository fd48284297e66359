// Wall Nusselt numbers without workspace scratch: the local heat-flux
// profiles and the reduced values live in a device array that the library
// holds for the life of the process, so the call allocates nothing and
// touches no caller memory beyond the handle's state and its outputs.
//
// The array is a file-scope __device__ variable: host code never uses its
// name as an address (that is a host-side stand-in); each device's copy is
// resolved once with hipGetSymbolAddress while that device is current, and
// that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lbm_handle.hpp"

namespace {

// Local Nusselt profiles of the two walls (ny*nz doubles each), then the
// eight reduced values.
constexpr size_t kMaxWallCells = (size_t)1 << 20;  // ny * nz of the largest cavity
constexpr size_t kScratchDoubles = 2 * kMaxWallCells + 8;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (dev must be current).
lbm_status scratch_of(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return lbm::fail(LBM_ERR_STATE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return lbm::hip_fail(e, "scratch symbol address");
        if (!p) return lbm::fail(LBM_ERR_HIP, "scratch symbol address is null");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_nusselt_noalloc(lbm_handle* h, lbm_nu* out, double* local_hot,
                               double* local_cold) {
    if (!h || !out) return lbm::fail(LBM_ERR_ARG, "null argument");
    const size_t wall = (size_t)h->p.ny * (size_t)h->p.nz;
    if (wall > kMaxWallCells)
        return lbm::fail(LBM_ERR_ARG, "ny * nz = " + std::to_string(wall) +
                                          " exceeds the static scratch limit of " +
                                          std::to_string(kMaxWallCells) + " wall cells");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lbm::hip_fail(e, "current device");
    if (dev != h->device)
        return lbm::fail(LBM_ERR_STATE, "the handle's device must be current");
    double* s = nullptr;
    lbm_status st = scratch_of(dev, &s);
    if (st != LBM_OK) return st;
    // every profile value and every reduced value is overwritten by the
    // kernels, so nothing has to start at zero
    return lbm::nusselt_into(h, s, s + wall, s + 2 * kMaxWallCells, out, local_hot, local_cold);
}

}  // extern "C"
