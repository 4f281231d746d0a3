// The allocation-free variant of the |E| quantile (spfd_percentile_noalloc).
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the radix
// selection's work area (per group: selection state and a 256-bin histogram)
// lives in a file-scope device array of fixed size instead of a handle's
// buffer.  Every GPU the library runs on holds its own copy of the array until
// the process ends; its device address is looked up once per device with that
// device current, and kernels get that address, never the array's name (in
// host code the name is a host-side stand-in).  Calls on one GPU share the
// array: calls that overlap on that GPU race.  The histograms are cleared at
// the start of every call (by a kernel, so the call can be captured).
#include <mutex>

#include "kernels.h"
#include "spfd.h"

namespace spfd {

constexpr int NOALLOC_GROUPS = 1 + MAX_LABELS;     // whole body + one group per label
constexpr int NOALLOC_DEVICES = 64;

// work area of launch_quantiles for up to NOALLOC_GROUPS groups, plus the output staging
static __device__ __align__(256) uint8_t scratch[272 * 1024];

namespace {
std::mutex scratch_mu;
void *scratch_ptr[NOALLOC_DEVICES] = {};

// device address of this device's copy of `scratch` (the device must be current)
hipError_t scratch_on(int device, void **out)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[device] = p;
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

}  // namespace spfd

using namespace spfd;

extern "C" spfd_status spfd_percentile_noalloc(int device, void *hip_stream, const uint8_t *labels,
                                               const double *sigma_table, int n_labels, const double *sigma_voxel,
                                               long long nvox, const double *emag, double q, double *out)
{
    if (!labels || !emag || !out || nvox <= 0) return SPFD_INVALID_ARG;
    if (!sigma_table && !sigma_voxel) return SPFD_INVALID_ARG;
    if (!(q > 0.0 && q <= 1.0)) return SPFD_INVALID_ARG;
    // the work area holds NOALLOC_GROUPS groups: 256 labels at most
    if (n_labels < 1 || n_labels > MAX_LABELS) return SPFD_INVALID_ARG;
    if (sel_work_bytes(NOALLOC_GROUPS) > sizeof(scratch)) return SPFD_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev || device >= NOALLOC_DEVICES)
        return SPFD_INVALID_ARG;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return SPFD_HIP_ERROR;
    hipError_t e = hipSetDevice(device);
    void *work = nullptr;
    if (e == hipSuccess) e = scratch_on(device, &work);
    if (e == hipSuccess)
        e = launch_quantiles(labels, sigma_table, sigma_voxel, nvox, emag, 1 + n_labels, q, work, out,
                             (hipStream_t)hip_stream);
    (void)hipSetDevice(prev);
    return e == hipSuccess ? SPFD_OK : SPFD_HIP_ERROR;
}
