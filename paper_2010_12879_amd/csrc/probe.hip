// Measurement aids: a STREAM-triad kernel that gives the HBM bandwidth a
// streaming kernel reaches on this part (the practical ceiling next to the
// 8 TB/s peak in the roofline of the stencil kernels), and the cache flush of
// the cold per-kernel timing.
#include "kernels.h"
#include "spfd.h"

namespace spfd {

// a[i] = b[i] + s c[i] over n doubles, U elements of two doubles per thread,
// consecutive blocks of 256*U pairs per workgroup (every load issued before
// the first use); nontemporal stores of a
template <int U>
__global__ __launch_bounds__(256) void k_triad(double *__restrict__ a, const double *__restrict__ b,
                                               const double *__restrict__ c, long long n2, double s)
{
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 *B = (const v2 *)b, *C = (const v2 *)c;
    v2 *A = (v2 *)a;
    const long long base = (long long)blockIdx.x * 256 * U + threadIdx.x;
    v2 bv[U], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long i = base + 256LL * u;
        if (i < n2) {
            bv[u] = B[i];
            cv[u] = C[i];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long i = base + 256LL * u;
        if (i < n2) {
            const v2 r = bv[u] + s * cv[u];
            __builtin_nontemporal_store(r, &A[i]);
        }
    }
}

hipError_t launch_triad(double *a, const double *b, const double *c, long long n, double s, int variant,
                        hipStream_t st)
{
    const long long n2 = n / 2;
    if (n2 <= 0) return hipSuccess;
    if (variant == 0) {
        const long long g = (n2 + 255) / 256;
        hipLaunchKernelGGL(k_triad<1>, dim3((unsigned)g), dim3(256), 0, st, a, b, c, n2, s);
    } else {
        const long long g = (n2 + 1023) / 1024;
        hipLaunchKernelGGL(k_triad<4>, dim3((unsigned)g), dim3(256), 0, st, a, b, c, n2, s);
    }
    return hipGetLastError();
}

// read and write every word of a buffer (evicts the L2 and the Infinity Cache before a cold timing)
__global__ void k_flush(unsigned *buf, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        buf[i] += 1u;
}

hipError_t launch_flush(void *buf, size_t bytes, hipStream_t st)
{
    hipLaunchKernelGGL(k_flush, dim3(8192), dim3(256), 0, st, (unsigned *)buf, (long long)(bytes / 4));
    return hipGetLastError();
}

}  // namespace spfd

using namespace spfd;

extern "C" spfd_status spfd_stream_triad(int device, void *hip_stream, double *a, const double *b, const double *c,
                                         long long n, int reps, double *best_gbs)
{
    if (!a || !b || !c || !best_gbs || n < 2 || reps < 1) return SPFD_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SPFD_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return SPFD_HIP_ERROR;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SPFD_HIP_ERROR;
    double best = 0.0;
    spfd_status rc = SPFD_OK;
    for (int variant = 0; variant < 2 && rc == SPFD_OK; ++variant) {
        for (int r = 0; r < reps + 1; ++r) {   // the first run of each variant is a warm-up
            if (hipEventRecord(e0, st) != hipSuccess || launch_triad(a, b, c, n, 1.5, variant, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = SPFD_HIP_ERROR;
                break;
            }
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = SPFD_HIP_ERROR;
                break;
            }
            const double gbs = 3.0 * 8.0 * (double)(n / 2 * 2) / (ms * 1e-3) / 1e9;
            if (r > 0 && gbs > best) best = gbs;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SPFD_OK) *best_gbs = best;
    return rc;
}
