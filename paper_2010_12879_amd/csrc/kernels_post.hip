// Post-processing on the voxel field: nearest-rank quantiles of |E|.
//
// Step 6 of the paper's technical summary (Sec. II.A) takes the 99th
// percentile of the voxel-averaged field (Sec. III.F) to exclude unphysical
// field enhancements.  The quantile of rank k = ceil(q n) among the n
// conducting voxels (whole body, and per tissue label) is found exactly by a
// radix select on the 64-bit patterns of |E|: for non-negative doubles the
// unsigned bit pattern orders like the value.  Eight passes of 8-bit digits,
// most significant first; per pass each workgroup builds LDS histograms for
// the whole body and every label, merged with integer atomics (exact, order
// independent), and one workgroup picks the digit of every group.
#include <math.h>

#include "kernels.h"

namespace spfd {

constexpr int SEL_BINS = 256;

// per group: prefix of the selected key, the rank still to find (1-based) and the count
struct SelState {
    unsigned long long prefix;
    long long k;
    long long n;
};

__global__ __launch_bounds__(256) void k_sel_hist(const uint8_t *__restrict__ labels, const double *__restrict__ table,
                                                  const double *__restrict__ sig_vox, long long nvox,
                                                  const double *__restrict__ emag, int ngroups, int shift,
                                                  const SelState *__restrict__ st, unsigned int *hist, int use_lds)
{
    extern __shared__ unsigned int lh[];
    const int nb = ngroups * SEL_BINS;
    if (use_lds) {
        for (int i = threadIdx.x; i < nb; i += blockDim.x) lh[i] = 0;
        __syncthreads();
    }
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x) {
        const double s = sig_vox ? sig_vox[v] : table[labels[v]];
        if (!(s > 0.0)) continue;
        const unsigned long long key = (unsigned long long)__double_as_longlong(emag[v]);
        const int digit = (int)((key >> shift) & 0xff);
        const int lab = labels[v];
        // group 0: whole body; group 1 + label: that tissue
        const int g2 = 1 + lab < ngroups ? 1 + lab : -1;
        const bool m0 = shift == 56 || (key >> (shift + 8)) == (st[0].prefix >> (shift + 8));
        const bool m2 = g2 >= 0 && (shift == 56 || (key >> (shift + 8)) == (st[g2].prefix >> (shift + 8)));
        if (use_lds) {
            if (m0) atomicAdd(lh + digit, 1u);
            if (m2) atomicAdd(lh + g2 * SEL_BINS + digit, 1u);
        } else {
            if (m0) atomicAdd(hist + digit, 1u);
            if (m2) atomicAdd(hist + g2 * SEL_BINS + digit, 1u);
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            if (lh[i]) atomicAdd(hist + i, lh[i]);
    }
}

// pick the digit that holds rank k of each group (one thread per group)
__global__ void k_sel_pick(int ngroups, int shift, double q, SelState *st, unsigned int *hist)
{
    for (int g = threadIdx.x; g < ngroups; g += blockDim.x) {
        unsigned int *h = hist + g * SEL_BINS;
        if (shift == 56) {
            long long n = 0;
            for (int d = 0; d < SEL_BINS; ++d) n += h[d];
            st[g].n = n;
            long long k = (long long)ceil(q * (double)n);
            st[g].k = k < 1 ? 1 : k;
            st[g].prefix = 0ull;
        }
        if (st[g].n > 0) {
            long long k = st[g].k, acc = 0;
            int d = 0;
            for (; d < SEL_BINS - 1; ++d) {
                if (acc + (long long)h[d] >= k) break;
                acc += h[d];
            }
            st[g].k = k - acc;
            st[g].prefix |= (unsigned long long)d << shift;
        }
        for (int d = 0; d < SEL_BINS; ++d) h[d] = 0u;
    }
}

__global__ void k_sel_out(int ngroups, const SelState *st, double *out)
{
    for (int g = threadIdx.x; g < ngroups; g += blockDim.x)
        out[g] = st[g].n > 0 ? __longlong_as_double((long long)st[g].prefix) : nan("");
}

size_t sel_work_bytes(int ngroups)
{
    return (size_t)ngroups * (sizeof(SelState) + SEL_BINS * sizeof(unsigned int) + sizeof(double)) + 256;
}

// work: sel_work_bytes(ngroups) bytes of device memory; out: ngroups doubles (device)
hipError_t launch_quantiles(const uint8_t *labels, const double *table, const double *sig_vox, long long nvox,
                            const double *emag, int ngroups, double q, void *work, double *out, hipStream_t s)
{
    SelState *st = (SelState *)work;
    unsigned int *hist = (unsigned int *)(st + ngroups);
    // cleared by a kernel, not a memset node: callers may capture this into a graph
    hipError_t e = launch_fill<int>((int *)hist, (long long)ngroups * SEL_BINS, 0, s);
    if (e != hipSuccess) return e;
    long long blocks = (nvox + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    const size_t lds = (size_t)ngroups * SEL_BINS * sizeof(unsigned int);
    const int use_lds = lds <= 64 * 1024;
    for (int shift = 56; shift >= 0; shift -= 8) {
        SPFD_LAUNCH(k_sel_hist, dim3((unsigned)blocks), dim3(256), use_lds ? lds : 0, s, labels, table, sig_vox,
                           nvox, emag, ngroups, shift, st, hist, use_lds);
        SPFD_LAUNCH(k_sel_pick, dim3(1), dim3(256), 0, s, ngroups, shift, q, st, hist);
    }
    SPFD_LAUNCH(k_sel_out, dim3(1), dim3(256), 0, s, ngroups, st, out);
    return hipGetLastError();
}

}  // namespace spfd
