// Dense inverse of the coarsest-level matrix by blocked Gauss-Jordan
// elimination on 64x64 tiles, spread over many workgroups.
//
// The matrix (after the rank-one regularisation of every connected component,
// which makes it symmetric positive definite) is copied into an ld x ld work
// array, ld = n rounded up to 64, with the identity on the padding.  For each
// diagonal tile k:
//   P       = A_kk^-1                      (one workgroup, in LDS)
//   A_kj   <- P A_kj  (j != k),  A_kk <- P (row block, one workgroup per tile)
//   A_ij   <- A_ij - A_ik A_kj  (i, j != k), A_ik <- -A_ik P (all other tiles)
// with the old column block A_ik saved before the row-block step.  No
// pivoting is needed for a symmetric positive definite matrix.
#include "kernels.h"

namespace spfd {

constexpr int GT = 64;        // tile edge
constexpr int GS = GT + 1;    // LDS row stride (bank spread)

__global__ __launch_bounds__(256) void k_gj_pad(int n, int ld, const double *__restrict__ A, double *__restrict__ W)
{
    const long long tot = (long long)ld * ld;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / ld), j = (int)(e % ld);
        W[e] = (i < n && j < n) ? A[(long long)i * n + j] : (i == j ? 1.0 : 0.0);
    }
}

__global__ __launch_bounds__(256) void k_gj_unpad(int n, int ld, const double *__restrict__ W, double *__restrict__ A)
{
    const long long tot = (long long)n * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        A[e] = W[(long long)i * ld + j];
    }
}

__device__ __forceinline__ void tile_load(const double *__restrict__ src, int ld, int r0, int c0, double *t)
{
    for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) {
        const int r = e / GT, c = e % GT;
        t[r * GS + c] = src[(long long)(r0 + r) * ld + c0 + c];
    }
}

// out (4x4 per thread, rows 4*(t/16).., cols 4*(t%16)..) = a * b for LDS tiles a, b
__device__ __forceinline__ void tile_mul(const double *a, const double *b, double acc[4][4])
{
    const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < GT; ++k) {
        double av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = a[(r0 + i) * GS + k];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = b[k * GS + c0 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
}

// P = A_kk^-1 by Gauss-Jordan: for pivot p with a = A_pp,
// A_pp <- 1/a, A_pj <- A_pj / a, A_ip <- -A_ip / a, A_ij <- A_ij - A_ip A_pj / a.
// 1024 threads hold four entries each in registers (row i = t/16, columns
// 4 (t%16) .. +3); per pivot only row p (with 1/a, formed once by its owner) and
// column p pass through LDS.  They are published for pivot p + 1 by the threads
// that hold them right after their update of pivot p, into the other of two LDS
// buffers, so each pivot needs one barrier.
__global__ __launch_bounds__(1024) void k_gj_diag(int ld, int k0, const double *__restrict__ W, double *__restrict__ P)
{
    __shared__ double row[2][GT + 1], col[2][GT];   // row[.][GT] = 1 / pivot
    const int t = threadIdx.x;
    const int i = t >> 4, j0 = (t & 15) * 4;
    double a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = W[(long long)(k0 + i) * ld + k0 + j0 + q];
    // publish row and column 0
    auto publish = [&](int p, int buf) {
        if (i == p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                row[buf][j0 + q] = a[q];
                if (j0 + q == p) row[buf][GT] = 1.0 / a[q];
            }
        }
        if (p >= j0 && p < j0 + 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j0 + q == p) col[buf][i] = a[q];
        }
    };
    publish(0, 0);
    __syncthreads();
    for (int p = 0; p < GT; ++p) {
        const int cur = p & 1;
        const double piv = row[cur][GT];
        const double ci = col[cur][i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + q;
            const double rpj = (j == p) ? 1.0 : row[cur][j];
            a[q] = (i == p) ? rpj * piv : (j == p ? 0.0 : a[q]) - ci * piv * rpj;
        }
        if (p + 1 < GT) publish(p + 1, cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) P[i * GT + j0 + q] = a[q];
}

// row block k <- P A_k*, A_kk <- P; and the old column block (rows outside k) into C [ld][64]
__global__ __launch_bounds__(256) void k_gj_row(int ld, int k0, double *__restrict__ W, const double *__restrict__ P,
                                                double *__restrict__ C)
{
    __shared__ double p[GT * GS];
    __shared__ double a[GT * GS];
    const int j0 = blockIdx.x * GT;
    // column block piece: rows j0..j0+63 of columns k0..k0+63 (not written by any workgroup here)
    if (j0 != k0)
        for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) {
            const int r = e / GT, c = e % GT;
            C[(long long)(j0 + r) * GT + c] = W[(long long)(j0 + r) * ld + k0 + c];
        }
    for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) p[(e / GT) * GS + e % GT] = P[e];
    if (j0 == k0) {
        __syncthreads();
        for (int e = threadIdx.x; e < GT * GT; e += blockDim.x)
            W[(long long)(k0 + e / GT) * ld + k0 + e % GT] = p[(e / GT) * GS + e % GT];
        return;
    }
    tile_load(W, ld, k0, j0, a);
    __syncthreads();
    double acc[4][4];
    tile_mul(p, a, acc);
    const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) W[(long long)(k0 + r0 + i) * ld + j0 + c0 + j] = acc[i][j];
}

// every tile outside row block k: A_ij -= C_i A_kj (j != k), A_ik = -C_i P
__global__ __launch_bounds__(256) void k_gj_update(int ld, int k0, double *__restrict__ W,
                                                   const double *__restrict__ P, const double *__restrict__ C)
{
    __shared__ double ct[GT * GS];
    __shared__ double rt[GT * GS];
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    if (i0 == k0) return;
    for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) ct[(e / GT) * GS + e % GT] = C[(long long)(i0 + e / GT) * GT + e % GT];
    if (j0 == k0) {
        for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) rt[(e / GT) * GS + e % GT] = P[e];
    } else {
        tile_load(W, ld, k0, j0, rt);
    }
    __syncthreads();
    double acc[4][4];
    tile_mul(ct, rt, acc);
    const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double *w = W + (long long)(i0 + r0 + i) * ld + j0 + c0 + j;
            *w = (j0 == k0) ? -acc[i][j] : *w - acc[i][j];
        }
}

size_t dense_inverse_work_doubles(int n)
{
    const long long ld = ((long long)n + GT - 1) / GT * GT;
    return (size_t)(ld * ld + ld * GT + GT * GT);
}

hipError_t launch_dense_inverse(int n, double *A, double *work, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int ld = (n + GT - 1) / GT * GT;
    const int nt = ld / GT;
    double *W = work, *C = work + (long long)ld * ld, *P = C + (long long)ld * GT;
    auto blocks = [](long long m) { return (unsigned)((m + 255) / 256 > 65536 ? 65536 : (m + 255) / 256); };
    SPFD_LAUNCH(k_gj_pad, dim3(blocks((long long)ld * ld)), dim3(256), 0, s, n, ld, A, W);
    for (int k = 0; k < nt; ++k) {
        const int k0 = k * GT;
        SPFD_LAUNCH(k_gj_diag, dim3(1), dim3(1024), 0, s, ld, k0, W, P);
        SPFD_LAUNCH(k_gj_row, dim3(nt), dim3(256), 0, s, ld, k0, W, P, C);
        SPFD_LAUNCH(k_gj_update, dim3(nt, nt), dim3(256), 0, s, ld, k0, W, P, C);
    }
    SPFD_LAUNCH(k_gj_unpad, dim3(blocks((long long)n * n)), dim3(256), 0, s, n, ld, W, A);
    return hipGetLastError();
}

}  // namespace spfd
