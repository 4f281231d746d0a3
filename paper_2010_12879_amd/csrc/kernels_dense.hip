// Dense inverse of the coarsest-level matrix by blocked Gauss-Jordan
// elimination on 64x64 tiles, one launch per tile step.
//
// The matrix (after the rank-one regularisation of every connected component,
// which makes it symmetric positive definite) is copied into an ld x ld work
// array, ld = n rounded up to 64, with the identity on the padding.  For each
// diagonal tile k, with P = A_kk^-1:
//   A_kk <- P,   A_kj <- P A_kj,   A_ik <- -A_ik P,
//   A_ij <- A_ij - (A_ik P) A_kj            (i, j != k; old A_ik, A_kj)
// Every tile of step k reads only the previous matrix and writes the next one
// (two work matrices used in turn), so one launch covers the whole step; P of
// the next step is formed by one workgroup from the new diagonal tile in
// between.  No pivoting is needed for a symmetric positive definite matrix.
#include "kernels.h"

namespace spfd {

constexpr int GT = 64;        // tile edge
constexpr int GS = GT + 1;    // LDS row stride (bank spread)
constexpr int GI = 4;         // columns per thread in the tile inverse (1024 threads: 16 per row)

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

// In-place Gauss-Jordan inverse of a 64x64 tile held by 1024 threads: thread
// t holds row t/16, columns 4 (t%16) .. +3.  For pivot p with d = A_pp:
//   A_pj <- A_pj / d (j != p),  A_pp <- 1/d,
//   A_ij <- A_ij - (A_ip / d) A_pj (i, j != p),  A_ip <- -A_ip / d,
// that is, one multiply-add per entry once row p carries 1 in place of d and
// the entries of column p outside row p start from 0.  Row p (with 1/d
// beside it) and column p pass through LDS; the threads that own row and
// column p + 1 publish them right after their update for pivot p, into the
// other of two buffers, so each pivot needs one barrier.
struct InvLds {
    double row[2][GT + 2];   // [GT]: reciprocal pivot; rows 16-byte aligned for wide loads
    double col[2][GT];
};

__device__ __forceinline__ void tile_inverse(double a[GI], InvLds &L)
{
    const int i = threadIdx.x >> 4, j0 = (threadIdx.x & 15) * GI;
    auto publish = [&](int p, int buf) {
        const bool mine = p >= j0 && p < j0 + GI;
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < GI; ++q)
            if (j0 + q == p) d = a[q];
        if (i == p) {
#pragma unroll
            for (int q = 0; q < GI; ++q) L.row[buf][j0 + q] = (j0 + q == p) ? 1.0 : a[q];
            if (mine) L.row[buf][GT] = 1.0 / d;
        }
        if (mine) L.col[buf][i] = d;
    };
    publish(0, 0);
    __syncthreads();
    for (int p = 0; p < GT; ++p) {
        const int cur = p & 1;
        const double piv = L.row[cur][GT];
        if (i == p) {
#pragma unroll
            for (int q = 0; q < GI; ++q) a[q] = L.row[cur][j0 + q] * piv;
        } else {
            const double cp = L.col[cur][i] * piv;
#pragma unroll
            for (int q = 0; q < GI; ++q) a[q] = __builtin_fma(-cp, L.row[cur][j0 + q], (j0 + q == p) ? 0.0 : a[q]);
        }
        if (p + 1 < GT) publish(p + 1, cur ^ 1);
        __syncthreads();
    }
}

// P = A_kk^-1 (the diagonal tile of step k)
__global__ __launch_bounds__(1024) void k_gj_diag(int ld, int k0, const double *__restrict__ W, double *__restrict__ P)
{
    __shared__ __align__(16) InvLds L;
    const int i = threadIdx.x >> 4, j0 = (threadIdx.x & 15) * GI;
    double a[GI];
#pragma unroll
    for (int q = 0; q < GI; ++q) a[q] = W[(long long)(k0 + i) * ld + k0 + j0 + q];
    tile_inverse(a, L);
#pragma unroll
    for (int q = 0; q < GI; ++q) P[i * GT + j0 + q] = a[q];
}

// Step k: tile (blockIdx.y, blockIdx.x) of Wn from Wo and P = (Wo)_kk^-1
__global__ __launch_bounds__(256) void k_gj_step(int ld, int k, const double *__restrict__ Wo,
                                                 double *__restrict__ Wn, const double *__restrict__ P)
{
    __shared__ double t0[GT * GS];
    __shared__ double t1[GT * GS];
    __shared__ double t2[GT * GS];
    const int bi = blockIdx.y, bj = blockIdx.x;
    const int k0 = k * GT, i0 = bi * GT, j0 = bj * GT;
    const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
    double acc[4][4];
    if (bi == k && bj == k) {   // A_kk <- P
        for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) Wn[(long long)(k0 + e / GT) * ld + k0 + e % GT] = P[e];
        return;
    }
    if (bi == k || bj == k) {   // row block: P A_kj;  column block: -A_ik P
        if (bi == k) {
            for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) t0[(e / GT) * GS + e % GT] = P[e];
            tile_load(Wo, ld, k0, j0, t1);
        } else {
            tile_load(Wo, ld, i0, k0, t0);
            for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) t1[(e / GT) * GS + e % GT] = P[e];
        }
        __syncthreads();
        tile_mul(t0, t1, acc);
        const double sg = bi == k ? 1.0 : -1.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) Wn[(long long)(i0 + r0 + i) * ld + j0 + c0 + j] = sg * acc[i][j];
        return;
    }
    // other tiles: A_ij - (A_ik P) A_kj; all three tiles and the old A_ij loaded up front
    double old[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) old[i][j] = Wo[(long long)(i0 + r0 + i) * ld + j0 + c0 + j];
    tile_load(Wo, ld, i0, k0, t0);
    for (int e = threadIdx.x; e < GT * GT; e += blockDim.x) t1[(e / GT) * GS + e % GT] = P[e];
    tile_load(Wo, ld, k0, j0, t2);
    __syncthreads();
    tile_mul(t0, t1, acc);      // T = A_ik P
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t0[(r0 + i) * GS + c0 + j] = acc[i][j];
    __syncthreads();
    tile_mul(t0, t2, acc);      // T A_kj
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = old[i][j] - acc[i][j];
            Wn[(long long)(i0 + r0 + i) * ld + j0 + c0 + j] = acc[i][j];
        }
}

size_t dense_inverse_work_doubles(int n)
{
    const long long ld = ((long long)n + GT - 1) / GT * GT;
    return (size_t)(2 * ld * ld + GT * GT);
}

hipError_t launch_dense_inverse(int n, double *A, double *work, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int ld = (n + GT - 1) / GT * GT;
    const int nt = ld / GT;
    double *W[2] = {work, work + (long long)ld * ld};
    double *P = work + 2LL * ld * ld;
    auto blocks = [](long long m) { return (unsigned)((m + 255) / 256 > 65536 ? 65536 : (m + 255) / 256); };
    SPFD_LAUNCH(k_gj_pad, dim3(blocks((long long)ld * ld)), dim3(256), 0, s, n, ld, A, W[0]);
    for (int k = 0; k < nt; ++k) {
        SPFD_LAUNCH(k_gj_diag, dim3(1), dim3(1024), 0, s, ld, k * GT, W[k & 1], P);
        SPFD_LAUNCH(k_gj_step, dim3(nt, nt), dim3(256), 0, s, ld, k, W[k & 1], W[(k + 1) & 1], P);
    }
    SPFD_LAUNCH(k_gj_unpad, dim3(blocks((long long)n * n)), dim3(256), 0, s, n, ld, W[nt & 1], A);
    return hipGetLastError();
}

}  // namespace spfd
