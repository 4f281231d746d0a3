// HIP kernels of the SPFD library for gfx950 (CDNA4, wave64).
//
// Paper: Sec. II (Eqs. (1), (3)), Sec. III.A (unknowns only in conducting
// voxels), Sec. III.F (voxel-averaged field).  The multigrid method replaces
// the paper's closed-library algebraic multigrid; see engine.hip.
#include <math.h>

#include "kernels.h"
#include <hip/hip_fp16.h>

namespace spfd {

// ============================================================================
// shared per-workgroup operator state
// ============================================================================

// Label-form operator, phase 1: stage the brick's 9x9x9 conductivity tile in
// LDS (two voxels per thread; the sigma table has 256 entries, zero beyond the
// labels in use, and is read through the cache).  A barrier must follow.
template <typename T>
__device__ __forceinline__ void stage_tile(const OpArgs<T> &op, int b, T *tile)
{
    const uint8_t *tl = op.tiles + (long long)b * TILE_BYTES;
    const int i0 = threadIdx.x, i1 = threadIdx.x + NT;
    const int l0 = tl[i0];
    const int l1 = i1 < TILE_VOX ? tl[i1] : 0;
    const T s0 = op.table[l0], s1 = op.table[l1];
    tile[i0] = s0;
    if (i1 < TILE_VOX) tile[i1] = s1;
}

// weights of node t (after stage_tile and a barrier for the label form)
template <typename T>
__device__ __forceinline__ void op_weights(const OpArgs<T> &op, const T *tile, long long base, int t, int tx, int ty,
                                           int tz, const long long I[6], T W[6])
{
    if (op.w)
        stored_weights(op.w, op.stride, base, t, I, W);
    else
        tile_weights(tile, tx, ty, tz, op.geo4, W);
}

template <typename T>
__device__ __forceinline__ void op_stage(const OpArgs<T> &op, int b, T *tile)
{
    if (!op.w) {
        stage_tile(op, b, tile);
        __syncthreads();
    }
}

// ============================================================================
// setup kernels
// ============================================================================

// Mark the finest-level bricks that contain a node of a conducting voxel and
// validate labels / conductivities (err: 1 = label out of table, 2 = bad sigma).
__global__ void k_brick_flags(const uint8_t *__restrict__ labels, const double *__restrict__ table, int nlab,
                              const double *__restrict__ sig_vox, Grid g, uint8_t *flags, int *err)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
         v += (long long)gridDim.x * blockDim.x) {
        double s;
        if (sig_vox) {
            s = sig_vox[v];
            if (!(s >= 0.0) || !isfinite(s)) { *err = 2; continue; }
        } else {
            const int lab = labels[v];
            if (lab >= nlab) { *err = 1; continue; }
            s = table[lab];
        }
        if (!(s > 0.0)) continue;
        const int i = (int)(v % g.nx), j = (int)((v / g.nx) % g.ny), k = (int)(v / ((long long)g.nx * g.ny));
        for (int c = 0; c < 8; ++c) {
            const int bi = (i + (c & 1)) >> 3, bj = (j + ((c >> 1) & 1)) >> 3, bk = (k + (c >> 2)) >> 3;
            flags[bi + (long long)g.Gx * (bj + (long long)g.Gy * bk)] = 1;
        }
    }
}

// out[0]: bits of the largest weight (starts at 0), out[1]: bits of the smallest positive one (starts at
// the bits of +inf); non-negative floats order like their bit patterns
__global__ __launch_bounds__(256) void k_wmax(const float *w, long long n, unsigned *out)
{
    __shared__ float smax[4], smin[4];
    float m = 0.0f, mp = INFINITY;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float v = w[i];
        m = fmaxf(m, v);
        if (v > 0.0f) mp = fminf(mp, v);
    }
    // wave, then workgroup, then one atomic per workgroup
    for (int off = 32; off > 0; off >>= 1) {
        m = fmaxf(m, __shfl_down(m, off, 64));
        mp = fminf(mp, __shfl_down(mp, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        smax[threadIdx.x >> 6] = m;
        smin[threadIdx.x >> 6] = mp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            m = fmaxf(m, smax[k]);
            mp = fminf(mp, smin[k]);
        }
        atomicMax(out, __float_as_uint(m));
        atomicMin(out + 1, __float_as_uint(mp));
    }
}
__global__ void k_w16(const float *w, long long n, float inv, uint16_t *h)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        h[i] = __half_as_ushort(__float2half_rn(w[i] * inv));
}
hipError_t launch_wmax(const float *w, long long n, unsigned *out, hipStream_t s)
{
    SPFD_LAUNCH(k_wmax, dim3(1024), dim3(256), 0, s, w, n, out);
    return hipGetLastError();
}
hipError_t launch_w16(const float *w, long long n, float inv, uint16_t *h, hipStream_t s)
{
    SPFD_LAUNCH(k_w16, dim3(1024), dim3(256), 0, s, w, n, inv, h);
    return hipGetLastError();
}

hipError_t launch_brick_flags(const uint8_t *labels, const double *table, int nlab, const double *sig_vox,
                              const Grid &g, uint8_t *flags, int *err, hipStream_t s)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    long long blocks = (nvox + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    SPFD_LAUNCH(k_brick_flags, dim3((unsigned)blocks), dim3(256), 0, s, labels, table, nlab, sig_vox, g,
                       flags, err);
    return hipGetLastError();
}

// label tile of a brick: voxels (8*bx - 1 + a, 8*by - 1 + b, 8*bz - 1 + c), a,b,c in 0..8; outside = air (0)
__global__ void k_label_tiles(const uint8_t *__restrict__ labels, Grid g, const int4 *__restrict__ coord,
                              uint8_t *tiles)
{
    const int b = blockIdx.x;
    const int4 c = coord[b];
    for (int idx = threadIdx.x; idx < TILE_BYTES; idx += blockDim.x) {
        uint8_t lab = 0;
        if (idx < TILE_VOX) {
            const int a = idx % 9, bb = (idx / 9) % 9, cc = idx / 81;
            const int i = c.x * 8 - 1 + a, j = c.y * 8 - 1 + bb, k = c.z * 8 - 1 + cc;
            if (i >= 0 && j >= 0 && k >= 0 && i < g.nx && j < g.ny && k < g.nz)
                lab = labels[i + (long long)g.nx * (j + (long long)g.ny * k)];
        }
        tiles[(long long)b * TILE_BYTES + idx] = lab;
    }
}

hipError_t launch_label_tiles(const uint8_t *labels, const Grid &g, const int4 *coord, int nb, uint8_t *tiles,
                              hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_label_tiles, dim3(nb), dim3(256), 0, s, labels, g, coord, tiles);
    return hipGetLastError();
}

__device__ __forceinline__ double vox_sig(const uint8_t *labels, const double *table, const double *sig_vox,
                                          const Grid &g, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz) return 0.0;
    const long long v = i + (long long)g.nx * (j + (long long)g.ny * k);
    return sig_vox ? sig_vox[v] : table[labels[v]];
}

// Stored finest-level conductances M_e (Eq. (3)) for the edges to +x, +y, +z
// of every brick node: mean sigma of the 4 voxels sharing the edge times
// dual area / length.
__global__ void k_weights0(const uint8_t *__restrict__ labels, const double *__restrict__ table,
                           const double *__restrict__ sig_vox, Grid g, double gx, double gy, double gz,
                           const int4 *__restrict__ coord, double *w64, float *w32, long long stride)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const int4 c = coord[b];
    const int i = c.x * 8 + tx, j = c.y * 8 + ty, k = c.z * 8 + tz;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (i < g.Nx && j < g.Ny && k < g.Nz) {
        sx = ((vox_sig(labels, table, sig_vox, g, i, j - 1, k - 1) + vox_sig(labels, table, sig_vox, g, i, j, k - 1)) +
              vox_sig(labels, table, sig_vox, g, i, j - 1, k)) + vox_sig(labels, table, sig_vox, g, i, j, k);
        sy = ((vox_sig(labels, table, sig_vox, g, i - 1, j, k - 1) + vox_sig(labels, table, sig_vox, g, i, j, k - 1)) +
              vox_sig(labels, table, sig_vox, g, i - 1, j, k)) + vox_sig(labels, table, sig_vox, g, i, j, k);
        sz = ((vox_sig(labels, table, sig_vox, g, i - 1, j - 1, k) + vox_sig(labels, table, sig_vox, g, i, j - 1, k)) +
              vox_sig(labels, table, sig_vox, g, i - 1, j, k)) + vox_sig(labels, table, sig_vox, g, i, j, k);
    }
    const long long n = (long long)b * BS + t;
    const double wx = sx * gx, wy = sy * gy, wz = sz * gz;
    w64[n] = wx;
    w64[stride + n] = wy;
    w64[2 * stride + n] = wz;
    if (w32) {
        w32[n] = (float)wx;
        w32[stride + n] = (float)wy;
        w32[2 * stride + n] = (float)wz;
    }
}

hipError_t launch_weights0(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                           const double geo4[3], const int4 *coord, int nb, double *w64, float *w32, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_weights0, dim3(nb), dim3(NT), 0, s, labels, table, sig_vox, g, geo4[0], geo4[1], geo4[2],
                       coord, w64, w32, (long long)nb * BS);
    return hipGetLastError();
}

// Galerkin coarse operator for piecewise-constant aggregation of 2x2x2 nodes:
// the coarse conductance between aggregates I and I+e_d is the sum of the four
// fine conductances that cross their interface (fine edges from the fine
// nodes 2I+1 along d).  P^T A P of a graph Laplacian is again one.
__device__ __forceinline__ double fine_w(const double *wf, long long fstride, const int *slot_of, int fGx, int fGy,
                                         int fGz, int fNx, int fNy, int fNz, int fi, int fj, int fk, int d)
{
    if (fi >= fNx || fj >= fNy || fk >= fNz) return 0.0;
    const int bi = fi >> 3, bj = fj >> 3, bk = fk >> 3;
    if (bi >= fGx || bj >= fGy || bk >= fGz) return 0.0;
    const int sl = slot_of[bi + fGx * (bj + fGy * bk)];
    if (sl < 0) return 0.0;
    return wf[d * fstride + (long long)sl * BS + (fi & 7) + 8 * (fj & 7) + 64 * (fk & 7)];
}

__global__ void k_galerkin(const double *__restrict__ wf, long long fstride, const int *__restrict__ slot_of,
                           int fGx, int fGy, int fGz, int fNx, int fNy, int fNz, const int4 *__restrict__ ccoord,
                           double *wc64, float *wc32, long long cstride)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const int4 c = ccoord[b];
    const int I = c.x * 8 + tx, J = c.y * 8 + ty, K = c.z * 8 + tz;
    double s[3];
    s[0] = ((fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J, 2 * K, 0) +
             fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J + 1, 2 * K, 0)) +
            fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J, 2 * K + 1, 0)) +
           fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J + 1, 2 * K + 1, 0);
    s[1] = ((fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I, 2 * J + 1, 2 * K, 1) +
             fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J + 1, 2 * K, 1)) +
            fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I, 2 * J + 1, 2 * K + 1, 1)) +
           fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J + 1, 2 * K + 1, 1);
    s[2] = ((fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I, 2 * J, 2 * K + 1, 2) +
             fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J, 2 * K + 1, 2)) +
            fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I, 2 * J + 1, 2 * K + 1, 2)) +
           fine_w(wf, fstride, slot_of, fGx, fGy, fGz, fNx, fNy, fNz, 2 * I + 1, 2 * J + 1, 2 * K + 1, 2);
    const long long n = (long long)b * BS + t;
    for (int d = 0; d < 3; ++d) {
        wc64[d * cstride + n] = s[d];
        wc32[d * cstride + n] = (float)s[d];
    }
}

hipError_t launch_galerkin(const double *wf, long long fstride, const int *f_slot_of, int fGx, int fGy, int fGz,
                           int fNx, int fNy, int fNz, const int4 *ccoord, int cnb, double *wc64, float *wc32,
                           long long cstride, hipStream_t s)
{
    if (cnb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_galerkin, dim3(cnb), dim3(NT), 0, s, wf, fstride, f_slot_of, fGx, fGy, fGz, fNx, fNy, fNz,
                       ccoord, wc64, wc32, cstride);
    return hipGetLastError();
}

// ---------------------------------------------------------------- connected components
// Union-find over the nodes with D > 0 (hook the larger root under the smaller
// with compare-and-swap, path halving on the way).  Loads and stores of the
// parent array go through L2 (agent scope) so that every lane sees the hooks.
__device__ __forceinline__ int pload(const int *p, int i)
{
    return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int pfind(int *p, int x)
{
    int px = pload(p, x);
    while (px != x) {
        const int ppx = pload(p, px);
        if (ppx != px) __hip_atomic_store(p + x, ppx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = px;
        px = ppx;
    }
    return x;
}

__device__ __forceinline__ void punite(int *p, int a, int b)
{
    while (true) {
        a = pfind(p, a);
        b = pfind(p, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        int expected = b;
        if (__hip_atomic_compare_exchange_strong(p + b, &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

__global__ void k_cc_init(const double *__restrict__ w, long long stride, Topo topo, int *parent)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int nb[6];
    brick_nbrs(topo.nbr, b, nb);
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    double W[6];
    const long long base = (long long)b * BS;
    long long I[6];
    nbr_index(base, t, tx, ty, tz, nb, I);
    stored_weights(w, stride, base, t, I, W);
    parent[base + t] = diag_of(W) > 0.0 ? (int)(base + t) : -1;
}

// union-find in LDS over the conducting edges inside one brick
__device__ __forceinline__ int lfind(int *p, int x)
{
    int px = __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (px != x) {
        x = px;
        px = __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return x;
}

__device__ __forceinline__ void lunite(int *p, int a, int b)
{
    while (true) {
        a = lfind(p, a);
        b = lfind(p, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        int expected = b;
        if (__hip_atomic_compare_exchange_strong(p + b, &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
    }
}

// Components in two stages: first inside each brick (LDS, workgroup atomics),
// storing every node's brick-local root as its parent; then, after the kernel
// boundary, across the brick faces only (global union-find), so the
// device-wide atomics see short chains.
__global__ void k_cc_local(const double *__restrict__ w, long long stride, int *parent)
{
    __shared__ int lp[BS];
    const int b = blockIdx.x, t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const long long base = (long long)b * BS;
    lp[t] = parent[base + t] >= 0 ? t : -1;
    __syncthreads();
    if (tx < 7 && w[base + t] > 0.0) lunite(lp, t, t + 1);
    if (ty < 7 && w[stride + base + t] > 0.0) lunite(lp, t, t + 8);
    if (tz < 7 && w[2 * stride + base + t] > 0.0) lunite(lp, t, t + 64);
    __syncthreads();
    if (lp[t] >= 0) parent[base + t] = (int)base + lfind(lp, t);
}

// Unions across the three plus faces of a brick.  Most face edges join the
// same pair of brick-local components as the face edge next to them: a face
// node whose (own parent, neighbour's parent) pair equals that of the previous
// node on the face skips its union (same sets, already joined or about to be).
__global__ void k_cc_union(const double *__restrict__ w, long long stride, Topo topo, int *parent)
{
    __shared__ int la[BS], lb[BS];
    const int b = blockIdx.x, t = threadIdx.x;
    int nb[6];
    brick_nbrs(topo.nbr, b, nb);
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const long long base = (long long)b * BS;
    const int me = (int)(base + t);
    for (int d = 0; d < 3; ++d) {
        const bool face = d == 0 ? tx == 7 : d == 1 ? ty == 7 : tz == 7;
        const int nbk = nb[d == 0 ? NPX : d == 1 ? NPY : NPZ];
        const int other = nbk * BS + t - (d == 0 ? 7 : d == 1 ? 56 : 448);
        const bool edge = face && nbk >= 0 && w[d * stride + base + t] > 0.0;
        la[t] = edge ? pload(parent, me) : -1;
        lb[t] = edge ? pload(parent, other) : -1;
        __syncthreads();
        // previous node on the face: one step along its first in-face axis, else its second
        int prev = -1;
        if (d == 0) prev = ty > 0 ? t - 8 : (tz > 0 ? t - 64 : -1);
        else if (d == 1) prev = tx > 0 ? t - 1 : (tz > 0 ? t - 64 : -1);
        else prev = tx > 0 ? t - 1 : (ty > 0 ? t - 8 : -1);
        const bool same = prev >= 0 && la[prev] == la[t] && lb[prev] == lb[t];
        if (edge && !same) punite(parent, me, other);
        __syncthreads();
    }
}

__global__ void k_cc_flatten(int *parent, long long n, int *flag)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        int r = -1;
        if (pload(parent, (int)i) >= 0) r = pfind(parent, (int)i);
        flag[i] = (r == (int)i) ? 1 : 0;
    }
}

__global__ void k_cc_store_root(int *parent, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int p = pload(parent, (int)i);
        if (p >= 0) parent[i] = pfind(parent, (int)i);
    }
}

// exclusive scan of int flags in three passes (block sums, one-block scan of
// the sums, offsets); SCAN_CHUNK elements per block
constexpr int SCAN_CHUNK = 2048;

__global__ void k_scan_blocks(const int *__restrict__ in, long long n, int *out, int *bsum)
{
    __shared__ int s[NT];
    const long long off = (long long)blockIdx.x * SCAN_CHUNK;
    const int t = threadIdx.x;
    int v[4], tot = 0;
    for (int q = 0; q < 4; ++q) {
        const long long i = off + t * 4 + q;
        v[q] = i < n ? in[i] : 0;
        tot += v[q];
    }
    s[t] = tot;
    __syncthreads();
    for (int d = 1; d < NT; d <<= 1) {
        const int add = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int run = s[t] - tot;
    for (int q = 0; q < 4; ++q) {
        const long long i = off + t * 4 + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
    if (t == NT - 1) bsum[blockIdx.x] = s[t];
}

__global__ void k_scan_sums(int *bsum, int nblk, int *total)
{
    __shared__ int s[NT];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += NT) {
        const int i = base + t;
        const int v = i < nblk ? bsum[i] : 0;
        s[t] = v;
        __syncthreads();
        for (int d = 1; d < NT; d <<= 1) {
            const int add = t >= d ? s[t - d] : 0;
            __syncthreads();
            s[t] += add;
            __syncthreads();
        }
        if (i < nblk) bsum[i] = carry + s[t] - v;
        __syncthreads();
        if (t == NT - 1) carry += s[t];
        __syncthreads();
    }
    if (t == 0) *total = carry;
}

__global__ void k_scan_add(int *out, long long n, const int *bsum)
{
    const long long off = (long long)blockIdx.x * SCAN_CHUNK;
    const int add = bsum[blockIdx.x];
    for (int q = threadIdx.x; q < SCAN_CHUNK; q += blockDim.x) {
        const long long i = off + q;
        if (i < n) out[i] += add;
    }
}

static hipError_t scan_exclusive(const int *in, long long n, int *out, int *bsum, int *total, hipStream_t s)
{
    const long long nblk = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nblk <= 0) return hipSuccess;
    SPFD_LAUNCH(k_scan_blocks, dim3((unsigned)nblk), dim3(NT), 0, s, in, n, out, bsum);
    SPFD_LAUNCH(k_scan_sums, dim3(1), dim3(NT), 0, s, bsum, (int)nblk, total);
    SPFD_LAUNCH(k_scan_add, dim3((unsigned)nblk), dim3(NT), 0, s, out, n, bsum);
    return hipGetLastError();
}

hipError_t scan_exclusive_ints(const int *in, long long n, int *out, int *tmp, int *total, hipStream_t s)
{
    return scan_exclusive(in, n, out, tmp, total, s);
}

__global__ void k_cc_assign(const int *__restrict__ parent, const int *__restrict__ idx, long long n, int *comp)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int p = parent[i];
        comp[i] = p >= 0 ? idx[p] : -1;
    }
}

// scan_tmp needs (n/2048 + 1) ints
hipError_t launch_components(const double *w64, long long stride, Topo topo, int *parent, int *flag, int *idx,
                             int *scan_tmp, int *comp, int *counts_or_null, int *ncomp_dev, hipStream_t s)
{
    (void)counts_or_null;
    const int nb = topo.nb;
    const long long n = (long long)nb * BS;
    if (nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_cc_init, dim3(nb), dim3(NT), 0, s, w64, stride, topo, parent);
    SPFD_LAUNCH(k_cc_local, dim3(nb), dim3(NT), 0, s, w64, stride, parent);
    SPFD_LAUNCH(k_cc_union, dim3(nb), dim3(NT), 0, s, w64, stride, topo, parent);
    const unsigned gb = (unsigned)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
    SPFD_LAUNCH(k_cc_store_root, dim3(gb), dim3(256), 0, s, parent, n);
    SPFD_LAUNCH(k_cc_flatten, dim3(gb), dim3(256), 0, s, parent, n, flag);
    hipError_t e = scan_exclusive(flag, n, idx, scan_tmp, ncomp_dev, s);
    if (e != hipSuccess) return e;
    SPFD_LAUNCH(k_cc_assign, dim3(gb), dim3(256), 0, s, parent, idx, n, comp);
    return hipGetLastError();
}

__global__ void k_comp_counts(const int *__restrict__ comp, long long n, int *counts)
{
    // the first 16 component ids are counted in LDS, one global atomic per block and id
    __shared__ int local[16];
    if (threadIdx.x < 16) local[threadIdx.x] = 0;
    __syncthreads();
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = comp[i];
        if (c >= 16) atomicAdd(counts + c, 1);
        else if (c >= 0) atomicAdd(local + c, 1);
    }
    __syncthreads();
    if (threadIdx.x < 16 && local[threadIdx.x]) atomicAdd(counts + threadIdx.x, local[threadIdx.x]);
}

hipError_t launch_comp_counts(const int *comp, long long n, int *counts, hipStream_t s)
{
    const unsigned gb = (unsigned)((n + 255) / 256 > 4096 ? 4096 : (n + 255) / 256);
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_comp_counts, dim3(gb), dim3(256), 0, s, comp, n, counts);
    return hipGetLastError();
}

// ---------------------------------------------------------------- coarsest level
// Enumerate the unknowns (D > 0) of the coarsest level in node order, one
// workgroup; adj[dof][6] = neighbour unknowns or -1.
__global__ void k_coarse_enum(const double *__restrict__ w, long long stride, Topo topo, int *dof_of_node,
                              int *node_of_dof, int *adj, int *ndof, int maxdof)
{
    __shared__ int s[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    const long long n = (long long)topo.nb * BS;
    if (t == 0) carry = 0;
    __syncthreads();
    for (long long base = 0; base < n; base += 1024) {
        const long long i = base + t;
        int isdof = 0;
        if (i < n) {
            const int b = (int)(i / BS), tt = (int)(i % BS);
            int tx, ty, tz;
            brick_xyz(tt, tx, ty, tz);
            double W[6];
            long long I[6];
            nbr_index((long long)b * BS, tt, tx, ty, tz, topo.nbr + b * 6, I);
            stored_weights(w, stride, (long long)b * BS, tt, I, W);
            isdof = diag_of(W) > 0.0;
        }
        s[t] = isdof;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int add = t >= d ? s[t - d] : 0;
            __syncthreads();
            s[t] += add;
            __syncthreads();
        }
        const int id = carry + s[t] - isdof;
        if (i < n) {
            dof_of_node[i] = isdof ? id : -1;
            if (isdof && id < maxdof) node_of_dof[id] = (int)i;
        }
        __syncthreads();
        if (t == 1023) carry += s[t];
        __syncthreads();
    }
    if (t == 0) *ndof = carry;
    __syncthreads();
    // adjacency among unknowns (only meaningful when ndof <= maxdof)
    const int nd = carry < maxdof ? carry : maxdof;
    for (int q = t; q < nd; q += blockDim.x) {
        const int i = node_of_dof[q];
        const int b = i / BS, tt = i % BS;
        int tx, ty, tz;
        brick_xyz(tt, tx, ty, tz);
        const int *nb = topo.nbr + b * 6;
        int m[6];
        m[NMX] = tx > 0 ? i - 1 : (nb[NMX] >= 0 ? nb[NMX] * BS + tt + 7 : -1);
        m[NPX] = tx < 7 ? i + 1 : (nb[NPX] >= 0 ? nb[NPX] * BS + tt - 7 : -1);
        m[NMY] = ty > 0 ? i - 8 : (nb[NMY] >= 0 ? nb[NMY] * BS + tt + 56 : -1);
        m[NPY] = ty < 7 ? i + 8 : (nb[NPY] >= 0 ? nb[NPY] * BS + tt - 56 : -1);
        m[NMZ] = tz > 0 ? i - 64 : (nb[NMZ] >= 0 ? nb[NMZ] * BS + tt + 448 : -1);
        m[NPZ] = tz < 7 ? i + 64 : (nb[NPZ] >= 0 ? nb[NPZ] * BS + tt - 448 : -1);
        double W[6];
        long long I[6];
        nbr_index((long long)b * BS, tt, tx, ty, tz, nb, I);
        stored_weights(w, stride, (long long)b * BS, tt, I, W);
        for (int k = 0; k < 6; ++k) adj[q * 6 + k] = (m[k] >= 0 && W[k] > 0.0) ? dof_of_node[m[k]] : -1;
    }
}

hipError_t launch_coarse_setup(const double *w64, long long stride, Topo topo, int *dof_of_node, int *node_of_dof,
                               int *adj, int *ndof_dev, int maxdof, hipStream_t s)
{
    SPFD_LAUNCH(k_coarse_enum, dim3(1), dim3(1024), 0, s, w64, stride, topo, dof_of_node, node_of_dof, adj,
                       ndof_dev, maxdof);
    return hipGetLastError();
}

// Dense matrix of the coarsest structured level over its unknowns (row-major n x n).
__global__ void k_coarse_assemble_brick(const double *__restrict__ w, long long stride, Topo topo,
                                        const int *__restrict__ node_of_dof, const int *__restrict__ adj, int n,
                                        double *A)
{
    const int t = threadIdx.x, nt = blockDim.x;
    for (long long e = t; e < (long long)n * n; e += nt) A[e] = 0.0;
    __syncthreads();
    for (int q = t; q < n; q += nt) {
        const int i = node_of_dof[q];
        const int b = i / BS, tt = i % BS;
        int tx, ty, tz;
        brick_xyz(tt, tx, ty, tz);
        double W[6];
        long long I[6];
        nbr_index((long long)b * BS, tt, tx, ty, tz, topo.nbr + b * 6, I);
        stored_weights(w, stride, (long long)b * BS, tt, I, W);
        double d = 0.0;
        for (int k = 0; k < 6; ++k) {
            const int m = adj[q * 6 + k];
            if (m >= 0) {
                A[(long long)q * n + m] -= W[k];
                d += W[k];
            }
        }
        A[(long long)q * n + q] += d;
    }
}

// Dense pseudo-inverse of the coarsest (singular) operator, in place: A_c +
// sum over components c of alpha_c 1_c 1_c^T is SPD, and for a right side
// orthogonal to every 1_c its solution has zero mean per component, i.e.
// equals A_c^+ r.  One workgroup: components by min-label propagation over
// the nonzeros, regularisation with alpha_c = mean diagonal / size^2, and
// Gauss-Jordan inversion (no pivoting needed for an SPD matrix).
// work: 2n ints + n doubles.
// Column masks of a structured level: bit tx + 8 ty of brick b is set when a
// node (tx,ty,*) of the brick has a positive diagonal (is an unknown).
__global__ __launch_bounds__(NT) void k_col_masks(const double *__restrict__ w, long long stride, Topo topo,
                                                  unsigned long long *__restrict__ mask)
{
    __shared__ unsigned long long m;
    const int bk = blockIdx.x;
    const int t = threadIdx.x;
    if (t == 0) m = 0ull;
    __syncthreads();
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    int nb[6];
    brick_nbrs(topo.nbr, bk, nb);
    const long long base = (long long)bk * BS;
    long long I[6];
    nbr_index(base, t, tx, ty, tz, nb, I);
    double W[6];
    stored_weights(w, stride, base, t, I, W);
    if (diag_of(W) > 0.0) atomicOr(&m, 1ull << (t & 63));
    __syncthreads();
    if (t == 0) mask[bk] = m;
}

// inverse diagonals of a structured level from its stored weights (0 where the diagonal vanishes)
__global__ __launch_bounds__(NT) void k_dinv_struct(const double *__restrict__ w, long long stride, Topo topo,
                                                    double *__restrict__ d64, float *__restrict__ d32)
{
    const int bk = blockIdx.x;
    const int t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    int nb[6];
    brick_nbrs(topo.nbr, bk, nb);
    const long long base = (long long)bk * BS;
    long long I[6];
    nbr_index(base, t, tx, ty, tz, nb, I);
    double W[6];
    stored_weights(w, stride, base, t, I, W);
    const double D = diag_of(W);
    const double v = D > 0.0 ? 1.0 / D : 0.0;
    d64[base + t] = v;
    d32[base + t] = (float)v;
}

hipError_t launch_dinv_struct(const double *w64, long long stride, Topo topo, double *d64, float *d32, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_dinv_struct, dim3(topo.nb), dim3(NT), 0, s, w64, stride, topo, d64, d32);
    return hipGetLastError();
}

hipError_t launch_col_masks(const double *w64, long long stride, Topo topo, unsigned long long *mask, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    Topo tp{topo.nb, topo.nbr, nullptr};
    SPFD_LAUNCH(k_col_masks, dim3(topo.nb), dim3(NT), 0, s, w64, stride, tp, mask);
    return hipGetLastError();
}

// Make the coarsest matrix definite: A += sum over its connected components c
// of (mean diagonal of c / |c|) 1_c 1_c^T.  For right sides with zero sum per
// component the inverse of the result applies the pseudo-inverse and returns
// the solution with zero sum per component.  Three kernels: the sparsity
// pattern as adjacency lists (one wave per row, many workgroups), the
// components by minimum-label propagation and their diagonal sums (one
// workgroup), the rank-one updates (many workgroups).
constexpr int CMAXADJ = 64;

struct CoarseWork {
    int *comp, *csize, *deg, *adj;  // labels, component sizes, row degree (-1: dense row), [n][CMAXADJ]
    double *cdiag;                  // diagonal sum per component (indexed by the component's label)
};

__host__ __device__ inline CoarseWork coarse_work(int n, int *work)
{
    CoarseWork w;
    w.comp = work;
    w.csize = work + n;
    w.cdiag = (double *)(work + 2 * n + ((2 * n) & 1));
    w.deg = work + 4 * n + 2;
    w.adj = w.deg + n;
    return w;
}

__global__ __launch_bounds__(256) void k_creg_pattern(int n, const double *__restrict__ A, int *work)
{
    const CoarseWork w = coarse_work(n, work);
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= n) return;
    if (lane == 0) {
        w.comp[q] = q;
        w.csize[q] = 0;
    }
    int d = 0;
    for (int m0 = 0; m0 < n; m0 += 64) {
        const int m = m0 + lane;
        const bool nz = m < n && m != q && A[(long long)q * n + m] != 0.0;
        const unsigned long long bal = __ballot(nz);
        const int pos = d + __popcll(bal & ((1ull << lane) - 1ull));
        if (nz && d >= 0 && pos < CMAXADJ) w.adj[(long long)q * CMAXADJ + pos] = m;
        if (d >= 0) d += __popcll(bal);
        if (d > CMAXADJ) d = -1;
    }
    if (lane == 0) w.deg[q] = d;
}

__global__ __launch_bounds__(1024) void k_creg_components(int n, const double *__restrict__ A, int *work)
{
    const CoarseWork w = coarse_work(n, work);
    const int t = threadIdx.x, nt = blockDim.x;
    __shared__ int changed;
    // minimum label over each component: neighbour minima plus pointer jumping
    do {
        __syncthreads();
        if (t == 0) changed = 0;
        __syncthreads();
        for (int q = t; q < n; q += nt) {
            int c = __hip_atomic_load(w.comp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int d = w.deg[q];
            const int cnt = d >= 0 ? d : n;
            for (int k = 0; k < cnt; ++k) {
                const int m = d >= 0 ? w.adj[(long long)q * CMAXADJ + k] : k;
                if (d < 0 && (m == q || A[(long long)q * n + m] == 0.0)) continue;
                const int cm = __hip_atomic_load(w.comp + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (cm < c) c = cm;
            }
            const int cc = __hip_atomic_load(w.comp + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cc < c) c = cc;
            if (c < __hip_atomic_load(w.comp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                __hip_atomic_store(w.comp + q, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                changed = 1;
            }
        }
        __syncthreads();
    } while (changed);
    for (int q = t; q < n; q += nt) atomicAdd(w.csize + w.comp[q], 1);
    // per-component diagonal sums in a fixed order (deterministic): diagonal and labels staged in LDS
    __shared__ double sdiag[1024], ssum[1024];
    __shared__ int scomp[1024];
    for (int q = t; q < n; q += nt) {
        sdiag[q] = A[(long long)q * n + q];
        scomp[q] = w.comp[q];
        ssum[q] = 0.0;
    }
    __syncthreads();
    if (t == 0)
        for (int q = 0; q < n; ++q) ssum[scomp[q]] += sdiag[q];
    __syncthreads();
    for (int q = t; q < n; q += nt) w.cdiag[q] = ssum[q];
}

__global__ __launch_bounds__(256) void k_creg_update(int n, double *A, const int *work)
{
    const CoarseWork w = coarse_work(n, const_cast<int *>(work));
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)n * n;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        const int c = w.comp[i];
        if (w.comp[j] == c) {
            const double sz = (double)w.csize[c];
            A[e] += (w.cdiag[c] / sz) / sz;
        }
    }
}

hipError_t launch_coarse_assemble_brick(const double *w64, long long stride, Topo topo, const int *node_of_dof,
                                        const int *adj, int n, double *A, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_coarse_assemble_brick, dim3(1), dim3(1024), 0, s, w64, stride, topo, node_of_dof, adj, n, A);
    return hipGetLastError();
}

size_t coarse_factor_work_ints(int n) { return (size_t)(5 + CMAXADJ) * n + 8; }

hipError_t launch_coarse_factor(int n, double *A, int *work, double *dwork, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_creg_pattern, dim3((n + 3) / 4), dim3(256), 0, s, n, A, work);
    SPFD_LAUNCH(k_creg_components, dim3(1), dim3(1024), 0, s, n, A, work);
    const long long nn = (long long)n * n;
    SPFD_LAUNCH(k_creg_update, dim3((unsigned)((nn + 255) / 256 > 4096 ? 4096 : (nn + 255) / 256)), dim3(256), 0, s,
                n, A, work);
    HIP_RETURN_IF(hipGetLastError());
    return launch_dense_inverse(n, A, dwork, s);
    return hipGetLastError();
}

// ============================================================================
// solve kernels
// ============================================================================

template <typename T>
__global__ void k_fill(T *x, long long n, T v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T>
hipError_t launch_fill(T *x, long long n, T v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned gb = (unsigned)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
    SPFD_LAUNCH(k_fill<T>, dim3(gb), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(double *, long long, double, hipStream_t);
template hipError_t launch_fill<float>(float *, long long, float, hipStream_t);
template hipError_t launch_fill<int>(int *, long long, int, hipStream_t);

// start of a solve: keeps ||b||^2 from the right-side kernel, arms the stop test
__global__ void k_scal_init(Scal *sc, double tol, int use_x0)
{
    (void)use_x0;
    sc += blockIdx.x;
    if (threadIdx.x == 0) {
        const double bb = sc->bb;
        sc->rz = 0.0; sc->pq = 0.0; sc->alpha = 0.0; sc->beta = 0.0; sc->zq = 0.0;
        sc->rr = bb;
        sc->tol2 = tol * tol * bb;
        sc->done = bb > 0.0 ? 0 : 1;
        sc->iters = 0; sc->status = 0; sc->hcount = 0; sc->happlied = 0; sc->pad = 0;
    }
}

hipError_t launch_scal_init(Scal *sc, double tol, int use_x0, int nbatch, hipStream_t s)
{
    SPFD_LAUNCH(k_scal_init, dim3(nbatch), dim3(64), 0, s, sc, tol, use_x0);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// Every reduction is two-stage and deterministic: each brick workgroup stores
// its partial sum with a plain store, and after the kernel boundary one
// workgroup (k_finish) sums the partials in a fixed order and updates the
// scalars of the solve.  No grid-wide fence is needed inside a kernel.

__device__ __forceinline__ double block_sum_any(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ void store_mirror(Scal *mirror, const Scal *sc)
{
    if (mirror) mirror[blockIdx.x] = *sc;
}

// rows.used: row r sums its first rows.n[r] partials (packed models: each model's own count), else n;
// the second set of partials (z.q) starts at part + n in every row
__global__ __launch_bounds__(1024) void k_finish(const double *__restrict__ part, int n, int mode, Scal *sc,
                                                 int max_iter, double *means, const int *counts, int comp, int ps,
                                                 Scal *mirror, FinRows rows)
{
    __shared__ double red[16];
    part += (long long)blockIdx.x * ps;
    if (sc) sc += blockIdx.x;
    // a stopped right side keeps its scalars; the flag is loaded with the partials and tested after them
    // (a test first would put one more memory round trip before the loads)
    const bool may_stop =
        mode == FIN_ALPHA || mode == FIN_RR || mode == FIN_BETA0 || mode == FIN_BETA || mode == FIN_BETA_STD;
    const int stopped = may_stop ? sc->done : 0;
    const int nr = rows.used ? rows.n[blockIdx.x] : n;
    // eight independent loads in flight per thread and round, summed in a fixed order (deterministic)
    constexpr int U = 8;
    const int nt = blockDim.x;
    double a = 0.0, b = 0.0;
    for (int i0 = threadIdx.x; i0 < nr; i0 += U * nt) {
        double v[U], w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nt;
            v[u] = i < nr ? part[i] : 0.0;
            w[u] = mode == FIN_BETA && i < nr ? part[n + i] : 0.0;
        }
        a += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        b += ((w[0] + w[1]) + (w[2] + w[3])) + ((w[4] + w[5]) + (w[6] + w[7]));
    }
    if (stopped) {
        if (threadIdx.x == 0) store_mirror(mirror, sc);
        return;
    }
    a = block_sum_any(a, red);
    if (mode == FIN_BETA) b = block_sum_any(b, red);
    if (threadIdx.x != 0) return;
    switch (mode) {
    case FIN_BB:
        sc->bb = a;
        break;
    case FIN_ALPHA: {
        sc->pq = a;
        double alpha = sc->rz / a;
        if (!(a > 0.0) || !isfinite(alpha)) {
            alpha = 0.0;
            sc->status = 6;
            sc->done = 1;
        }
        sc->alpha = alpha;
        break;
    }
    case FIN_RR:
        sc->rr = a;
        sc->iters += 1;
        sc->hcount += 1;   // the step's search direction and step size are kept
        if (a <= sc->tol2) {
            sc->done = 1;
        } else if (!isfinite(a)) {
            sc->status = 6;
            sc->done = 1;
        } else if (sc->iters >= max_iter) {
            sc->status = 5;
            sc->done = 1;
        }
        break;
    case FIN_BETA0:
    case FIN_BETA:
    case FIN_BETA_STD: {
        double beta = 0.0;
        if (mode == FIN_BETA) beta = -sc->alpha * b / sc->rz;
        if (mode == FIN_BETA_STD) beta = a / sc->rz;
        if (!(a > 0.0) || !isfinite(beta)) {
            sc->status = 6;
            sc->done = 1;
            beta = 0.0;
        }
        sc->zq = b;
        sc->rz = a;
        sc->beta = beta;
        break;
    }
    case FIN_RESID0:
        sc->rr = a;
        if (a <= sc->tol2) sc->done = 1;
        break;
    case FIN_RESID1:
        sc->zq = a;
        break;
    case FIN_MEAN:
        means[comp] = counts[comp] > 0 ? a / (double)counts[comp] : 0.0;
        break;
    }
    if (sc) store_mirror(mirror, sc);
}

hipError_t launch_finish(const double *part, int n, int mode, Scal *sc, int max_iter, hipStream_t s, double *means,
                         const int *counts, int comp, int nbatch, int ps, Scal *mirror, const FinRows *rows)
{
    if (mirror && !sc) return hipErrorInvalidValue;
    if (rows && rows->used && nbatch > MAX_MODELS) return hipErrorInvalidValue;
    const FinRows fr = rows ? *rows : FinRows{};
    SPFD_LAUNCH(k_finish, dim3(nbatch), dim3(1024), 0, s, part, n, mode, sc, max_iter, means, counts, comp, ps,
                mirror, fr);
    return hipGetLastError();
}

// b = -G^T M a on the unknowns of the finest level (Eq. (3), right side):
// b_n = sum over edges leaving n of M_e a_e - sum over edges entering n of M_e a_e,
// and ||b||^2.  a is read only on conducting edges (M_e > 0), which all lie in the grid.
// With packed models (topo.np > 0, one launch row): g is the model's grid, zoff its first node layer in
// the packed grid, and the bricks are the model's.
template <bool LABEL>
__global__ __launch_bounds__(NT) void k_rhs(OpArgs<double> op, Topo topo, const int4 *__restrict__ coord, Grid g,
                                            int zoff, const double *__restrict__ a, double *b, double *part)
{
    __shared__ double tile[TILE_VOX + 7];
    __shared__ double red[8];
    int loc;
    const int bk = topo_brick(topo, loc);
    if (bk < 0) return;
    int nb[6];
    brick_nbrs(topo.nbr, bk, nb);
    const int t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const long long base = (long long)bk * BS;
    long long I[6];
    nbr_index(base, t, tx, ty, tz, nb, I);
    op_stage(op, bk, tile);
    double W[6];
    op_weights(op, tile, base, t, tx, ty, tz, I, W);
    const int4 c = coord[bk];
    const long long i = c.x * 8 + tx, j = c.y * 8 + ty, k = c.z * 8 + tz - zoff;
    const long long n = i + (long long)g.Nx * (j + (long long)g.Ny * k);
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    double s = 0.0;
    if (W[NPX] != 0.0) s += W[NPX] * a[n];
    if (W[NMX] != 0.0) s -= W[NMX] * a[n - 1];
    if (W[NPY] != 0.0) s += W[NPY] * a[nn + n];
    if (W[NMY] != 0.0) s -= W[NMY] * a[nn + n - g.Nx];
    if (W[NPZ] != 0.0) s += W[NPZ] * a[2 * nn + n];
    if (W[NMZ] != 0.0) s -= W[NMZ] * a[2 * nn + n - (long long)g.Nx * g.Ny];
    b[base + t] = s;
    const double tot = block_sum(s * s, red);
    if (t == 0) part[loc] = tot;
}

hipError_t launch_rhs(const OpArgs<double> &op, Topo topo, const int4 *coord, const Grid &g, const double *a,
                      double *b, double *part, Scal *sc, hipStream_t s, int zoff)
{
    if (topo.nb <= 0) return hipSuccess;
    if (topo.np > 1) return hipErrorInvalidValue;   // one model per call
    const dim3 grid(xcd_grid(topo_count(topo)));
    if (op.w)
        SPFD_LAUNCH(k_rhs<false>, grid, dim3(NT), 0, s, op, topo, coord, g, zoff, a, b, part);
    else
        SPFD_LAUNCH(k_rhs<true>, grid, dim3(NT), 0, s, op, topo, coord, g, zoff, a, b, part);
    return hipGetLastError();
}

// x += sum_j alpha_j p_j over the search directions kept in the window and not yet added (slots happlied ..
// hcount-1, filled in step order), in step order: x receives the same sequence of updates as with one
// update per step, whatever the window length and whenever the updates happen.  k_hist_reset then starts
// the next window (full) or marks the directions added (an update before the window is full).
template <typename TP>
__global__ __launch_bounds__(NT) void k_x_flush(Topo topo, double *__restrict__ x, const TP *__restrict__ ph,
                                                long long hs, const double *__restrict__ ahist, int nh, long long vs,
                                                const Scal *sc)
{
    int loc;
    const int bk = topo_brick(topo, loc);
    if (bk < 0) return;
    const double *ah = ahist + (long long)blockIdx.y * nh;
    const int m = min(sc[blockIdx.y].hcount, nh);
    const int lo = max(sc[blockIdx.y].happlied, 0);
    if (m <= lo) return;
    // a node column without unknowns holds zeros in x and every p: nothing to read or write
    if (topo.cmask && !((topo.cmask[bk] >> (threadIdx.x & 63)) & 1ull)) return;
    const long long n = blockIdx.y * vs + (long long)bk * BS + threadIdx.x;
    // every direction's load in flight (fully unrolled, wave-uniform conditions: no indexed private
    // array), then the updates in step order
    double a[MAX_PHIST];
    TP pv[MAX_PHIST];
#pragma unroll
    for (int j = 0; j < MAX_PHIST; ++j) {
        a[j] = 0.0;
        pv[j] = TP(0);
        if (j >= lo && j < m) {
            a[j] = ah[j];
            pv[j] = ph[(long long)j * hs + n];
        }
    }
    double xv = x[n];
#pragma unroll
    for (int j = 0; j < MAX_PHIST; ++j)
        if (j >= lo && j < m) xv = __builtin_fma(a[j], (double)pv[j], xv);
    x[n] = xv;
}

// full: the next window starts empty; else the window goes on, its directions so far marked as added
__global__ void k_hist_reset(Scal *sc, int n, int full)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (full) {
        sc[i].hcount = 0;
        sc[i].happlied = 0;
    } else {
        sc[i].happlied = sc[i].hcount;
    }
}

template <typename TP>
hipError_t launch_x_flush(Topo topo, double *x, const TP *ph, long long hs, const double *ahist, int nh, Scal *sc,
                          const Batch &bt, hipStream_t s, int full)
{
    if (topo.nb <= 0 || bt.n <= 0) return hipSuccess;
    if (nh < 2 || nh > MAX_PHIST || !ph || !ahist || !sc) return hipErrorInvalidValue;
    SPFD_LAUNCH(k_x_flush<TP>, dim3(xcd_grid(topo_count(topo)), bt.n), dim3(NT), 0, s, topo, x, ph, hs, ahist, nh,
                bt.vs, sc);
    SPFD_LAUNCH(k_hist_reset, dim3((bt.n + 63) / 64), dim3(64), 0, s, sc, bt.n, full);
    return hipGetLastError();
}
template hipError_t launch_x_flush<float>(Topo, double *, const float *, long long, const double *, int, Scal *,
                                          const Batch &, hipStream_t, int);
template hipError_t launch_x_flush<double>(Topo, double *, const double *, long long, const double *, int, Scal *,
                                           const Batch &, hipStream_t, int);

// r -= alpha q, ||r||^2 partials and the FP32 copy of r (x is updated once per window of steps, k_x_flush)
__global__ __launch_bounds__(NT) void k_rupdate(Topo topo, double *__restrict__ r, const double *__restrict__ q,
                                                double *part, const Scal *sc, long long vs, int ps,
                                                float *__restrict__ r32, double *ahist, int nh)
{
    __shared__ double red[8];
    sc += blockIdx.y;
    // the step size of this search direction (window slot hcount), for the update of x at the window's end
    if (blockIdx.x == 0 && threadIdx.x == 0 && sc->done == 0 && sc->hcount < nh)
        ahist[blockIdx.y * nh + sc->hcount] = sc->alpha;
    int loc;
    const int bk = topo_brick(topo, loc);
    if (bk < 0) return;
    const long long n = blockIdx.y * vs + (long long)bk * BS + threadIdx.x;
    // The loads do not wait for the stop flag (a test before them would cost one more memory round
    // trip): a stopped right side loads, but stores nothing.
    const double rv = r[n], qv = q[n];
    const bool run = sc->done == 0;
    const double rn = rv - sc->alpha * qv;
    if (run) {
        r[n] = rn;
        if (r32) r32[n] = (float)rn;
    }
    const double tot = block_sum(run ? rn * rn : 0.0, red);
    if (threadIdx.x == 0 && run) part[(long long)blockIdx.y * ps + loc] = tot;
}

hipError_t launch_rupdate(Topo topo, double *r, const double *q, double *part, Scal *sc, const Batch &bt, float *r32,
                          hipStream_t s, double *ahist, int nh)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!ahist || nh < 2 || nh > MAX_PHIST) return hipErrorInvalidValue;
    SPFD_LAUNCH(k_rupdate, dim3(xcd_grid(topo_count(topo)), bt.n), dim3(NT), 0, s, topo, r, q, part, sc, bt.vs,
                bt.ps, r32, ahist, nh);
    return hipGetLastError();
}

// partials of r.z and z.q (flexible beta follows in k_finish)
template <typename TZ>
__global__ __launch_bounds__(NT) void k_dots(Topo topo, const TZ *__restrict__ z, const double *__restrict__ r,
                                             const double *__restrict__ q, double *part, const Scal *sc, int first,
                                             long long vs, int ps)
{
    __shared__ double red[8];
    sc += blockIdx.y;
    if (sc->done) return;
    int loc;
    const int bk = topo_brick(topo, loc);
    if (bk < 0) return;
    z += blockIdx.y * vs;
    r += blockIdx.y * vs;
    q += blockIdx.y * vs;
    part += (long long)blockIdx.y * ps;
    const long long n = (long long)bk * BS + threadIdx.x;
    const double zv = (double)z[n];
    const double a = block_sum(zv * r[n], red);
    const double c = first ? 0.0 : block_sum(zv * q[n], red);
    if (threadIdx.x == 0) {
        // z.q partials follow the topo_count(topo) partials of r.z
        part[loc] = a;
        part[topo_count(topo) + loc] = c;
    }
}

template <typename TZ>
hipError_t launch_dots(Topo topo, const TZ *z, const double *r, const double *q, double *part, Scal *sc, int first,
                       const Batch &bt, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_dots<TZ>, dim3(xcd_grid(topo_count(topo)), bt.n), dim3(NT), 0, s, topo, z, r, q, part, sc, first,
                bt.vs, bt.ps);
    return hipGetLastError();
}
template hipError_t launch_dots<double>(Topo, const double *, const double *, const double *, double *, Scal *, int,
                                        const Batch &, hipStream_t);
template hipError_t launch_dots<float>(Topo, const float *, const double *, const double *, double *, Scal *, int,
                                       const Batch &, hipStream_t);

template <typename TZ>
__global__ __launch_bounds__(NT) void k_pupdate(Topo topo, const TZ *__restrict__ z, double *__restrict__ p,
                                                const Scal *sc, int first, long long vs)
{
    sc += blockIdx.y;
    if (sc->done) return;
    int loc;
    const int bk = topo_brick(topo, loc);
    if (bk < 0) return;
    z += blockIdx.y * vs;
    p += blockIdx.y * vs;
    const long long n = (long long)bk * BS + threadIdx.x;
    const double zv = (double)z[n];
    p[n] = first ? zv : zv + sc->beta * p[n];
}

template <typename TZ>
hipError_t launch_pupdate(Topo topo, const TZ *z, double *p, const Scal *sc, int first, const Batch &bt,
                          hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_pupdate<TZ>, dim3(xcd_grid(topo_count(topo)), bt.n), dim3(NT), 0, s, topo, z, p, sc, first, bt.vs);
    return hipGetLastError();
}
template hipError_t launch_pupdate<double>(Topo, const double *, double *, const Scal *, int, const Batch &,
                                           hipStream_t);
template hipError_t launch_pupdate<float>(Topo, const float *, double *, const Scal *, int, const Batch &, hipStream_t);

// ---------------------------------------------------------------- multigrid level kernels
__device__ __forceinline__ bool stopped(const Scal *sc)
{
    return sc && sc[blockIdx.y].done;   // written by an earlier kernel only: a plain (scalar) load
}

// x += s * P x_c
template <typename T>
__global__ __launch_bounds__(NT) void k_prolong(Topo topo, T *__restrict__ x, const T *__restrict__ xc,
                                                const int *__restrict__ parent_slot, const int4 *__restrict__ fcoord,
                                                T scale, const Scal *sc, long long vs, long long vsc)
{
    if (stopped(sc)) return;
    const int bk = xcd_brick(blockIdx.x, topo.nb);
    if (bk < 0) return;
    x += blockIdx.y * vs;
    xc += blockIdx.y * vsc;
    const int t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const int4 c = fcoord[bk];
    const int cxl = (c.x & 1) * 4 + (tx >> 1), cyl = (c.y & 1) * 4 + (ty >> 1), czl = (c.z & 1) * 4 + (tz >> 1);
    const long long n = (long long)bk * BS + t;
    x[n] += scale * xc[(long long)parent_slot[bk] * BS + cxl + 8 * cyl + 64 * czl];
}

// coarsest solve z_c = A_c^+ r_c (dense FP64 GEMV); 4 rows per workgroup of 256
template <typename T, typename TB>
__global__ __launch_bounds__(256) void k_coarse_apply(const TB *__restrict__ bc, T *__restrict__ xc,
                                                      const double *__restrict__ Ainv,
                                                      const int *__restrict__ node_of_dof, int n, const Scal *sc,
                                                      long long vs)
{
    __shared__ double rv[1024];
    bc += blockIdx.y * vs;
    xc += blockIdx.y * vs;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + wv;
    // the wave's row of the inverse is loaded first (n <= 1024: 16 values per
    // lane), in flight together with the gather of b_c and the stop flag
    const double *a = Ainv + (long long)(row < n ? row : n - 1) * n;
    double av[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = lane + 64 * k;
        av[k] = a[j < n ? j : n - 1];
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) rv[i] = (double)bc[node_of_dof[i]];
    const bool stop = stopped(sc);
    __syncthreads();
    if (stop || row >= n) return;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = lane + 64 * k;
        if (j < n) s += av[k] * rv[j];
    }
    s = wave_sum(s);
    if (lane == 0) xc[node_of_dof[row]] = (T)s;
}

template <typename T>
hipError_t launch_prolong(Topo topo, T *x, const T *xc, const int *parent_slot, const int4 *fcoord, T scale,
                          const Scal *sc, const Batch &bt, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_prolong<T>, dim3(xcd_grid(topo.nb), bt.n), dim3(NT), 0, s, topo, x, xc, parent_slot, fcoord,
                       scale, sc, bt.vs, bt.vsc);
    return hipGetLastError();
}

template <typename T, typename TB>
hipError_t launch_coarse_apply(const TB *bc, T *xc, const double *Ainv, const int *node_of_dof, int n, const Scal *sc,
                               const Batch &bt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > 1024) return hipErrorInvalidValue;
    SPFD_LAUNCH((k_coarse_apply<T, TB>), dim3((n + 3) / 4, bt.n), dim3(256), 0, s, bc, xc, Ainv, node_of_dof, n,
                       sc, bt.vs);
    return hipGetLastError();
}

template hipError_t launch_prolong<double>(Topo, double *, const double *, const int *, const int4 *, double,
                                           const Scal *, const Batch &, hipStream_t);
template hipError_t launch_prolong<float>(Topo, float *, const float *, const int *, const int4 *, float, const Scal *,
                                          const Batch &, hipStream_t);
template hipError_t launch_coarse_apply<double, double>(const double *, double *, const double *, const int *, int,
                                                        const Scal *, const Batch &, hipStream_t);
template hipError_t launch_coarse_apply<float, float>(const float *, float *, const double *, const int *, int,
                                                      const Scal *, const Batch &, hipStream_t);
template hipError_t launch_coarse_apply<float, double>(const double *, float *, const double *, const int *, int,
                                                       const Scal *, const Batch &, hipStream_t);

// ============================================================================
// gauge, output, post-processing
// ============================================================================

// Component means in a fixed summation order (bitwise reproducible for any
// number of components): up to COMP_PASS components per pass; every brick
// workgroup forms the sum of each component over its 512 nodes (wave sums,
// then the eight waves in order) and stores one partial per (component,
// brick); one workgroup per component then adds its partials in brick order.
constexpr int COMP_PASS = 16;

__global__ __launch_bounds__(NT) void k_comp_sum(Topo topo, const double *__restrict__ x, const int *__restrict__ comp,
                                                 int c0, int nk, double *part)
{
    __shared__ double red[COMP_PASS][NT / 64];
    const int bk = xcd_brick(blockIdx.x, topo.nb);
    if (bk < 0) return;
    const long long n = (long long)bk * BS + threadIdx.x;
    const int c = comp[n] - c0;
    const double v = x[n];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < nk; ++k) {
        const double t = wave_sum(c == k ? v : 0.0);
        if (lane == 0) red[k][wv] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < nk) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += red[threadIdx.x][w];
        part[(long long)threadIdx.x * topo.nb + bk] = t;
    }
}

// mean of component c0 + blockIdx.x: its nb partials summed in a fixed order
__global__ __launch_bounds__(1024) void k_comp_finish(const double *__restrict__ part, int nb, int c0,
                                                      const int *__restrict__ counts, double *means)
{
    __shared__ double red[16];
    const int k = blockIdx.x;
    const double *p = part + (long long)k * nb;
    double t = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) t += p[i];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        const int cnt = counts[c0 + k];
        means[c0 + k] = cnt > 0 ? s / (double)cnt : 0.0;
    }
}

size_t comp_mean_parts(int nb) { return (size_t)COMP_PASS * (nb > 0 ? nb : 1); }

hipError_t launch_comp_mean(Topo topo, const double *x, const int *comp, int ncomp, const int *counts, double *means,
                            double *part, hipStream_t s)
{
    if (topo.nb <= 0 || ncomp <= 0) return hipSuccess;
    for (int c0 = 0; c0 < ncomp; c0 += COMP_PASS) {
        const int nk = ncomp - c0 < COMP_PASS ? ncomp - c0 : COMP_PASS;
        SPFD_LAUNCH(k_comp_sum, dim3(xcd_grid(topo.nb)), dim3(NT), 0, s, topo, x, comp, c0, nk, part);
        SPFD_LAUNCH(k_comp_finish, dim3(nk), dim3(1024), 0, s, part, topo.nb, c0, counts, means);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- several voxel models in one handle
// model m's labels (nx, ny, nz voxels) into the packed label grid (NX, NY voxels per layer) from voxel
// layer zoff on; the rest of the packed grid stays as it is (air)
__global__ void k_pack_labels(const uint8_t *__restrict__ src, int nx, int ny, int nz, uint8_t *__restrict__ dst,
                              int NX, int NY, int zoff)
{
    const long long n = (long long)nx * ny * nz;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long long)nx * ny));
        dst[i + (long long)NX * (j + (long long)NY * (k + zoff))] = src[v];
    }
}

hipError_t launch_pack_labels(const uint8_t *src, int nx, int ny, int nz, uint8_t *dst, int NX, int NY, int zoff,
                              hipStream_t s)
{
    const long long n = (long long)nx * ny * nz;
    const unsigned gb = (unsigned)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
    SPFD_LAUNCH(k_pack_labels, dim3(gb), dim3(256), 0, s, src, nx, ny, nz, dst, NX, NY, zoff);
    return hipGetLastError();
}

// conductivity of every voxel of the packed grid: its model's table at its label (tables [np][256]),
// 0 outside every model's box
__global__ void k_pack_sigma(const uint8_t *__restrict__ labels, Grid g, ModelBoxes mb,
                             const double *__restrict__ tables, double *__restrict__ sig)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(v % g.nx), j = (int)((v / g.nx) % g.ny), k = (int)(v / ((long long)g.nx * g.ny));
        double sv = 0.0;
        for (int m = 0; m < mb.np; ++m)
            if (k >= mb.zoff[m] && k < mb.zoff[m] + mb.nz[m] && i < mb.nx[m] && j < mb.ny[m])
                sv = tables[m * MAX_LABELS + labels[v]];
        sig[v] = sv;
    }
}

hipError_t launch_pack_sigma(const uint8_t *labels, const Grid &g, const ModelBoxes &mb, const double *tables,
                             double *sig, hipStream_t s)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    const unsigned gb = (unsigned)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
    SPFD_LAUNCH(k_pack_sigma, dim3(gb), dim3(256), 0, s, labels, g, mb, tables, sig);
    return hipGetLastError();
}

// dense node array from the brick layout: psi = x - mean(component), 0 outside the conductor.  g: the
// output's grid; gb: the grid of the brick layout (the same, or the packed grid of several models, in
// which the output's model starts at node layer zoff)
constexpr int PSI_ROWS = 8;   // node rows per workgroup: the eight y rows of one brick row

__global__ __launch_bounds__(256) void k_psi_out(const double *__restrict__ x, const int *__restrict__ comp,
                                                 const double *__restrict__ means, const int *__restrict__ slot_of,
                                                 Grid g, Grid gb, int zoff, double *psi)
{
    // workgroup: node rows j0..j0+7 of layer k (contiguous stores, no 64-bit index division).  The eight
    // rows lie in the same bricks, so one slot lookup per lane serves all of them, and each lane keeps the
    // eight rows' loads in flight together.  Rows past the grid's end (the last brick row) are loaded, as
    // they lie inside their bricks, but not stored.
    const int gy = (g.Ny + PSI_ROWS - 1) / PSI_ROWS;
    const int jb = blockIdx.x % gy, k = blockIdx.x / gy;
    const int kb = k + zoff, j0 = jb * PSI_ROWS;
    const int nr = g.Ny - j0 < PSI_ROWS ? g.Ny - j0 : PSI_ROWS;
    const int *srow = slot_of + gb.Gx * (jb + gb.Gy * (kb >> 3));
    double *prow = psi + ((long long)k * g.Ny + j0) * g.Nx;
    for (int i = threadIdx.x; i < g.Nx; i += blockDim.x) {
        const int sl = srow[i >> 3];
        // slot 0 stands in outside the bricks; the values are masked below
        const long long base = sl >= 0 ? (long long)sl * BS + (i & 7) + 64 * (kb & 7) : 0;
        int c[PSI_ROWS];
        double xv[PSI_ROWS];
#pragma unroll
        for (int r = 0; r < PSI_ROWS; ++r) {
            const long long idx = sl >= 0 ? base + 8 * r : 0;
            c[r] = comp[idx];
            xv[r] = x[idx];
        }
#pragma unroll
        for (int r = 0; r < PSI_ROWS; ++r) {
            const double m = means[c[r] >= 0 ? c[r] : 0];
            if (r < nr) prow[(long long)r * g.Nx + i] = (sl >= 0 && c[r] >= 0) ? xv[r] - m : 0.0;
        }
    }
}

hipError_t launch_psi_out(const double *x, const int *comp, const double *means, const int *slot_of, const Grid &g,
                          double *psi, hipStream_t s, const Grid *gbricks, int zoff)
{
    const long long groups = (long long)((g.Ny + PSI_ROWS - 1) / PSI_ROWS) * g.Nz;
    if (groups <= 0 || g.Nx <= 0) return hipSuccess;
    SPFD_LAUNCH(k_psi_out, dim3((unsigned)groups), dim3(256), 0, s, x, comp, means, slot_of, g, gbricks ? *gbricks : g,
                zoff, psi);
    return hipGetLastError();
}

// start of a solve from x = 0: x = 0, r = b (right side i at b + i*bvs, vectors at i*n) and, for an
// FP32 cycle, the FP32 copy of r that the first cycle reads
__global__ void k_start(long long n, const double *__restrict__ b, long long bvs, double *__restrict__ x,
                        double *__restrict__ r, float *__restrict__ r32, const float *__restrict__ dinv)
{
    const long long off = (long long)blockIdx.y * n;
    b += (long long)blockIdx.y * bvs;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const double v = b[k];
        x[off + k] = 0.0;
        r[off + k] = v;
        if (r32) r32[off + k] = dinv ? (float)(v * (double)dinv[k]) : (float)v;
    }
}

hipError_t launch_start(long long n, const double *b, long long bvs, double *x, double *r, float *r32, int nvec,
                        hipStream_t s, const float *dinv)
{
    if (n <= 0 || nvec <= 0) return hipSuccess;
    if (dinv && !r32) return hipErrorInvalidValue;
    const long long blocks = (n + 255) / 256;
    SPFD_LAUNCH(k_start, dim3((unsigned)(blocks > 65536 ? 65536 : blocks), nvec), dim3(256), 0, s, n, b, bvs, x, r, r32,
                dinv);
    return hipGetLastError();
}

// brick layout from a dense node array (start iterate), 0 outside the conductor
__global__ void k_psi_in(const double *__restrict__ psi, const int *__restrict__ comp, const int4 *__restrict__ coord,
                         Grid g, double *x)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const int4 c = coord[b];
    const int i = c.x * 8 + tx, j = c.y * 8 + ty, k = c.z * 8 + tz;
    const long long idx = (long long)b * BS + t;
    double v = 0.0;
    if (comp[idx] >= 0) v = psi[i + (long long)g.Nx * (j + (long long)g.Ny * k)];
    x[idx] = v;
}

hipError_t launch_psi_in(const double *psi, const int *comp, const int4 *coord, int nb, const Grid &g, double *x,
                         hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_psi_in, dim3(nb), dim3(NT), 0, s, psi, comp, coord, g, x);
    return hipGetLastError();
}

// Eq. (1) and the voxel average: for a conducting voxel, u = a + G psi on its
// twelve edges (all conducting), ubar_d = mean of the four d-edges and
// |E| = omega * sqrt(sum (ubar_d / h_d)^2); air voxels get 0.
__global__ void k_efield(const uint8_t *__restrict__ labels, const double *__restrict__ table,
                         const double *__restrict__ sig_vox, Grid g, double hx, double hy, double hz, double omega,
                         const double *__restrict__ a, const double *__restrict__ psi, double *emag)
{
    // one workgroup per voxel row (j, k): contiguous loads and stores, no 64-bit index division
    const int row = blockIdx.x;
    const int j = row % g.ny, k = row / g.ny;
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    const long long sy = g.Nx, sz = (long long)g.Nx * g.Ny;
    const long long v0 = (long long)row * g.nx, nrow = j * sy + k * sz;
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
        const long long v = v0 + i;
        const double s = sig_vox ? sig_vox[v] : table[labels[v]];
        if (!(s > 0.0)) {
            emag[v] = 0.0;
            continue;
        }
        const long long n0 = nrow + i;
        // x-edges start at (i, j..j+1, k..k+1)
        const long long ex[4] = {n0, n0 + sy, n0 + sz, n0 + sy + sz};
        const long long ey[4] = {n0, n0 + 1, n0 + sz, n0 + 1 + sz};
        const long long ez[4] = {n0, n0 + 1, n0 + sy, n0 + 1 + sy};
        double ux = 0.0, uy = 0.0, uz = 0.0;
        for (int q = 0; q < 4; ++q) {
            ux += (a[ex[q]] + psi[ex[q] + 1]) - psi[ex[q]];
            uy += (a[nn + ey[q]] + psi[ey[q] + sy]) - psi[ey[q]];
            uz += (a[2 * nn + ez[q]] + psi[ez[q] + sz]) - psi[ez[q]];
        }
        const double fx = 0.25 * ux / hx, fy = 0.25 * uy / hy, fz = 0.25 * uz / hz;
        emag[v] = omega * sqrt(fx * fx + fy * fy + fz * fz);
    }
}

hipError_t launch_efield(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                         const double h[3], double omega, const double *a, const double *psi, double *emag,
                         hipStream_t s)
{
    const long long rows = (long long)g.ny * g.nz;
    if (rows <= 0) return hipSuccess;
    SPFD_LAUNCH(k_efield, dim3((unsigned)rows), dim3(256), 0, s, labels, table, sig_vox, g, h[0], h[1], h[2], omega, a,
                psi, emag);
    return hipGetLastError();
}

// u = a + G psi on conducting edges (any of the four voxels around the edge conducts), 0 elsewhere
__global__ void k_uedges(const uint8_t *__restrict__ labels, const double *__restrict__ table,
                         const double *__restrict__ sig_vox, Grid g, const double *__restrict__ a,
                         const double *__restrict__ psi, double *u)
{
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    // one workgroup per node row (j, k): contiguous loads and stores, no 64-bit index division
    const int row = blockIdx.x;
    const int j = row % g.Ny, k = row / g.Ny;
    for (int i = threadIdx.x; i < g.Nx; i += blockDim.x) {
        const long long n = (long long)row * g.Nx + i;
        // x-edge: voxels (i, j-1..j, k-1..k)
        double sx = 0.0, sy = 0.0, sz = 0.0;
        if (i < g.nx)
            sx = vox_sig(labels, table, sig_vox, g, i, j - 1, k - 1) + vox_sig(labels, table, sig_vox, g, i, j, k - 1) +
                 vox_sig(labels, table, sig_vox, g, i, j - 1, k) + vox_sig(labels, table, sig_vox, g, i, j, k);
        if (j < g.ny)
            sy = vox_sig(labels, table, sig_vox, g, i - 1, j, k - 1) + vox_sig(labels, table, sig_vox, g, i, j, k - 1) +
                 vox_sig(labels, table, sig_vox, g, i - 1, j, k) + vox_sig(labels, table, sig_vox, g, i, j, k);
        if (k < g.nz)
            sz = vox_sig(labels, table, sig_vox, g, i - 1, j - 1, k) + vox_sig(labels, table, sig_vox, g, i, j - 1, k) +
                 vox_sig(labels, table, sig_vox, g, i - 1, j, k) + vox_sig(labels, table, sig_vox, g, i, j, k);
        u[n] = sx > 0.0 ? (a[n] + psi[n + 1]) - psi[n] : 0.0;
        u[nn + n] = sy > 0.0 ? (a[nn + n] + psi[n + g.Nx]) - psi[n] : 0.0;
        u[2 * nn + n] = sz > 0.0 ? (a[2 * nn + n] + psi[n + (long long)g.Nx * g.Ny]) - psi[n] : 0.0;
    }
}

hipError_t launch_uedges(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                         const double *a, const double *psi, double *u, hipStream_t s)
{
    const long long rows = (long long)g.Ny * g.Nz;
    if (rows <= 0) return hipSuccess;
    SPFD_LAUNCH(k_uedges, dim3((unsigned)rows), dim3(256), 0, s, labels, table, sig_vox, g, a, psi, u);
    return hipGetLastError();
}

}  // namespace spfd

namespace spfd {

// ============================================================================
// adjoint gradient of an objective J(|E|) with respect to the conductivities
// ============================================================================
// With A Psi = -G^T M a, u = a + G Psi and dA = G^T dM G, a change of M gives
// A dPsi = -G^T dM u; for dJ = g^T du = (G^T g)^T dPsi the adjoint solve
// A lambda = G^T g yields dJ = -(G lambda)^T dM u, and dM_e/dsigma_v = (dual
// area / length)/4 for the four voxels v around edge e.

// per conducting voxel: c_d = dJ/d|E| * omega^2 * ubar_d / (4 h_d^2 |E|), the
// derivative of J with respect to each of the voxel's four d-edge voltages
__global__ void k_adj_voxel(const uint8_t *__restrict__ labels, const double *__restrict__ table,
                            const double *__restrict__ sig_vox, Grid g, double hx, double hy, double hz, double omega,
                            const double *__restrict__ a, const double *__restrict__ psi,
                            const double *__restrict__ grad_emag, double *c)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    const long long sy = g.Nx, sz = (long long)g.Nx * g.Ny;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x) {
        const double s = sig_vox ? sig_vox[v] : table[labels[v]];
        double cx = 0.0, cy = 0.0, cz = 0.0;
        if (s > 0.0) {
            const long long i = v % g.nx, j = (v / g.nx) % g.ny, k = v / ((long long)g.nx * g.ny);
            const long long n0 = i + g.Nx * (j + (long long)g.Ny * k);
            const long long ex[4] = {n0, n0 + sy, n0 + sz, n0 + sy + sz};
            const long long ey[4] = {n0, n0 + 1, n0 + sz, n0 + 1 + sz};
            const long long ez[4] = {n0, n0 + 1, n0 + sy, n0 + 1 + sy};
            double ux = 0.0, uy = 0.0, uz = 0.0;
            for (int q = 0; q < 4; ++q) {
                ux += (a[ex[q]] + psi[ex[q] + 1]) - psi[ex[q]];
                uy += (a[nn + ey[q]] + psi[ey[q] + sy]) - psi[ey[q]];
                uz += (a[2 * nn + ez[q]] + psi[ez[q] + sz]) - psi[ez[q]];
            }
            const double fx = 0.25 * ux / hx, fy = 0.25 * uy / hy, fz = 0.25 * uz / hz;
            const double E = omega * sqrt(fx * fx + fy * fy + fz * fz);
            if (E > 0.0) {
                const double ge = grad_emag[v];
                cx = ge * omega * omega * (0.25 * ux) / (4.0 * hx * hx * E);
                cy = ge * omega * omega * (0.25 * uy) / (4.0 * hy * hy * E);
                cz = ge * omega * omega * (0.25 * uz) / (4.0 * hz * hz * E);
            }
        }
        c[v] = cx;
        c[nvox + v] = cy;
        c[2 * nvox + v] = cz;
    }
}

// adjoint right side at the nodes: (G^T g)_n, where each of the 8 voxels
// around n passes its d-edge through n; n is the head of that edge when the
// voxel lies on the minus side along d (+c) and its tail otherwise (-c)
__global__ __launch_bounds__(NT) void k_adj_rhs(Topo topo, const int4 *__restrict__ coord, Grid g,
                                                const double *__restrict__ c, double *b, double *part)
{
    __shared__ double red[8];
    const int bk = xcd_brick(blockIdx.x, topo.nb);
    if (bk < 0) return;
    const int t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const int4 q = coord[bk];
    const int i = q.x * 8 + tx, j = q.y * 8 + ty, k = q.z * 8 + tz;
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    double s = 0.0;
    for (int oz = -1; oz <= 0; ++oz)
        for (int oy = -1; oy <= 0; ++oy)
            for (int ox = -1; ox <= 0; ++ox) {
                const int vi = i + ox, vj = j + oy, vk = k + oz;
                if (vi < 0 || vj < 0 || vk < 0 || vi >= g.nx || vj >= g.ny || vk >= g.nz) continue;
                const long long v = vi + (long long)g.nx * (vj + (long long)g.ny * vk);
                s += (ox < 0 ? c[v] : -c[v]);
                s += (oy < 0 ? c[nvox + v] : -c[nvox + v]);
                s += (oz < 0 ? c[2 * nvox + v] : -c[2 * nvox + v]);
            }
    b[(long long)bk * BS + t] = s;
    const double tot = block_sum(s * s, red);
    if (t == 0) part[bk] = tot;
}

// dJ/dsigma_v = -sum over the 12 edges of v of (area/length/4) (G lambda)_e u_e,
// and per-block partial sums per label (LDS atomics, then a fixed-order sum)
__global__ __launch_bounds__(256) void k_adj_grad(const uint8_t *__restrict__ labels, const double *__restrict__ table,
                                                  const double *__restrict__ sig_vox, Grid g, double gx, double gy,
                                                  double gz, const double *__restrict__ a,
                                                  const double *__restrict__ psi, const double *__restrict__ lam,
                                                  double *grad, double *lab_part, int nlab)
{
    __shared__ double hist[MAX_LABELS];
    for (int l = threadIdx.x; l < nlab; l += blockDim.x) hist[l] = 0.0;
    __syncthreads();
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    const long long sy = g.Nx, sz = (long long)g.Nx * g.Ny;
    const double geo[3] = {gx, gy, gz};
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x) {
        const double s = sig_vox ? sig_vox[v] : table[labels[v]];
        double out = 0.0;
        if (s > 0.0) {
            const long long i = v % g.nx, j = (v / g.nx) % g.ny, k = v / ((long long)g.nx * g.ny);
            const long long n0 = i + g.Nx * (j + (long long)g.Ny * k);
            const long long e[3][4] = {{n0, n0 + sy, n0 + sz, n0 + sy + sz},
                                       {n0, n0 + 1, n0 + sz, n0 + 1 + sz},
                                       {n0, n0 + 1, n0 + sy, n0 + 1 + sy}};
            const long long st[3] = {1, sy, sz};
            double acc = 0.0;
            for (int d = 0; d < 3; ++d)
                for (int q = 0; q < 4; ++q) {
                    const long long n = e[d][q];
                    const double glam = lam[n + st[d]] - lam[n];
                    const double u = (a[d * nn + n] + psi[n + st[d]]) - psi[n];
                    acc += geo[d] * glam * u;
                }
            out = -acc;
            if (labels[v] < nlab) atomicAdd(hist + labels[v], out);
        }
        grad[v] = out;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < nlab; l += blockDim.x) lab_part[(long long)blockIdx.x * nlab + l] = hist[l];
}

// per-label totals: fixed-order sum of the block partials
__global__ void k_adj_labsum(const double *__restrict__ lab_part, int nblocks, int nlab, double *out)
{
    const int l = blockIdx.x;
    __shared__ double red[8];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += lab_part[(long long)b * nlab + l];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[l] = s;
}

hipError_t launch_adj_voxel(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                            const double h[3], double omega, const double *a, const double *psi,
                            const double *grad_emag, double *c, hipStream_t s)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    const unsigned gb = (unsigned)((nvox + 255) / 256 > 131072 ? 131072 : (nvox + 255) / 256);
    SPFD_LAUNCH(k_adj_voxel, dim3(gb), dim3(256), 0, s, labels, table, sig_vox, g, h[0], h[1], h[2], omega, a,
                       psi, grad_emag, c);
    return hipGetLastError();
}

hipError_t launch_adj_rhs(Topo topo, const int4 *coord, const Grid &g, const double *c, double *b, double *part,
                          hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_adj_rhs, dim3(xcd_grid(topo.nb)), dim3(NT), 0, s, topo, coord, g, c, b, part);
    return hipGetLastError();
}

int adj_grad_blocks(const Grid &g)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    const long long b = (nvox + 255) / 256;
    return (int)(b > 8192 ? 8192 : b);
}

hipError_t launch_adj_grad(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                           const double geo4[3], const double *a, const double *psi, const double *lam, double *grad,
                           double *lab_part, int nlab, double *lab_out, hipStream_t s)
{
    const int gb = adj_grad_blocks(g);
    SPFD_LAUNCH(k_adj_grad, dim3(gb), dim3(256), 0, s, labels, table, sig_vox, g, geo4[0], geo4[1], geo4[2], a,
                       psi, lam, grad, lab_part, nlab);
    SPFD_LAUNCH(k_adj_labsum, dim3(nlab), dim3(NT), 0, s, lab_part, gb, nlab, lab_out);
    return hipGetLastError();
}

}  // namespace spfd
