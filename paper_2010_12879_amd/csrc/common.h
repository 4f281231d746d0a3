// Shared device-side definitions of the SPFD library (gfx950, wave64).
//
// Node arrays of every multigrid level live in 8x8x8 bricks: only bricks that
// hold unknowns are stored, brick b occupies elements [b*512, b*512+512) and
// node (tx,ty,tz) of a brick sits at tx + 8*ty + 64*tz.  A workgroup of 512
// threads owns one brick, so each wave covers one 8x8 z-slice (512 contiguous
// bytes in FP64).  Neighbour bricks come from a [nb][6] table (-1 = absent).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spfd {

constexpr int BD = 8;              // brick edge in nodes
constexpr int BS = 512;            // nodes per brick
constexpr int TILE = 9;            // label tile edge: the brick's voxels plus one layer on the minus side
constexpr int TILE_VOX = 729;
constexpr int TILE_BYTES = 768;    // 729 padded
constexpr int MAX_LABELS = 256;
constexpr int NT = 512;            // threads per brick workgroup

// neighbour slots
enum { NMX = 0, NPX = 1, NMY = 2, NPY = 3, NMZ = 4, NPZ = 5 };

// per right-hand side scalars of the outer CG, resident in device memory
struct Scal {
    double rz;       // r.z of the current iterate
    double pq;       // p.q
    double alpha;
    double beta;
    double rr;       // ||r||^2
    double bb;       // ||b||^2
    double zq;       // z.q (flexible beta)
    double tol2;     // (rel_tol)^2 * ||b||^2
    int done;        // 1 = converged or stopped: later kernels of this solve return at once
    int iters;
    int status;      // 0 ok, 5 not converged, 6 breakdown
    int hcount;      // CG steps of the current window of kept search directions (the next one's slot)
    int happlied;    // of these, the directions already added to x (an update of x before the window is full)
    int pad;
};

constexpr int MAX_MODELS = 16;     // voxel models packed into one handle

struct Topo {
    int nb;                                    // active bricks
    const int *nbr;                            // [nb*6]
    const unsigned long long *cmask = nullptr; // [nb]: bit tx + 8 ty set when the node column (tx,ty,*)
                                               // holds an unknown (nullptr: all columns)
    // np > 0: the bricks of np voxel models packed into one level; launch row blockIdx.y = m works on
    // model m's bricks [prange[m].x, prange[m].x + prange[m].y) (its own scalars and partial sums).
    // The ranges live in device memory (a uniform load), not in the kernel arguments: an argument
    // array indexed by blockIdx.y would be copied to scratch memory in every kernel.
    int np = 0;
    int pmax = 0;                    // largest range
    const int2 *prange = nullptr;    // [np] (first brick, bricks)
};

// bricks per launch row: all bricks, or the largest model's
__host__ __device__ __forceinline__ int topo_count(const Topo &t) { return t.np ? t.pmax : t.nb; }

// XCD-aware workgroup -> brick map: the hardware hands consecutive workgroup
// ids to the 8 XCDs in turn; giving each XCD a contiguous run of bricks keeps
// neighbour bricks (halo reads) in the same L2.  Returns -1 for padding ids.
__device__ __forceinline__ int xcd_brick(int wg, int nb)
{
    int per = (nb + 7) >> 3;
    int b = (wg & 7) * per + (wg >> 3);
    return b < nb ? b : -1;
}

__host__ __forceinline__ int xcd_grid(int nb) { return ((nb + 7) >> 3) << 3; }

// The brick of a one-brick workgroup (-1 for padding) and its index within its
// launch row (local; the index of its partial sum): with packed models, row
// blockIdx.y = m covers model m's bricks.
__device__ __forceinline__ int topo_brick(const Topo &t, int &local)
{
    if (t.np == 0) {
        local = xcd_brick(blockIdx.x, t.nb);
        return local;
    }
    // the map is taken over the launch row's full length (the largest model), so that every brick of
    // a smaller model has exactly one workgroup; the rest of the row has none
    const int2 r = t.prange[blockIdx.y];
    local = xcd_brick(blockIdx.x, t.pmax);
    if (local >= r.y) local = -1;
    return local < 0 ? -1 : r.x + local;
}

__device__ __forceinline__ void brick_xyz(int t, int &tx, int &ty, int &tz)
{
    tx = t & 7;
    ty = (t >> 3) & 7;
    tz = t >> 6;
}

// Index of each face neighbour of node t of brick b.  A neighbour in an absent
// brick is never a conductor node, and the edge to it has conductance 0, so
// it is replaced by the node itself: every lane issues exactly one load per
// direction and the stencil term w (x_n - x_n) vanishes.
__device__ __forceinline__ void nbr_index(long long base, int t, int tx, int ty, int tz, const int *nb,
                                          long long I[6])
{
    const long long self = base + t;
    I[NMX] = tx > 0 ? self - 1 : (nb[NMX] >= 0 ? (long long)nb[NMX] * BS + t + 7 : self);
    I[NPX] = tx < 7 ? self + 1 : (nb[NPX] >= 0 ? (long long)nb[NPX] * BS + t - 7 : self);
    I[NMY] = ty > 0 ? self - 8 : (nb[NMY] >= 0 ? (long long)nb[NMY] * BS + t + 56 : self);
    I[NPY] = ty < 7 ? self + 8 : (nb[NPY] >= 0 ? (long long)nb[NPY] * BS + t - 56 : self);
    I[NMZ] = tz > 0 ? self - 64 : (nb[NMZ] >= 0 ? (long long)nb[NMZ] * BS + t + 448 : self);
    I[NPZ] = tz < 7 ? self + 64 : (nb[NPZ] >= 0 ? (long long)nb[NPZ] * BS + t - 448 : self);
}

template <typename T>
__device__ __forceinline__ void nbr_vals(const T *__restrict__ x, const long long I[6], T X[6])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = x[I[k]];
}

// edge weights of node t from stored arrays w[d*stride + node] (edge to +d);
// the minus-side weights are the plus-side weights of the minus neighbours
// (0 when that neighbour's brick is absent)
template <typename T>
__device__ __forceinline__ void stored_weights(const T *__restrict__ w, long long stride, long long base, int t,
                                               const long long I[6], T W[6])
{
    const long long n = base + t;
    W[NPX] = w[n];
    W[NPY] = w[stride + n];
    W[NPZ] = w[2 * stride + n];
    const T mx = w[I[NMX]], my = w[stride + I[NMY]], mz = w[2 * stride + I[NMZ]];
    W[NMX] = I[NMX] != n ? mx : T(0);
    W[NMY] = I[NMY] != n ? my : T(0);
    W[NMZ] = I[NMZ] != n ? mz : T(0);
}

// the six neighbour slots of a brick (uniform across the workgroup: scalar loads)
__device__ __forceinline__ void brick_nbrs(const int *nbr, int b, int nb[6])
{
    const int *p = nbr + b * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) nb[k] = p[k];
}

// Conductances of the six edges of a node from the conductivities of its eight
// surrounding voxels, held in an LDS tile s[a + 9*(b + 9*c)] where (a,b,c) =
// (tx,ty,tz) + {0,1}^3.  Edge to +x: the four voxels at a = tx+1, and so on.
// geo4[d] = (area of the dual facet) / (length) / 4 of a d-edge.  The sums keep
// the order (j-1,k-1), (j,k-1), (j-1,k), (j,k) of the other two axes.
template <typename T>
__device__ __forceinline__ void tile_weights(const T *s, int tx, int ty, int tz, const T geo4[3], T W[6])
{
    const T *p = s + tx + 9 * (ty + 9 * tz);
    const T s000 = p[0], s100 = p[1], s010 = p[9], s110 = p[10];
    const T s001 = p[81], s101 = p[82], s011 = p[90], s111 = p[91];
    W[NPX] = (((s100 + s110) + s101) + s111) * geo4[0];
    W[NMX] = (((s000 + s010) + s001) + s011) * geo4[0];
    W[NPY] = (((s010 + s110) + s011) + s111) * geo4[1];
    W[NMY] = (((s000 + s100) + s001) + s101) * geo4[1];
    W[NPZ] = (((s001 + s101) + s011) + s111) * geo4[2];
    W[NMZ] = (((s000 + s100) + s010) + s110) * geo4[2];
}

// (A x)_n = sum over edges of w (x_n - x_m); exact zero for a constant field
template <typename T>
__device__ __forceinline__ T stencil_apply(T x0, const T X[6], const T W[6])
{
    T y = W[0] * (x0 - X[0]);
    y += W[1] * (x0 - X[1]);
    y += W[2] * (x0 - X[2]);
    y += W[3] * (x0 - X[3]);
    y += W[4] * (x0 - X[4]);
    y += W[5] * (x0 - X[5]);
    return y;
}

template <typename T>
__device__ __forceinline__ T diag_of(const T W[6])
{
    return ((((W[0] + W[1]) + W[2]) + W[3]) + W[4]) + W[5];
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// sum over a 512-thread block, valid in thread 0; lds needs 8 doubles
__device__ __forceinline__ double block_sum(double v, double *lds)
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

}  // namespace spfd
