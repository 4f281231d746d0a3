// Unstructured (ELL) coarse levels of the aggregation multigrid.
//
// On the coarse end of the hierarchy, 2x2x2 aggregates are split into the
// pieces that are connected inside the aggregate, so that one coarse unknown
// never glues together conductor regions that touch only through air (an arm
// and the torso across a thin gap, two legs).  A coarse unknown is then no
// longer a grid node: these levels store, per unknown, its grid position and
// up to K neighbours with conductances (ELL, column-major: entry k of row i at
// k*n + i, column -1 = empty).  The Galerkin product for piecewise-constant
// aggregation is still exact: the coarse conductance between two pieces is
// the sum of the fine conductances that join them.
#include <math.h>

#include "kernels.h"

namespace spfd {

// ---------------------------------------------------------------- union-find helpers (agent-scope, lock-free)
__device__ __forceinline__ int uf_load(const int *p, int i)
{
    return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int *p, int x)
{
    int px = uf_load(p, x);
    while (px != x) {
        const int ppx = uf_load(p, px);
        if (ppx != px) __hip_atomic_store(p + x, ppx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = px;
        px = ppx;
    }
    return x;
}

__device__ __forceinline__ void uf_unite(int *p, int a, int b)
{
    while (true) {
        a = uf_find(p, a);
        b = uf_find(p, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        int expected = b;
        if (__hip_atomic_compare_exchange_strong(p + b, &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// ---------------------------------------------------------------- pieces of a structured (brick) level
// parent[n] = n for unknowns (D > 0), -1 otherwise
__global__ void k_piece_init_brick(const double *__restrict__ w, long long stride, Topo topo, int *parent)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int nb[6];
    brick_nbrs(topo.nbr, b, nb);
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const long long base = (long long)b * BS;
    long long I[6];
    nbr_index(base, t, tx, ty, tz, nb, I);
    double W[6];
    stored_weights(w, stride, base, t, I, W);
    parent[base + t] = diag_of(W) > 0.0 ? (int)(base + t) : -1;
}

// unite across the edges that stay inside a 2x2x2 aggregate: the +d edge of a
// node with an even grid coordinate along d (bricks start at multiples of 8,
// so both ends are in the same brick)
__global__ void k_piece_union_brick(const double *__restrict__ w, long long stride, Topo topo, int *parent)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const long long base = (long long)b * BS;
    const int me = (int)(base + t);
    if ((tx & 1) == 0 && w[base + t] > 0.0) uf_unite(parent, me, me + 1);
    if ((ty & 1) == 0 && w[stride + base + t] > 0.0) uf_unite(parent, me, me + 8);
    if ((tz & 1) == 0 && w[2 * stride + base + t] > 0.0) uf_unite(parent, me, me + 64);
}

// position (at the coarse level) of the piece rooted at node n
__global__ void k_piece_pos_brick(const int *__restrict__ parent, const int *__restrict__ idx, Topo topo,
                                  const int4 *__restrict__ coord, int4 *pos)
{
    const int b = blockIdx.x, t = threadIdx.x;
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    const long long n = (long long)b * BS + t;
    if (parent[n] == (int)n) {
        const int4 c = coord[b];
        pos[idx[n]] = make_int4((c.x * 8 + tx) >> 1, (c.y * 8 + ty) >> 1, (c.z * 8 + tz) >> 1, 0);
    }
}

// ---------------------------------------------------------------- pieces of an ELL level
__global__ void k_piece_init_ell(int n, int K, const int *__restrict__ col, const double *__restrict__ val,
                                 int *parent)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int k = 0; k < K; ++k)
            if (col[(long long)k * n + i] >= 0) d += val[(long long)k * n + i];
        parent[i] = d > 0.0 ? i : -1;
    }
}

__global__ void k_piece_union_ell(int n, int K, const int *__restrict__ col, const double *__restrict__ val,
                                  const int4 *__restrict__ pos, int *parent)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (parent[i] < 0) continue;
        const int4 pi = pos[i];
        for (int k = 0; k < K; ++k) {
            const int j = col[(long long)k * n + i];
            if (j <= i || !(val[(long long)k * n + i] > 0.0)) continue;
            const int4 pj = pos[j];
            if ((pi.x >> 1) == (pj.x >> 1) && (pi.y >> 1) == (pj.y >> 1) && (pi.z >> 1) == (pj.z >> 1))
                uf_unite(parent, i, j);
        }
    }
}

__global__ void k_piece_pos_ell(int n, const int *__restrict__ parent, const int *__restrict__ idx,
                                const int4 *__restrict__ fpos, int4 *pos)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (parent[i] == i) {
            const int4 p = fpos[i];
            pos[idx[i]] = make_int4(p.x >> 1, p.y >> 1, p.z >> 1, 0);
        }
}

// ---------------------------------------------------------------- shared steps
__global__ void k_piece_flatten(int *parent, long long n, int *flag)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        int r = -1;
        if (uf_load(parent, (int)i) >= 0) r = uf_find(parent, (int)i);
        flag[i] = (r == (int)i) ? 1 : 0;
    }
}

__global__ void k_piece_store_root(int *parent, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int p = uf_load(parent, (int)i);
        if (p >= 0) parent[i] = uf_find(parent, (int)i);
    }
}

__global__ void k_piece_assign(const int *__restrict__ parent, const int *__restrict__ idx, long long n, int *agg,
                               int *count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int p = parent[i];
        const int a = p >= 0 ? idx[p] : -1;
        agg[i] = a;
        if (a >= 0) atomicAdd(count + a, 1);
    }
}

// members of each coarse unknown, in increasing fine index (deterministic order)
__global__ void k_members_fill(const int *__restrict__ agg, long long n, const int *__restrict__ mptr, int *cursor,
                               int *mem)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int a = agg[i];
        if (a >= 0) mem[mptr[a] + atomicAdd(cursor + a, 1)] = (int)i;
    }
}

__global__ void k_members_sort(int nc, const int *__restrict__ mptr, int *mem)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x) {
        const int b = mptr[p], e = mptr[p + 1];
        for (int i = b + 1; i < e; ++i) {
            const int v = mem[i];
            int j = i - 1;
            while (j >= b && mem[j] > v) {
                mem[j + 1] = mem[j];
                --j;
            }
            mem[j + 1] = v;
        }
    }
}

// Direct member table of the restriction: memb[p*8 + j] = member j of aggregate p (-1: none), one load
// instead of the CSR pair (pointer, then member); an aggregate with more than eight members sets *over
// (the restriction then keeps the CSR form).
__global__ void k_members8(int nc, const int *__restrict__ mptr, const int *__restrict__ mem, int *__restrict__ memb,
                           int *over)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x) {
        const int b = mptr[p], e = mptr[p + 1];
        if (e - b > 8) *over = 1;
#pragma unroll
        for (int j = 0; j < 8; ++j) memb[(long long)p * 8 + j] = b + j < e ? mem[b + j] : -1;
    }
}

// ---------------------------------------------------------------- Galerkin rows
constexpr int GAL_MAX = 48;   // distinct coarse neighbours a row may collect

// visit the edges of fine unknown i: f(j, w) for every neighbour j with w > 0
struct FineLevel {
    // structured
    const double *w;
    long long stride;
    const int *nbr;
    // ELL
    int n, K;
    const int *col;
    const double *val;
};

template <typename F>
__device__ __forceinline__ void fine_edges(const FineLevel &f, int i, F &&fn)
{
    if (f.w) {
        const int b = i / BS, t = i % BS;
        int tx, ty, tz;
        brick_xyz(t, tx, ty, tz);
        int nb[6];
        brick_nbrs(f.nbr, b, nb);
        long long I[6];
        nbr_index((long long)b * BS, t, tx, ty, tz, nb, I);
        double W[6];
        stored_weights(f.w, f.stride, (long long)b * BS, t, I, W);
        for (int k = 0; k < 6; ++k)
            if (W[k] > 0.0 && I[k] != i) fn((int)I[k], W[k]);
    } else {
        for (int k = 0; k < f.K; ++k) {
            const int j = f.col[(long long)k * f.n + i];
            if (j >= 0 && f.val[(long long)k * f.n + i] > 0.0) fn(j, f.val[(long long)k * f.n + i]);
        }
    }
}

// pass 0: row lengths (len[p]); pass 1: fill ELL with width K (entries in
// order of first appearance over members and their edges; sums in that order)
__global__ void k_galerkin_rows(FineLevel f, const int *__restrict__ agg, int nc, const int *__restrict__ mptr,
                                const int *__restrict__ mem, int pass, int *len, int K, int *col, double *val64,
                                float *val32, int *overflow)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x) {
        int cols[GAL_MAX];
        double ws[GAL_MAX];
        int m = 0;
        bool over = false;
        for (int q = mptr[p]; q < mptr[p + 1]; ++q) {
            const int i = mem[q];
            fine_edges(f, i, [&](int j, double wj) {
                const int a = agg[j];
                if (a < 0 || a == p) return;
                int s = 0;
                while (s < m && cols[s] != a) ++s;
                if (s == m) {
                    if (m == GAL_MAX) { over = true; return; }
                    cols[m] = a;
                    ws[m] = 0.0;
                    ++m;
                }
                ws[s] += wj;
            });
        }
        if (over) *overflow = 1;
        if (pass == 0) {
            len[p] = m;
        } else {
            for (int k = 0; k < K; ++k) {
                const long long e = (long long)k * nc + p;
                if (k < m) {
                    col[e] = cols[k];
                    val64[e] = ws[k];
                    val32[e] = (float)ws[k];
                } else {
                    col[e] = -1;
                    val64[e] = 0.0;
                    val32[e] = 0.0f;
                }
            }
        }
    }
}

__global__ void k_max_int(const int *__restrict__ v, int n, int *out)
{
    __shared__ int s[256];
    int m = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = max(m, v[i]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + d]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

static unsigned gblocks(long long n, int bs = 256, long long cap = 65536)
{
    long long b = (n + bs - 1) / bs;
    if (b < 1) b = 1;
    return (unsigned)(b > cap ? cap : b);
}

hipError_t launch_pieces_brick(const double *w64, long long stride, Topo topo, const int4 *coord, int *parent,
                               hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_piece_init_brick, dim3(topo.nb), dim3(NT), 0, s, w64, stride, topo, parent);
    SPFD_LAUNCH(k_piece_union_brick, dim3(topo.nb), dim3(NT), 0, s, w64, stride, topo, parent);
    (void)coord;
    return hipGetLastError();
}

hipError_t launch_pieces_ell(int n, int K, const int *col, const double *val, const int4 *pos, int *parent,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_piece_init_ell, dim3(gblocks(n)), dim3(256), 0, s, n, K, col, val, parent);
    SPFD_LAUNCH(k_piece_union_ell, dim3(gblocks(n)), dim3(256), 0, s, n, K, col, val, pos, parent);
    return hipGetLastError();
}

hipError_t launch_pieces_finish(int *parent, long long n, int *flag, hipStream_t s)
{
    SPFD_LAUNCH(k_piece_store_root, dim3(gblocks(n)), dim3(256), 0, s, parent, n);
    SPFD_LAUNCH(k_piece_flatten, dim3(gblocks(n)), dim3(256), 0, s, parent, n, flag);
    return hipGetLastError();
}

hipError_t launch_pieces_assign(const int *parent, const int *idx, long long n, int *agg, int *count, hipStream_t s)
{
    SPFD_LAUNCH(k_piece_assign, dim3(gblocks(n)), dim3(256), 0, s, parent, idx, n, agg, count);
    return hipGetLastError();
}

hipError_t launch_piece_pos_brick(const int *parent, const int *idx, Topo topo, const int4 *coord, int4 *pos,
                                  hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    SPFD_LAUNCH(k_piece_pos_brick, dim3(topo.nb), dim3(NT), 0, s, parent, idx, topo, coord, pos);
    return hipGetLastError();
}

hipError_t launch_piece_pos_ell(int n, const int *parent, const int *idx, const int4 *fpos, int4 *pos, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_piece_pos_ell, dim3(gblocks(n)), dim3(256), 0, s, n, parent, idx, fpos, pos);
    return hipGetLastError();
}

hipError_t launch_members(const int *agg, long long n, int nc, const int *mptr, int *cursor, int *mem, hipStream_t s)
{
    SPFD_LAUNCH(k_members_fill, dim3(gblocks(n)), dim3(256), 0, s, agg, n, mptr, cursor, mem);
    if (nc > 0) SPFD_LAUNCH(k_members_sort, dim3(gblocks(nc)), dim3(256), 0, s, nc, mptr, mem);
    return hipGetLastError();
}

hipError_t launch_members8(int nc, const int *mptr, const int *mem, int *memb, int *over, hipStream_t s)
{
    if (nc <= 0) return hipSuccess;
    SPFD_LAUNCH(k_members8, dim3(gblocks(nc)), dim3(256), 0, s, nc, mptr, mem, memb, over);
    return hipGetLastError();
}

hipError_t launch_galerkin_ell(const FineLevelArgs &fa, const int *agg, int nc, const int *mptr, const int *mem,
                               int pass, int *len, int K, int *col, double *val64, float *val32, int *overflow,
                               int *maxlen, hipStream_t s)
{
    FineLevel f;
    f.w = fa.w;
    f.stride = fa.stride;
    f.nbr = fa.nbr;
    f.n = fa.n;
    f.K = fa.K;
    f.col = fa.col;
    f.val = fa.val;
    if (nc <= 0) return hipSuccess;
    SPFD_LAUNCH(k_galerkin_rows, dim3(gblocks(nc, 128)), dim3(128), 0, s, f, agg, nc, mptr, mem, pass, len, K,
                       col, val64, val32, overflow);
    if (pass == 0) SPFD_LAUNCH(k_max_int, dim3(1), dim3(256), 0, s, len, nc, maxlen);
    return hipGetLastError();
}

// ============================================================================
// cycle kernels on ELL levels (T = arithmetic of the cycle)
// ============================================================================
__device__ __forceinline__ bool ell_stopped(const Scal *sc)
{
    return sc && sc[blockIdx.y].done;   // written by an earlier kernel only: a plain (scalar) load
}

// (A x)_i and the diagonal D of an ELL row.  Padding entries (col < 0) read
// the row's own value and count with weight 0: every load is unconditional,
// so a thread has all of its row's loads in flight at once (a load under a
// condition becomes a branch that waits for it).
template <typename T>
__device__ __forceinline__ T ell_row(int n, int K, const int *__restrict__ col, const T *__restrict__ val,
                                     const T *__restrict__ x, int i, T xi, T &D)
{
    T y = T(0), d = T(0);
#pragma unroll 8
    for (int k = 0; k < K; ++k) {
        const int j = col[(long long)k * n + i];
        const T v = val[(long long)k * n + i];
        const T xj = x[j >= 0 ? j : i];
        const T w = j >= 0 ? v : T(0);
        d += w;
        y += w * (xi - xj);
    }
    D = d;
    return y;
}

template <typename T>
__global__ void k_ell_cheb_first(int n, int K, const int *__restrict__ col, const T *__restrict__ val,
                                 const T *__restrict__ b, T *__restrict__ x, T c0, const Scal *sc, long long vs)
{
    if (ell_stopped(sc)) return;
    b += blockIdx.y * vs;
    x += blockIdx.y * vs;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T bi = b[i];
        T d = T(0);
#pragma unroll 8
        for (int k = 0; k < K; ++k) {
            const int j = col[(long long)k * n + i];
            const T v = val[(long long)k * n + i];
            d += j >= 0 ? v : T(0);
        }
        x[i] = d > T(0) ? c0 * bi / d : T(0);
    }
}

// x with the coarse-grid correction of the prolongation applied: x_i + s x_c[agg_i] (agg_i < 0: none)
template <typename T>
__device__ __forceinline__ T corrected(const T *__restrict__ x, const int *__restrict__ agg, const T *__restrict__ xc,
                                       T scale, int i)
{
    const T v = x[i];
    const int a = agg[i];
    const T c = xc[a >= 0 ? a : 0];
    return a >= 0 ? v + scale * c : v;
}

// general Chebyshev step on an ELL level; with agg the prolongation from the
// coarser ELL level (x += s x_c[agg]) is applied to every value read (the
// first post-smoothing step)
template <typename T>
__global__ void k_ell_cheb_step(int n, int K, const int *__restrict__ col, const T *__restrict__ val,
                                const T *__restrict__ b, const T *__restrict__ xin, T *__restrict__ xout,
                                const T *__restrict__ din, T *__restrict__ dout, T c1, T c2, const Scal *sc,
                                long long vs, const int *__restrict__ agg, const T *__restrict__ xc, T scale,
                                long long vsc)
{
    if (ell_stopped(sc)) return;
    b += blockIdx.y * vs;
    xin += blockIdx.y * vs;
    xout += blockIdx.y * vs;
    if (din) din += blockIdx.y * vs;
    if (dout) dout += blockIdx.y * vs;
    if (agg) xc += blockIdx.y * vsc;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T xi = agg ? corrected(xin, agg, xc, scale, i) : xin[i];
        const T bi = b[i];
        const T di = din ? din[i] : T(0);
        T D;
        T ax;
        if (agg) {
            // as ell_row, with every value read corrected (unconditional loads)
            T y = T(0), d = T(0);
#pragma unroll 8
            for (int k = 0; k < K; ++k) {
                const int j = col[(long long)k * n + i];
                const T v = val[(long long)k * n + i];
                const T xj = corrected(xin, agg, xc, scale, j >= 0 ? j : i);
                const T w = j >= 0 ? v : T(0);
                d += w;
                y += w * (xi - xj);
            }
            D = d;
            ax = y;
        } else {
            ax = ell_row(n, K, col, val, xin, i, xi, D);
        }
        T xo = T(0), dn = T(0);
        if (D > T(0)) {
            const T dold = din ? di : xi;
            dn = c1 * dold + c2 * (bi - ax) / D;
            xo = xi + dn;
        }
        xout[i] = xo;
        if (dout) dout[i] = dn;
    }
}

// (b - A x)_i of row i of the finer level (structured stencil or ELL rows)
template <typename T>
__device__ __forceinline__ T fine_resid(const FineLevelT<T> &f, const T *__restrict__ b, const T *__restrict__ x,
                                        long long i)
{
    const T xi = x[i];
    T ax;
    if (f.w) {
        const int bk = (int)(i / BS), t = (int)(i % BS);
        int tx, ty, tz;
        brick_xyz(t, tx, ty, tz);
        int nb[6];
        brick_nbrs(f.nbr, bk, nb);
        long long I[6];
        nbr_index((long long)bk * BS, t, tx, ty, tz, nb, I);
        T W[6], X[6];
        stored_weights(f.w, f.stride, (long long)bk * BS, t, I, W);
        nbr_vals(x, I, X);
        ax = stencil_apply(xi, X, W);
    } else {
        T D;
        ax = ell_row(f.n, f.K, f.col, f.val, x, (int)i, xi, D);
    }
    return b[i] - ax;
}

// Coarse right side b_c[p] = sum over the members i of p of (b - A x)_i.
// Eight lanes per aggregate (an aggregate of the split 2x2x2 aggregation has
// at most eight members): lane j forms the residuals of members j, j+8, ...
// and the eight partial sums meet in a fixed butterfly, so the result does not
// depend on scheduling.  With xc: also the coarse level's first Chebyshev
// step, xc = c0 D^-1 b_c.
constexpr int RLANES = 8;
constexpr int ELL_K8 = 8;   // row width of the fixed-width ELL kernels

template <typename T>
__global__ __launch_bounds__(256) void k_restrict_rows(FineLevelT<T> f, int nc, const int *__restrict__ mptr,
                                                       const int *__restrict__ mem, const T *__restrict__ b,
                                                       const T *__restrict__ x, T *__restrict__ bc, const Scal *sc,
                                                       long long vs, long long vsc, T *__restrict__ xc,
                                                       const T *__restrict__ dinv, T c0)
{
    const bool done = ell_stopped(sc);
    b += blockIdx.y * vs;
    x += blockIdx.y * vs;
    bc += blockIdx.y * vsc;
    if (xc) xc += blockIdx.y * vsc;
    const int j = threadIdx.x % RLANES;
    // the eight lanes of a group share p, so they run the same rounds (the butterfly needs all of them)
    for (int p = (blockIdx.x * blockDim.x + threadIdx.x) / RLANES; p < nc; p += gridDim.x * blockDim.x / RLANES) {
        const int q0 = mptr[p], q1 = mptr[p + 1];
        T s = T(0);
        for (int q = q0 + j; q < q1; q += RLANES) s += fine_resid(f, b, x, mem[q]);
#pragma unroll
        for (int m = 1; m < RLANES; m <<= 1) s += __shfl_xor(s, m, RLANES);
        if (j == 0 && !done) {
            bc[p] = s;
            if (xc) xc[p] = c0 * s * dinv[p];
        }
    }
}

// The same restriction from the direct member table (aggregates of at most eight members; lane j of a
// group takes member j): the member index, then the member's row or stencil, then the neighbours, with no
// wait inside a round.  FELL: the finer level is an ELL level stored with 8 entries per row; otherwise a
// structured level with stored weights.  The stop flag only guards the stores.
template <typename T, bool FELL>
__global__ __launch_bounds__(256) void k_restrict8(FineLevelT<T> f, int nc, const int *__restrict__ memb,
                                                   const T *__restrict__ b, const T *__restrict__ x,
                                                   T *__restrict__ bc, const Scal *sc, long long vs, long long vsc,
                                                   T *__restrict__ xc, const T *__restrict__ dinv, T c0)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int p = (int)(t / RLANES), j = (int)(t % RLANES);
    const bool inr = p < nc;   // (every lane of a group reaches the butterfly)
    const int stop = sc[blockIdx.y].done;
    b += blockIdx.y * vs;
    x += blockIdx.y * vs;
    bc += blockIdx.y * vsc;
    // unconditional loads at clamped indices (a load under a condition becomes a branch that waits for it)
    const int mi = memb[inr ? (long long)p * RLANES + j : 0];
    const T dq = (xc ? dinv : b)[inr ? p : 0];
    const int i = inr ? mi : -1;
    const T dp = xc ? dq : T(0);
    const long long ii = i >= 0 ? i : 0;   // a valid row for the loads of a lane without a member
    T r;
    if constexpr (FELL) {
        int jj[ELL_K8];
        T vv[ELL_K8];
#pragma unroll
        for (int k = 0; k < ELL_K8; ++k) {
            jj[k] = f.col[(long long)k * f.n + ii];
            vv[k] = f.val[(long long)k * f.n + ii];
        }
        const T xi = x[ii], bi = b[ii];
        T xj[ELL_K8];
#pragma unroll
        for (int k = 0; k < ELL_K8; ++k) xj[k] = x[jj[k] >= 0 ? jj[k] : ii];
        T y = T(0);
#pragma unroll
        for (int k = 0; k < ELL_K8; ++k) y += (jj[k] >= 0 ? vv[k] : T(0)) * (xi - xj[k]);
        r = bi - y;
    } else {
        r = fine_resid(f, b, x, ii);
    }
    T sum = i >= 0 ? r : T(0);
#pragma unroll
    for (int m = 1; m < RLANES; m <<= 1) sum += __shfl_xor(sum, m, RLANES);
    if (j == 0 && inr && !stop) {
        bc[p] = sum;
        if (xc) xc[blockIdx.y * vsc + p] = c0 * sum * dp;
    }
}

// inverse diagonals (0 where the diagonal vanishes) of an ELL level
__global__ void k_dinv_ell(int n, int K, const int *__restrict__ col, const double *__restrict__ val,
                           double *__restrict__ d64, float *__restrict__ d32)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int k = 0; k < K; ++k)
            if (col[(long long)k * n + i] >= 0) d += val[(long long)k * n + i];
        const double v = d > 0.0 ? 1.0 / d : 0.0;
        d64[i] = v;
        d32[i] = (float)v;
    }
}

hipError_t launch_dinv_ell(int n, int K, const int *col, const double *val, double *d64, float *d32, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_dinv_ell, dim3(gblocks(n)), dim3(256), 0, s, n, K, col, val, d64, d32);
    return hipGetLastError();
}

// The same step for levels stored with ELL_K8 entries per row (every level with rows of at most that many;
// the build pads them to it), one row per thread, written so that a
// thread's loads go out in two rounds without a wait in between the loads of a round: first its row (the
// eight column indices and values, b, d and its own x, and with the prolongation its aggregate), then the
// gathers of the neighbours' x (and their aggregates and coarse values).  The stop flag is loaded with the
// first round and tested after it was issued (the opaque copy keeps the compiler from testing it first,
// which would put one more memory round trip in front of the loads).
// (No __restrict__ here: with it the compiler may move the row loads past the opaque flag and its test.)
template <typename T, bool PRO>
__global__ __launch_bounds__(256) void k_ell_cheb_step8(int n, int K, const int *col, const T *val, const T *b,
                                                        const T *xin, T *xout, const T *din, T *dout, T c1, T c2,
                                                        const Scal *sc, long long vs, const int *agg, const T *xc,
                                                        T scale, long long vsc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int stop = sc[blockIdx.y].done;
    b += blockIdx.y * vs;
    xin += blockIdx.y * vs;
    xout += blockIdx.y * vs;
    const bool has_d = din != nullptr;
    const T *dsrc = has_d ? din + blockIdx.y * vs : xin;   // (a valid address either way)
    if (dout) dout += blockIdx.y * vs;
    if (PRO) xc += blockIdx.y * vsc;
    int j[ELL_K8];
    T v[ELL_K8];
#pragma unroll
    for (int k = 0; k < ELL_K8; ++k) {
        j[k] = col[(long long)k * n + i];
        v[k] = val[(long long)k * n + i];
    }
    const T bi = b[i];
    const T dd = dsrc[i];
    const T x0 = xin[i];
    const int a0 = PRO ? agg[i] : -1;
    asm volatile("" : "+s"(stop) : : "memory");
    if (stop) return;
    // second round: the neighbours (padding entries read the row's own slot with weight 0)
    T xj[ELL_K8];
    int aj[ELL_K8];
#pragma unroll
    for (int k = 0; k < ELL_K8; ++k) {
        const int jj = j[k] >= 0 ? j[k] : i;
        xj[k] = xin[jj];
        if (PRO) aj[k] = agg[jj];
    }
    T xi = x0;
    if (PRO) {
        const T c0v = xc[a0 >= 0 ? a0 : 0];
        T cj[ELL_K8];
#pragma unroll
        for (int k = 0; k < ELL_K8; ++k) cj[k] = xc[aj[k] >= 0 ? aj[k] : 0];
        xi = a0 >= 0 ? x0 + scale * c0v : x0;
#pragma unroll
        for (int k = 0; k < ELL_K8; ++k) xj[k] = aj[k] >= 0 ? xj[k] + scale * cj[k] : xj[k];
    }
    T y = T(0), d = T(0);
#pragma unroll
    for (int k = 0; k < ELL_K8; ++k) {
        const T w = j[k] >= 0 ? v[k] : T(0);
        d += w;
        y += w * (xi - xj[k]);
    }
    T xo = T(0), dn = T(0);
    if (d > T(0)) {
        const T dold = has_d ? dd : xi;
        dn = c1 * dold + c2 * (bi - y) / d;
        xo = xi + dn;
    }
    xout[i] = xo;
    if (dout) dout[i] = dn;
}

// x_f += scale * x_c[agg]
template <typename T>
__global__ void k_prolong_agg(long long n, const int *__restrict__ agg, T *__restrict__ x, const T *__restrict__ xc,
                              T scale, const Scal *sc, long long vs, long long vsc)
{
    // the stop flag guards the stores only (tested before the loads it would cost one more round trip)
    const bool stop = ell_stopped(sc);
    x += blockIdx.y * vs;
    xc += blockIdx.y * vsc;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int a = agg[i];
        const T xv = x[i];
        const T cv = xc[a >= 0 ? a : 0];
        // (stored unconditionally, unchanged where nothing applies, so that the load of x is not moved
        // behind the aggregate's)
        x[i] = a >= 0 && !stop ? xv + scale * cv : xv;
    }
}

template <typename T>
hipError_t launch_ell_cheb_first(int n, int K, const int *col, const T *val, const T *b, T *x, T c0, const Scal *sc,
                                 const Batch &bt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_ell_cheb_first<T>, dim3(gblocks(n), bt.n), dim3(256), 0, s, n, K, col, val, b, x, c0, sc,
                       bt.vs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ell_cheb_step(int n, int K, const int *col, const T *val, const T *b, const T *xin, T *xout,
                                const T *din, T *dout, T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s,
                                const int *agg, const T *xc, T scale)
{
    if (n <= 0) return hipSuccess;
    if (agg && !xc) return hipErrorInvalidValue;
    const long long nb = (n + 255) / 256;
    if (K == ELL_K8 && sc && nb <= 65536) {
        if (agg)
            SPFD_LAUNCH((k_ell_cheb_step8<T, true>), dim3((unsigned)nb, bt.n), dim3(256), 0, s, n, K, col, val, b, xin,
                        xout, din, dout, c1, c2, sc, bt.vs, agg, xc, scale, bt.vsc);
        else
            SPFD_LAUNCH((k_ell_cheb_step8<T, false>), dim3((unsigned)nb, bt.n), dim3(256), 0, s, n, K, col, val, b, xin,
                        xout, din, dout, c1, c2, sc, bt.vs, agg, xc, scale, bt.vsc);
        return hipGetLastError();
    }
    SPFD_LAUNCH(k_ell_cheb_step<T>, dim3(gblocks(n), bt.n), dim3(256), 0, s, n, K, col, val, b, xin, xout, din, dout,
                c1, c2, sc, bt.vs, agg, xc, scale, bt.vsc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_members(const FineLevelT<T> &f, long long nrows, const T *b, const T *x, int nc,
                                   const int *mptr, const int *mem, T *bc, const Scal *sc, const Batch &bt,
                                   hipStream_t s, T *xc, const T *dinv_c, T c0, const int *memb)
{
    if (nc <= 0 || nrows <= 0) return hipSuccess;
    if (xc && !dinv_c) return hipErrorInvalidValue;
    const long long nt = (long long)nc * RLANES, nbk = (nt + 255) / 256;
    if (memb && sc && nbk <= 65536 && (f.w || f.K == ELL_K8)) {
        if (f.w)
            SPFD_LAUNCH((k_restrict8<T, false>), dim3((unsigned)nbk, bt.n), dim3(256), 0, s, f, nc, memb, b, x, bc, sc,
                        bt.vs, bt.vsc, xc, dinv_c, c0);
        else
            SPFD_LAUNCH((k_restrict8<T, true>), dim3((unsigned)nbk, bt.n), dim3(256), 0, s, f, nc, memb, b, x, bc, sc,
                        bt.vs, bt.vsc, xc, dinv_c, c0);
        return hipGetLastError();
    }
    SPFD_LAUNCH(k_restrict_rows<T>, dim3(gblocks((long long)nc * RLANES, 256), bt.n), dim3(256), 0, s, f, nc, mptr,
                mem, b, x, bc, sc, bt.vs, bt.vsc, xc, dinv_c, c0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_agg(long long n, const int *agg, T *x, const T *xc, T scale, const Scal *sc,
                              const Batch &bt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_prolong_agg<T>, dim3(gblocks(n), bt.n), dim3(256), 0, s, n, agg, x, xc, scale, sc, bt.vs,
                       bt.vsc);
    return hipGetLastError();
}

#define SPFD_INST_ELL(T)                                                                                            \
    template hipError_t launch_ell_cheb_first<T>(int, int, const int *, const T *, const T *, T *, T, const Scal *, \
                                                 const Batch &, hipStream_t);                                       \
    template hipError_t launch_ell_cheb_step<T>(int, int, const int *, const T *, const T *, const T *, T *,         \
                                                const T *, T *, T, T, const Scal *, const Batch &, hipStream_t,     \
                                                const int *, const T *, T);                                         \
    template hipError_t launch_restrict_members<T>(const FineLevelT<T> &, long long, const T *, const T *, int,      \
                                                   const int *, const int *, T *, const Scal *, const Batch &,      \
                                                   hipStream_t, T *, const T *, T, const int *);                    \
    template hipError_t launch_prolong_agg<T>(long long, const int *, T *, const T *, T, const Scal *,             \
                                              const Batch &, hipStream_t);
SPFD_INST_ELL(double)
SPFD_INST_ELL(float)

// ---------------------------------------------------------------- coarsest level given as ELL
// unknowns = rows with D > 0, in row order; adjacency among them
__global__ void k_coarse_enum_ell(int n, int K, const int *__restrict__ col, const double *__restrict__ val,
                                  int *dof_of_row, int *row_of_dof, int *ndof, int maxdof)
{
    __shared__ int s[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + t;
        int isdof = 0;
        if (i < n) {
            double d = 0.0;
            for (int k = 0; k < K; ++k)
                if (col[(long long)k * n + i] >= 0) d += val[(long long)k * n + i];
            isdof = d > 0.0;
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
            dof_of_row[i] = isdof ? id : -1;
            if (isdof && id < maxdof) row_of_dof[id] = i;
        }
        __syncthreads();
        if (t == 1023) carry += s[t];
        __syncthreads();
    }
    if (t == 0) *ndof = carry;
}

hipError_t launch_coarse_enum_ell(int n, int K, const int *col, const double *val, int *dof_of_row, int *row_of_dof,
                                  int *ndof, int maxdof, hipStream_t s)
{
    SPFD_LAUNCH(k_coarse_enum_ell, dim3(1), dim3(1024), 0, s, n, K, col, val, dof_of_row, row_of_dof, ndof,
                       maxdof);
    return hipGetLastError();
}

// dense matrix of the coarsest ELL level over its unknowns (row-major n x n)
__global__ void k_coarse_dense_ell(int nrow, int K, const int *__restrict__ col, const double *__restrict__ val,
                                   const int *__restrict__ dof_of_row, const int *__restrict__ row_of_dof, int n,
                                   double *A)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)n * n;
         e += (long long)gridDim.x * blockDim.x)
        A[e] = 0.0;
}

__global__ void k_coarse_fill_ell(int nrow, int K, const int *__restrict__ col, const double *__restrict__ val,
                                  const int *__restrict__ dof_of_row, const int *__restrict__ row_of_dof, int n,
                                  double *A)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int i = row_of_dof[q];
        double d = 0.0;
        for (int k = 0; k < K; ++k) {
            const int j = col[(long long)k * nrow + i];
            if (j < 0) continue;
            const double w = val[(long long)k * nrow + i];
            d += w;
            const int m = dof_of_row[j];
            if (m >= 0) A[(long long)q * n + m] -= w;
        }
        A[(long long)q * n + q] += d;
    }
}

hipError_t launch_coarse_dense_ell(int nrow, int K, const int *col, const double *val, const int *dof_of_row,
                                   const int *row_of_dof, int n, double *A, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    SPFD_LAUNCH(k_coarse_dense_ell, dim3(gblocks((long long)n * n)), dim3(256), 0, s, nrow, K, col, val,
                       dof_of_row, row_of_dof, n, A);
    SPFD_LAUNCH(k_coarse_fill_ell, dim3(gblocks(n)), dim3(256), 0, s, nrow, K, col, val, dof_of_row,
                       row_of_dof, n, A);
    return hipGetLastError();
}

}  // namespace spfd
