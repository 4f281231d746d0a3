// Stencil kernels of the structured multigrid levels in column form.
//
// One wave owns a column segment of a brick: lane (tx, ty) = (lane & 7,
// lane >> 3) holds the nodes (tx, ty, z0 .. z0+ZPL-1) in registers.  The z
// neighbours of a node come from the lane's own registers; the lateral
// neighbours inside the brick from the lanes l-1, l+1, l-8, l+8 (cross-lane
// permutes, no memory access), and only the lanes on an x or y face of the
// brick load one extra column from the neighbour brick.  Compared with four
// lateral column loads per lane (cache hits), this frees registers, i.e.
// more HBM bytes in flight per register, and cache bandwidth: the CG step
// went from 118 to 99-104 us on the 8.9M-unknown body, the smoothing steps
// by 5-15 % (measured).  Every load of the wave is independent of the
// others, so a wave has all of them in flight at once.  The stencil needs no workgroup barrier: this is
// what keeps HBM busy (a 512-thread brick workgroup with a barrier holds too
// few bytes in flight per compute unit for the latency of HBM3E).  The
// permutes need all 64 lanes: the stencil loops run in wave-uniform control
// flow and only the stores depend on the lane.
//
// Operator forms (Eq. (3), the matrix G^T M_sigma G):
//  * label form (finest level): the conductivities of the voxel planes the
//    segment touches are staged per wave in LDS, label -> sigma through a
//    per-wave copy of the sigma table, and the six edge conductances of a node
//    are formed on the fly with the same summation order as the setup kernel;
//  * stored form (coarser structured levels, or per-voxel conductivities):
//    three weight arrays (edge to +x, +y, +z); the minus-side weights are the
//    plus-side weights of the minus neighbours.
#include <math.h>
#include <type_traits>
#include <hip/hip_fp16.h>

#include "kernels.h"

namespace spfd {

constexpr int CWAVES = 4;                 // waves per workgroup
constexpr int CTHREADS = 64 * CWAVES;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// value of v in lane `src` of the wave (src taken modulo 64)
template <typename T>
__device__ __forceinline__ T lane_get(T v, int src)
{
    return __shfl(v, src & 63, 64);
}

// 1/d: the hardware reciprocal in FP32 (about 1 ulp, the FP32 smoother's own
// precision), a correctly rounded division in FP64
template <typename T>
__device__ __forceinline__ T recip(T d)
{
    return T(1) / d;
}
template <>
__device__ __forceinline__ float recip<float>(float d)
{
    return __builtin_amdgcn_rcpf(d);
}

// Where a wave's segment lies.  Absent neighbour bricks hold no unknowns and
// the edges into them have conductance 0: in their place a lane reads its own
// slot (a finite stand-in that only meets weights of 0).  Columns without
// unknowns hold zeros and are never written.
template <int ZPL>
struct Seg {
    static constexpr int WPB = 8 / ZPL;           // waves per brick
    static constexpr int BPG = CWAVES / WPB;      // bricks per workgroup
    int bk;                                       // brick (-1: this wave has none)
    int grp;                                      // brick group of the workgroup (-1: padding)
    int z0, lane, tx, ty;
    int nb[6];                                    // neighbour bricks of bk (-1: absent)
    long long self;                               // slot of (tx, ty, z0)
    long long xe, ye;                             // lanes with tx = 0 or 7 (ty = 0 or 7): slot of the x (y)
                                                  // neighbour of (tx, ty, z0) in the next brick
    long long zm, zp;                             // (tx, ty, z0-1) and (tx, ty, z0+ZPL)
    bool has[6];                                  // neighbour slot exists
    bool bx, by;                                  // xe (ye) is to be read: face lane, neighbour brick present
    bool active;                                  // the lane's node column holds an unknown
    bool stop;                                    // the launch row's right side has stopped: return at once
    int hc;                                       // the launch row's Scal::hcount (CG search-direction slot)
};

template <int ZPL>
__host__ __device__ __forceinline__ int col_ngroups(int nb)
{
    return (nb + Seg<ZPL>::BPG - 1) / Seg<ZPL>::BPG;
}

// (with packed models, launch row blockIdx.y = m covers model m's bricks; grp
// is the group's index within the row, the index of its partial sum)
//
// The uniform records a wave needs before its first vector load (the brick's
// neighbour table and column mask) and the stop flag of its right side are
// scalar loads from memory.  They are issued as one batch (at brick 0 for a
// wave without a brick) and waited for once: a branch on any of them, or on
// whether a pointer is given, before the others were issued would cost one
// more memory round trip per wave, a large part of a wave's life in these
// short kernels.  So the column mask and the scalars are required (launches
// that never stop pass zeroed scalars).  The stop flag is written only by an
// earlier kernel of the stream, so a plain load sees it.
template <int ZPL, bool FLAG = true>
__device__ __forceinline__ Seg<ZPL> make_seg(const Topo &topo, const Scal *sc)
{
    Seg<ZPL> s;
    const int2 rg = topo.np ? topo.prange[blockIdx.y] : make_int2(0, topo.nb);
    const int cnt = rg.y, first = rg.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the map covers the launch row's full length (with packed models, the largest model's groups), so
    // that each group of a smaller model has exactly one workgroup
    s.grp = xcd_brick(blockIdx.x, col_ngroups<ZPL>(topo_count(topo)));
    if (s.grp >= col_ngroups<ZPL>(cnt)) s.grp = -1;
    s.lane = threadIdx.x & 63;
    s.tx = s.lane & 7;
    s.ty = s.lane >> 3;
    s.z0 = (wave % Seg<ZPL>::WPB) * ZPL;
    const int b = s.grp < 0 ? -1 : s.grp * Seg<ZPL>::BPG + wave / Seg<ZPL>::WPB;
    s.bk = b >= 0 && b < cnt ? first + b : -1;
    const int bl = s.bk < 0 ? 0 : s.bk;
    const unsigned long long cm = topo.cmask[bl];
    if constexpr (FLAG) {
        // (adjacent fields of the row's scalars: loaded together)
        s.stop = sc[blockIdx.y].done != 0;
        s.hc = sc[blockIdx.y].hcount;
    } else {
        s.stop = false;
        s.hc = 0;
    }
    brick_nbrs(topo.nbr, bl, s.nb);
    s.active = false;
    if (s.bk < 0) return s;
    // a column without unknowns stores nothing (its slots stay zero) and
    // loads only what its neighbours' stencils need (nothing in most kernels);
    // edges into it have conductance 0
    s.active = (cm >> s.lane) & 1ull;
    const int *nb = s.nb;
    const long long base = (long long)s.bk * BS;
    const int t0 = s.lane + 64 * s.z0;
    s.self = base + t0;
    s.has[NMX] = s.tx > 0 || nb[NMX] >= 0;
    s.has[NPX] = s.tx < 7 || nb[NPX] >= 0;
    s.has[NMY] = s.ty > 0 || nb[NMY] >= 0;
    s.has[NPY] = s.ty < 7 || nb[NPY] >= 0;
    const int ex = s.tx == 0 ? nb[NMX] : (s.tx == 7 ? nb[NPX] : -1);
    const int ey = s.ty == 0 ? nb[NMY] : (s.ty == 7 ? nb[NPY] : -1);
    s.bx = ex >= 0;
    s.by = ey >= 0;
    s.xe = s.bx ? (long long)ex * BS + t0 + (s.tx == 0 ? 7 : -7) : s.self;
    s.ye = s.by ? (long long)ey * BS + t0 + (s.ty == 0 ? 56 : -56) : s.self;
    if (s.z0 > 0) {
        s.has[NMZ] = true;
        s.zm = s.self - 64;
    } else {
        s.has[NMZ] = nb[NMZ] >= 0;
        s.zm = s.has[NMZ] ? (long long)nb[NMZ] * BS + s.lane + 448 : s.self;
    }
    if (s.z0 + ZPL < 8) {
        s.has[NPZ] = true;
        s.zp = s.self + 64 * ZPL;
    } else {
        s.has[NPZ] = nb[NPZ] >= 0;
        s.zp = s.has[NPZ] ? (long long)nb[NPZ] * BS + s.lane : s.self + 64 * (ZPL - 1);
    }
    return s;
}

// LDS per wave of the label form: sigma table copy + sigma of ZPL+1 voxel planes
template <typename T, int ZPL>
struct ColLds {
    static constexpr int NE = 81 * (ZPL + 1);
    static constexpr int PER_WAVE = MAX_LABELS + ((NE + 3) & ~3);
};

template <typename T, int ZPL, bool LABEL>
struct SegOp;

// Label form.  Plane c of the wave holds the voxels of tile plane z0 + c
// (tile plane k = voxel layer below node layer k of the brick).
template <typename T, int ZPL>
struct SegOp<T, ZPL, true> {
    static constexpr int NE = ColLds<T, ZPL>::NE;
    static constexpr int NWD = (NE + 3) / 4;      // label dwords (81 z0 is a multiple of 4)
    static constexpr int NLD = (NWD + 63) / 64;
    uint32_t lab[NLD];
    T tv[4];
    T *tab, *sig;
    T g[3];
    T lo[4];

    __device__ __forceinline__ void load(const OpArgs<T> &op, const Seg<ZPL> &s, T *lds)
    {
        tab = lds + (threadIdx.x >> 6) * ColLds<T, ZPL>::PER_WAVE;
        sig = tab + MAX_LABELS;
        g[0] = op.geo4[0];
        g[1] = op.geo4[1];
        g[2] = op.geo4[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) tv[k] = (s.lane + 64 * k < op.nlab) ? op.table[s.lane + 64 * k] : T(0);
        const uint32_t *tl = (const uint32_t *)(op.tiles + (long long)s.bk * TILE_BYTES + 81 * s.z0);
#pragma unroll
        for (int k = 0; k < NLD; ++k) lab[k] = (s.lane + 64 * k < NWD) ? tl[s.lane + 64 * k] : 0u;
    }

    __device__ __forceinline__ void stage(const OpArgs<T> &op, const Seg<ZPL> &s)
    {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (s.lane + 64 * k < op.nlab) tab[s.lane + 64 * k] = tv[k];
        wave_sync();
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int e = 4 * (s.lane + 64 * k);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (e + m < NE) sig[e + m] = tab[(lab[k] >> (8 * m)) & 255u];
        }
        wave_sync();
        plane(s, 0, lo);
    }

    __device__ __forceinline__ void plane(const Seg<ZPL> &s, int c, T q[4]) const
    {
        const T *p = sig + 81 * c + s.tx + 9 * s.ty;
        q[0] = p[0];
        q[1] = p[1];
        q[2] = p[9];
        q[3] = p[10];
    }

    // weights of node z0+z (call with z = 0, 1, ... in order); the sums keep the
    // order of the setup kernel: (j-1,k-1), (j,k-1), (j-1,k), (j,k) of the other axes
    __device__ __forceinline__ void weights(const Seg<ZPL> &s, int z, T W[6])
    {
        T hi[4];
        plane(s, z + 1, hi);
        W[NPX] = (((lo[1] + lo[3]) + hi[1]) + hi[3]) * g[0];
        W[NMX] = (((lo[0] + lo[2]) + hi[0]) + hi[2]) * g[0];
        W[NPY] = (((lo[2] + lo[3]) + hi[2]) + hi[3]) * g[1];
        W[NMY] = (((lo[0] + lo[1]) + hi[0]) + hi[1]) * g[1];
        W[NPZ] = (((hi[0] + hi[1]) + hi[2]) + hi[3]) * g[2];
        W[NMZ] = (((lo[0] + lo[1]) + lo[2]) + lo[3]) * g[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) lo[k] = hi[k];
    }
};

// Stored form: w[d*stride + n] = conductance of the edge from n to +d; the
// minus-side weights are the plus-side weights of the minus neighbours, inside
// the brick taken from lanes l-1 and l-8, on the minus faces loaded from the
// neighbour brick.  Columns without unknowns have weights 0 (every edge at
// such a node has conductance 0).
template <typename T, int ZPL>
struct SegOp<T, ZPL, false> {
    T wp[3][ZPL], wmx[ZPL], wmy[ZPL], wmz;

    // Lanes of columns with unknowns load their own weights, the lanes of
    // the minus faces also the neighbour brick's (stand-in slots where it is
    // absent, masked afterwards).  Nothing converts a value loaded under a
    // lane condition: a use sunk into such a branch would wait for its load
    // there, one load at a time.
    // FP16 weights (scaled by op.whs): every load unconditional, including
    // the faces', since each value is converted where it is used
    __device__ __forceinline__ void load_h(const OpArgs<T> &op, const Seg<ZPL> &s)
    {
        const uint16_t *w = op.wh;
        const long long st = op.stride;
        uint16_t hp[3][ZPL], hx[ZPL], hy[ZPL];
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            hp[0][z] = w[s.self + 64 * z];
            hp[1][z] = w[st + s.self + 64 * z];
            hp[2][z] = w[2 * st + s.self + 64 * z];
            hx[z] = w[s.xe + 64 * z];
            hy[z] = w[st + s.ye + 64 * z];
        }
        const uint16_t hz = w[2 * st + s.zm];
        const T sc = (T)op.whs;
        const bool mx = s.active && s.bx && s.tx == 0, my = s.active && s.by && s.ty == 0;
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
#pragma unroll
            for (int d = 0; d < 3; ++d) wp[d][z] = (T)__half2float(__ushort_as_half(hp[d][z])) * sc;
            wmx[z] = mx ? (T)__half2float(__ushort_as_half(hx[z])) * sc : T(0);
            wmy[z] = my ? (T)__half2float(__ushort_as_half(hy[z])) * sc : T(0);
        }
        wmz = s.active && s.has[NMZ] ? (T)__half2float(__ushort_as_half(hz)) * sc : T(0);
    }

    __device__ __forceinline__ void load(const OpArgs<T> &op, const Seg<ZPL> &s, T *)
    {
        if constexpr (std::is_same<T, float>::value) {
            if (op.wh) {
                load_h(op, s);
                return;
            }
        }
        const T *w = op.w;
        const long long st = op.stride;
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            wp[0][z] = wp[1][z] = wp[2][z] = T(0);
            wmx[z] = wmy[z] = T(0);
        }
        // a column without unknowns has weights 0 (not loaded)
        if (s.active) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) {
                wp[0][z] = w[s.self + 64 * z];
                wp[1][z] = w[st + s.self + 64 * z];
                wp[2][z] = w[2 * st + s.self + 64 * z];
            }
        }
        wmz = w[2 * st + s.zm];
        // minus-face weights: only the lanes on that face load (as in SegVals)
        if (s.active && s.tx == 0) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) wmx[z] = w[s.xe + 64 * z];
        }
        if (s.active && s.ty == 0) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) wmy[z] = w[st + s.ye + 64 * z];
        }
        const bool mx = s.active && s.bx && s.tx == 0, my = s.active && s.by && s.ty == 0;
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            wmx[z] = mx ? wmx[z] : T(0);
            wmy[z] = my ? wmy[z] : T(0);
        }
        wmz = s.active && s.has[NMZ] ? wmz : T(0);
    }

    __device__ __forceinline__ void stage(const OpArgs<T> &, const Seg<ZPL> &) {}

    // all 64 lanes of the wave must call this
    __device__ __forceinline__ void weights(const Seg<ZPL> &s, int z, T W[6])
    {
        const T mx = lane_get(wp[0][z], s.lane - 1), my = lane_get(wp[1][z], s.lane - 8);
        W[NPX] = wp[0][z];
        W[NPY] = wp[1][z];
        W[NPZ] = wp[2][z];
        W[NMX] = s.tx > 0 ? mx : wmx[z];
        W[NMY] = s.ty > 0 ? my : wmy[z];
        W[NMZ] = z > 0 ? wp[2][z - 1] : wmz;
    }
};

// values of x along the segment, the face lanes' columns in the neighbour
// bricks (ex, ey) and the two z ends.  Nothing is masked: a column without
// unknowns holds zeros (read from its slots, or set without a load), and
// where a neighbour is absent the value read is a finite stand-in (the
// lane's own slot) whose edge weight is exactly 0, so every term W (x0 - N)
// it enters is 0.
template <typename T, int ZPL>
struct SegVals {
    T c[ZPL], ex[ZPL], ey[ZPL], zm, zp;

    // FACES: only the lanes on an x (y) face load ex (ey), the others read 0
    // (they never use it); a quarter of the lanes per face load instruction
    // (finest first two smoothing steps 44 -> 39.5 us); lanes of columns
    // without unknowns load nothing (-1.2 % per solve).  Off where the
    // caller converts the values (a conversion sunk into the branch would
    // wait for each load there).
    template <bool FACES = true>
    __device__ __forceinline__ void load(const T *__restrict__ x, const Seg<ZPL> &s)
    {
        if constexpr (FACES) {
            // lanes of columns without unknowns load nothing (their slots hold 0)
#pragma unroll
            for (int z = 0; z < ZPL; ++z) c[z] = ex[z] = ey[z] = T(0);
            zm = zp = T(0);
            if (s.active) {
#pragma unroll
                for (int z = 0; z < ZPL; ++z) c[z] = x[s.self + 64 * z];
                zm = x[s.zm];
                zp = x[s.zp];
            }
            if (s.active && (s.tx == 0 || s.tx == 7)) {
#pragma unroll
                for (int z = 0; z < ZPL; ++z) ex[z] = x[s.xe + 64 * z];
            }
            if (s.active && (s.ty == 0 || s.ty == 7)) {
#pragma unroll
                for (int z = 0; z < ZPL; ++z) ey[z] = x[s.ye + 64 * z];
            }
        } else {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) c[z] = x[s.self + 64 * z];
            zm = x[s.zm];
            zp = x[s.zp];
#pragma unroll
            for (int z = 0; z < ZPL; ++z) {
                ex[z] = x[s.xe + 64 * z];
                ey[z] = x[s.ye + 64 * z];
            }
        }
    }

    // the six neighbours of node z0+z; all 64 lanes of the wave must call this
    __device__ __forceinline__ void nbrs(const Seg<ZPL> &s, int z, T N[6]) const
    {
        const T xm = lane_get(c[z], s.lane - 1), xp = lane_get(c[z], s.lane + 1);
        const T ym = lane_get(c[z], s.lane - 8), yp = lane_get(c[z], s.lane + 8);
        N[NMX] = s.tx > 0 ? xm : ex[z];
        N[NPX] = s.tx < 7 ? xp : ex[z];
        N[NMY] = s.ty > 0 ? ym : ey[z];
        N[NPY] = s.ty < 7 ? yp : ey[z];
        N[NMZ] = z > 0 ? c[z - 1] : zm;
        N[NPZ] = z < ZPL - 1 ? c[z + 1] : zp;
    }
};

template <typename T, int ZPL, bool LABEL>
__device__ __forceinline__ T *col_lds()
{
    if constexpr (LABEL) {
        __shared__ T lds[CWAVES * ColLds<T, ZPL>::PER_WAVE];
        return lds;
    } else {
        return nullptr;
    }
}

// ---------------------------------------------------------------- Chebyshev smoothing
// first step from a zero start: x = c0 D^-1 b (0 where D = 0)
template <typename T, typename TB, int ZPL, bool LABEL>
__global__ __launch_bounds__(CTHREADS) void k_col_cheb_first(OpArgs<T> op, Topo topo, const TB *__restrict__ b,
                                                             T *__restrict__ x, T c0, const Scal *sc, long long vs)
{
    T *lds = col_lds<T, ZPL, LABEL>();
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    if (s.bk < 0 || s.stop) return;
    b += blockIdx.y * vs;
    x += blockIdx.y * vs;
    SegOp<T, ZPL, LABEL> A;
    A.load(op, s, lds);
    TB braw[ZPL];
#pragma unroll
    for (int z = 0; z < ZPL; ++z) braw[z] = b[s.self + 64 * z];
    T bv[ZPL];
#pragma unroll
    for (int z = 0; z < ZPL; ++z) bv[z] = (T)braw[z];
    A.stage(op, s);
#pragma unroll
    for (int z = 0; z < ZPL; ++z) {
        T W[6];
        A.weights(s, z, W);
        const T D = diag_of(W);
        // (a scaled right side already holds D^-1 b)
        const T v = op.bscale ? c0 * bv[z] : c0 * bv[z] * recip(D);
        if (s.active) x[s.self + 64 * z] = D > T(0) ? v : T(0);
    }
}

// The first two Chebyshev steps from a zero start in one pass: the first step
// x1 = c0 D^-1 b is formed wherever the second step reads it (own segment,
// face columns, z ends; D^-1 from the stored inverse diagonal, so every wave
// forms the same value for a node) and never stored; then
//   r = b - A x1, d = c1 x1 + c2 D^-1 r, xout = x1 + d (dout = d if given).
// SB: b holds D^-1 b (op.bscale), so x1 = c0 b needs no inverse diagonal at
// all, and the own nodes form D b and D^-1 from their weights: one of the
// kernel's two vectors with halo less to load.
template <typename T, typename TB, int ZPL, bool LABEL, bool SB>
__global__ __launch_bounds__(CTHREADS) void k_col_cheb_first2(OpArgs<T> op, Topo topo, const TB *__restrict__ b,
                                                              const T *__restrict__ dinv, T *__restrict__ xout,
                                                              T *__restrict__ dout, T c0, T c1, T c2, const Scal *sc,
                                                              long long vs)
{
    T *lds = col_lds<T, ZPL, LABEL>();
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    if (s.bk < 0 || s.stop) return;
    b += blockIdx.y * vs;
    xout += blockIdx.y * vs;
    if (dout) dout += blockIdx.y * vs;
    SegOp<T, ZPL, LABEL> A;
    A.load(op, s, lds);
    SegVals<TB, ZPL> B;
    B.template load<std::is_same<T, TB>::value>(b, s);
    SegVals<T, ZPL> DI;
    if constexpr (!SB) DI.load(dinv, s);
    // x1 on the segment, the face columns and the z ends
    SegVals<T, ZPL> X;
#pragma unroll
    for (int z = 0; z < ZPL; ++z) {
        if constexpr (SB) {
            X.c[z] = c0 * (T)B.c[z];
            X.ex[z] = c0 * (T)B.ex[z];
            X.ey[z] = c0 * (T)B.ey[z];
        } else {
            X.c[z] = c0 * (T)B.c[z] * DI.c[z];
            X.ex[z] = c0 * (T)B.ex[z] * DI.ex[z];
            X.ey[z] = c0 * (T)B.ey[z] * DI.ey[z];
        }
    }
    if constexpr (SB) {
        X.zm = c0 * (T)B.zm;
        X.zp = c0 * (T)B.zp;
    } else {
        X.zm = c0 * (T)B.zm * DI.zm;
        X.zp = c0 * (T)B.zp * DI.zp;
    }
    A.stage(op, s);
#pragma unroll
    for (int z = 0; z < ZPL; ++z) {
        T W[6], N[6];
        A.weights(s, z, W);
        X.nbrs(s, z, N);
        // the stored inverse diagonal (0 where the diagonal vanishes), as in x1; SB: from the weights
        T di, bz;
        if constexpr (SB) {
            const T D = diag_of(W);
            di = D > T(0) ? recip(D) : T(0);
            bz = D * (T)B.c[z];
        } else {
            di = DI.c[z];
            bz = (T)B.c[z];
        }
        T xo = T(0), dn = T(0);
        if (s.active && di > T(0)) {
            const T r = bz - stencil_apply(X.c[z], N, W);
            dn = c1 * X.c[z] + c2 * r * di;
            xo = X.c[z] + dn;
        }
        if (s.active) {
            xout[s.self + 64 * z] = xo;
            if (dout) dout[s.self + 64 * z] = dn;
        }
    }
}

// Coarse-grid correction of a structured level, x += scale * P x_c, applied
// to the values a segment reads: the coarse node of fine node (tx,ty,tz) of
// brick b is node (4 (f.x & 1) + tx/2, ...) of the parent brick, f = coord of b.
// (From an unstructured coarser level the correction is a kernel of its own:
// fused here, its dependent index and gather loads made the step slower than
// the two kernels, measured.)
struct Prolong {
    const void *xc;
    const int *parent_slot;
    const int4 *fcoord;
    double scale;
    long long vsc;
};

__device__ __forceinline__ long long coarse_slot(const Prolong &pr, int b, int tx, int ty, int tz)
{
    const int4 f = pr.fcoord[b];
    return (long long)pr.parent_slot[b] * BS + ((f.x & 1) * 4 + (tx >> 1)) + 8 * ((f.y & 1) * 4 + (ty >> 1)) +
           64 * ((f.z & 1) * 4 + (tz >> 1));
}

template <typename T, int ZPL>
__device__ __forceinline__ void apply_prolong(const Prolong &pr, const Topo &topo, const Seg<ZPL> &s,
                                              SegVals<T, ZPL> &X)
{
    // every lane loads from a valid slot
    const T *xc = (const T *)pr.xc + blockIdx.y * pr.vsc;
    const T sc = (T)pr.scale;
    const int *nb = s.nb;
    const int tx = s.tx, ty = s.ty, z0 = s.z0;
    // coarse slots of the lane's own column, of its face column in the x (y)
    // neighbour brick and of the two z ends (absent -> own column, never read)
    const long long c0 = coarse_slot(pr, s.bk, tx, ty, z0);
    const long long cx = s.bx ? coarse_slot(pr, tx == 0 ? nb[NMX] : nb[NPX], tx == 0 ? 7 : 0, ty, z0) : c0;
    const long long cy = s.by ? coarse_slot(pr, ty == 0 ? nb[NMY] : nb[NPY], tx, ty == 0 ? 7 : 0, z0) : c0;
    const long long czm = z0 > 0 ? coarse_slot(pr, s.bk, tx, ty, z0 - 1)
                                 : (nb[NMZ] >= 0 ? coarse_slot(pr, nb[NMZ], tx, ty, 7) : c0);
    const int ze = z0 + ZPL;
    const long long czp = ze < 8 ? coarse_slot(pr, s.bk, tx, ty, ze) : (nb[NPZ] >= 0 ? coarse_slot(pr, nb[NPZ], tx, ty, 0) : c0);
    T v0[ZPL / 2], vx[ZPL / 2], vy[ZPL / 2];
#pragma unroll
    for (int h = 0; h < ZPL / 2; ++h) {
        v0[h] = xc[c0 + 64 * h];
        vx[h] = xc[cx + 64 * h];
        vy[h] = xc[cy + 64 * h];
    }
    const T vm = xc[czm], vp = xc[czp];
    // unmasked, like SegVals: a stand-in value only meets edge weights of 0
#pragma unroll
    for (int z = 0; z < ZPL; ++z) {
        X.c[z] += sc * v0[z >> 1];
        X.ex[z] += sc * vx[z >> 1];
        X.ey[z] += sc * vy[z >> 1];
    }
    X.zm += sc * vm;
    X.zp += sc * vp;
}

// Dot products of the outer flexible CG that ride on the last finest-level
// smoothing step: partials (one per workgroup) of z.r into part[g] and of
// z.q into part[nparts + g], z being the step's output.
struct Dots {
    const double *q;
    double *part;
    int ps;        // partial stride per right side
    int nparts;
};

// general step: r = b - A xin; d = c1 d_old + c2 D^-1 r; xout = xin + d.
// d_old, the previous step's update x_k - x_{k-1} (dmode, CHEB_D_*):
//   FROM_X   d_old = xin (right after a zero start, or unused when c1 = 0);
//   STORED   read from din;
//   PREV     xin - x_{k-1}, with x_{k-1} read from xout before it is
//            overwritten: the ping-pong buffer the step writes holds the
//            iterate before xin, so no d has to be stored (4 bytes per node
//            written and read less);
//   PREV_PRO as PREV where the previous step applied the coarse-grid
//            correction to its input on the fly: x_{k-1} in xout lacks it,
//            so it is applied again here (pr, own column only).
// With PRO, xin is first corrected from the coarser level (the prolongation
// of the upward leg, fused into the first post-smoothing step); with DOT the
// step also forms the CG dot products of its output with b (the residual the
// cycle was given, as the cycle reads it) and with q.
template <typename T, typename TB, int ZPL, bool LABEL, bool PRO, bool DOT>
__global__ __launch_bounds__(CTHREADS) void k_col_cheb_step(OpArgs<T> op, Topo topo, const TB *__restrict__ b,
                                                            const T *__restrict__ xin, T *__restrict__ xout,
                                                            const T *__restrict__ din, T *__restrict__ dout, T c1,
                                                            T c2, const Scal *sc, long long vs, Prolong pr, Dots dt,
                                                            int dmode)
{
    T *lds = col_lds<T, ZPL, LABEL>();
    __shared__ double red[2][CWAVES];
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    if ((DOT ? s.grp < 0 : s.bk < 0) || s.stop) return;
    double dzr = 0.0, dzq = 0.0;
    if (s.bk >= 0) {
        b += blockIdx.y * vs;
        xin += blockIdx.y * vs;
        xout += blockIdx.y * vs;
        if (din) din += blockIdx.y * vs;
        if (dout) dout += blockIdx.y * vs;
        SegOp<T, ZPL, LABEL> A;
        A.load(op, s, lds);
        SegVals<T, ZPL> X;
        X.load(xin, s);
        // (loaded by every lane, used only where the column holds unknowns)
        TB braw[ZPL];
        T dv[ZPL], xprev[ZPL];
        double qv[DOT ? ZPL : 1];
#pragma unroll
        for (int z = 0; z < ZPL; ++z) braw[z] = dv[z] = xprev[z] = 0;
        if (s.active || !std::is_same<T, TB>::value) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) braw[z] = b[s.self + 64 * z];
        }
        if (dmode == CHEB_D_STORED && s.active) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) dv[z] = din[s.self + 64 * z];
        }
        if (dmode >= CHEB_D_PREV && s.active) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) xprev[z] = xout[s.self + 64 * z];
        }
        // PREV_PRO: the correction of the own column, as apply_prolong forms it (every lane loads from a valid slot)
        T vpro[ZPL / 2];
        if (dmode == CHEB_D_PREV_PRO) {
            const T *xc = (const T *)pr.xc + blockIdx.y * pr.vsc;
            const long long cs = coarse_slot(pr, s.bk, s.tx, s.ty, s.z0);
#pragma unroll
            for (int h = 0; h < ZPL / 2; ++h) vpro[h] = xc[cs + 64 * h];
        }
        if constexpr (DOT) {
            // z.q only for the flexible beta (q == nullptr: partials of 0)
#pragma unroll
            for (int z = 0; z < ZPL; ++z) qv[z] = 0.0;
            if (dt.q && s.active) {
                const double *q = dt.q + blockIdx.y * vs;
#pragma unroll
                for (int z = 0; z < ZPL; ++z) qv[z] = q[s.self + 64 * z];
            }
        }
        T bv[ZPL];
#pragma unroll
        for (int z = 0; z < ZPL; ++z) bv[z] = (T)braw[z];
        if constexpr (PRO) apply_prolong(pr, topo, s, X);
        if (dmode == CHEB_D_FROM_X) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) dv[z] = X.c[z];
        } else if (dmode == CHEB_D_PREV_PRO) {
            const T ps = (T)pr.scale;
#pragma unroll
            for (int z = 0; z < ZPL; ++z) {
                T xp = xprev[z];
                xp += ps * vpro[z >> 1];
                dv[z] = X.c[z] - xp;
            }
        } else if (dmode == CHEB_D_PREV) {
#pragma unroll
            for (int z = 0; z < ZPL; ++z) dv[z] = X.c[z] - xprev[z];
        }
        A.stage(op, s);
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            T W[6], N[6];
            A.weights(s, z, W);
            X.nbrs(s, z, N);
            const T D = diag_of(W);
            // b as the cycle takes it (a scaled right side holds D^-1 b)
            const T bz = op.bscale ? D * bv[z] : bv[z];
            T xo = T(0), dn = T(0);
            if (s.active && D > T(0)) {
                const T r = bz - stencil_apply(X.c[z], N, W);
                dn = c1 * dv[z] + c2 * r * recip(D);
                xo = X.c[z] + dn;
            }
            if (s.active) {
                xout[s.self + 64 * z] = xo;
                if (dout) dout[s.self + 64 * z] = dn;
                if constexpr (DOT) {
                    dzr += (double)xo * (double)bz;
                    dzq += (double)xo * qv[z];
                }
            }
        }
    }
    if constexpr (DOT) {
        dzr = wave_sum(dzr);
        dzq = wave_sum(dzq);
        if (s.lane == 0) {
            red[0][threadIdx.x >> 6] = dzr;
            red[1][threadIdx.x >> 6] = dzq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, c = 0.0;
#pragma unroll
            for (int w = 0; w < CWAVES; ++w) {
                a += red[0][w];
                c += red[1][w];
            }
            double *part = dt.part + (long long)blockIdx.y * dt.ps;
            part[s.grp] = a;
            part[dt.nparts + s.grp] = c;
        }
    }
}

// coarse right side b_c = P^T (b - A x), P = 2x2x2 piecewise-constant
// aggregation: z pairs add in the lane, x pairs across lanes l, l+1, y pairs
// across l, l+8; the lane of the even corner stores the aggregate.
// SB: b holds D^-1 b (op.bscale); then b - A x = -sum_k W_k ((x - b) - N_k),
// the stencil applied to x - b, which needs no diagonal.
template <typename T, typename TB, int ZPL, bool LABEL, bool SB>
__global__ __launch_bounds__(CTHREADS) void k_col_resid_restrict(OpArgs<T> op, Topo topo, const TB *__restrict__ b,
                                                                 const T *__restrict__ x, T *__restrict__ bc,
                                                                 const int *__restrict__ parent_slot,
                                                                 const int4 *__restrict__ fcoord, const Scal *sc,
                                                                 long long vs, long long vsc, T *__restrict__ xc,
                                                                 const T *__restrict__ dinv_c, T c0)
{
    T *lds = col_lds<T, ZPL, LABEL>();
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    if (s.bk < 0 || s.stop) return;
    b += blockIdx.y * vs;
    x += blockIdx.y * vs;
    bc += blockIdx.y * vsc;
    SegOp<T, ZPL, LABEL> A;
    A.load(op, s, lds);
    SegVals<T, ZPL> X;
    X.load(x, s);
    TB braw[ZPL];
#pragma unroll
    for (int z = 0; z < ZPL; ++z) braw[z] = b[s.self + 64 * z];
    T bv[ZPL];
#pragma unroll
    for (int z = 0; z < ZPL; ++z) bv[z] = (T)braw[z];
    const int4 fc = fcoord[s.bk];
    const long long pbase = (long long)parent_slot[s.bk] * BS;
    const int ox = (fc.x & 1) * 4 + (s.tx >> 1), oy = (fc.y & 1) * 4 + (s.ty >> 1);
    const int oz = (fc.z & 1) * 4 + (s.z0 >> 1);
    const bool corner = ((s.tx | s.ty) & 1) == 0;
    // inverse diagonals of the coarse nodes this lane may store (loaded early: no tail latency)
    T dc[ZPL / 2];
    if (xc && corner)
#pragma unroll
        for (int k = 0; k < ZPL / 2; ++k) dc[k] = dinv_c[pbase + ox + 8 * oy + 64 * (oz + k)];
    A.stage(op, s);
    T r[ZPL];
#pragma unroll
    for (int z = 0; z < ZPL; ++z) {
        T W[6], N[6];
        A.weights(s, z, W);
        X.nbrs(s, z, N);
        const T rz = SB ? -stencil_apply(X.c[z] - bv[z], N, W) : bv[z] - stencil_apply(X.c[z], N, W);
        r[z] = s.active ? rz : T(0);
    }
#pragma unroll
    for (int k = 0; k < ZPL / 2; ++k) {
        T a = r[2 * k] + r[2 * k + 1];
        a += __shfl_down(a, 1, 64);
        a += __shfl_down(a, 8, 64);
        if (corner) {
            const long long n = pbase + ox + 8 * oy + 64 * (oz + k);
            bc[n] = a;
            // the coarse level's first Chebyshev step from zero: x_c = c0 D_c^-1 b_c
            if (xc) xc[blockIdx.y * vsc + n] = c0 * a * dc[k];
        }
    }
}

// ---------------------------------------------------------------- outer CG step
// Fused CG step:
//   p_k = z_k + beta_{k-1} p_{k-1}        (p_k = z_k on the first step)
//   q_k = A p_k and the partials of p_k.q_k (one per workgroup)
// q_k is stored only where a later kernel reads it (q == nullptr: not
// stored; the residual update then forms A p_k again, k_col_rupdate).
// p_k at the neighbours is formed from z and p_{k-1}.  x is not touched: the
// search directions of a window of steps are kept (p_k in the window slot
// hcount, p_{k-1} in the slot before it), with their step sizes, and
// x += sum alpha_j p_j is formed once per window (k_x_flush), which saves
// reading and writing x (FP64) in every step.
//
// p is kept in the cycle's precision TZ (FP32 with the FP32 cycle): it is formed by one fused
// multiply-add in TZ wherever it is needed, so every wave forms the same value at a node, and q = A p
// (FP64 operator and arithmetic) and the later x += alpha p use exactly the stored p.  x and r then stay
// consistent to FP64 rounding; the rounding of p only perturbs the search directions, by as much as the
// FP32 cycle already perturbs z.
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename TZ, int ZPL, bool LABEL, bool FIRST>
__global__ __launch_bounds__(CTHREADS) void k_col_cg_step(OpArgs<double> op, Topo topo, const TZ *__restrict__ zv,
                                                          TZ *ph, long long hs, int nh, double *__restrict__ q,
                                                          double *part, Scal *sc, long long vs, int ps)
{
    constexpr bool WIDE = std::is_same<TZ, double>::value;
    double *lds = col_lds<double, ZPL, LABEL>();
    __shared__ double red[CWAVES];
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    sc += blockIdx.y;
    // a stopped right side (batched solves, a step queued past the stop) returns before its loads; a full
    // window (not reached: the host updates x first) stores nothing
    if (s.grp < 0 || s.stop || s.hc < 0 || s.hc >= nh) return;
    zv += blockIdx.y * vs;
    const TZ *__restrict__ pin = ph + (long long)(s.hc == 0 ? nh - 1 : s.hc - 1) * hs + blockIdx.y * vs;
    TZ *__restrict__ pout = ph + (long long)s.hc * hs + blockIdx.y * vs;
    if (q) q += blockIdx.y * vs;
    part += (long long)blockIdx.y * ps;
    double dot = 0.0;
    if (s.bk >= 0) {
        SegOp<double, ZPL, LABEL> A;
        A.load(op, s, lds);
        SegVals<TZ, ZPL> Z;
        Z.template load<WIDE>(zv, s);
        SegVals<TZ, ZPL> Pi;
        if constexpr (!FIRST) Pi.template load<WIDE>(pin, s);
        const TZ beta = FIRST ? TZ(0) : (TZ)sc->beta;
        // p_k on the segment, the face columns and the z ends
        SegVals<TZ, ZPL> P;
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            P.c[z] = FIRST ? Z.c[z] : fma_t<TZ>(beta, Pi.c[z], Z.c[z]);
            P.ex[z] = FIRST ? Z.ex[z] : fma_t<TZ>(beta, Pi.ex[z], Z.ex[z]);
            P.ey[z] = FIRST ? Z.ey[z] : fma_t<TZ>(beta, Pi.ey[z], Z.ey[z]);
        }
        P.zm = FIRST ? Z.zm : fma_t<TZ>(beta, Pi.zm, Z.zm);
        P.zp = FIRST ? Z.zp : fma_t<TZ>(beta, Pi.zp, Z.zp);
        A.stage(op, s);
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            double W[6], N[6];
            TZ Nt[6];
            A.weights(s, z, W);
            P.nbrs(s, z, Nt);
#pragma unroll
            for (int k = 0; k < 6; ++k) N[k] = (double)Nt[k];
            const double pc = (double)P.c[z];
            const double y = stencil_apply(pc, N, W);
            if (s.active) {
                const long long n = s.self + 64 * z;
                pout[n] = P.c[z];
                if (q) q[n] = y;
                dot += pc * y;
            }
        }
    }
    dot = wave_sum(dot);
    if (s.lane == 0) red[threadIdx.x >> 6] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < CWAVES; ++w) t += red[w];
        part[s.grp] = t;
    }
}

// ---------------------------------------------------------------- residual update
// r_{k+1} = r_k - alpha_k A p_k, the partials of ||r_{k+1}||^2 (one per
// workgroup, as in the CG step) and the FP32 copy of r (r32 nullable; with
// r32_scaled, of D^-1 r, the form an FP32 cycle in label form reads); alpha_k
// goes to the window slot of p_k for the later update of x.  A p_k
// is formed again from the stored p_k with the CG step's operator, segment
// and order of operations, so it equals the q_k that step formed for p.q bit
// for bit; reading p_k in the cycle's precision and the labels costs fewer
// bytes than storing q_k in FP64 and reading it back.
template <typename TZ, int ZPL, bool LABEL>
__global__ __launch_bounds__(CTHREADS) void k_col_rupdate(OpArgs<double> op, Topo topo, const TZ *ph, long long hs,
                                                          int nh, double *__restrict__ r, float *__restrict__ r32,
                                                          double *part, const Scal *sc, long long vs, int ps,
                                                          int r32_scaled, double *ahist)
{
    constexpr bool WIDE = std::is_same<TZ, double>::value;
    double *lds = col_lds<double, ZPL, LABEL>();
    __shared__ double red[CWAVES];
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    if (s.stop || s.hc < 0 || s.hc >= nh) return;
    const double alpha = sc[blockIdx.y].alpha;
    // the step size of this search direction, for the update of x at the end of the window
    if (blockIdx.x == 0 && threadIdx.x == 0) ahist[blockIdx.y * nh + s.hc] = alpha;
    if (s.grp < 0) return;
    const TZ *__restrict__ pv = ph + (long long)s.hc * hs + blockIdx.y * vs;
    r += blockIdx.y * vs;
    if (r32) r32 += blockIdx.y * vs;
    double rr = 0.0;
    if (s.bk >= 0) {
        SegOp<double, ZPL, LABEL> A;
        A.load(op, s, lds);
        SegVals<TZ, ZPL> P;
        P.template load<WIDE>(pv, s);
        double rv[ZPL];
#pragma unroll
        for (int z = 0; z < ZPL; ++z) rv[z] = 0.0;
        if (s.active)
#pragma unroll
            for (int z = 0; z < ZPL; ++z) rv[z] = r[s.self + 64 * z];
        A.stage(op, s);
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            double W[6], N[6];
            TZ Nt[6];
            A.weights(s, z, W);
            P.nbrs(s, z, Nt);
#pragma unroll
            for (int k = 0; k < 6; ++k) N[k] = (double)Nt[k];
            const double y = stencil_apply((double)P.c[z], N, W);
            if (s.active) {
                const long long n = s.self + 64 * z;
                const double rn = rv[z] - alpha * y;
                r[n] = rn;
                // the FP32 copy the cycle reads; scaled: D^-1 r with the FP32 reciprocal (the cycle's own
                // precision; the first smoothing steps then need no inverse diagonal), 0 at the nodes of
                // the column that are no unknowns (D = 0, r = 0)
                const float D = (float)diag_of(W);
                if (r32) r32[n] = r32_scaled ? (D > 0.0f ? (float)rn * recip(D) : 0.0f) : (float)rn;
                rr += rn * rn;
            }
        }
    }
    rr = wave_sum(rr);
    if (s.lane == 0) red[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < CWAVES; ++w) t += red[w];
        part[(long long)blockIdx.y * ps + s.grp] = t;
    }
}

// ---------------------------------------------------------------- true residual
// r = b - A x (FP64 operator, r nullable) and the partials of ||r||^2, one per
// workgroup.  (The CG's deferred x update is applied before this kernel: here
// waves read x at the neighbours of their segments while others would store.)
template <int ZPL, bool LABEL>
__global__ __launch_bounds__(CTHREADS) void k_col_resid(OpArgs<double> op, Topo topo, const double *__restrict__ b,
                                                        const double *__restrict__ x, double *__restrict__ r,
                                                        double *part, long long bvs, long long vs, int ps)
{
    double *lds = col_lds<double, ZPL, LABEL>();
    __shared__ double red[CWAVES];
    const Seg<ZPL> s = make_seg<ZPL, false>(topo, nullptr);
    if (s.grp < 0) return;
    double rr = 0.0;
    if (s.bk >= 0) {
        b += blockIdx.y * bvs;
        x += blockIdx.y * vs;
        if (r) r += blockIdx.y * vs;
        SegOp<double, ZPL, LABEL> A;
        A.load(op, s, lds);
        SegVals<double, ZPL> X;
        X.load(x, s);
        double bv[ZPL];
#pragma unroll
        for (int z = 0; z < ZPL; ++z) bv[z] = b[s.self + 64 * z];
        A.stage(op, s);
#pragma unroll
        for (int z = 0; z < ZPL; ++z) {
            double W[6], N[6];
            A.weights(s, z, W);
            X.nbrs(s, z, N);
            const double rv = bv[z] - stencil_apply(X.c[z], N, W);
            if (s.active) {
                if (r) r[s.self + 64 * z] = rv;
                rr += rv * rv;
            }
        }
    }
    rr = wave_sum(rr);
    if (s.lane == 0) red[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < CWAVES; ++w) t += red[w];
        part[(long long)blockIdx.y * ps + s.grp] = t;
    }
}

// ---------------------------------------------------------------- plain operator application
// w = A z (FP64 operator, z in the cycle's precision): the Krylov vector of
// the flexible GMRES outer solver
template <typename TZ, int ZPL, bool LABEL>
__global__ __launch_bounds__(CTHREADS) void k_col_spmv(OpArgs<double> op, Topo topo, const TZ *__restrict__ zv,
                                                       double *__restrict__ w, const Scal *sc, long long vs)
{
    double *lds = col_lds<double, ZPL, LABEL>();
    const Seg<ZPL> s = make_seg<ZPL>(topo, sc);
    if (s.bk < 0 || s.stop) return;
    zv += blockIdx.y * vs;
    w += blockIdx.y * vs;
    SegOp<double, ZPL, LABEL> A;
    A.load(op, s, lds);
    SegVals<TZ, ZPL> Z;
    Z.template load<std::is_same<TZ, double>::value>(zv, s);
    A.stage(op, s);
#pragma unroll
    for (int z = 0; z < ZPL; ++z) {
        double W[6], P[6];
        TZ N[6];
        A.weights(s, z, W);
        Z.nbrs(s, z, N);
#pragma unroll
        for (int k = 0; k < 6; ++k) P[k] = (double)N[k];
        const double y = stencil_apply((double)Z.c[z], P, W);
        if (s.active) w[s.self + 64 * z] = y;
    }
}

// ---------------------------------------------------------------- launchers
// segment lengths: 8 nodes per lane in FP32 (one wave per brick), 4 in FP64
// and in the CG step (two waves per brick), which hold twice the registers per node
template <typename T>
constexpr int zpl_cycle() { return sizeof(T) == 4 ? 8 : 4; }
constexpr int ZPL_CG = 4;

int cg_step_parts(int nb) { return col_ngroups<ZPL_CG>(nb); }
// segment of the residual update (8 nodes per lane, one wave per brick, measured no faster on the body
// phantom: 53.5 against 54.7 us, within the spread between machines, at half the occupancy in FP64)
constexpr int ZPL_RU = 4;
int rupdate_parts(int nb) { return col_ngroups<ZPL_RU>(nb); }

// the column kernels read the level's column mask and (except the true
// residual) the scalars of every launch row unconditionally
static bool col_args_ok(const Topo &topo, const Scal *sc, bool need_sc = true)
{
    return topo.cmask && topo.nbr && (sc || !need_sc);
}

template <int ZPL>
static dim3 col_grid(int nb, int nbatch)
{
    return dim3(xcd_grid(col_ngroups<ZPL>(nb)), nbatch);
}

// Coarser structured levels (stored weights) with few bricks (op.short_below,
// 8192 by default) run shorter segments: all their waves are resident at once,
// so a kernel lasts about one wave's load-to-store latency, which shrinks with
// the segment (body phantom: 8 -> 4 nodes per lane saves 0.3 ms per solve, 2
// is no better than 4).
constexpr int ZPL_SMALL = 4;

template <typename T, typename TB, int ZPL, bool LABEL>
static void cheb_first_z(const OpArgs<T> &op, Topo topo, const TB *b, T *x, T c0, const Scal *sc, const Batch &bt,
                         hipStream_t s)
{
    SPFD_LAUNCH((k_col_cheb_first<T, TB, ZPL, LABEL>), col_grid<ZPL>(topo_count(topo), bt.n), dim3(CTHREADS), 0, s, op, topo,
                b, x, c0, sc, bt.vs);
}

template <typename T, typename TB>
hipError_t launch_cheb_first(const OpArgs<T> &op, Topo topo, const TB *b, T *x, T c0, const Scal *sc, const Batch &bt,
                             hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    constexpr int Z = zpl_cycle<T>();
    if (!op.w)
        cheb_first_z<T, TB, Z, true>(op, topo, b, x, c0, sc, bt, s);
    else if (topo.nb < op.short_below)
        cheb_first_z<T, TB, ZPL_SMALL, false>(op, topo, b, x, c0, sc, bt, s);
    else
        cheb_first_z<T, TB, Z, false>(op, topo, b, x, c0, sc, bt, s);
    return hipGetLastError();
}

template <typename T, typename TB>
hipError_t launch_cheb_first2(const OpArgs<T> &op, Topo topo, const TB *b, const T *dinv, T *xout, T *dout, T c0,
                              T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    if (!dinv && !op.bscale) return hipErrorInvalidValue;
    constexpr int Z = zpl_cycle<T>();
    const dim3 g = col_grid<Z>(topo_count(topo), bt.n);
#define SPFD_F2(LB, SB) SPFD_LAUNCH((k_col_cheb_first2<T, TB, Z, LB, SB>), g, dim3(CTHREADS), 0, s, op, topo, b, dinv, \
                                    xout, dout, c0, c1, c2, sc, bt.vs)
    if (op.w) {
        if (op.bscale) SPFD_F2(false, true);
        else SPFD_F2(false, false);
    } else {
        if (op.bscale) SPFD_F2(true, true);
        else SPFD_F2(true, false);
    }
#undef SPFD_F2
    return hipGetLastError();
}

template <typename T, typename TB, int ZPL, bool LAB, bool PRO, bool DOT>
static void cheb_step_z(const OpArgs<T> &op, Topo topo, const TB *b, const T *xin, T *xout, const T *din, T *dout,
                        T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s, const Prolong &pr, Dots dt,
                        int dmode)
{
    dt.nparts = col_ngroups<ZPL>(topo_count(topo));
    SPFD_LAUNCH((k_col_cheb_step<T, TB, ZPL, LAB, PRO, DOT>), col_grid<ZPL>(topo_count(topo), bt.n), dim3(CTHREADS), 0, s, op,
                topo, b, xin, xout, din, dout, c1, c2, sc, bt.vs, pr, dt, dmode);
}

template <typename T, typename TB>
hipError_t launch_cheb_step(const OpArgs<T> &op, Topo topo, const TB *b, const T *xin, T *xout, const T *din, T *dout,
                            T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s, const T *xc,
                            const int *parent_slot, const int4 *fcoord, T pscale, const double *dot_q,
                            double *dot_part, int dmode)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    if (xin == xout) return hipErrorInvalidValue;
    if (xc && !(parent_slot && fcoord)) return hipErrorInvalidValue;
    // the legacy selection by din; the previous iterate in xout (xc: the correction to apply to it)
    if (dmode == CHEB_D_AUTO) dmode = din ? CHEB_D_STORED : CHEB_D_FROM_X;
    if (dmode < CHEB_D_FROM_X || dmode > CHEB_D_PREV_PRO) return hipErrorInvalidValue;
    if (dmode == CHEB_D_STORED && !din) return hipErrorInvalidValue;
    if (dmode == CHEB_D_PREV_PRO && !xc) return hipErrorInvalidValue;
    constexpr int Z = zpl_cycle<T>();
    const Prolong pr{xc, parent_slot, fcoord, (double)pscale, bt.vsc};
    const Dots dt{dot_q, dot_part, bt.ps, 0};
    // the dot-product partials are counted by cheb_dot_parts (segment length Z)
    const bool small = op.w && !dot_part && topo.nb < op.short_below;
    const bool pro = xc && dmode != CHEB_D_PREV_PRO;
    const int sel = (small ? 8 : 0) | (op.w ? 0 : 4) | (pro ? 2 : 0) | (dot_part ? 1 : 0);
#define SPFD_CHEB_CASE(K, ZZ, LAB, PRO, DOT)                                                                          \
    case K:                                                                                                           \
        cheb_step_z<T, TB, ZZ, LAB, PRO, DOT>(op, topo, b, xin, xout, din, dout, c1, c2, sc, bt, s, pr, dt, dmode);  \
        break;
    switch (sel) {
        SPFD_CHEB_CASE(0, Z, false, false, false)
        SPFD_CHEB_CASE(1, Z, false, false, true)
        SPFD_CHEB_CASE(2, Z, false, true, false)
        SPFD_CHEB_CASE(3, Z, false, true, true)
        SPFD_CHEB_CASE(4, Z, true, false, false)
        SPFD_CHEB_CASE(5, Z, true, false, true)
        SPFD_CHEB_CASE(6, Z, true, true, false)
        SPFD_CHEB_CASE(7, Z, true, true, true)
        SPFD_CHEB_CASE(8, ZPL_SMALL, false, false, false)
        SPFD_CHEB_CASE(10, ZPL_SMALL, false, true, false)
    default: return hipErrorInvalidValue;
    }
#undef SPFD_CHEB_CASE
    return hipGetLastError();
}

template <typename T>
int cheb_dot_parts(int nb)
{
    return col_ngroups<zpl_cycle<T>()>(nb);
}
template int cheb_dot_parts<float>(int);
template int cheb_dot_parts<double>(int);

template <typename T, typename TB, int ZPL, bool LABEL>
static void resid_restrict_z(const OpArgs<T> &op, Topo topo, const TB *b, const T *x, T *bc, const int *parent_slot,
                             const int4 *fcoord, const Scal *sc, const Batch &bt, hipStream_t s, T *xc,
                             const T *dinv_c, T c0)
{
    if (op.bscale)
        SPFD_LAUNCH((k_col_resid_restrict<T, TB, ZPL, LABEL, true>), col_grid<ZPL>(topo_count(topo), bt.n),
                    dim3(CTHREADS), 0, s, op, topo, b, x, bc, parent_slot, fcoord, sc, bt.vs, bt.vsc, xc, dinv_c, c0);
    else
        SPFD_LAUNCH((k_col_resid_restrict<T, TB, ZPL, LABEL, false>), col_grid<ZPL>(topo_count(topo), bt.n),
                    dim3(CTHREADS), 0, s, op, topo, b, x, bc, parent_slot, fcoord, sc, bt.vs, bt.vsc, xc, dinv_c, c0);
}

template <typename T, typename TB>
hipError_t launch_resid_restrict(const OpArgs<T> &op, Topo topo, const TB *b, const T *x, T *bc, const int *parent_slot,
                                 const int4 *fcoord, const Scal *sc, const Batch &bt, hipStream_t s, T *xc,
                                 const T *dinv_c, T c0)
{
    if (xc && !dinv_c) return hipErrorInvalidValue;
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    constexpr int Z = zpl_cycle<T>();
    if (!op.w)
        resid_restrict_z<T, TB, Z, true>(op, topo, b, x, bc, parent_slot, fcoord, sc, bt, s, xc, dinv_c, c0);
    else if (topo.nb < op.short_below)
        resid_restrict_z<T, TB, ZPL_SMALL, false>(op, topo, b, x, bc, parent_slot, fcoord, sc, bt, s, xc, dinv_c, c0);
    else
        resid_restrict_z<T, TB, Z, false>(op, topo, b, x, bc, parent_slot, fcoord, sc, bt, s, xc, dinv_c, c0);
    return hipGetLastError();
}

template <typename TZ>
hipError_t launch_cg_step(const OpArgs<double> &op, Topo topo, const TZ *z, TZ *ph, long long hs, int nh, double *q,
                          double *part, Scal *sc, int first, const Batch &bt, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    if (!ph || nh < 2 || nh > MAX_PHIST) return hipErrorInvalidValue;
    const dim3 g = col_grid<ZPL_CG>(topo_count(topo), bt.n);
#define SPFD_CG(LB, F) SPFD_LAUNCH((k_col_cg_step<TZ, ZPL_CG, LB, F>), g, dim3(CTHREADS), 0, s, op, topo, z, ph, hs, \
                                   nh, q, part, sc, bt.vs, bt.ps)
    if (op.w) {
        if (first) SPFD_CG(false, true);
        else SPFD_CG(false, false);
    } else {
        if (first) SPFD_CG(true, true);
        else SPFD_CG(true, false);
    }
#undef SPFD_CG
    return hipGetLastError();
}

template <typename TZ>
hipError_t launch_col_rupdate(const OpArgs<double> &op, Topo topo, const TZ *ph, long long hs, int nh, double *r,
                              float *r32, double *part, const Scal *sc, const Batch &bt, hipStream_t s, int r32_scaled,
                              double *ahist)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    if (r32_scaled && !r32) return hipErrorInvalidValue;
    if (!ph || !ahist || nh < 2 || nh > MAX_PHIST) return hipErrorInvalidValue;
    const dim3 g = col_grid<ZPL_RU>(topo_count(topo), bt.n);
    if (op.w)
        SPFD_LAUNCH((k_col_rupdate<TZ, ZPL_RU, false>), g, dim3(CTHREADS), 0, s, op, topo, ph, hs, nh, r, r32, part,
                    sc, bt.vs, bt.ps, r32_scaled, ahist);
    else
        SPFD_LAUNCH((k_col_rupdate<TZ, ZPL_RU, true>), g, dim3(CTHREADS), 0, s, op, topo, ph, hs, nh, r, r32, part,
                    sc, bt.vs, bt.ps, r32_scaled, ahist);
    return hipGetLastError();
}
template hipError_t launch_col_rupdate<double>(const OpArgs<double> &, Topo, const double *, long long, int, double *,
                                               float *, double *, const Scal *, const Batch &, hipStream_t, int,
                                               double *);
template hipError_t launch_col_rupdate<float>(const OpArgs<double> &, Topo, const float *, long long, int, double *,
                                              float *, double *, const Scal *, const Batch &, hipStream_t, int,
                                              double *);

hipError_t launch_resid(const OpArgs<double> &op, Topo topo, const double *b, const double *x, double *r,
                        double *part, long long bvs, const Batch &bt, hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, nullptr, false)) return hipErrorInvalidValue;
    const dim3 g = col_grid<ZPL_CG>(topo_count(topo), bt.n);
    if (op.w)
        SPFD_LAUNCH((k_col_resid<ZPL_CG, false>), g, dim3(CTHREADS), 0, s, op, topo, b, x, r, part, bvs, bt.vs, bt.ps);
    else
        SPFD_LAUNCH((k_col_resid<ZPL_CG, true>), g, dim3(CTHREADS), 0, s, op, topo, b, x, r, part, bvs, bt.vs, bt.ps);
    return hipGetLastError();
}

template <typename TZ>
hipError_t launch_spmv(const OpArgs<double> &op, Topo topo, const TZ *z, double *w, const Scal *sc, const Batch &bt,
                       hipStream_t s)
{
    if (topo.nb <= 0) return hipSuccess;
    if (!col_args_ok(topo, sc)) return hipErrorInvalidValue;
    const dim3 g = col_grid<ZPL_CG>(topo_count(topo), bt.n);
    if (op.w)
        SPFD_LAUNCH((k_col_spmv<TZ, ZPL_CG, false>), g, dim3(CTHREADS), 0, s, op, topo, z, w, sc, bt.vs);
    else
        SPFD_LAUNCH((k_col_spmv<TZ, ZPL_CG, true>), g, dim3(CTHREADS), 0, s, op, topo, z, w, sc, bt.vs);
    return hipGetLastError();
}
template hipError_t launch_spmv<double>(const OpArgs<double> &, Topo, const double *, double *, const Scal *,
                                        const Batch &, hipStream_t);
template hipError_t launch_spmv<float>(const OpArgs<double> &, Topo, const float *, double *, const Scal *,
                                       const Batch &, hipStream_t);

#define SPFD_INST_COL(T, TB)                                                                                          \
    template hipError_t launch_cheb_first<T, TB>(const OpArgs<T> &, Topo, const TB *, T *, T, const Scal *,       \
                                                 const Batch &, hipStream_t);                                       \
    template hipError_t launch_cheb_first2<T, TB>(const OpArgs<T> &, Topo, const TB *, const T *, T *, T *, T, T, T, \
                                                  const Scal *, const Batch &, hipStream_t);                        \
    template hipError_t launch_cheb_step<T, TB>(const OpArgs<T> &, Topo, const TB *, const T *, T *, const T *, T *, \
                                                T, T, const Scal *, const Batch &, hipStream_t, const T *,          \
                                                const int *, const int4 *, T, const double *, double *, int);        \
    template hipError_t launch_resid_restrict<T, TB>(const OpArgs<T> &, Topo, const TB *, const T *, T *,           \
                                                     const int *, const int4 *, const Scal *, const Batch &,        \
                                                     hipStream_t, T *, const T *, T);
SPFD_INST_COL(double, double)
SPFD_INST_COL(float, float)
SPFD_INST_COL(float, double)

template hipError_t launch_cg_step<double>(const OpArgs<double> &, Topo, const double *, double *, long long, int,
                                           double *, double *, Scal *, int, const Batch &, hipStream_t);
template hipError_t launch_cg_step<float>(const OpArgs<double> &, Topo, const float *, float *, long long, int,
                                          double *, double *, Scal *, int, const Batch &, hipStream_t);

}  // namespace spfd
