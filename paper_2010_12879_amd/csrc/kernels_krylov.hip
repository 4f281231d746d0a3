// Flexible GMRES outer solver (the Krylov method of the paper, Sec. III: FGMRES
// with an algebraic multigrid preconditioner), right preconditioned with the
// same multigrid cycle as the flexible CG:
//   v_0 = r / beta,  for j = 0, 1, ...:  z_j = B v_j,  w = A z_j,
//   h_{i,j} = v_i . w (i <= j) by classical Gram-Schmidt applied twice,
//   h_{j+1,j} = ||w||,  v_{j+1} = w / h_{j+1,j},
//   Givens rotations keep the least-squares problem min ||beta e_1 - H y||
//   triangular; |g_{j+1}| is the residual norm of x_0 + Z y.
// At convergence or after m columns: y = R^-1 g and x += Z y (restart from
// the true residual).  Vectors are the finest level's slot arrays (zero at
// slots without an unknown); the small least-squares problem lives in device
// memory and is updated by one thread per column.
#include <math.h>

#include "kernels.h"

namespace spfd {

constexpr int KT = 256;   // threads per workgroup of the vector kernels

__device__ __forceinline__ double block_reduce(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < KT / 64; ++i) s += lds[i];
    return s;
}

// partials of NV rows at once: row i of the workgroup into part[i*gridDim.x + blockIdx.x], i < nv
template <int NV>
__device__ __forceinline__ void rows_reduce(double (&acc)[NV], int nv, double *__restrict__ part)
{
    __shared__ double lds[NV][KT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double t = wave_sum(acc[i]);
        if (lane == 0) lds[i][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < KT / 64; ++k) t += lds[threadIdx.x][k];
        part[(long long)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// The basis kernels are templated on NV >= nv, the smallest of 4, 8, 16, 32:
// every thread loads rows 0..NV-1 (rows from nv on repeat row nv-1, cache
// hits) before it uses any of them, so all loads of an element are in flight
// together; rows from nv on are masked out.  (A load under a condition on its
// row index becomes a branch that waits for it inside, one row at a time.)

// partials (one per workgroup g, stored at part[i*ng + g]) of V_i . w, i < nv
template <int NV>
__global__ __launch_bounds__(KT) void k_mdot(const double *__restrict__ V, long long ldv, const double *__restrict__ w,
                                             long long n, int nv, double *__restrict__ part, const Scal *sc)
{
    if (sc->done) return;
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < n; e += (long long)gridDim.x * KT) {
        const double wv = w[e];
        double v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = V[(i < nv ? i : nv - 1) * ldv + e];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v[i] * wv;
    }
    rows_reduce<NV>(acc, nv, part);
}

// w -= sum_i h_i V_i; then either the partials of V_i . w (mode 0) or of w.w (mode 1)
template <int NV>
__global__ __launch_bounds__(KT) void k_mupdate(const double *__restrict__ V, long long ldv, double *__restrict__ w,
                                                long long n, int nv, const double *__restrict__ h, int mode,
                                                double *__restrict__ part, const Scal *sc)
{
    __shared__ double lds[KT / 64];
    if (sc->done) return;
    double hv[NV], acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        hv[i] = i < nv ? h[i] : 0.0;
        acc[i] = 0.0;
    }
    double nrm = 0.0;
    for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < n; e += (long long)gridDim.x * KT) {
        double wv = w[e];
        double v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = V[(i < nv ? i : nv - 1) * ldv + e];
#pragma unroll
        for (int i = 0; i < NV; ++i) wv -= hv[i] * v[i];
        w[e] = wv;
        if (mode == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] += v[i] * wv;
        } else {
            nrm += wv * wv;
        }
    }
    if (mode == 0) {
        rows_reduce<NV>(acc, nv, part);
    } else {
        const double t = block_reduce(nrm, lds);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

// out[i] = sum over g of part[i*ng + g] (one workgroup per i, fixed order)
__global__ __launch_bounds__(KT) void k_msum(const double *__restrict__ part, int ng, double *__restrict__ out,
                                             const Scal *sc)
{
    __shared__ double lds[KT / 64];
    if (sc->done) return;
    const double *p = part + (long long)blockIdx.x * ng;
    double a = 0.0;
    for (int g = threadIdx.x; g < ng; g += KT) a += p[g];
    a = block_reduce(a, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// start of a cycle from the residual norm^2 in sc->rr: beta, g = beta e_1
__global__ void k_fg_start(FGState *st, const Scal *sc)
{
    if (sc->done) return;
    const double beta = sqrt(sc->rr);
    st->beta = beta;
    for (int i = 0; i <= FG_MAXM; ++i) st->g[i] = 0.0;
    st->g[0] = beta;
    st->scale = beta > 0.0 ? 1.0 / beta : 0.0;
}

// column j of H from the two Gram-Schmidt passes and ||w||; rotations; stop test
__global__ void k_fg_column(FGState *st, Scal *sc, int j, int max_iter)
{
    if (sc->done) return;
    double *H = st->H + (long long)j * (FG_MAXM + 1);
    for (int i = 0; i <= j; ++i) H[i] = st->h1[i] + st->h2[i];
    const double hn = sqrt(st->hnext);
    H[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = st->cs[i] * H[i] + st->sn[i] * H[i + 1];
        H[i + 1] = -st->sn[i] * H[i] + st->cs[i] * H[i + 1];
        H[i] = t;
    }
    const double a = H[j], b = H[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
    st->cs[j] = c;
    st->sn[j] = s;
    H[j] = r;
    H[j + 1] = 0.0;
    st->g[j + 1] = -s * st->g[j];
    st->g[j] = c * st->g[j];
    st->scale = hn > 0.0 ? 1.0 / hn : 0.0;
    const double res2 = st->g[j + 1] * st->g[j + 1];
    sc->rr = res2;
    sc->iters += 1;
    if (!isfinite(res2) || !(r > 0.0)) {
        sc->status = 6;
        sc->done = 1;
    } else if (res2 <= sc->tol2 || !(hn > 0.0)) {
        sc->done = 1;   // converged (hn = 0: the Krylov space holds the solution)
    } else if (sc->iters >= max_iter) {
        sc->status = 5;
        sc->done = 1;
    }
}

// y = R^-1 g over the first k columns (back substitution); runs also after the stop flag is set
__global__ void k_fg_ysolve(FGState *st, int k)
{
    for (int i = k - 1; i >= 0; --i) {
        double t = st->g[i];
        for (int l = i + 1; l < k; ++l) t -= st->H[(long long)l * (FG_MAXM + 1) + i] * st->y[l];
        const double d = st->H[(long long)i * (FG_MAXM + 1) + i];
        st->y[i] = d != 0.0 ? t / d : 0.0;
    }
}

// v = src * st->scale (and its FP32 copy for an FP32 cycle)
__global__ __launch_bounds__(KT) void k_fg_scale(const double *__restrict__ src, double *__restrict__ v,
                                                 float *__restrict__ v32, long long n, const FGState *st,
                                                 const Scal *sc)
{
    if (sc->done) return;
    const double f = st->scale;
    for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < n; e += (long long)gridDim.x * KT) {
        const double t = src[e] * f;
        v[e] = t;
        if (v32) v32[e] = (float)t;
    }
}

// x += sum_{i<k} y_i Z_i (runs also after the stop flag is set)
template <typename TZ, int NV>
__global__ __launch_bounds__(KT) void k_fg_xupdate(double *__restrict__ x, const TZ *__restrict__ Z, long long ldz,
                                                   long long n, int k, const FGState *st)
{
    double y[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) y[i] = i < k ? st->y[i] : 0.0;
    for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < n; e += (long long)gridDim.x * KT) {
        double t = x[e];
        TZ zv[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) zv[i] = Z[(i < k ? i : k - 1) * ldz + e];
#pragma unroll
        for (int i = 0; i < NV; ++i) t += y[i] * (double)zv[i];
        x[e] = t;
    }
}

// smallest of 4, 8, 16, 32 that holds m rows
static int nv_bucket(int m)
{
    return m <= 4 ? 4 : m <= 8 ? 8 : m <= 16 ? 16 : 32;
}

static unsigned kgrid(long long n)
{
    long long b = (n + KT - 1) / KT;
    if (b > FG_PARTS) b = FG_PARTS;
    return (unsigned)(b < 1 ? 1 : b);
}

int fg_parts(long long n) { return (int)kgrid(n); }

hipError_t launch_mdot(const double *V, long long ldv, const double *w, long long n, int nv, double *part,
                       const Scal *sc, hipStream_t s)
{
    if (nv < 1 || nv > FG_MAXM) return hipErrorInvalidValue;
    switch (nv_bucket(nv)) {
    case 4: SPFD_LAUNCH(k_mdot<4>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, part, sc); break;
    case 8: SPFD_LAUNCH(k_mdot<8>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, part, sc); break;
    case 16: SPFD_LAUNCH(k_mdot<16>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, part, sc); break;
    default: SPFD_LAUNCH(k_mdot<32>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, part, sc); break;
    }
    return hipGetLastError();
}

hipError_t launch_mupdate(const double *V, long long ldv, double *w, long long n, int nv, const double *h, int mode,
                          double *part, const Scal *sc, hipStream_t s)
{
    if (nv < 1 || nv > FG_MAXM) return hipErrorInvalidValue;
    switch (nv_bucket(nv)) {
    case 4: SPFD_LAUNCH(k_mupdate<4>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, h, mode, part, sc); break;
    case 8: SPFD_LAUNCH(k_mupdate<8>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, h, mode, part, sc); break;
    case 16: SPFD_LAUNCH(k_mupdate<16>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, h, mode, part, sc); break;
    default: SPFD_LAUNCH(k_mupdate<32>, dim3(kgrid(n)), dim3(KT), 0, s, V, ldv, w, n, nv, h, mode, part, sc); break;
    }
    return hipGetLastError();
}

hipError_t launch_msum(const double *part, int ng, int nv, double *out, const Scal *sc, hipStream_t s)
{
    SPFD_LAUNCH(k_msum, dim3(nv), dim3(KT), 0, s, part, ng, out, sc);
    return hipGetLastError();
}

hipError_t launch_fg_start(FGState *st, const Scal *sc, hipStream_t s)
{
    SPFD_LAUNCH(k_fg_start, dim3(1), dim3(1), 0, s, st, sc);
    return hipGetLastError();
}

hipError_t launch_fg_column(FGState *st, Scal *sc, int j, int max_iter, hipStream_t s)
{
    if (j < 0 || j >= FG_MAXM) return hipErrorInvalidValue;
    SPFD_LAUNCH(k_fg_column, dim3(1), dim3(1), 0, s, st, sc, j, max_iter);
    return hipGetLastError();
}

hipError_t launch_fg_ysolve(FGState *st, int k, hipStream_t s)
{
    if (k < 0 || k > FG_MAXM) return hipErrorInvalidValue;
    SPFD_LAUNCH(k_fg_ysolve, dim3(1), dim3(1), 0, s, st, k);
    return hipGetLastError();
}

hipError_t launch_fg_scale(const double *src, double *v, float *v32, long long n, const FGState *st, const Scal *sc,
                           hipStream_t s)
{
    SPFD_LAUNCH(k_fg_scale, dim3(kgrid(n)), dim3(KT), 0, s, src, v, v32, n, st, sc);
    return hipGetLastError();
}

template <typename TZ>
hipError_t launch_fg_xupdate(double *x, const TZ *Z, long long ldz, long long n, int k, const FGState *st,
                             hipStream_t s)
{
    if (k < 0 || k > FG_MAXM) return hipErrorInvalidValue;
    if (k == 0) return hipSuccess;
    switch (nv_bucket(k)) {
    case 4: SPFD_LAUNCH((k_fg_xupdate<TZ, 4>), dim3(kgrid(n)), dim3(KT), 0, s, x, Z, ldz, n, k, st); break;
    case 8: SPFD_LAUNCH((k_fg_xupdate<TZ, 8>), dim3(kgrid(n)), dim3(KT), 0, s, x, Z, ldz, n, k, st); break;
    case 16: SPFD_LAUNCH((k_fg_xupdate<TZ, 16>), dim3(kgrid(n)), dim3(KT), 0, s, x, Z, ldz, n, k, st); break;
    default: SPFD_LAUNCH((k_fg_xupdate<TZ, 32>), dim3(kgrid(n)), dim3(KT), 0, s, x, Z, ldz, n, k, st); break;
    }
    return hipGetLastError();
}
template hipError_t launch_fg_xupdate<double>(double *, const double *, long long, long long, int, const FGState *,
                                              hipStream_t);
template hipError_t launch_fg_xupdate<float>(double *, const float *, long long, long long, int, const FGState *,
                                             hipStream_t);

}  // namespace spfd
