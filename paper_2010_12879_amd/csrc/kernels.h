// Host-side launchers of the SPFD kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <hip/hip_ext.h>

#include "common.h"

namespace spfd {

// Timing events for the next kernel launch, set by the host's timing scope and
// consumed by that launch: the dispatch itself records the start and stop
// times (no separate marker packets in the stream).
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents &next_launch_events();

#define SPFD_LAUNCH(kernel, grid, block, shmem, stream, ...)                                                \
    do {                                                                                                    \
        LaunchEvents &le_ = next_launch_events();                                                           \
        if (le_.start) {                                                                                    \
            const LaunchEvents ev_ = le_;                                                                   \
            le_ = LaunchEvents{};                                                                           \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0, __VA_ARGS__); \
        } else {                                                                                            \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                            \
        }                                                                                                   \
    } while (0)

#define HIP_RETURN_IF(...)                        \
    do {                                          \
        hipError_t e_ = (__VA_ARGS__);            \
        if (e_ != hipSuccess) return e_;          \
    } while (0)


// Operator of one level: stored edge weights (w != nullptr) or, on the finest
// level, conductances rebuilt from the per-brick label tiles and a sigma table.
template <typename T>
struct OpArgs {
    const T *w;              // [3][stride] or nullptr
    long long stride;        // nb * 512
    const uint8_t *tiles;    // [nb][768] or nullptr
    const T *table;          // sigma per label (device)
    int nlab;
    T geo4[3];               // dual area / length / 4 per direction
    const uint16_t *wh = nullptr;  // FP16 bits of w / whs (first coarse level of an FP32 cycle), read instead of w
    float whs = 0.0f;
    int short_below = 8192;        // stored-weight levels with fewer bricks run 4-node column segments
    int bscale = 0;                // the right side b is held as D^-1 b (finest level of an FP32 cycle in label
                                   // form): the kernels form D b where they need b
};

// A batch of right sides solved together: launch grids get a y-dimension of
// n, and block y offsets every vector by vs (the level's stride; vsc for the
// coarser level's vectors), the partial sums by ps and the scalars by one Scal.
struct Batch {
    int n;
    long long vs;
    long long vsc;
    int ps;
};

struct Grid {
    int nx, ny, nz;          // voxels
    int Nx, Ny, Nz;          // nodes
    int Gx, Gy, Gz;          // bricks of the finest level
};

// ---------------------------------------------------------------- setup
hipError_t launch_brick_flags(const uint8_t *labels, const double *table, int nlab, const double *sig_vox,
                              const Grid &g, uint8_t *flags, int *err, hipStream_t s);
hipError_t launch_label_tiles(const uint8_t *labels, const Grid &g, const int4 *coord, int nb, uint8_t *tiles,
                              hipStream_t s);
hipError_t launch_weights0(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                           const double geo4[3], const int4 *coord, int nb, double *w64, float *w32, hipStream_t s);
// largest and smallest positive of n non-negative weights (bits atomically maxed into out[0], which
// starts at 0, and minned into out[1], which starts at the bits of +inf), and FP16 copies
// h = w * inv rounded to nearest
hipError_t launch_wmax(const float *w, long long n, unsigned *out, hipStream_t s);
hipError_t launch_w16(const float *w, long long n, float inv, uint16_t *h, hipStream_t s);
hipError_t launch_galerkin(const double *wf, long long fstride, const int *f_slot_of, int fGx, int fGy, int fGz,
                           int fNx, int fNy, int fNz, const int4 *ccoord, int cnb, double *wc64, float *wc32,
                           long long cstride, hipStream_t s);
hipError_t launch_components(const double *w64, long long stride, Topo topo, int *parent, int *flag, int *idx,
                             int *scan_tmp, int *comp, int *counts_or_null, int *ncomp_dev, hipStream_t s);
hipError_t launch_comp_counts(const int *comp, long long n, int *counts, hipStream_t s);
hipError_t launch_coarse_setup(const double *w64, long long stride, Topo topo, int *dof_of_node, int *node_of_dof,
                               int *adj, int *ndof_dev, int maxdof, hipStream_t s);
hipError_t launch_coarse_assemble_brick(const double *w64, long long stride, Topo topo, const int *node_of_dof,
                                        const int *adj, int n, double *A, hipStream_t s);
// dense pseudo-inverse in place; work: 2n ints + n doubles (+1 int of padding)
// per brick, the node columns (tx,ty) that hold unknowns (bit tx + 8 ty)
hipError_t launch_col_masks(const double *w64, long long stride, Topo topo, unsigned long long *mask, hipStream_t s);
// A <- inverse of the regularised coarsest matrix (work: coarse_factor_work_ints(n)
// ints; dwork: dense_inverse_work_doubles(n) doubles)
size_t coarse_factor_work_ints(int n);
hipError_t launch_coarse_factor(int n, double *A, int *work, double *dwork, hipStream_t s);
size_t dense_inverse_work_doubles(int n);
hipError_t launch_dense_inverse(int n, double *A, double *work, hipStream_t s);

// ---------------------------------------------------------------- solve
// Reductions are two-stage: a producer kernel stores one partial per brick
// workgroup, then launch_finish (one workgroup) sums them in a fixed order and
// updates the solve's scalars according to `mode`.
enum {
    FIN_BB = 0,       // ||b||^2 of a new right side
    FIN_ALPHA = 1,    // alpha = r.z / p.q
    FIN_RR = 2,       // ||r||^2, iteration count and stop test
    FIN_BETA0 = 3,    // r.z of the first preconditioned residual
    FIN_BETA = 4,     // flexible beta = -alpha z.q / (r.z)_old (partials of z.q follow those of r.z)
    FIN_RESID0 = 5,   // ||b - A x0||^2 at the start of a warm-started solve
    FIN_RESID1 = 6,   // true ||b - A x||^2 at the end of a solve (kept in zq)
    FIN_MEAN = 7,     // mean of one component
    FIN_BETA_STD = 8  // standard beta = r.z / (r.z)_old
};
// mirror != nullptr: the scalars of right side i are also written to
// mirror[i] (host-visible memory) when the kernel ends, also when the solve
// had already stopped: the host reads them after the stream has passed here.
// rows (nullable, used != 0): row r sums only its first n[r] partials (packed models: each model's own
// count of bricks or groups); the z.q partials of FIN_BETA start at part + n in every row
struct FinRows {
    int used;
    int n[MAX_MODELS];
};
hipError_t launch_finish(const double *part, int n, int mode, Scal *sc, int max_iter, hipStream_t s,
                         double *means = nullptr, const int *counts = nullptr, int comp = 0, int nbatch = 1,
                         int ps = 0, Scal *mirror = nullptr, const FinRows *rows = nullptr);

template <typename T>
hipError_t launch_fill(T *x, long long n, T v, hipStream_t s);

// b = -G^T M a and the ||b||^2 partials (one per brick of the launch row).  Packed models: topo holds one
// model (np = 1), g is that model's grid and zoff its first node layer in the packed grid.
hipError_t launch_rhs(const OpArgs<double> &op, Topo topo, const int4 *coord, const Grid &g, const double *a,
                      double *b, double *part, Scal *sc, hipStream_t s, int zoff = 0);
hipError_t launch_scal_init(Scal *sc, double tol, int use_x0, int nbatch, hipStream_t s);
// fused CG step: p = z + beta p (p = z when first), x += alpha p_old (deferred), q = A p, p.q partials;
// pin and pout are different buffers (neighbours read p_old)
// edge potentials a [3][Nz][Ny][Nx] from divergence-free facet fluxes (tree-cotree gauge)
hipError_t launch_tree_cotree(const double *flux, double *a, const Grid &g, hipStream_t s);

// ---------------------------------------------------------------- flexible GMRES
constexpr int FG_MAXM = 32;     // largest restart length (basis vectors per cycle)
constexpr int MAX_PHIST = 32;   // most CG search directions kept between two updates of x
constexpr int FG_PARTS = 1024;  // partial sums per dot product
// least-squares state of one cycle (device memory): H column-major with leading dimension FG_MAXM + 1
struct FGState {
    double H[FG_MAXM * (FG_MAXM + 1)];
    double cs[FG_MAXM], sn[FG_MAXM], g[FG_MAXM + 1], y[FG_MAXM];
    double h1[FG_MAXM], h2[FG_MAXM];
    double hnext;   // ||w||^2 after the second Gram-Schmidt pass
    double beta;    // norm of the cycle's start residual
    double scale;   // 1 / norm of the vector to be stored next
};
int fg_parts(long long n);
hipError_t launch_mdot(const double *V, long long ldv, const double *w, long long n, int nv, double *part,
                       const Scal *sc, hipStream_t s);
hipError_t launch_mupdate(const double *V, long long ldv, double *w, long long n, int nv, const double *h, int mode,
                          double *part, const Scal *sc, hipStream_t s);
hipError_t launch_msum(const double *part, int ng, int nv, double *out, const Scal *sc, hipStream_t s);
hipError_t launch_fg_start(FGState *st, const Scal *sc, hipStream_t s);
hipError_t launch_fg_column(FGState *st, Scal *sc, int j, int max_iter, hipStream_t s);
hipError_t launch_fg_ysolve(FGState *st, int k, hipStream_t s);
hipError_t launch_fg_scale(const double *src, double *v, float *v32, long long n, const FGState *st, const Scal *sc,
                           hipStream_t s);
template <typename TZ>
hipError_t launch_fg_xupdate(double *x, const TZ *Z, long long ldz, long long n, int k, const FGState *st,
                             hipStream_t s);

// w = A z on the finest level (FP64 operator)
template <typename TZ>
hipError_t launch_spmv(const OpArgs<double> &op, Topo topo, const TZ *z, double *w, const Scal *sc, const Batch &bt,
                       hipStream_t s);
// number of partial sums launch_cg_step (launch_col_rupdate) writes per right side (nb: bricks per launch
// row, topo_count)
int cg_step_parts(int nb);
int rupdate_parts(int nb);
// Window of search directions: p_j of window slot j at ph + j * hs (+ row * vs), its step size at
// ahist[row * nh + j]; a right side's current slot is its Scal::hcount (steps since x was last updated).
// p = z + beta p_prev into the current slot, q = A p (q nullable: not stored), p.q partials
template <typename TZ>
hipError_t launch_cg_step(const OpArgs<double> &op, Topo topo, const TZ *z, TZ *ph, long long hs, int nh, double *q,
                          double *part, Scal *sc, int first, const Batch &bt, hipStream_t s);
// x += sum_j alpha_j p_j over the window's slots happlied .. hcount-1, in step order; then (full) an empty
// window, else happlied = hcount
template <typename TP>
hipError_t launch_x_flush(Topo topo, double *x, const TP *ph, long long hs, const double *ahist, int nh, Scal *sc,
                          const Batch &bt, hipStream_t s, int full);
// r -= alpha q, ||r||^2 partials, the FP32 copy of r; alpha also into the window slot hcount
hipError_t launch_rupdate(Topo topo, double *r, const double *q, double *part, Scal *sc, const Batch &bt, float *r32,
                          hipStream_t s, double *ahist, int nh);
// r -= alpha A p with A p formed again from p in the window slot hcount (the CG step then stores no q),
// ||r||^2 partials (rupdate_parts(nb) per right side) and the FP32 copy of r (r32 nullable); alpha also
// into that slot
template <typename TZ>
hipError_t launch_col_rupdate(const OpArgs<double> &op, Topo topo, const TZ *ph, long long hs, int nh, double *r,
                              float *r32, double *part, const Scal *sc, const Batch &bt, hipStream_t s, int r32_scaled,
                              double *ahist);
// r = b - A x (r nullable) and the partials of ||r||^2 (cg_step_parts(nb) per right side).  b has its own
// batch stride bvs (the right sides may live apart from the solve vectors).
hipError_t launch_resid(const OpArgs<double> &op, Topo topo, const double *b, const double *x, double *r,
                        double *part, long long bvs, const Batch &bt, hipStream_t s);
template <typename TZ>
hipError_t launch_dots(Topo topo, const TZ *z, const double *r, const double *q, double *part, Scal *sc,
                       int first, const Batch &bt, hipStream_t s);
template <typename TZ>
hipError_t launch_pupdate(Topo topo, const TZ *z, double *p, const Scal *sc, int first, const Batch &bt,
                          hipStream_t s);

// multigrid level kernels (T = arithmetic of the cycle, TB = type of the level's right side)
template <typename T, typename TB>
hipError_t launch_cheb_first(const OpArgs<T> &op, Topo topo, const TB *b, T *x, T c0, const Scal *sc,
                             const Batch &bt, hipStream_t s);
// the first two Chebyshev steps from zero in one pass (x1 = c0 dinv b formed where read, never stored)
template <typename T, typename TB>
hipError_t launch_cheb_first2(const OpArgs<T> &op, Topo topo, const TB *b, const T *dinv, T *xout, T *dout, T c0,
                              T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s);
// Where a Chebyshev step takes the previous update d_old = x_k - x_{k-1} from: AUTO (din if given, else
// FROM_X), FROM_X (d_old = xin: right after a zero start, or unused with c1 = 0), STORED (din), PREV (xin minus
// x_{k-1}, which the output buffer holds before the step overwrites it), PREV_PRO (as PREV, x_{k-1} first
// corrected by pscale * P xc: the previous step applied that correction on the fly)
enum { CHEB_D_AUTO = -1, CHEB_D_FROM_X = 0, CHEB_D_STORED = 1, CHEB_D_PREV = 2, CHEB_D_PREV_PRO = 3 };
// xc != nullptr (dmode other than PREV_PRO): xin is first corrected by pscale * P xc from the structured
// coarser level (parent_slot / fcoord of this level), i.e. the prolongation
// fused into the step.  dot_part != nullptr: the step also writes the
// partials of xout.b (dot_part[g]) and xout.dot_q (dot_part[n + g]),
// n = cheb_dot_parts<T>(nb), for the outer CG.
template <typename T, typename TB>
hipError_t launch_cheb_step(const OpArgs<T> &op, Topo topo, const TB *b, const T *xin, T *xout, const T *din,
                            T *dout, T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s,
                            const T *xc = nullptr, const int *parent_slot = nullptr, const int4 *fcoord = nullptr,
                            T pscale = T(0), const double *dot_q = nullptr, double *dot_part = nullptr,
                            int dmode = CHEB_D_AUTO);
template <typename T>
int cheb_dot_parts(int nb);
// xc != nullptr: also the coarse level's first Chebyshev step, xc = c0 dinv_c bc
template <typename T, typename TB>
hipError_t launch_resid_restrict(const OpArgs<T> &op, Topo topo, const TB *b, const T *x, T *bc,
                                 const int *parent_slot, const int4 *fcoord, const Scal *sc, const Batch &bt,
                                 hipStream_t s, T *xc = nullptr, const T *dinv_c = nullptr, T c0 = T(0));
template <typename T>
hipError_t launch_prolong(Topo topo, T *x, const T *xc, const int *parent_slot, const int4 *fcoord, T scale,
                          const Scal *sc, const Batch &bt, hipStream_t s);
template <typename T, typename TB>
hipError_t launch_coarse_apply(const TB *bc, T *xc, const double *Ainv, const int *node_of_dof, int n,
                               const Scal *sc, const Batch &bt, hipStream_t s);

// ---------------------------------------------------------------- several voxel models in one handle
// model boxes in the packed grid: model m has nx x ny x nz voxels from voxel layer zoff on
struct ModelBoxes {
    int np;
    int nx[MAX_MODELS], ny[MAX_MODELS], nz[MAX_MODELS], zoff[MAX_MODELS];
};
hipError_t launch_pack_labels(const uint8_t *src, int nx, int ny, int nz, uint8_t *dst, int NX, int NY, int zoff,
                              hipStream_t s);
hipError_t launch_pack_sigma(const uint8_t *labels, const Grid &g, const ModelBoxes &mb, const double *tables,
                             double *sig, hipStream_t s);

// ---------------------------------------------------------------- gauge, output, post-processing
// means[c] = mean of x over component c, in a fixed summation order; part holds comp_mean_parts(nb) doubles
size_t comp_mean_parts(int nb);
hipError_t launch_comp_mean(Topo topo, const double *x, const int *comp, int ncomp, const int *counts,
                            double *means, double *part, hipStream_t s);
// gbricks (nullable): the grid of the brick layout when it is not g (packed models; the output's model
// starts at node layer zoff of it)
hipError_t launch_psi_out(const double *x, const int *comp, const double *means, const int *slot_of, const Grid &g,
                          double *psi, hipStream_t s, const Grid *gbricks = nullptr, int zoff = 0);
// start of a solve from x = 0 for nvec right sides: x = 0, r = b and r32 = (float)b (r32 may be null;
// dinv given: r32 = (float)(dinv b), the scaled form an FP32 cycle in label form reads)
hipError_t launch_start(long long n, const double *b, long long bvs, double *x, double *r, float *r32, int nvec,
                        hipStream_t s, const float *dinv = nullptr);
hipError_t launch_psi_in(const double *psi, const int *comp, const int4 *coord, int nb, const Grid &g, double *x,
                         hipStream_t s);
hipError_t launch_efield(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                         const double h[3], double omega, const double *a, const double *psi, double *emag,
                         hipStream_t s);
hipError_t launch_uedges(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                         const double *a, const double *psi, double *u, hipStream_t s);

// ---------------------------------------------------------------- unstructured (ELL) coarse levels
// A fine level for the Galerkin product and the restriction: structured
// (w != nullptr: stored weights of a brick level) or ELL (col/val, n rows, width K).
struct FineLevelArgs {
    const double *w;
    long long stride;
    const int *nbr;
    int n, K;
    const int *col;
    const double *val;
};
template <typename T>
struct FineLevelT {
    const T *w;
    long long stride;
    const int *nbr;
    int n, K;
    const int *col;
    const T *val;
};
// pieces = connected parts of each 2x2x2 aggregate; parent = union-find forest
hipError_t launch_pieces_brick(const double *w64, long long stride, Topo topo, const int4 *coord, int *parent,
                               hipStream_t s);
hipError_t launch_pieces_ell(int n, int K, const int *col, const double *val, const int4 *pos, int *parent,
                             hipStream_t s);
hipError_t launch_pieces_finish(int *parent, long long n, int *flag, hipStream_t s);
hipError_t launch_pieces_assign(const int *parent, const int *idx, long long n, int *agg, int *count, hipStream_t s);
hipError_t launch_piece_pos_brick(const int *parent, const int *idx, Topo topo, const int4 *coord, int4 *pos,
                                  hipStream_t s);
hipError_t launch_piece_pos_ell(int n, const int *parent, const int *idx, const int4 *fpos, int4 *pos, hipStream_t s);
hipError_t launch_members(const int *agg, long long n, int nc, const int *mptr, int *cursor, int *mem, hipStream_t s);
hipError_t launch_galerkin_ell(const FineLevelArgs &fa, const int *agg, int nc, const int *mptr, const int *mem,
                               int pass, int *len, int K, int *col, double *val64, float *val32, int *overflow,
                               int *maxlen, hipStream_t s);
hipError_t scan_exclusive_ints(const int *in, long long n, int *out, int *tmp, int *total, hipStream_t s);
template <typename T>
hipError_t launch_ell_cheb_first(int n, int K, const int *col, const T *val, const T *b, T *x, T c0, const Scal *sc,
                                 const Batch &bt, hipStream_t s);
// agg != nullptr: the prolongation xin += scale xc[agg] from the coarser ELL level is applied to every value read
template <typename T>
hipError_t launch_ell_cheb_step(int n, int K, const int *col, const T *val, const T *b, const T *xin, T *xout,
                                const T *din, T *dout, T c1, T c2, const Scal *sc, const Batch &bt, hipStream_t s,
                                const int *agg = nullptr, const T *xc = nullptr, T scale = T(0));
// b_c = P^T (b - A x) onto an ELL level (nrows rows of the finer level, nc aggregates);
// xc != nullptr: also the coarse level's first Chebyshev step, xc = c0 dinv_c b_c
template <typename T>
hipError_t launch_restrict_members(const FineLevelT<T> &f, long long nrows, const T *b, const T *x, int nc,
                                   const int *mptr, const int *mem, T *bc, const Scal *sc, const Batch &bt,
                                   hipStream_t s, T *xc = nullptr, const T *dinv_c = nullptr, T c0 = T(0),
                                   const int *memb = nullptr);
// direct member table memb[p*8 + j] of the restriction (*over = 1 if an aggregate has more than 8 members)
hipError_t launch_members8(int nc, const int *mptr, const int *mem, int *memb, int *over, hipStream_t s);
// inverse diagonals (0 where the diagonal vanishes): ELL level, structured level
hipError_t launch_dinv_ell(int n, int K, const int *col, const double *val, double *d64, float *d32, hipStream_t s);
hipError_t launch_dinv_struct(const double *w64, long long stride, Topo topo, double *d64, float *d32,
                              hipStream_t s);
template <typename T>
hipError_t launch_prolong_agg(long long n, const int *agg, T *x, const T *xc, T scale, const Scal *sc,
                              const Batch &bt, hipStream_t s);
hipError_t launch_coarse_enum_ell(int n, int K, const int *col, const double *val, int *dof_of_row, int *row_of_dof,
                                  int *ndof, int maxdof, hipStream_t s);
hipError_t launch_coarse_dense_ell(int nrow, int K, const int *col, const double *val, const int *dof_of_row,
                                   const int *row_of_dof, int n, double *A, hipStream_t s);

// ---------------------------------------------------------------- quantiles of |E|
size_t sel_work_bytes(int ngroups);
// nearest-rank q-quantile over the conducting voxels: out[0] whole body,
// out[1 + l] voxels with label l (NaN when empty); out and work on the device
hipError_t launch_quantiles(const uint8_t *labels, const double *table, const double *sig_vox, long long nvox,
                            const double *emag, int ngroups, double q, void *work, double *out, hipStream_t s);

// ---------------------------------------------------------------- adjoint gradient
hipError_t launch_adj_voxel(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                            const double h[3], double omega, const double *a, const double *psi,
                            const double *grad_emag, double *c, hipStream_t s);
hipError_t launch_adj_rhs(Topo topo, const int4 *coord, const Grid &g, const double *c, double *b, double *part,
                          hipStream_t s);
int adj_grad_blocks(const Grid &g);
hipError_t launch_adj_grad(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                           const double geo4[3], const double *a, const double *psi, const double *lam, double *grad,
                           double *lab_part, int nlab, double *lab_out, hipStream_t s);

// ---------------------------------------------------------------- measurement aids
// a = b + s c over n doubles (variant 0: one pair of doubles per thread; 1: four pairs)
hipError_t launch_triad(double *a, const double *b, const double *c, long long n, double s, int variant,
                        hipStream_t st);
// read and write every 32-bit word of buf (evicts the caches before a cold timing)
hipError_t launch_flush(void *buf, size_t bytes, hipStream_t st);

}  // namespace spfd
