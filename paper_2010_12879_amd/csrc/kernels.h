// Host-side launchers of the SPFD kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace spfd {

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
hipError_t launch_galerkin(const double *wf, long long fstride, const int *f_slot_of, int fGx, int fGy, int fGz,
                           int fNx, int fNy, int fNz, const int4 *ccoord, int cnb, double *wc64, float *wc32,
                           long long cstride, hipStream_t s);
hipError_t launch_components(const double *w64, long long stride, Topo topo, int *parent, int *flag, int *idx,
                             int *scan_tmp, int *comp, int *counts_or_null, int *ncomp_dev, hipStream_t s);
hipError_t launch_comp_counts(const int *comp, long long n, int *counts, hipStream_t s);
hipError_t launch_coarse_setup(const double *w64, long long stride, Topo topo, int *dof_of_node, int *node_of_dof,
                               int *adj, int *ndof_dev, int maxdof, hipStream_t s);
hipError_t launch_coarse_factor(const double *w64, long long stride, Topo topo, const int *dof_of_node,
                                const int *node_of_dof, int *adj, int n, double *A, int *work, hipStream_t s);

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
    FIN_MEAN = 7      // mean of one component
};
hipError_t launch_finish(const double *part, int n, int mode, Scal *sc, int max_iter, hipStream_t s,
                         double *means = nullptr, const int *counts = nullptr, int comp = 0);

template <typename T>
hipError_t launch_fill(T *x, long long n, T v, hipStream_t s);

hipError_t launch_rhs(const OpArgs<double> &op, Topo topo, const int4 *coord, const Grid &g, const double *a,
                      double *b, double *part, Scal *sc, hipStream_t s);
hipError_t launch_scal_init(Scal *sc, double tol, int use_x0, hipStream_t s);
hipError_t launch_spmv_dot(const OpArgs<double> &op, Topo topo, const double *p, double *q, double *part,
                           Scal *sc, hipStream_t s);
hipError_t launch_update(Topo topo, double *x, double *r, const double *p, const double *q, double *part,
                         Scal *sc, int max_iter, hipStream_t s);
hipError_t launch_resid(const OpArgs<double> &op, Topo topo, const double *b, const double *x, double *r,
                        double *part, Scal *sc, int mode, hipStream_t s);
template <typename TZ>
hipError_t launch_dots(Topo topo, const TZ *z, const double *r, const double *q, double *part, Scal *sc,
                       int first, hipStream_t s);
template <typename TZ>
hipError_t launch_pupdate(Topo topo, const TZ *z, double *p, const Scal *sc, int first, hipStream_t s);

// multigrid level kernels (T = arithmetic of the cycle, TB = type of the level's right side)
template <typename T, typename TB>
hipError_t launch_cheb_first(const OpArgs<T> &op, Topo topo, const TB *b, T *x, T c0, const Scal *sc, hipStream_t s);
template <typename T, typename TB>
hipError_t launch_cheb_step(const OpArgs<T> &op, Topo topo, const TB *b, const T *xin, T *xout, const T *din,
                            T *dout, T c1, T c2, const Scal *sc, hipStream_t s);
template <typename T, typename TB>
hipError_t launch_resid_restrict(const OpArgs<T> &op, Topo topo, const TB *b, const T *x, T *bc,
                                 const int *parent_slot, const int4 *fcoord, const Scal *sc, hipStream_t s);
template <typename T>
hipError_t launch_prolong(Topo topo, T *x, const T *xc, const int *parent_slot, const int4 *fcoord, T scale,
                          const Scal *sc, hipStream_t s);
template <typename T, typename TB>
hipError_t launch_coarse_apply(const TB *bc, T *xc, const double *Ainv, const int *node_of_dof, int n,
                               const Scal *sc, hipStream_t s);

// ---------------------------------------------------------------- gauge, output, post-processing
hipError_t launch_comp_mean(Topo topo, const double *x, const int *comp, int ncomp, const int *counts,
                            double *sums, double *part, hipStream_t s);
hipError_t launch_psi_out(const double *x, const int *comp, const double *means, const int *slot_of, const Grid &g,
                          double *psi, hipStream_t s);
hipError_t launch_psi_in(const double *psi, const int *comp, const int4 *coord, int nb, const Grid &g, double *x,
                         hipStream_t s);
hipError_t launch_efield(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                         const double h[3], double omega, const double *a, const double *psi, double *emag,
                         hipStream_t s);
hipError_t launch_uedges(const uint8_t *labels, const double *table, const double *sig_vox, const Grid &g,
                         const double *a, const double *psi, double *u, hipStream_t s);

}  // namespace spfd
