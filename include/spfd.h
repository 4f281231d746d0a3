/*
 * spfd.h -- C-ABI of the MI355X (gfx950) library for the Co-Sim. SPFD Poisson
 * solve and E-field post-processing.
 *
 * The operation (paper, Sec. II, Eqs. (1) and (3); Sec. III.A; Sec. III.F):
 *   on a voxel body model with per-voxel tissue conductivity sigma, let
 *   M_kappa be the diagonal matrix of edge conductances
 *       M_e = (mean sigma of the four voxels sharing edge e) * (dual facet area) / (edge length),
 *   G the node-to-edge gradient ((G Psi)_e = Psi_head - Psi_tail) and a the
 *   source edge potentials (line integrals of the magnetic vector potential).
 *   Solve  G^T M_kappa G Psi = -G^T M_kappa a  (Eq. (3)) for the nodal
 *   potentials Psi of the conducting voxels only (Sec. III.A), then form the
 *   edge voltages e = -j omega (a + G Psi) (Eq. (1)) and the voxel-averaged
 *   field magnitude |E| (Sec. III.F).  Eq. (3) is singular (constants per
 *   connected conductor); the library returns the solution with zero mean
 *   over every connected component.
 *
 * Index conventions (all arrays contiguous):
 *   voxel (i,j,k)  -> i + nx*(j + ny*k)                       [nvox = nx*ny*nz]
 *   node  (i,j,k)  -> i + (nx+1)*(j + (ny+1)*k)               [nnodes = (nx+1)(ny+1)(nz+1)]
 *   edge arrays [3][nnodes]: entry [d][n] is the edge from node n to node n + e_d
 *   (d = 0,1,2 = x,y,z); entries of edges that leave the grid are ignored.
 *   Voxel (i,j,k) spans nodes i..i+1, j..j+1, k..k+1; h = (hx,hy,hz) metres.
 *   labels: uint8 per voxel, looked up in a sigma table; sigma_table[label] = 0 is air.
 *
 * Memory: every array argument marked "device" is a device pointer on the
 * handle's GPU, owned by the caller; the library never frees it and does not
 * keep it after the call returns.  Arguments marked "host" are host memory.
 * Work is enqueued on the stream given at creation; every call returns after
 * its work has completed, so the caller may reuse its buffers immediately.
 *
 * Errors: every function returns a status; no C++ exception crosses the ABI.
 * On SPFD_INVALID_ARG or SPFD_BAD_STATE nothing is written.  On
 * SPFD_NOT_CONVERGED / SPFD_BREAKDOWN the best iterate and the info are still
 * written.  spfd_last_error() gives a message for the last failing call.
 * A handle must be used by one thread at a time.
 */
#ifndef SPFD_H
#define SPFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spfd_ctx *spfd_handle;

typedef enum {
    SPFD_OK = 0,
    SPFD_INVALID_ARG = 1,     /* bad size, pointer, NaN/negative sigma, zero conducting voxels ... */
    SPFD_BAD_STATE = 2,       /* call order violated (geometry -> sigma -> build -> source -> solve) */
    SPFD_OUT_OF_MEMORY = 3,
    SPFD_HIP_ERROR = 4,
    SPFD_NOT_CONVERGED = 5,   /* max_iter reached; best iterate written */
    SPFD_BREAKDOWN = 6        /* non-positive or non-finite curvature in CG; best iterate written */
} spfd_status;

enum { SPFD_FP64 = 0, SPFD_MIXED = 1 };          /* precision of the multigrid cycle */
enum { SPFD_CYCLE_V = 0 };
enum { SPFD_SMOOTH_CHEBYSHEV = 0, SPFD_SMOOTH_L1_JACOBI = 1, SPFD_SMOOTH_CHEBYSHEV4 = 2 };  /* smoother of every level */

/* Multigrid preconditioner (the paper uses an algebraic multigrid
 * preconditioner inside a Krylov solver, Sec. III; its configuration is not
 * given).  Zero-initialised options select the defaults. */
typedef struct {
    int precision;        /* SPFD_FP64 (default) or SPFD_MIXED: FP32 cycle (FP16 weights on its first coarse
                             level), FP64 outer CG (x, r, q = A p, dots; the search direction p is stored
                             in FP32 and q is formed from the stored value) and coarsest solve */
    int cycle;            /* SPFD_CYCLE_V (the only cycle; any other value is rejected) */
    int smooth_degree;    /* Chebyshev degree per pre/post smoothing, default 2, max 4 */
    int coarsest_max;     /* coarsen until the coarsest level has <= this many unknowns, default and max 1024 */
    double cheby_ratio;   /* smoothing interval [2/ratio, 2] of D^-1 A, default 8 */
    double coarse_scale;  /* scaling of the coarse-grid correction (over-correction of the piecewise-constant
                             aggregation), default 1.9; keep below 2 */
    int split_level;      /* aggregates of this level and coarser ones are split into their connected pieces
                             (coarse unknowns become unstructured), default 2 */
    int no_split;         /* nonzero: never split aggregates (structured 7-point levels only) */
    int level1_degree;    /* Chebyshev degree per pre/post smoothing on the first coarse level, default 4,
                             max 8 (that level costs about an eighth of the finest one per step, and
                             smoothing it harder lowers the iteration count) */
    int smoother;         /* SPFD_SMOOTH_CHEBYSHEV (default) or SPFD_SMOOTH_L1_JACOBI: smooth_degree
                             (level1_degree) sweeps x += D_l1^-1 (b - A x), D_l1 the row l1 norms,
                             which equal twice the diagonal here (every level's rows sum to zero);
                             any other value is rejected with SPFD_INVALID_ARG */
    int short_segment_bricks; /* column segment (nodes per lane) of the stencil kernels of structured levels
                             with stored weights in an FP32 cycle: 0 (default) = tuned per level at build
                             (one Chebyshev step timed with 4- and 8-node segments, the faster kept; the
                             results are the same either way); > 0 = levels with fewer bricks than this run
                             4-node segments, larger ones 8; negative = 8-node segments everywhere.
                             FP64 cycles always run 4-node segments */
    int level1_fp32;      /* SPFD_MIXED only.  0 (default): the first coarse level's smoothing and
                             restriction read FP16 copies of its weights, scaled so that the largest is
                             2^15, unless the smallest nonzero weight would then fall below FP16's normal
                             range (then FP32 weights are kept); nonzero: always FP32 weights */
    int cg_window;        /* CG search directions kept (in the cycle's precision) before x is updated from
                             them: 0 (default) = up to 32, as many as fit in about 16 GiB for the handle's
                             right sides, at least 2; else an even number 2..32.  x receives the same
                             updates in the same order whatever the window (the results are bitwise the
                             same); a longer window saves reading and writing x in FP64 per CG step */
} spfd_amg_options;

typedef struct {
    double rel_tol;       /* stop when ||b - A Psi||_2 <= rel_tol * ||b||_2 (true residual at exit); default 1e-8 */
    int max_iter;         /* default 500 */
    int use_x0;           /* nonzero: psi holds the start iterate on entry */
    int eager;            /* nonzero: launch every kernel from the host instead of replaying the
                             captured HIP graph of a CG iteration (same kernels, same results) */
    int method;           /* SPFD_CG (default): preconditioned CG (see flexible); SPFD_FGMRES: flexible GMRES
                             (the paper's Krylov method, Sec. III), one right side per handle only */
    int restart;          /* FGMRES basis vectors per cycle, 1..32, default 30 */
    int flexible;         /* SPFD_CG only.  0 (default): standard beta = (r.z)_k / (r.z)_{k-1};
                             nonzero: flexible beta = -alpha_{k-1} (z_k.q_{k-1}) / (r.z)_{k-1}
                             (Polak-Ribiere form, robust to a preconditioner that varies
                             between iterations; reads q once more per iteration) */
} spfd_solve_options;

enum { SPFD_CG = 0, SPFD_FGMRES = 1 };

typedef struct {
    int iterations;
    double rel_residual;  /* true ||b - A Psi||_2 / ||b||_2 of the returned Psi */
    int status;           /* spfd_status of this right-hand side */
} spfd_rhs_info;

/* Device memory of a handle.  alloc(bytes, user) returns a device pointer on
 * the handle's GPU (NULL on failure: the call reports SPFD_OUT_OF_MEMORY) and
 * free(ptr, user) releases one; both are called from the thread that calls
 * the library, only inside spfd_* calls, and every buffer is freed again by
 * spfd_destroy at the latest, after the handle's work has completed.  A caller
 * that owns a caching allocator (e.g. PyTorch's) passes it here so that the
 * handle's working memory is accounted and reused there. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} spfd_allocator;

/* Create a handle on HIP device `device`; `hip_stream` is a hipStream_t (NULL
 * = default stream).  Each call orders its work after the work already on
 * hip_stream and runs it on streams the handle owns (default priority;
 * spfd_build overlaps two parts of the setup on two of them).  alloc (host,
 * nullable; copied): the allocator of the handle's device memory,
 * hipMalloc/hipFree when NULL or when both of its functions are NULL;
 * SPFD_INVALID_ARG when only one of them is given. */
spfd_status spfd_create(int device, void *hip_stream, const spfd_allocator *alloc, spfd_handle *out);
void spfd_destroy(spfd_handle h);
/* Message of the last failing call on h (valid until the next call on h). */
const char *spfd_last_error(spfd_handle h);

/* Voxel geometry (Sec. III.A): grid sizes, voxel edge lengths in metres,
 * labels [nvox] (device, uint8).  Finds the bricks that hold conducting
 * voxels once the conductivities are known (spfd_build). */
spfd_status spfd_set_geometry(spfd_handle h, int nx, int ny, int nz, double hx, double hy, double hz,
                              const uint8_t *labels);
/* Conductivity per label, S/m (host, n_labels <= 256, finite, >= 0; 0 = air).
 * M_kappa at the field's frequency (Eq. (3)). */
spfd_status spfd_set_sigma_table(spfd_handle h, const double *sigma, int n_labels);
/* Conductivity per voxel (device, [nvox], finite, >= 0): overrides the table. */
spfd_status spfd_set_sigma_voxel(spfd_handle h, const double *sigma_voxel);
/* Assemble the edge conductances M_kappa of Eq. (3) from the conductivities
 * (mean of the four voxels around each edge times dual facet area over edge
 * length; Sec. III.A: nodes of conducting voxels are the unknowns), find the
 * connected conductors (the constants of Eq. (3)'s null space), and build the
 * multigrid hierarchy of the preconditioner (the paper solves Eq. (3) with an
 * algebraic multigrid preconditioner inside a Krylov method, Sec. III).
 * opt (host) may be NULL (defaults).  SPFD_INVALID_ARG when no voxel conducts
 * or an option is out of range; the previous hierarchy is released first. */
spfd_status spfd_build(spfd_handle h, const spfd_amg_options *opt);
/* Sizes after build (any pointer may be NULL): unknowns, connected
 * components, multigrid levels, device bytes held by the handle. */
spfd_status spfd_get_info(spfd_handle h, long long *n_dofs, int *n_components, int *n_levels,
                          size_t *device_bytes);
/* One level of the multigrid hierarchy after build (0 = finest; any pointer
 * may be NULL): kind 0 = structured brick level (7-point stencil), 1 =
 * unstructured level (rows of the split aggregation, ELL storage); its
 * unknowns; the slots of its vectors (bricks x 512, or rows); the entries per
 * matrix row (7, or 1 + the ELL width); the column segment of its smoothing
 * kernels in the cycle (nodes per lane, 4 or 8; 0 for ELL levels and the
 * coarsest level).  The last level is the one solved directly.
 * SPFD_INVALID_ARG for a level outside [0, n_levels). */
spfd_status spfd_level_info(spfd_handle h, int level, int *kind, long long *unknowns, long long *slots,
                            int *row_entries, int *segment);
/* Number of right-hand sides solved together (default 1); resets the sources. */
spfd_status spfd_set_num_rhs(spfd_handle h, int nrhs);
/* Right-hand side of Eq. (3) for source `rhs`: b = -G^T M_kappa a, with
 * a [3][nnodes] (device, FP64, V*s). */
spfd_status spfd_set_source(spfd_handle h, int rhs, const double *a);
/* Solve Eq. (3) for every right-hand side.  psi [nrhs][nnodes] (device,
 * FP64): start iterate on entry if opt->use_x0, on exit the solution with zero
 * mean per connected component and 0 at nodes outside the conductor.
 * info [nrhs] (host) may be NULL.  opt may be NULL (defaults). */
spfd_status spfd_solve(spfd_handle h, const spfd_solve_options *opt, double *psi, spfd_rhs_info *info);
/* Eq. (1) and the voxel average (Sec. III.F) for nsrc >= 1 sources:
 * a [nsrc][3][nnodes] and psi [nsrc][nnodes] (device) as in spfd_set_source /
 * spfd_solve; u_edges [nsrc][3][nnodes] (device, nullable) = a + G psi on
 * conducting edges (0 elsewhere), so that Im(e) = -omega*u and Re(e) = 0;
 * emag [nsrc][nvox] (device) = omega * |mean of the voxel's d-edges / h_d|
 * per conducting voxel, 0 in air. */
spfd_status spfd_efield(spfd_handle h, double omega, int nsrc, const double *a, const double *psi,
                        double *u_edges, double *emag);

/* Edge potentials from facet fluxes, Eq. (2) b = C a, solved in a tree-cotree
 * gauge (technical summary of Sec. II.A, step 3).  flux [3][Nz][Ny][Nx]
 * (device): magnetic flux through each voxel facet, normal d, anchored at the
 * facet's lowest corner node (entries beyond the grid are ignored); it must be
 * discretely divergence-free (zero net flux out of every voxel), else the
 * z-facets above the bottom node plane are not reproduced.  a [3][Nz][Ny][Nx]
 * (device, written): edge potentials in the layout of spfd_set_source, zero on
 * the tree (every z-edge, the y-edges of the plane k = 0, the x-edges of the
 * line j = k = 0) and on entries beyond the grid.  Any two solutions differ by
 * a discrete gradient, which leaves the field of Eq. (1) unchanged.  Needs the
 * geometry only. */
spfd_status spfd_edge_potentials(spfd_handle h, const double *flux, double *a);

/* Nearest-rank q-quantile of the voxel field |E| (step 6 of the paper's
 * technical summary, Sec. II.A: the 99th percentile of the voxel-averaged
 * field, Sec. III.F, q = 0.99): among the n conducting voxels (sigma > 0) the
 * value of rank ceil(q n) in ascending order.  emag [nvox] (device), e.g. from
 * spfd_efield.  out_body (host): whole body; out_labels (host, nullable): one
 * value per label of the sigma table (256 in per-voxel mode), NaN for labels
 * without conducting voxels.  Exact (radix selection on the FP64 values). */
spfd_status spfd_percentile(spfd_handle h, const double *emag, double q, double *out_body, double *out_labels);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * quantile of spfd_percentile without a handle and without any allocation.
 * Its work area is a fixed device array inside the library (272 KiB per GPU,
 * held until the process ends), which limits it to n_labels <= 256; larger
 * values give SPFD_INVALID_ARG.  All arrays are device memory: labels [nvox]
 * (uint8); sigma_table [n_labels] (FP64, nullable when sigma_voxel is given);
 * sigma_voxel [nvox] (FP64, nullable: then sigma_table[labels[v]]); emag
 * [nvox]; out [1 + n_labels] (FP64, written): out[0] the whole body's value,
 * out[1 + l] the value over the conducting voxels of label l (NaN if none).
 * The body is the voxels with sigma > 0, the rule nearest rank (as in
 * spfd_percentile).  The work is enqueued on hip_stream (NULL = default
 * stream) of `device` and not waited for: out is valid once that stream has
 * passed it.  Calls that overlap on one GPU share the work area and race;
 * calls in order on one stream do not.  SPFD_INVALID_ARG for a null required
 * pointer, nvox <= 0, q outside (0, 1] or a bad device; SPFD_HIP_ERROR if a
 * launch fails. */
spfd_status spfd_percentile_noalloc(int device, void *hip_stream, const uint8_t *labels, const double *sigma_table,
                                    int n_labels, const double *sigma_voxel, long long nvox, const double *emag,
                                    double q, double *out);

/* A measurement aid for the roofline of the bandwidth-bound kernels: the
 * STREAM triad a = b + 1.5 c over n doubles (device arrays, caller-owned,
 * 16-byte aligned), in two launch shapes, each timed reps times with HIP
 * events on hip_stream of `device` after one untimed run; *best_gbs (host)
 * = the best 24 n bytes / time in GB/s.  Arrays much larger than the
 * 256 MB Infinity Cache measure HBM.  SPFD_INVALID_ARG for null pointers,
 * n < 2, reps < 1 or a bad device. */
spfd_status spfd_stream_triad(int device, void *hip_stream, double *a, const double *b, const double *c,
                              long long n, int reps, double *best_gbs);

/* Several voxel models in one handle (many phantoms of uneven size solved
 * together, each with its own conductivities, source and CG scalars): the
 * models are stacked along z in one packed grid, each starting on a node
 * layer that is a multiple of 64 and at least one empty voxel layer above the
 * previous one, so that no brick of the structured multigrid levels and no
 * aggregate spans two models.  One hierarchy serves all of them: every level
 * kernel runs once over all models (the cycle is block-diagonal), and the
 * finest-level CG kernels run one launch row per model over that model's
 * bricks, with the model's own alpha, beta, residual norms and stop test
 * (so each model's iterates are those of its own preconditioned CG).
 * n (1..16) models; dims [n][3] (host): nx, ny, nz voxels of model m; labels
 * [n] (host array of device pointers to uint8 [nz][ny][nx] arrays, copied);
 * h as for spfd_set_geometry.  Then spfd_set_sigma_tables, spfd_build (split
 * aggregation from level 3 or finer), spfd_set_source(h, m, a_m) with a_m in
 * model m's own layout [3][(nx+1)(ny+1)(nz+1)], and spfd_solve, whose psi is
 * the models' node arrays one after the other and info one entry per model.
 * The number of right sides is the number of models.  spfd_efield,
 * spfd_adjoint, spfd_percentile, spfd_edge_potentials, spfd_solve_many, the
 * per-label and per-voxel conductivity calls, FGMRES and warm starts give
 * SPFD_BAD_STATE / SPFD_INVALID_ARG on such a handle. */
spfd_status spfd_set_geometry_many(spfd_handle h, int n, const int *dims, double hx, double hy, double hz,
                                   const uint8_t *const *labels);
/* Conductivity tables of the packed models: tables [n] (host array of host
 * arrays), n_labels [n] (1..256 each; finite, >= 0; 0 = air).  A voxel whose
 * label its model's table does not cover makes spfd_build fail with
 * SPFD_INVALID_ARG. */
spfd_status spfd_set_sigma_tables(spfd_handle h, const double *const *tables, const int *n_labels);

/* Solve Eq. (3) on several voxel models at once (each handle built, with its
 * sources set, on the same device).  The CG iterations of all handles advance
 * in lockstep, each handle's kernels on its own stream, so that problems of
 * uneven size share the GPU.  psi[k] is handle k's output as in spfd_solve;
 * info (host, nullable) holds the right sides of all handles in order.
 * opt as in spfd_solve (use_x0 ignored).  Errors are reported on hs[0]. */
spfd_status spfd_solve_many(spfd_handle *hs, int n, const spfd_solve_options *opt, double **psi,
                            spfd_rhs_info *info);

/* Adjoint gradient of a scalar objective J(|E|) with respect to the voxel
 * conductivities, by one extra solve of Eq. (3) on the built hierarchy.
 * Inputs: omega, a and psi of a forward solution (as for spfd_efield), and
 * grad_emag [nvox] (device) = dJ/d|E_v|.  Computes g_e = dJ/du_e on the edges,
 * solves A lambda = G^T g (opt as for spfd_solve, use_x0 ignored) and writes
 *   grad_sigma_voxel [nvox] (device) = -sum over the 12 edges e of v of
 *       (dual area / length / 4) (G lambda)_e u_e   (0 for air voxels);
 *   grad_sigma_table (host, nullable) = per-label sums of grad_sigma_voxel
 *       (n_labels entries of the sigma table; 256 in per-voxel mode).
 * Follows from A Psi = -G^T M a, u = a + G Psi (Eqs. (1), (3)) and dA = G^T dM G.
 * info (host, nullable) reports the adjoint solve. */
spfd_status spfd_adjoint(spfd_handle h, double omega, const double *a, const double *psi, const double *grad_emag,
                         const spfd_solve_options *opt, double *grad_sigma_voxel, double *grad_sigma_table,
                         spfd_rhs_info *info);

/* Per-launch timing, a tracing aid.  Kernel classes: */
enum {
    SPFD_K_SPMV = 0,          /* outer CG: p = z + beta p, q = A p, p.q partials (FP64); q is stored only for
                                 the flexible beta */
    SPFD_K_UPDATE = 1,        /* outer CG: r -= alpha q (standard beta: q = A p formed again from the stored p),
                                 ||r||^2 partials, FP32 copy of r */
    SPFD_K_DOTS = 2,          /* outer CG: last finest-level smoothing step with the r.z and z.q partials */
    SPFD_K_PUPDATE = 3,       /* outer CG: x += sum alpha_j p_j over a window of kept search directions */
    SPFD_K_SMOOTH0 = 4,       /* finest level: Chebyshev step with a stencil application */
    SPFD_K_SMOOTH0_FIRST = 5, /* finest level: first Chebyshev step from zero (no stencil) */
    SPFD_K_RESTRICT0 = 6,     /* finest level: residual and restriction */
    SPFD_K_PROLONG0 = 7,      /* finest level: first post-smoothing step with the prolongation */
    SPFD_K_COARSE = 8,        /* every kernel of the coarser levels and the coarsest solve */
    SPFD_K_FINISH = 9,        /* one-workgroup reduction finishers */
    SPFD_K_RHS = 10,          /* right side b = -G^T M a */
    SPFD_K_EFIELD = 11,       /* E-field and edge voltages */
    SPFD_K_GAUGE = 12,        /* component means and the output of psi */
    SPFD_K_RESID = 13,        /* true residual b - A x on the finest level (start, restart, exit) */
    SPFD_K_COUNT = 14
};
/* Enable timing for the classes in the bit mask (1 << class); resets all
 * counters.  While enabled, the launches of such a class in the second CG
 * iteration of every solve (run from the host, not from the captured graph)
 * are bracketed by two HIP events on the handle's stream: a sample of every
 * solve, at the cost of one eagerly launched iteration.  With
 * SPFD_TIMING_COLD in the mask, a kernel that reads and writes a 1 GiB buffer
 * (four times the Infinity Cache) runs before every timed launch, outside
 * its events, so each sample starts from cold caches; the buffer is held
 * until timing is set again without the flag. */
#define SPFD_TIMING_COLD 0x80000000u
spfd_status spfd_timing(spfd_handle h, unsigned int class_mask);
/* Counters of a class since the last spfd_timing call: all launches and their
 * algorithmic bytes (counted whether or not the class is timed), and the timed
 * launches with their summed event time (ms) and algorithmic bytes.
 * Algorithmic bytes count, per unknown of the level, one read or write of each
 * array the kernel touches (1 byte per voxel label, 3 weights per node where
 * weights are stored).  Any output pointer may be NULL. */
spfd_status spfd_timing_get(spfd_handle h, int kclass, long long *launches, double *algorithmic_bytes,
                            long long *timed_launches, double *timed_ms, double *timed_bytes);

#ifdef __cplusplus
}
#endif
#endif /* SPFD_H */
