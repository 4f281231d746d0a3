/*
 * CPU oracle of the Co-Sim. SPFD Poisson solve and E-field post-processing.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * FP64 reference that the HIP library is checked against.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it.  It shares no code with the HIP library.
 *
 * What it computes (paper: Sec. II, Eqs. (1) and (3); Sec. III.A; Sec. III.F):
 *   - M_kappa: a diagonal matrix of edge conductances of the voxel grid,
 *     M_e = kbar_e * (dual facet area) / (edge length), kbar_e the mean of the
 *     conductivities of the four voxels that share edge e (voxels outside the
 *     grid are air);
 *   - unknowns: only nodes touched by conductive voxels (Sec. III.A);
 *   - Eq. (3): G^T M G Psi = -G^T M a with (G Psi)_e = Psi_head - Psi_tail,
 *     solved by Jacobi-preconditioned CG in double precision; the singular
 *     system is made unique by a zero mean of Psi over each connected
 *     component of the conductor;
 *   - Eq. (1): e = -j omega (a + G Psi); this code returns the real edge
 *     voltage u = a + G Psi (so Im(e) = -omega u) and the voxel-averaged field
 *     magnitude |E|_v = omega * |ubar_v / h| with ubar_{v,d} the mean of the
 *     four d-directed edges of voxel v (Sec. III.F: voxel averaged field);
 *   - an adjoint gradient of a scalar objective of |E| with respect to the
 *     voxel conductivities (one extra solve of Eq. (3) with another source).
 *
 * Layout: voxel (i,j,k) -> i + nx*(j + ny*k); node (i,j,k) -> i + Nx*(j + Ny*k)
 * with Nx = nx+1, Ny = ny+1; edge arrays [3][Nnodes], entry [d][n] is the edge
 * from node n to node n + e_d.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int nx, ny, nz;
    long Nx, Ny, Nz, nn;   /* node grid */
    double h[3];
} grid_t;

static grid_t make_grid(int nx, int ny, int nz, const double *h)
{
    grid_t g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.Nx = nx + 1; g.Ny = ny + 1; g.Nz = nz + 1;
    g.nn = g.Nx * g.Ny * g.Nz;
    g.h[0] = h[0]; g.h[1] = h[1]; g.h[2] = h[2];
    return g;
}

static inline long node_id(const grid_t *g, long i, long j, long k) { return i + g->Nx * (j + g->Ny * k); }

/* conductivity of voxel (i,j,k); outside the grid = air */
static inline double vox_sigma(const grid_t *g, const double *sig, long i, long j, long k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return 0.0;
    return sig[i + (long)g->nx * (j + (long)g->ny * k)];
}

/* ---------------------------------------------------------------------------
 * M_kappa (Eq. (3)): edge conductances.  Edge of direction d at node (i,j,k)
 * runs to the node one step along d; the four voxels sharing it are those
 * with index i (resp. j, k) along d and index {c-1, c} along the two other
 * axes.  M = (sum of the four sigmas / 4) * h_a * h_b / h_d.
 * ------------------------------------------------------------------------- */
void oracle_edge_conductance(int nx, int ny, int nz, const double *h, const double *sig, double *M)
{
    grid_t g = make_grid(nx, ny, nz, h);
    const double geo[3] = { h[1] * h[2] / h[0], h[0] * h[2] / h[1], h[0] * h[1] / h[2] };
    #pragma omp parallel for schedule(static)
    for (long k = 0; k < g.Nz; ++k)
        for (long j = 0; j < g.Ny; ++j)
            for (long i = 0; i < g.Nx; ++i) {
                long n = node_id(&g, i, j, k);
                double sx = 0.0, sy = 0.0, sz = 0.0;
                if (i < nx)
                    sx = vox_sigma(&g, sig, i, j - 1, k - 1) + vox_sigma(&g, sig, i, j, k - 1)
                       + vox_sigma(&g, sig, i, j - 1, k) + vox_sigma(&g, sig, i, j, k);
                if (j < ny)
                    sy = vox_sigma(&g, sig, i - 1, j, k - 1) + vox_sigma(&g, sig, i, j, k - 1)
                       + vox_sigma(&g, sig, i - 1, j, k) + vox_sigma(&g, sig, i, j, k);
                if (k < nz)
                    sz = vox_sigma(&g, sig, i - 1, j - 1, k) + vox_sigma(&g, sig, i, j - 1, k)
                       + vox_sigma(&g, sig, i - 1, j, k) + vox_sigma(&g, sig, i, j, k);
                M[0 * g.nn + n] = 0.25 * sx * geo[0];
                M[1 * g.nn + n] = 0.25 * sy * geo[1];
                M[2 * g.nn + n] = 0.25 * sz * geo[2];
            }
}

/* neighbour of node (i,j,k) across edge slot s = 0..5: (+x,-x,+y,-y,+z,-z);
 * returns the neighbour node and the conductance of the connecting edge */
static inline long nbr(const grid_t *g, const double *M, long i, long j, long k, int s, double *w)
{
    long n = node_id(g, i, j, k);
    *w = 0.0;
    switch (s) {
    case 0: if (i + 1 < g->Nx) { *w = M[n];              return n + 1; } break;
    case 1: if (i > 0)         { *w = M[n - 1];          return n - 1; } break;
    case 2: if (j + 1 < g->Ny) { *w = M[g->nn + n];      return n + g->Nx; } break;
    case 3: if (j > 0)         { *w = M[g->nn + n - g->Nx]; return n - g->Nx; } break;
    case 4: if (k + 1 < g->Nz) { *w = M[2 * g->nn + n];  return n + g->Nx * g->Ny; } break;
    case 5: if (k > 0)         { *w = M[2 * g->nn + n - g->Nx * g->Ny]; return n - g->Nx * g->Ny; } break;
    }
    return -1;
}

/* ---------------------------------------------------------------------------
 * Unknowns and connected components (Sec. III.A: only conductive voxels).
 * A node is an unknown (DOF) iff one of its edges has M > 0.  DOFs are
 * numbered in node order; components are found by breadth-first search over
 * edges with M > 0.  comp[n] = component id or -1 for non-DOF nodes.
 * Returns the number of components.
 * ------------------------------------------------------------------------- */
int oracle_components(int nx, int ny, int nz, const double *h, const double *M, int32_t *comp)
{
    grid_t g = make_grid(nx, ny, nz, h);
    for (long n = 0; n < g.nn; ++n) comp[n] = -2;          /* -2: unvisited */
    for (long k = 0; k < g.Nz; ++k)
        for (long j = 0; j < g.Ny; ++j)
            for (long i = 0; i < g.Nx; ++i) {
                int any = 0;
                for (int s = 0; s < 6; ++s) { double w; if (nbr(&g, M, i, j, k, s, &w) >= 0 && w > 0.0) any = 1; }
                if (!any) comp[node_id(&g, i, j, k)] = -1;
            }
    long *queue = (long *)malloc(sizeof(long) * (size_t)g.nn);
    int nc = 0;
    for (long start = 0; start < g.nn; ++start) {
        if (comp[start] != -2) continue;
        long head = 0, tail = 0;
        queue[tail++] = start;
        comp[start] = nc;
        while (head < tail) {
            long n = queue[head++];
            long k = n / (g.Nx * g.Ny), rem = n % (g.Nx * g.Ny), j = rem / g.Nx, i = rem % g.Nx;
            for (int s = 0; s < 6; ++s) {
                double w;
                long m = nbr(&g, M, i, j, k, s, &w);
                if (m >= 0 && w > 0.0 && comp[m] == -2) { comp[m] = nc; queue[tail++] = m; }
            }
        }
        ++nc;
    }
    free(queue);
    return nc;
}

/* ---------------------------------------------------------------------------
 * Explicit CSR assembly of A = G^T M G over the DOFs (Eq. (3) left side):
 * A_nn = sum of the conductances of the edges at n, A_nm = -M_e for the edge
 * e joining n and m.
 * ------------------------------------------------------------------------- */
typedef struct {
    long ndof;
    long *rowptr;
    long *col;
    double *val;
    long *node_of;     /* DOF -> node */
    long *dof_of;      /* node -> DOF or -1 */
    int32_t *comp_dof; /* DOF -> component */
    int ncomp;
    long *comp_size;
} csr_t;

static void csr_free(csr_t *A)
{
    free(A->rowptr); free(A->col); free(A->val); free(A->node_of); free(A->dof_of);
    free(A->comp_dof); free(A->comp_size);
}

static void assemble(const grid_t *g, const double *M, const int32_t *comp, int ncomp, csr_t *A)
{
    A->dof_of = (long *)malloc(sizeof(long) * (size_t)g->nn);
    long nd = 0;
    for (long n = 0; n < g->nn; ++n) A->dof_of[n] = comp[n] >= 0 ? nd++ : -1;
    A->ndof = nd;
    A->node_of = (long *)malloc(sizeof(long) * (size_t)(nd + 1));
    A->comp_dof = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nd + 1));
    A->ncomp = ncomp;
    A->comp_size = (long *)calloc((size_t)ncomp + 1, sizeof(long));
    for (long n = 0; n < g->nn; ++n)
        if (A->dof_of[n] >= 0) {
            A->node_of[A->dof_of[n]] = n;
            A->comp_dof[A->dof_of[n]] = comp[n];
            A->comp_size[comp[n]]++;
        }
    A->rowptr = (long *)malloc(sizeof(long) * (size_t)(nd + 1));
    A->col = (long *)malloc(sizeof(long) * (size_t)(7 * nd + 1));
    A->val = (double *)malloc(sizeof(double) * (size_t)(7 * nd + 1));
    /* fixed 7 slots per row (diagonal first), trailing unused slots have value 0
     * and point to the row itself, so every row has the same layout */
    #pragma omp parallel for schedule(static)
    for (long r = 0; r < nd; ++r) {
        long n = A->node_of[r];
        long k = n / (g->Nx * g->Ny), rem = n % (g->Nx * g->Ny), j = rem / g->Nx, i = rem % g->Nx;
        long p = 7 * r;
        double diag = 0.0;
        A->col[p] = r;
        int q = 1;
        for (int s = 0; s < 6; ++s) {
            double w;
            long m = nbr(g, M, i, j, k, s, &w);
            if (m >= 0 && w > 0.0) {
                diag += w;
                A->col[p + q] = A->dof_of[m];
                A->val[p + q] = -w;
                ++q;
            }
        }
        for (; q < 7; ++q) { A->col[p + q] = r; A->val[p + q] = 0.0; }
        A->val[p] = diag;
        A->rowptr[r] = p;
    }
    A->rowptr[nd] = 7 * nd;
}

static void spmv(const csr_t *A, const double *x, double *y)
{
    #pragma omp parallel for schedule(static)
    for (long r = 0; r < A->ndof; ++r) {
        double s = 0.0;
        for (long p = A->rowptr[r]; p < A->rowptr[r + 1]; ++p) s += A->val[p] * x[A->col[p]];
        y[r] = s;
    }
}

static double dot(long n, const double *x, const double *y)
{
    double s = 0.0;
    #pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* the gauge: subtract the mean over each connected component */
static void project_mean_zero(const csr_t *A, double *x)
{
    int nc = A->ncomp;
    double *sum = (double *)calloc((size_t)nc + 1, sizeof(double));
    for (long r = 0; r < A->ndof; ++r) sum[A->comp_dof[r]] += x[r];
    for (int c = 0; c < nc; ++c) sum[c] /= (double)A->comp_size[c];
    #pragma omp parallel for schedule(static)
    for (long r = 0; r < A->ndof; ++r) x[r] -= sum[A->comp_dof[r]];
    free(sum);
}

/* Jacobi-PCG for A x = b with b orthogonal to the component constants and the
 * preconditioner z = P D^{-1} r, P the mean-zero projection (symmetric positive
 * definite on the range of A).  x starts at 0.  Stops when ||r|| <= tol ||b||.
 * Returns the iteration count. */
static int jacobi_pcg(const csr_t *A, const double *b, double *x, double tol, int max_iter)
{
    long n = A->ndof;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *dinv = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; dinv[i] = 1.0 / A->val[A->rowptr[i]]; }
    double bnorm = sqrt(dot(n, b, b));
    int it = 0;
    if (bnorm > 0.0) {
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        project_mean_zero(A, z);
        memcpy(p, z, sizeof(double) * (size_t)n);
        double rz = dot(n, r, z);
        while (it < max_iter) {
            spmv(A, p, q);
            double alpha = rz / dot(n, p, q);
            #pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            ++it;
            if (sqrt(dot(n, r, r)) <= tol * bnorm) break;
            #pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
            project_mean_zero(A, z);
            double rz_new = dot(n, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            #pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
    }
    project_mean_zero(A, x);
    free(r); free(z); free(p); free(q); free(dinv);
    return it;
}

static double true_relres(const csr_t *A, const double *b, const double *x)
{
    long n = A->ndof;
    double *q = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    spmv(A, x, q);
    double rr = 0.0, bb = 0.0;
    for (long i = 0; i < n; ++i) { double d = b[i] - q[i]; rr += d * d; bb += b[i] * b[i]; }
    free(q);
    return bb > 0.0 ? sqrt(rr / bb) : 0.0;
}

/* b = -G^T M a on the DOFs (Eq. (3) right side):
 * b_n = sum_{edges leaving n} M_e a_e - sum_{edges entering n} M_e a_e */
static void rhs_div(const grid_t *g, const double *M, const double *edge_field, const csr_t *A, double *b)
{
    #pragma omp parallel for schedule(static)
    for (long r = 0; r < A->ndof; ++r) {
        long n = A->node_of[r];
        long k = n / (g->Nx * g->Ny), rem = n % (g->Nx * g->Ny), j = rem / g->Nx, i = rem % g->Nx;
        double s = 0.0;
        if (i + 1 < g->Nx) s += M[n] * edge_field[n];
        if (i > 0) s -= M[n - 1] * edge_field[n - 1];
        if (j + 1 < g->Ny) s += M[g->nn + n] * edge_field[g->nn + n];
        if (j > 0) s -= M[g->nn + n - g->Nx] * edge_field[g->nn + n - g->Nx];
        if (k + 1 < g->Nz) s += M[2 * g->nn + n] * edge_field[2 * g->nn + n];
        if (k > 0) s -= M[2 * g->nn + n - g->Nx * g->Ny] * edge_field[2 * g->nn + n - g->Nx * g->Ny];
        b[r] = s;
    }
}

typedef struct {
    int iterations;
    int ncomp;
    long ndof;
    double relres;      /* true ||b - A psi|| / ||b|| */
    double bnorm;
    double t_assemble;  /* s */
    double t_solve;     /* s */
} oracle_info;

/* ---------------------------------------------------------------------------
 * Solve Eq. (3) for Psi on all nodes (0 at non-DOF nodes), mean-zero per
 * component.  a: [3][Nnodes].  nthreads <= 0 keeps the OpenMP default.
 * ------------------------------------------------------------------------- */
int oracle_solve(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                 double tol, int max_iter, int nthreads, double *psi, oracle_info *info)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    grid_t g = make_grid(nx, ny, nz, h);
    double t0 = omp_get_wtime();
    double *M = (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.nn);
    oracle_edge_conductance(nx, ny, nz, h, sig, M);
    int nc = oracle_components(nx, ny, nz, h, M, comp);
    csr_t A;
    assemble(&g, M, comp, nc, &A);
    double *b = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    double *x = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    rhs_div(&g, M, a, &A, b);
    project_mean_zero(&A, b);   /* exact in exact arithmetic: 1^T G^T = 0 per component */
    double t1 = omp_get_wtime();
    int it = jacobi_pcg(&A, b, x, tol, max_iter);
    double t2 = omp_get_wtime();
    memset(psi, 0, sizeof(double) * (size_t)g.nn);
    for (long r = 0; r < A.ndof; ++r) psi[A.node_of[r]] = x[r];
    if (info) {
        info->iterations = it;
        info->ncomp = nc;
        info->ndof = A.ndof;
        info->relres = true_relres(&A, b, x);
        info->bnorm = sqrt(dot(A.ndof, b, b));
        info->t_assemble = t1 - t0;
        info->t_solve = t2 - t1;
    }
    free(M); free(comp); free(b); free(x);
    csr_free(&A);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Residual of a given Psi: r = b - A Psi over the DOFs, with b = -G^T M a
 * projected to mean zero per component.  Writes r on all nodes (0 elsewhere)
 * if r != NULL and returns ||r|| / ||b||.  Used to check a solution computed
 * elsewhere at sizes where a second solve on the CPU is too slow.
 * ------------------------------------------------------------------------- */
double oracle_residual(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                       const double *psi, int nthreads, double *r_nodes)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    grid_t g = make_grid(nx, ny, nz, h);
    double *M = (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.nn);
    oracle_edge_conductance(nx, ny, nz, h, sig, M);
    int nc = oracle_components(nx, ny, nz, h, M, comp);
    csr_t A;
    assemble(&g, M, comp, nc, &A);
    double *b = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    double *x = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    rhs_div(&g, M, a, &A, b);
    project_mean_zero(&A, b);
    for (long r = 0; r < A.ndof; ++r) x[r] = psi[A.node_of[r]];
    spmv(&A, x, q);
    double rr = 0.0, bb = 0.0;
    if (r_nodes) memset(r_nodes, 0, sizeof(double) * (size_t)g.nn);
    for (long r = 0; r < A.ndof; ++r) {
        double d = b[r] - q[r];
        rr += d * d; bb += b[r] * b[r];
        if (r_nodes) r_nodes[A.node_of[r]] = d;
    }
    free(M); free(comp); free(b); free(x); free(q);
    csr_free(&A);
    return bb > 0.0 ? sqrt(rr / bb) : 0.0;
}

/* ---------------------------------------------------------------------------
 * Eq. (1) and the voxel average (Sec. III.F).  u_e = a_e + Psi_head - Psi_tail
 * on edges with M_e > 0 (0 elsewhere).  For a conductive voxel the mean of
 * its four d-directed edges gives ubar_d and |E| = omega*sqrt(sum (ubar_d/h_d)^2);
 * air voxels get 0.  u (nullable) is [3][Nnodes], emag is [nvox].
 * ------------------------------------------------------------------------- */
void oracle_efield(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                   const double *psi, double omega, double *u, double *emag)
{
    grid_t g = make_grid(nx, ny, nz, h);
    double *M = (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    double *ue = u ? u : (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    oracle_edge_conductance(nx, ny, nz, h, sig, M);
    const long step[3] = { 1, g.Nx, g.Nx * g.Ny };
    #pragma omp parallel for schedule(static)
    for (long n = 0; n < g.nn; ++n)
        for (int d = 0; d < 3; ++d) {
            double w = M[d * g.nn + n];
            ue[d * g.nn + n] = w > 0.0 ? a[d * g.nn + n] + psi[n + step[d]] - psi[n] : 0.0;
        }
    #pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + (long)nx * (j + (long)ny * k);
                if (!(sig[v] > 0.0)) { emag[v] = 0.0; continue; }
                /* the four x-edges of the voxel start at nodes (i, j..j+1, k..k+1), etc. */
                double ux = ue[node_id(&g, i, j, k)] + ue[node_id(&g, i, j + 1, k)]
                          + ue[node_id(&g, i, j, k + 1)] + ue[node_id(&g, i, j + 1, k + 1)];
                double uy = ue[g.nn + node_id(&g, i, j, k)] + ue[g.nn + node_id(&g, i + 1, j, k)]
                          + ue[g.nn + node_id(&g, i, j, k + 1)] + ue[g.nn + node_id(&g, i + 1, j, k + 1)];
                double uz = ue[2 * g.nn + node_id(&g, i, j, k)] + ue[2 * g.nn + node_id(&g, i + 1, j, k)]
                          + ue[2 * g.nn + node_id(&g, i, j + 1, k)] + ue[2 * g.nn + node_id(&g, i + 1, j + 1, k)];
                double ex = 0.25 * ux / h[0], ey = 0.25 * uy / h[1], ez = 0.25 * uz / h[2];
                emag[v] = omega * sqrt(ex * ex + ey * ey + ez * ez);
            }
    free(M);
    if (!u) free(ue);
}

/* ---------------------------------------------------------------------------
 * Adjoint gradient of a scalar J(|E|) with respect to the voxel conductivities.
 * Given dJ/d|E_v| (grad_emag, [nvox]) and the forward solution psi:
 *   g_e   = sum over the conductive voxels v sharing edge e (direction d) of
 *           grad_emag_v * omega^2 * ubar_{v,d} / (4 h_d^2 |E_v|)   (|E_v| > 0)
 *   solve A lambda = G^T g (mean-zero, Jacobi-PCG to tol)
 *   dJ/dsigma_v = - sum over the 12 edges e of v of
 *           (1/4) (dual area_e / length_e) (G lambda)_e u_e       (conductive v)
 * which follows from A Psi = -G^T M a, u = a + G Psi and dA = G^T dM G.
 * Air voxels get 0.  grad_table (nullable, [n_labels]) sums the voxel
 * gradient per label when labels != NULL.
 * ------------------------------------------------------------------------- */
int oracle_adjoint(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                   const double *psi, double omega, const double *grad_emag, double tol, int max_iter,
                   int nthreads, const uint8_t *labels, int n_labels,
                   double *grad_sigma, double *grad_table, oracle_info *info)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    grid_t g = make_grid(nx, ny, nz, h);
    long nvox = (long)nx * ny * nz;
    double *M = (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.nn);
    double *u = (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    double *E = (double *)malloc(sizeof(double) * (size_t)(nvox + 1));
    double *ge = (double *)calloc((size_t)(3 * g.nn), sizeof(double));
    oracle_edge_conductance(nx, ny, nz, h, sig, M);
    int nc = oracle_components(nx, ny, nz, h, M, comp);
    oracle_efield(nx, ny, nz, h, sig, a, psi, omega, u, E);
    /* scatter dJ/du_e (serial: several voxels share an edge) */
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + (long)nx * (j + (long)ny * k);
                if (!(sig[v] > 0.0) || !(E[v] > 0.0)) continue;
                long nx_[4] = { node_id(&g, i, j, k), node_id(&g, i, j + 1, k), node_id(&g, i, j, k + 1), node_id(&g, i, j + 1, k + 1) };
                long ny_[4] = { node_id(&g, i, j, k), node_id(&g, i + 1, j, k), node_id(&g, i, j, k + 1), node_id(&g, i + 1, j, k + 1) };
                long nz_[4] = { node_id(&g, i, j, k), node_id(&g, i + 1, j, k), node_id(&g, i, j + 1, k), node_id(&g, i + 1, j + 1, k) };
                const long *ed[3] = { nx_, ny_, nz_ };
                for (int d = 0; d < 3; ++d) {
                    double ub = 0.0;
                    for (int q = 0; q < 4; ++q) ub += u[d * g.nn + ed[d][q]];
                    ub *= 0.25;
                    double c = grad_emag[v] * omega * omega * ub / (4.0 * h[d] * h[d] * E[v]);
                    for (int q = 0; q < 4; ++q) ge[d * g.nn + ed[d][q]] += c;
                }
            }
    csr_t A;
    assemble(&g, M, comp, nc, &A);
    double *b = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    double *lam = (double *)malloc(sizeof(double) * (size_t)(A.ndof + 1));
    /* (G^T g)_n = sum of g over edges entering n - sum over edges leaving n */
    {
        #pragma omp parallel for schedule(static)
        for (long r = 0; r < A.ndof; ++r) {
            long n = A.node_of[r];
            long k = n / (g.Nx * g.Ny), rem = n % (g.Nx * g.Ny), j = rem / g.Nx, i = rem % g.Nx;
            double s = 0.0;
            if (i + 1 < g.Nx) s -= ge[n];
            if (i > 0) s += ge[n - 1];
            if (j + 1 < g.Ny) s -= ge[g.nn + n];
            if (j > 0) s += ge[g.nn + n - g.Nx];
            if (k + 1 < g.Nz) s -= ge[2 * g.nn + n];
            if (k > 0) s += ge[2 * g.nn + n - g.Nx * g.Ny];
            b[r] = s;
        }
    }
    project_mean_zero(&A, b);
    int it = jacobi_pcg(&A, b, lam, tol, max_iter);
    if (info) {
        info->iterations = it;
        info->ncomp = nc;
        info->ndof = A.ndof;
        info->relres = true_relres(&A, b, lam);
        info->bnorm = sqrt(dot(A.ndof, b, b));
        info->t_assemble = 0.0;
        info->t_solve = 0.0;
    }
    double *lam_n = (double *)calloc((size_t)g.nn, sizeof(double));
    for (long r = 0; r < A.ndof; ++r) lam_n[A.node_of[r]] = lam[r];
    const double geo[3] = { h[1] * h[2] / h[0], h[0] * h[2] / h[1], h[0] * h[1] / h[2] };
    const long step[3] = { 1, g.Nx, g.Nx * g.Ny };
    #pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + (long)nx * (j + (long)ny * k);
                if (!(sig[v] > 0.0)) { grad_sigma[v] = 0.0; continue; }
                long nx_[4] = { node_id(&g, i, j, k), node_id(&g, i, j + 1, k), node_id(&g, i, j, k + 1), node_id(&g, i, j + 1, k + 1) };
                long ny_[4] = { node_id(&g, i, j, k), node_id(&g, i + 1, j, k), node_id(&g, i, j, k + 1), node_id(&g, i + 1, j, k + 1) };
                long nz_[4] = { node_id(&g, i, j, k), node_id(&g, i + 1, j, k), node_id(&g, i, j + 1, k), node_id(&g, i + 1, j + 1, k) };
                const long *ed[3] = { nx_, ny_, nz_ };
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int q = 0; q < 4; ++q) {
                        long n = ed[d][q];
                        double glam = lam_n[n + step[d]] - lam_n[n];
                        s += 0.25 * geo[d] * glam * u[d * g.nn + n];
                    }
                grad_sigma[v] = -s;
            }
    if (grad_table && labels) {
        for (int t = 0; t < n_labels; ++t) grad_table[t] = 0.0;
        for (long v = 0; v < nvox; ++v)
            if (labels[v] < n_labels) grad_table[labels[v]] += grad_sigma[v];
    }
    free(M); free(comp); free(u); free(E); free(ge); free(b); free(lam); free(lam_n);
    csr_free(&A);
    return 0;
}

/* Dense matrix A (ndof x ndof, row-major) and rhs b for tiny grids, with the
 * DOF -> node map, so that a dense direct solve can check the iterative one. */
long oracle_dense_system(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                         double *A_dense, double *b, long *node_of, int32_t *comp_of, long max_dof)
{
    grid_t g = make_grid(nx, ny, nz, h);
    double *M = (double *)malloc(sizeof(double) * (size_t)(3 * g.nn));
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.nn);
    oracle_edge_conductance(nx, ny, nz, h, sig, M);
    int nc = oracle_components(nx, ny, nz, h, M, comp);
    csr_t A;
    assemble(&g, M, comp, nc, &A);
    long nd = A.ndof;
    if (nd <= max_dof && A_dense) {
        memset(A_dense, 0, sizeof(double) * (size_t)(nd * nd));
        for (long r = 0; r < nd; ++r)
            for (long p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) A_dense[r * nd + A.col[p]] += A.val[p];
        rhs_div(&g, M, a, &A, b);
        for (long r = 0; r < nd; ++r) { node_of[r] = A.node_of[r]; comp_of[r] = A.comp_dof[r]; }
    }
    free(M); free(comp);
    csr_free(&A);
    return nd;
}
