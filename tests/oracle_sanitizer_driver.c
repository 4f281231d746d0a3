/* Host-side sanitizer run of the CPU oracle (test infrastructure): every oracle entry point on tiny
 * grids with holes and several components, built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py.  Exits 0 when every call returns a sane result; any out-of-bounds
 * access, leak or undefined operation in the oracle aborts the run with the sanitizer's report. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int iterations;
    int ncomp;
    long ndof;
    double relres;
    double bnorm;
    double t_assemble;
    double t_solve;
} oracle_info;

void oracle_edge_conductance(int nx, int ny, int nz, const double *h, const double *sig, double *M);
int oracle_components(int nx, int ny, int nz, const double *h, const double *M, int32_t *comp);
int oracle_solve(int nx, int ny, int nz, const double *h, const double *sig, const double *a, double tol,
                 int max_iter, int nthreads, double *psi, oracle_info *info);
double oracle_residual(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                       const double *psi, int nthreads, double *r_nodes);
void oracle_efield(int nx, int ny, int nz, const double *h, const double *sig, const double *a, const double *psi,
                   double omega, double *u, double *emag);
int oracle_adjoint(int nx, int ny, int nz, const double *h, const double *sig, const double *a, const double *psi,
                   double omega, const double *grad_emag, double tol, int max_iter, int nthreads,
                   const uint8_t *labels, int n_labels, double *grad_sigma, double *grad_table, oracle_info *info);
long oracle_dense_system(int nx, int ny, int nz, const double *h, const double *sig, const double *a,
                         double *A_dense, double *b, long *node_of, int32_t *comp_of, long max_dof);

static const double OMEGA = 2.0 * 3.14159265358979323846 * 85e3;   /* 85 kHz */
static unsigned long long rng = 12879ull;
static double urand(void)
{
    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int nx, int ny, int nz, int nthreads)
{
    const double h[3] = {2e-3, 1.5e-3, 1e-3};
    const long nvox = (long)nx * ny * nz;
    const long nn = (long)(nx + 1) * (ny + 1) * (nz + 1);
    double *sig = malloc(sizeof(double) * nvox);
    uint8_t *lab = malloc(nvox);
    const double table[4] = {0.0, 0.2, 0.9, 0.05};
    for (long v = 0; v < nvox; ++v) {
        const int k = v / ((long)nx * ny);
        /* a layer of air splits the conductor into two components; random holes inside */
        lab[v] = (k == nz / 2 || urand() < 0.2) ? 0 : (uint8_t)(1 + (int)(urand() * 3.0));
        sig[v] = table[lab[v]];
    }
    double *a = malloc(sizeof(double) * 3 * nn), *psi = malloc(sizeof(double) * nn);
    double *r = malloc(sizeof(double) * nn), *u = malloc(sizeof(double) * 3 * nn);
    double *emag = malloc(sizeof(double) * nvox), *gE = malloc(sizeof(double) * nvox);
    double *gs = malloc(sizeof(double) * nvox), *gt = malloc(sizeof(double) * 4);
    double *M = malloc(sizeof(double) * 3 * nn);
    int32_t *comp = malloc(sizeof(int32_t) * nn);
    for (long e = 0; e < 3 * nn; ++e) a[e] = urand() - 0.5;
    for (long v = 0; v < nvox; ++v) gE[v] = urand();
    oracle_info info;
    const int st = oracle_solve(nx, ny, nz, h, sig, a, 1e-12, 2000, nthreads, psi, &info);
    const double rel = oracle_residual(nx, ny, nz, h, sig, a, psi, nthreads, r);
    oracle_efield(nx, ny, nz, h, sig, a, psi, OMEGA, u, emag);
    oracle_edge_conductance(nx, ny, nz, h, sig, M);
    const int nc = oracle_components(nx, ny, nz, h, M, comp);
    oracle_info ainfo;
    const int sta = oracle_adjoint(nx, ny, nz, h, sig, a, psi, OMEGA, gE, 1e-12, 2000, nthreads, lab, 4, gs,
                                   gt, &ainfo);
    long nd = info.ndof > 0 ? info.ndof : 1;
    double *A = malloc(sizeof(double) * nd * nd), *b = malloc(sizeof(double) * nd);
    long *node_of = malloc(sizeof(long) * nd);
    int32_t *comp_of = malloc(sizeof(int32_t) * nd);
    const long nd2 = oracle_dense_system(nx, ny, nz, h, sig, a, A, b, node_of, comp_of, nd);
    int ok = st == 0 && sta == 0 && info.relres <= 1e-11 && fabs(rel - info.relres) <= 1e-6 * info.relres + 1e-15 &&
             nc == info.ncomp && nc >= 2 && nd2 == info.ndof;
    for (long v = 0; v < nvox; ++v) ok = ok && isfinite(emag[v]) && isfinite(gs[v]) && (sig[v] > 0.0 || emag[v] == 0.0);
    printf("case %dx%dx%d: status %d/%d, %ld unknowns, %d components, %d iterations, relres %.2e (%.2e)\n", nx, ny, nz,
           st, sta, info.ndof, nc, info.iterations, info.relres, rel);
    free(sig); free(lab); free(a); free(psi); free(r); free(u); free(emag); free(gE); free(gs); free(gt);
    free(M); free(comp); free(A); free(b); free(node_of); free(comp_of);
    return ok;
}

int main(void)
{
    int ok = 1;
    ok = run_case(5, 4, 7, 1) && ok;
    ok = run_case(9, 6, 5, 2) && ok;
    ok = run_case(1, 1, 3, 1) && ok;
    printf(ok ? "sanitized oracle ok\n" : "sanitized oracle FAILED\n");
    return ok ? 0 : 1;
}
