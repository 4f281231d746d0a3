// Edge potentials from facet fluxes, Eq. (2) b = C a, in a tree-cotree gauge
// (technical summary of Sec. II.A, step 3).
//
// On the structured voxel grid a spanning tree of the nodes is fixed: every
// z-edge, the y-edges of the node plane k = 0 and the x-edges of the node line
// j = k = 0 carry a = 0.  Every cotree edge then closes one facet whose other
// three edges are known, so the over-determined system becomes prefix sums:
//   plane k = 0 (z-facets):  a_x(i, j+1, 0) = a_x(i, j, 0) - b_z(i, j, 0)   (one thread per i)
//   columns (y- and x-facets): a_x(i, j, k+1) = a_x(i, j, k) + b_y(i, j, k),
//                              a_y(i, j, k+1) = a_y(i, j, k) - b_x(i, j, k)  (one thread per (i, j))
// and the remaining z-facets hold when the fluxes are divergence-free.  Arrays
// are [3][Nz][Ny][Nx] node-anchored (flux of normal d and edge along d start
// at node (i, j, k)), as the sources of spfd_set_source.  The sums run in the
// order of the recurrences.
#include "kernels.h"

namespace spfd {

__global__ __launch_bounds__(256) void k_tc_plane(const double *__restrict__ flux, double *__restrict__ a, Grid g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nx) return;
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    const double *bz = flux + 2 * nn;
    double acc = 0.0;
    a[i] = 0.0;
    for (int j = 0; j < g.ny; ++j) {
        acc -= bz[(long long)j * g.Nx + i];
        a[(long long)(j + 1) * g.Nx + i] = acc;
    }
}

__global__ __launch_bounds__(256) void k_tc_columns(const double *__restrict__ flux, double *__restrict__ a, Grid g)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.Nx * g.Ny) return;
    const int i = e % g.Nx, j = e / g.Nx;
    const long long nn = (long long)g.Nx * g.Ny * g.Nz;
    const long long plane = (long long)g.Nx * g.Ny;
    const bool hx = i < g.nx, hy = j < g.ny;
    const double *bx = flux, *by = flux + nn;
    double *ax = a, *ay = a + nn, *az = a + 2 * nn;
    double sx = hx ? ax[e] : 0.0;   // the plane k = 0, written by k_tc_plane
    double sy = 0.0;
    if (!hx) ax[e] = 0.0;
    ay[e] = 0.0;
    for (int k = 0; k < g.nz; ++k) {
        const long long o = (long long)k * plane + e;
        const double fy = hx ? by[o] : 0.0;
        const double fx = hy ? bx[o] : 0.0;
        sx += fy;
        sy -= fx;
        ax[o + plane] = hx ? sx : 0.0;
        ay[o + plane] = hy ? sy : 0.0;
        az[o] = 0.0;
    }
    az[(long long)g.nz * plane + e] = 0.0;
}

hipError_t launch_tree_cotree(const double *flux, double *a, const Grid &g, hipStream_t s)
{
    SPFD_LAUNCH(k_tc_plane, dim3((g.nx + 255) / 256), dim3(256), 0, s, flux, a, g);
    SPFD_LAUNCH(k_tc_columns, dim3((g.Nx * g.Ny + 255) / 256), dim3(256), 0, s, flux, a, g);
    return hipGetLastError();
}

}  // namespace spfd
