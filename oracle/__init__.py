"""CPU oracle of the Co-Sim. SPFD Poisson solve (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.
It wraps ``spfd_oracle.c`` (plain C + OpenMP, FP64) through ctypes and adds a
dense NumPy reference for tiny grids (``oracle.dense``).  It shares no code
with the HIP library.

All arrays use the index conventions of ``workloads``: voxel arrays
(nz, ny, nx), node arrays (nz+1, ny+1, nx+1), edge arrays (3, nz+1, ny+1, nx+1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spfd_oracle.c")
_LIB = os.path.join(_HERE, "libspfd_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE FP64 round-to-nearest)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OracleInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("ncomp", ctypes.c_int), ("ndof", ctypes.c_long),
                ("relres", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("t_assemble", ctypes.c_double), ("t_solve", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.oracle_edge_conductance.argtypes = [I, I, I, P, P, P]
        lib.oracle_edge_conductance.restype = None
        lib.oracle_components.argtypes = [I, I, I, P, P, P]
        lib.oracle_components.restype = I
        lib.oracle_solve.argtypes = [I, I, I, P, P, P, D, I, I, P, ctypes.POINTER(OracleInfo)]
        lib.oracle_solve.restype = I
        lib.oracle_residual.argtypes = [I, I, I, P, P, P, P, I, P]
        lib.oracle_residual.restype = D
        lib.oracle_efield.argtypes = [I, I, I, P, P, P, P, D, P, P]
        lib.oracle_efield.restype = None
        lib.oracle_adjoint.argtypes = [I, I, I, P, P, P, P, D, P, D, I, I, P, I, P, P,
                                       ctypes.POINTER(OracleInfo)]
        lib.oracle_adjoint.restype = I
        lib.oracle_dense_system.argtypes = [I, I, I, P, P, P, P, P, P, P, ctypes.c_long]
        lib.oracle_dense_system.restype = ctypes.c_long
        _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p) if x is not None else None


def _dims(sigma):
    nz, ny, nx = sigma.shape
    return nx, ny, nz


def edge_conductance(sigma, h):
    """M_kappa as an edge array (3, nz+1, ny+1, nx+1)."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    M = np.empty((3, nz + 1, ny + 1, nx + 1))
    _load().oracle_edge_conductance(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(M))
    return M


def components(sigma, h):
    """(comp (nz+1,ny+1,nx+1) int32 with -1 at non-DOF nodes, number of components)."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    M = edge_conductance(sigma, h)
    comp = np.empty((nz + 1, ny + 1, nx + 1), np.int32)
    nc = _load().oracle_components(nx, ny, nz, _ptr(h), _ptr(M), _ptr(comp))
    return comp, nc


def solve(sigma, h, a, tol=1e-12, max_iter=200000, nthreads=0):
    """Mean-zero solution psi of Eq. (3) (node array) and an info dict."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    a = _f64(a)
    assert a.shape == (3, nz + 1, ny + 1, nx + 1)
    psi = np.empty((nz + 1, ny + 1, nx + 1))
    info = OracleInfo()
    _load().oracle_solve(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(a), tol, max_iter, nthreads,
                         _ptr(psi), ctypes.byref(info))
    return psi, info.as_dict()


def residual(sigma, h, a, psi, nthreads=0, want_nodes=False):
    """||b - A psi|| / ||b|| of a given psi (and optionally the residual node array)."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    a = _f64(a)
    psi = _f64(psi)
    r = np.empty((nz + 1, ny + 1, nx + 1)) if want_nodes else None
    rel = _load().oracle_residual(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(a), _ptr(psi), nthreads, _ptr(r))
    return (rel, r) if want_nodes else rel


def efield(sigma, h, a, psi, omega):
    """(u edge array, |E| voxel array) from Eq. (1) and the voxel average."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    a = _f64(a)
    psi = _f64(psi)
    u = np.empty((3, nz + 1, ny + 1, nx + 1))
    emag = np.empty((nz, ny, nx))
    _load().oracle_efield(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(a), _ptr(psi), omega, _ptr(u), _ptr(emag))
    return u, emag


def adjoint(sigma, h, a, psi, omega, grad_emag, tol=1e-12, max_iter=200000, nthreads=0,
            labels=None, n_labels=0):
    """(dJ/dsigma per voxel, dJ/dsigma per label or None, info) for a given dJ/d|E|."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    a = _f64(a)
    psi = _f64(psi)
    ge = _f64(grad_emag)
    gs = np.empty((nz, ny, nx))
    gt = np.empty(n_labels) if labels is not None else None
    lab = np.ascontiguousarray(labels, dtype=np.uint8) if labels is not None else None
    info = OracleInfo()
    _load().oracle_adjoint(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(a), _ptr(psi), omega, _ptr(ge),
                           tol, max_iter, nthreads, _ptr(lab), n_labels, _ptr(gs), _ptr(gt),
                           ctypes.byref(info))
    return gs, gt, info.as_dict()


def dense_system(sigma, h, a, max_dof=4000):
    """Dense A (ndof x ndof), b, DOF->node map and DOF->component for tiny grids."""
    sigma = _f64(sigma)
    nx, ny, nz = _dims(sigma)
    h = _f64(h)
    a = _f64(a)
    nd = _load().oracle_dense_system(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(a), None, None, None, None, 0)
    if nd > max_dof:
        raise ValueError(f"{nd} DOFs exceed max_dof={max_dof}")
    A = np.empty((nd, nd))
    b = np.empty(nd)
    node_of = np.empty(nd, np.int64)
    comp_of = np.empty(nd, np.int32)
    _load().oracle_dense_system(nx, ny, nz, _ptr(h), _ptr(sigma), _ptr(a), _ptr(A), _ptr(b),
                                _ptr(node_of), _ptr(comp_of), max_dof)
    return A, b, node_of, comp_of


def pnorm_objective(emag, p=8):
    """J = (sum |E_v|^p)^(1/p) over body voxels and dJ/d|E| (air voxels have |E| = 0)."""
    e = np.asarray(emag, dtype=np.float64)
    J = float(np.sum(e ** p) ** (1.0 / p))
    g = (e / J) ** (p - 1) if J > 0 else np.zeros_like(e)
    return J, g


def percentile_nearest_rank(emag, labels, sigma, q=0.99, n_labels=None):
    """Nearest-rank q-quantile of the voxel |E| over the conducting voxels (step 6 of the
    paper's technical summary, Sec. II.A; the voxel-averaged field, Sec. III.F), whole body
    and per label: sort the n values ascending and take the one of rank ceil(q n) (1-based).
    The body is the set of voxels with sigma > 0 (Sec. III.A: only conducting tissue is
    modelled), so a labelled voxel whose conductivity is 0 is excluded as air is; per label
    the set is the body voxels carrying that label, and a label without any gets NaN.
    sigma is the per-voxel conductivity array (same shape as emag and labels).
    Returns (whole-body value, per-label array)."""
    e = np.asarray(emag, dtype=np.float64).reshape(-1)
    lab = np.asarray(labels).reshape(-1)
    sig = np.asarray(sigma, dtype=np.float64).reshape(-1)
    if not (e.shape == lab.shape == sig.shape):
        raise ValueError("emag, labels and sigma must have the same number of voxels")
    body = sig > 0

    def nearest_rank(v):
        if v.size == 0:
            return float("nan")
        v = np.sort(v)
        r = int(np.ceil(q * v.size))
        return float(v[max(r, 1) - 1])

    n_labels = int(lab.max()) + 1 if n_labels is None else n_labels
    per = np.array([nearest_rank(e[body & (lab == t)]) for t in range(n_labels)])
    return nearest_rank(e[body]), per


def tree_cotree_potentials(flux):
    """Edge potentials a with C a = flux (Eq. (2)) in a tree-cotree gauge (technical summary
    of Sec. II.A, step 3).  flux is a (3, Nz, Ny, Nx) array of facet fluxes (normal d, anchored at
    the facet's lowest corner node, as in tests/discrete.py) and must be discretely divergence-free.

    Tree (a = 0 there): every z-edge, the y-edges of the node plane k = 0 and the x-edges of the node
    line j = k = 0.  Each cotree edge closes exactly one facet whose other edges are known:
      z-facets of the plane k = 0:  a_x(i, j+1, 0) = a_x(i, j, 0) - flux_z(i, j, 0),
      y-facets:                     a_x(i, j, k+1) = a_x(i, j, k) + flux_y(i, j, k),
      x-facets:                     a_y(i, j, k+1) = a_y(i, j, k) - flux_x(i, j, k);
    the z-facets above the bottom plane then hold because every cell's outgoing flux sums to zero.
    The recurrences are evaluated in this order (sequential sums)."""
    f = np.asarray(flux, dtype=np.float64)
    _, Nz, Ny, Nx = f.shape
    nx, ny, nz = Nx - 1, Ny - 1, Nz - 1
    a = np.zeros_like(f)
    for j in range(ny):
        a[0, 0, j + 1, :nx] = a[0, 0, j, :nx] - f[2, 0, j, :nx]
    for k in range(nz):
        a[0, k + 1, :, :nx] = a[0, k, :, :nx] + f[1, k, :, :nx]
        a[1, k + 1, :ny, :] = a[1, k, :ny, :] - f[0, k, :ny, :]
    return a
