"""MI355X (gfx950) Co-Sim. SPFD solver: Python binding of ``libspfd.so``.

The binding only marshals arguments: every step of the solve runs in the HIP
kernels behind the C-ABI declared in ``include/spfd.h``.  Arrays are torch
tensors on the GPU (PyTorch supplies device memory and the stream).  If the
library has not been built, every entry point raises; there is no CPU path.

Low-level functions carry the C names (``spfd_create``, ``spfd_set_geometry``,
...); :class:`Solver` strings them together.

Shapes (numpy/torch order, x fastest): voxel arrays (nz, ny, nx), node arrays
(nz+1, ny+1, nx+1), edge arrays (3, nz+1, ny+1, nx+1).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspfd.so")

FP64, MIXED = 0, 1
CYCLE_V = 0
SMOOTH_CHEBYSHEV, SMOOTH_L1_JACOBI, SMOOTH_CHEBYSHEV4 = 0, 1, 2
CG, FGMRES = 0, 1
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "BAD_STATE", 3: "OUT_OF_MEMORY", 4: "HIP_ERROR", 5: "NOT_CONVERGED",
          6: "BREAKDOWN"}


class SPFDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class AmgOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("cycle", ctypes.c_int), ("smooth_degree", ctypes.c_int),
                ("coarsest_max", ctypes.c_int), ("cheby_ratio", ctypes.c_double), ("coarse_scale", ctypes.c_double),
                ("split_level", ctypes.c_int), ("no_split", ctypes.c_int), ("level1_degree", ctypes.c_int),
                ("smoother", ctypes.c_int), ("short_segment_bricks", ctypes.c_int), ("level1_fp32", ctypes.c_int),
                ("cg_window", ctypes.c_int)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """spfd_allocator: device memory of a handle (alloc(bytes, user) -> pointer or NULL, free(ptr, user))."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


def torch_allocator(device, stream=None):
    """An Allocator that takes the handle's device memory from PyTorch's caching allocator on `device`
    (blocks tied to `stream`, default the current stream).  spfd_create keeps it alive until
    spfd_destroy: the library calls its functions until then."""
    import torch

    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:   # out of memory: NULL, reported as SPFD_OUT_OF_MEMORY
            return None

    def _free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:   # interpreter shutdown: the process releases the memory
            pass

    return Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)


class SolveOptions(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("use_x0", ctypes.c_int),
                ("eager", ctypes.c_int), ("method", ctypes.c_int), ("restart", ctypes.c_int),
                ("flexible", ctypes.c_int)]


class RhsInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return {"iterations": self.iterations, "rel_residual": self.rel_residual, "status": STATUS[self.status]}


_lib = None
# allocator of each live handle (by address), held here so that its ctypes callbacks stay valid
_HANDLE_ALLOCATORS = {}
EXPORTS = ["spfd_create", "spfd_destroy", "spfd_last_error", "spfd_set_geometry", "spfd_set_sigma_table",
           "spfd_set_sigma_voxel", "spfd_build", "spfd_get_info", "spfd_level_info", "spfd_set_num_rhs", "spfd_set_source",
           "spfd_solve", "spfd_solve_many", "spfd_efield", "spfd_edge_potentials", "spfd_percentile",
           "spfd_percentile_noalloc", "spfd_adjoint", "spfd_timing", "spfd_timing_get", "spfd_stream_triad",
           "spfd_set_geometry_many", "spfd_set_sigma_tables"]
TIMING_COLD = 0x80000000
# kernel classes of spfd_timing / spfd_timing_get (order of the enum in spfd.h)
KERNEL_CLASSES = ["spmv", "update", "dots", "pupdate", "smooth0", "smooth0_first", "restrict0", "prolong0", "coarse",
                  "finish", "rhs", "efield", "gauge", "resid"]


def load_library(path: str = LIB_PATH):
    """Load libspfd.so (torch first, so that its HIP runtime is the one in use)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (shares one HIP runtime with the library)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2010_12879_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    H = ctypes.c_void_p
    lib.spfd_create.argtypes = [I, P, ctypes.POINTER(Allocator), ctypes.POINTER(H)]
    lib.spfd_destroy.argtypes = [H]
    lib.spfd_destroy.restype = None
    lib.spfd_last_error.argtypes = [H]
    lib.spfd_last_error.restype = ctypes.c_char_p
    lib.spfd_set_geometry.argtypes = [H, I, I, I, D, D, D, P]
    lib.spfd_set_sigma_table.argtypes = [H, P, I]
    lib.spfd_set_sigma_voxel.argtypes = [H, P]
    lib.spfd_set_geometry_many.argtypes = [H, I, ctypes.POINTER(I), D, D, D, ctypes.POINTER(P)]
    lib.spfd_set_sigma_tables.argtypes = [H, ctypes.POINTER(ctypes.POINTER(D)), ctypes.POINTER(I)]
    lib.spfd_build.argtypes = [H, ctypes.POINTER(AmgOptions)]
    lib.spfd_get_info.argtypes = [H, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(I), ctypes.POINTER(I),
                                  ctypes.POINTER(ctypes.c_size_t)]
    lib.spfd_level_info.argtypes = [H, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.spfd_set_num_rhs.argtypes = [H, I]
    lib.spfd_set_source.argtypes = [H, I, P]
    lib.spfd_solve.argtypes = [H, ctypes.POINTER(SolveOptions), P, ctypes.POINTER(RhsInfo)]
    lib.spfd_efield.argtypes = [H, D, I, P, P, P, P]
    lib.spfd_adjoint.argtypes = [H, D, P, P, P, ctypes.POINTER(SolveOptions), P, P, ctypes.POINTER(RhsInfo)]
    lib.spfd_percentile.argtypes = [H, P, D, ctypes.POINTER(D), P]
    lib.spfd_edge_potentials.argtypes = [H, P, P]
    lib.spfd_percentile_noalloc.argtypes = [I, P, P, P, I, P, ctypes.c_longlong, P, D, P]
    lib.spfd_solve_many.argtypes = [ctypes.POINTER(H), I, ctypes.POINTER(SolveOptions), ctypes.POINTER(P),
                                    ctypes.POINTER(RhsInfo)]
    lib.spfd_timing.argtypes = [H, ctypes.c_uint]
    lib.spfd_stream_triad.argtypes = [I, P, P, P, P, ctypes.c_longlong, I, ctypes.POINTER(D)]
    LL = ctypes.POINTER(ctypes.c_longlong)
    lib.spfd_timing_get.argtypes = [H, I, LL, ctypes.POINTER(D), LL, ctypes.POINTER(D), ctypes.POINTER(D)]
    for name in EXPORTS:
        if name not in ("spfd_destroy", "spfd_last_error"):
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(h, status, allow=()):
    if status != 0 and status not in allow:
        msg = load_library().spfd_last_error(h)
        raise SPFDError(status, msg.decode() if msg else "")
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_cuda(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


# ---------------------------------------------------------------- the C names
def spfd_create(device: int = 0, stream=None, allocator: Allocator | None = None):
    """A handle on `device` working on the hipStream_t `stream` (an int, None = default stream);
    allocator: its device memory (torch_allocator(...)), hipMalloc when None."""
    lib = load_library()
    h = ctypes.c_void_p()
    st = lib.spfd_create(device, ctypes.c_void_p(stream) if stream else None,
                         ctypes.byref(allocator) if allocator is not None else None, ctypes.byref(h))
    if st != 0:
        raise SPFDError(st, "spfd_create failed")
    if allocator is not None:
        _HANDLE_ALLOCATORS[h.value] = allocator   # its callbacks must outlive the handle
    return h


def spfd_destroy(h):
    load_library().spfd_destroy(h)
    _HANDLE_ALLOCATORS.pop(h.value if isinstance(h, ctypes.c_void_p) else h, None)


def spfd_last_error(h) -> str:
    m = load_library().spfd_last_error(h)
    return m.decode() if m else ""


def spfd_set_geometry(h, nx, ny, nz, hx, hy, hz, labels):
    import torch
    _require_cuda(labels, torch.uint8, (nz, ny, nx), "labels")
    return _check(h, load_library().spfd_set_geometry(h, nx, ny, nz, hx, hy, hz, _ptr(labels)))


def spfd_set_geometry_many(h, labels_list, hx, hy, hz):
    """Several voxel models (uint8 CUDA tensors (nz, ny, nx) each) packed into one handle."""
    import torch
    n = len(labels_list)
    dims = (ctypes.c_int * (3 * n))()
    ptrs = (ctypes.c_void_p * n)()
    for m, lab in enumerate(labels_list):
        _require_cuda(lab, torch.uint8, None, f"labels[{m}]")
        nz, ny, nx = lab.shape
        dims[3 * m], dims[3 * m + 1], dims[3 * m + 2] = nx, ny, nz
        ptrs[m] = lab.data_ptr()
    return _check(h, load_library().spfd_set_geometry_many(h, n, dims, hx, hy, hz, ptrs))


def spfd_set_sigma_tables(h, tables):
    """One conductivity table (sequence per label) per packed model."""
    n = len(tables)
    arrs = [(ctypes.c_double * len(t))(*[float(v) for v in t]) for t in tables]
    ptrs = (ctypes.POINTER(ctypes.c_double) * n)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_double)) for a in arrs])
    counts = (ctypes.c_int * n)(*[len(t) for t in tables])
    return _check(h, load_library().spfd_set_sigma_tables(h, ptrs, counts))


def spfd_set_sigma_table(h, sigma):
    arr = (ctypes.c_double * len(sigma))(*[float(s) for s in sigma])
    return _check(h, load_library().spfd_set_sigma_table(h, arr, len(sigma)))


def spfd_set_sigma_voxel(h, sigma_voxel):
    import torch
    _require_cuda(sigma_voxel, torch.float64, None, "sigma_voxel")
    return _check(h, load_library().spfd_set_sigma_voxel(h, _ptr(sigma_voxel)))


def spfd_build(h, opts: AmgOptions | None = None):
    return _check(h, load_library().spfd_build(h, ctypes.byref(opts) if opts is not None else None))


def spfd_get_info(h):
    nd, nc, nl, nbytes = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    _check(h, load_library().spfd_get_info(h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nl), ctypes.byref(nbytes)))
    return {"n_dofs": nd.value, "n_components": nc.value, "n_levels": nl.value, "device_bytes": nbytes.value}


def spfd_level_info(h, level):
    """kind ("structured" or "ell"), unknowns, slots, entries per row and column segment of one level."""
    k, n, sl, re, sg = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int()
    _check(h, load_library().spfd_level_info(h, level, ctypes.byref(k), ctypes.byref(n), ctypes.byref(sl),
                                             ctypes.byref(re), ctypes.byref(sg)))
    return {"kind": "ell" if k.value else "structured", "unknowns": n.value, "slots": sl.value,
            "row_entries": re.value, "segment": sg.value}


def spfd_set_num_rhs(h, nrhs):
    return _check(h, load_library().spfd_set_num_rhs(h, nrhs))


def spfd_set_source(h, rhs, a):
    import torch
    _require_cuda(a, torch.float64, None, "a")
    return _check(h, load_library().spfd_set_source(h, rhs, _ptr(a)))


def spfd_solve(h, opts: SolveOptions | None, psi, nrhs: int):
    import torch
    _require_cuda(psi, torch.float64, None, "psi")
    info = (RhsInfo * nrhs)()
    st = load_library().spfd_solve(h, ctypes.byref(opts) if opts is not None else None, _ptr(psi), info)
    _check(h, st, allow=(5, 6))
    return st, [i.as_dict() for i in info]


def spfd_solve_many(handles, opts: SolveOptions | None, psis, nrhs_total: int):
    """Solve several built handles together; psis[k] is handle k's output tensor."""
    import torch
    for t in psis:
        _require_cuda(t, torch.float64, None, "psi")
    n = len(handles)
    harr = (ctypes.c_void_p * n)(*[h.value for h in handles])
    parr = (ctypes.c_void_p * n)(*[t.data_ptr() for t in psis])
    info = (RhsInfo * nrhs_total)()
    st = load_library().spfd_solve_many(harr, n, ctypes.byref(opts) if opts is not None else None, parr, info)
    _check(handles[0], st, allow=(5, 6))
    return st, [i.as_dict() for i in info]


def solve_many(solvers, sources, tol=1e-8, max_iter=500):
    """Solve one source per Solver (each with its own stream) in lockstep; returns (psis, infos)."""
    import torch
    torch.cuda.current_stream().synchronize()   # inputs written on the current stream are complete
    psis = []
    for s, a in zip(solvers, sources):
        s.set_sources(a)
        psis.append(torch.empty((s.nrhs,) + s.node_shape, dtype=torch.float64, device=s.device))
    st, info = spfd_solve_many([s.handle for s in solvers], SolveOptions(tol, max_iter, 0), psis,
                               sum(s.nrhs for s in solvers))
    return [p[0] if p.shape[0] == 1 else p for p in psis], info


def spfd_efield(h, omega, a, psi, u_edges, emag, nsrc=1):
    """|E| (and u) of nsrc sources: a [nsrc][3][nnodes], psi [nsrc][nnodes], emag [nsrc][nvox]."""
    import torch
    for t, n in ((a, "a"), (psi, "psi"), (emag, "emag")):
        _require_cuda(t, torch.float64, None, n)
    if u_edges is not None:
        _require_cuda(u_edges, torch.float64, None, "u_edges")
    return _check(h, load_library().spfd_efield(h, float(omega), int(nsrc), _ptr(a), _ptr(psi), _ptr(u_edges),
                                                _ptr(emag)))


def spfd_adjoint(h, omega, a, psi, grad_emag, opts: SolveOptions | None, grad_sigma_voxel, n_table: int = 0):
    """Adjoint gradient: fills grad_sigma_voxel; returns (status, per-label sums or None, info)."""
    import torch
    for t, n in ((a, "a"), (psi, "psi"), (grad_emag, "grad_emag"), (grad_sigma_voxel, "grad_sigma_voxel")):
        _require_cuda(t, torch.float64, None, n)
    table = (ctypes.c_double * n_table)() if n_table else None
    info = RhsInfo()
    st = load_library().spfd_adjoint(h, float(omega), _ptr(a), _ptr(psi), _ptr(grad_emag),
                                     ctypes.byref(opts) if opts is not None else None, _ptr(grad_sigma_voxel),
                                     table, ctypes.byref(info))
    _check(h, st, allow=(5, 6))
    return st, (list(table) if table is not None else None), info.as_dict()


def spfd_edge_potentials(h, flux, a):
    """a = edge potentials with C a = flux in the tree-cotree gauge (both (3, Nz, Ny, Nx) float64 CUDA)."""
    import torch
    _require_cuda(flux, torch.float64, None, "flux")
    _require_cuda(a, torch.float64, None, "a")
    return _check(h, load_library().spfd_edge_potentials(h, _ptr(flux), _ptr(a)))


def spfd_percentile(h, emag, q=0.99, n_labels=0):
    """(whole-body quantile, per-label list or None) of the voxel |E| (nearest rank)."""
    import torch
    _require_cuda(emag, torch.float64, None, "emag")
    body = ctypes.c_double()
    labs = (ctypes.c_double * n_labels)() if n_labels else None
    _check(h, load_library().spfd_percentile(h, _ptr(emag), float(q), ctypes.byref(body), labs))
    return body.value, (list(labs) if labs is not None else None)


def spfd_percentile_noalloc(labels, sigma_table, sigma_voxel, emag, q, out, device=0, stream=None):
    """Allocation-free quantile: writes out[0] (whole body) and out[1 + l] (label l) on the device;
    sigma_table (n_labels,) and/or sigma_voxel, labels, emag and out are CUDA tensors.  Enqueued on
    `stream` (a hipStream_t int, None = default stream), not waited for."""
    import torch
    _require_cuda(labels, torch.uint8, None, "labels")
    _require_cuda(emag, torch.float64, None, "emag")
    _require_cuda(out, torch.float64, None, "out")
    n_labels = sigma_table.numel() if sigma_table is not None else out.numel() - 1
    if sigma_table is not None:
        _require_cuda(sigma_table, torch.float64, None, "sigma_table")
    if sigma_voxel is not None:
        _require_cuda(sigma_voxel, torch.float64, None, "sigma_voxel")
    if out.numel() < 1 + n_labels or labels.numel() != emag.numel():
        raise ValueError("out needs 1 + n_labels entries and labels one per voxel of emag")
    st = load_library().spfd_percentile_noalloc(int(device), ctypes.c_void_p(stream) if stream else None,
                                                _ptr(labels), _ptr(sigma_table), int(n_labels), _ptr(sigma_voxel),
                                                int(emag.numel()), _ptr(emag), float(q), _ptr(out))
    if st != 0:
        raise SPFDError(st, "spfd_percentile_noalloc failed")
    return st


def spfd_stream_triad(a, b, c, reps=5, device=0, stream=None):
    """Best STREAM-triad bandwidth (GB/s) a = b + 1.5 c over three float64 CUDA tensors of equal size."""
    import torch
    for t, n in ((a, "a"), (b, "b"), (c, "c")):
        _require_cuda(t, torch.float64, None, n)
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("a, b and c must have the same size")
    best = ctypes.c_double()
    st = load_library().spfd_stream_triad(int(device), ctypes.c_void_p(stream) if stream else None, _ptr(a), _ptr(b),
                                          _ptr(c), int(a.numel()), int(reps), ctypes.byref(best))
    if st != 0:
        raise SPFDError(st, "spfd_stream_triad failed")
    return best.value


def spfd_timing(h, class_mask: int):
    return _check(h, load_library().spfd_timing(h, class_mask))


def spfd_timing_get(h, kclass: int):
    """Counters of a kernel class: dict with launches, bytes (algorithmic, all launches),
    timed_launches, timed_ms and timed_bytes (the event-timed sample)."""
    n, by, tn, tms, tby = (ctypes.c_longlong(), ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double(),
                           ctypes.c_double())
    _check(h, load_library().spfd_timing_get(h, kclass, ctypes.byref(n), ctypes.byref(by), ctypes.byref(tn),
                                             ctypes.byref(tms), ctypes.byref(tby)))
    return {"launches": n.value, "bytes": by.value, "timed_launches": tn.value, "timed_ms": tms.value,
            "timed_bytes": tby.value}


# ---------------------------------------------------------------- convenience
class Solver:
    """Eq. (3) solver on one voxel model; the hierarchy is reused for every source.

    labels: uint8 CUDA tensor (nz, ny, nx); sigma: sequence per label (label 0 = air
    normally) or a float64 CUDA tensor per voxel; h: voxel edge lengths (m).
    """

    def __init__(self, labels, sigma, h, precision="fp64", device=None, smooth_degree=2, coarsest_max=1024,
                 cheby_ratio=8.0, coarse_scale=1.9, split_level=2, split=True, stream=None, level1_degree=4,
                 smoother="chebyshev", short_segment_bricks=0, level1_fp32=False, torch_memory=True, cg_window=0):
        """torch_memory: the handle's device memory comes from PyTorch's caching allocator
        (torch.cuda.memory_allocated() accounts for it); False: hipMalloc inside the library.
        cg_window: CG search directions kept before x is updated (0: the library's choice)."""
        import torch
        self.device = labels.device if device is None else torch.device(device)
        self.nz, self.ny, self.nx = labels.shape
        self.h = tuple(float(v) for v in h)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        stream = self.stream.cuda_stream
        self._allocator = torch_allocator(self.device, self.stream) if torch_memory else None
        self.version = 0    # bumped by every set_sigma (the hierarchy an adjoint needs)
        self.handle = spfd_create(self.device.index or 0, stream, self._allocator)
        try:
            spfd_set_geometry(self.handle, self.nx, self.ny, self.nz, *self.h, labels)
            if isinstance(sigma, torch.Tensor):
                spfd_set_sigma_voxel(self.handle, sigma)
            else:
                spfd_set_sigma_table(self.handle, list(sigma))
            self.opts = AmgOptions(MIXED if precision == "mixed" else FP64, CYCLE_V,
                                   smooth_degree, coarsest_max, cheby_ratio, coarse_scale, split_level,
                                   0 if split else 1, level1_degree,
                                   {"chebyshev": SMOOTH_CHEBYSHEV, "l1jacobi": SMOOTH_L1_JACOBI, "chebyshev4": SMOOTH_CHEBYSHEV4}[smoother],
                                   short_segment_bricks, 1 if level1_fp32 else 0, cg_window)
            spfd_build(self.handle, self.opts)
        except Exception:
            spfd_destroy(self.handle)
            self.handle = None
            raise
        self.nrhs = 1
        self.n_table = 0 if isinstance(sigma, torch.Tensor) else len(sigma)

    def set_sigma(self, sigma):
        """New conductivities (table sequence / 1-D tensor, or per-voxel CUDA tensor) and a rebuilt hierarchy."""
        import torch
        if isinstance(sigma, torch.Tensor) and sigma.dim() == 3:
            spfd_set_sigma_voxel(self.handle, sigma.detach().to(torch.float64).contiguous())
            self.n_table = 0
        else:
            vals = sigma.detach().cpu().tolist() if isinstance(sigma, torch.Tensor) else list(sigma)
            spfd_set_sigma_table(self.handle, vals)
            self.n_table = len(vals)
        self.version += 1
        spfd_build(self.handle, self.opts)
        self.nrhs = 1

    def adjoint(self, a, psi, omega, grad_emag, tol=1e-8, max_iter=500):
        """(dJ/dsigma per voxel (nz,ny,nx), per-label list or None, info) for dJ/d|E| = grad_emag."""
        import torch
        gvox = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        n_table = self.n_table if self.n_table else 256
        st, gtab, info = spfd_adjoint(self.handle, omega, a.contiguous(), psi.contiguous(),
                                      grad_emag.to(torch.float64).contiguous(), SolveOptions(tol, max_iter, 0), gvox,
                                      n_table)
        return gvox, gtab, info

    @property
    def node_shape(self):
        return (self.nz + 1, self.ny + 1, self.nx + 1)

    def info(self):
        return spfd_get_info(self.handle)

    def set_sources(self, a):
        """a: (3, Nz, Ny, Nx) or (nrhs, 3, Nz, Ny, Nx) float64 CUDA tensor."""
        a = a if a.dim() == 5 else a.unsqueeze(0)
        if tuple(a.shape[1:]) != (3,) + self.node_shape:
            raise ValueError(f"a must have shape (nrhs, 3) + {self.node_shape}")
        if a.shape[0] != self.nrhs:
            spfd_set_num_rhs(self.handle, a.shape[0])
            self.nrhs = a.shape[0]
        for r in range(a.shape[0]):
            spfd_set_source(self.handle, r, a[r].contiguous())

    def solve(self, a=None, tol=1e-8, max_iter=500, x0=None, check=True, eager=False, method="cg", restart=30,
              flexible=False):
        """Psi (nrhs or none, Nz, Ny, Nx) and the per-source info dicts (eager: no graph replay;
        method "cg" or "fgmres" with `restart` basis vectors per cycle; flexible: the CG's
        Polak-Ribiere beta instead of the standard one)."""
        import torch
        squeeze = a is not None and a.dim() == 4
        if a is not None:
            self.set_sources(a)
        if x0 is not None:
            psi = x0.reshape((self.nrhs,) + self.node_shape).clone().contiguous()
        else:
            psi = torch.empty((self.nrhs,) + self.node_shape, dtype=torch.float64, device=self.device)
        opts = SolveOptions(tol, max_iter, 1 if x0 is not None else 0, 1 if eager else 0,
                            FGMRES if method == "fgmres" else CG, restart, 1 if flexible else 0)
        st, info = spfd_solve(self.handle, opts, psi, self.nrhs)
        if check and st != 0:
            raise SPFDError(st, spfd_last_error(self.handle))
        return (psi[0] if squeeze else psi), (info[0] if squeeze else info)

    def efield(self, a, psi, omega, want_u=False):
        """|E| per voxel (nz, ny, nx) [and u edges (3, Nz, Ny, Nx)] for one source; for n sources
        (a (n, 3, Nz, Ny, Nx), psi (n, Nz, Ny, Nx)) the same with a leading dimension n."""
        import torch
        many = a.dim() == 5
        n = a.shape[0] if many else 1
        nn = (self.nz + 1) * (self.ny + 1) * (self.nx + 1)
        if tuple(a.shape[-4:]) != (3,) + self.node_shape or psi.numel() != n * nn:
            raise ValueError(f"a must be ([n,] 3) + {self.node_shape} and psi hold n * {nn} node values")
        lead = (n,) if many else ()
        emag = torch.empty(lead + (self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        u = torch.empty(lead + (3,) + self.node_shape, dtype=torch.float64, device=self.device) if want_u else None
        spfd_efield(self.handle, omega, a.contiguous(), psi.contiguous(), u, emag, n)
        return (emag, u) if want_u else emag

    def edge_potentials(self, flux):
        """Edge potentials (3, Nz, Ny, Nx) from facet fluxes of the same shape (tree-cotree gauge)."""
        import torch
        if tuple(flux.shape) != (3,) + self.node_shape:
            raise ValueError(f"flux must have shape (3,) + {self.node_shape}")
        a = torch.empty_like(flux, dtype=torch.float64)
        spfd_edge_potentials(self.handle, flux.to(torch.float64).contiguous(), a)
        return a

    def percentile(self, emag, q=0.99):
        """(whole body, per-label list) nearest-rank q-quantile of |E| over conducting voxels."""
        if emag.numel() != self.nx * self.ny * self.nz:
            raise ValueError(f"emag must hold {self.nx * self.ny * self.nz} voxel values")
        return spfd_percentile(self.handle, emag.contiguous(), q, self.n_table if self.n_table else 256)

    def close(self):
        if getattr(self, "handle", None) is not None:
            spfd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiSolver:
    """Eq. (3) on several voxel models of uneven size in one handle (packed along z, one hierarchy,
    every level kernel launched once for all models, one CG per model).

    labels_list: uint8 CUDA tensors (nz, ny, nx), one per model; tables: one conductivity sequence
    per model; h: voxel edge lengths shared by all models (m).
    """

    def __init__(self, labels_list, tables, h, precision="fp64", device=None, stream=None, torch_memory=True,
                 **amg):
        import torch
        self.device = labels_list[0].device if device is None else torch.device(device)
        self.shapes = [tuple(l.shape) for l in labels_list]
        self.node_shapes = [(nz + 1, ny + 1, nx + 1) for nz, ny, nx in self.shapes]
        self.h = tuple(float(v) for v in h)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._allocator = torch_allocator(self.device, self.stream) if torch_memory else None
        self.handle = spfd_create(self.device.index or 0, self.stream.cuda_stream, self._allocator)
        try:
            spfd_set_geometry_many(self.handle, labels_list, *self.h)
            spfd_set_sigma_tables(self.handle, [list(t) for t in tables])
            opts = AmgOptions(MIXED if precision == "mixed" else FP64, CYCLE_V, amg.get("smooth_degree", 2),
                              amg.get("coarsest_max", 1024), amg.get("cheby_ratio", 8.0), amg.get("coarse_scale", 1.9),
                              amg.get("split_level", 2), 0, amg.get("level1_degree", 4), SMOOTH_CHEBYSHEV,
                              amg.get("short_segment_bricks", 0), 1 if amg.get("level1_fp32") else 0,
                              amg.get("cg_window", 0))
            spfd_build(self.handle, opts)
        except Exception:
            spfd_destroy(self.handle)
            self.handle = None
            raise

    @property
    def n_models(self):
        return len(self.shapes)

    def info(self):
        return spfd_get_info(self.handle)

    def set_sources(self, sources):
        """sources: one float64 CUDA tensor (3, Nz, Ny, Nx) per model."""
        import torch
        if len(sources) != self.n_models:
            raise ValueError("one source per model")
        for m, a in enumerate(sources):
            if tuple(a.shape) != (3,) + self.node_shapes[m]:
                raise ValueError(f"source {m} must have shape {(3,) + self.node_shapes[m]}")
            spfd_set_source(self.handle, m, a.to(torch.float64).contiguous())

    def solve(self, sources=None, tol=1e-8, max_iter=500, check=True, flexible=False, eager=False):
        """(list of psi (Nz, Ny, Nx) per model, list of info dicts)."""
        import torch
        if sources is not None:
            self.set_sources(sources)
        sizes = [nz * ny * nx for nz, ny, nx in self.node_shapes]
        flat = torch.empty(sum(sizes), dtype=torch.float64, device=self.device)
        opts = SolveOptions(tol, max_iter, 0, 1 if eager else 0, CG, 30, 1 if flexible else 0)
        st, info = spfd_solve(self.handle, opts, flat, self.n_models)
        if check and st != 0:
            raise SPFDError(st, spfd_last_error(self.handle))
        out, off = [], 0
        for n, shp in zip(sizes, self.node_shapes):
            out.append(flat[off:off + n].view(shp))
            off += n
        return out, info

    def close(self):
        if getattr(self, "handle", None) is not None:
            spfd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class SPFDField(torch.autograd.Function):
        """|E| per voxel as a differentiable function of the conductivities.

        forward(sigma, solver, a, omega, tol): sigma is a 1-D float64 tensor (one value
        per label) or a (nz, ny, nx) float64 CUDA tensor (per voxel).  The solver's
        hierarchy is rebuilt for sigma, Eq. (3) is solved and |E| returned.
        backward: one adjoint solve (spfd_adjoint) gives dJ/dsigma.
        """

        @staticmethod
        def forward(ctx, sigma, solver, a, omega, tol=1e-10):
            solver.set_sigma(sigma)
            psi, info = solver.solve(a, tol=tol)
            emag = solver.efield(a, psi, omega)
            ctx.solver, ctx.omega, ctx.tol = solver, omega, tol
            ctx.per_voxel = sigma.dim() == 3
            ctx.n = sigma.numel()
            ctx.sigma_device, ctx.sigma_dtype = sigma.device, sigma.dtype
            # the conductivities this forward ran with, and the solver state they gave
            ctx.sigma_used = sigma.detach().clone()
            ctx.version = solver.version
            ctx.save_for_backward(a, psi)
            return emag

        @staticmethod
        def backward(ctx, grad_emag):
            a, psi = ctx.saved_tensors
            if ctx.solver.version != ctx.version:
                # another forward changed the solver's conductivities since: the adjoint solve and
                # dM/dsigma need this forward's, so its hierarchy is rebuilt first
                ctx.solver.set_sigma(ctx.sigma_used)
            gvox, gtab, info = ctx.solver.adjoint(a, psi, ctx.omega, grad_emag.contiguous(), tol=ctx.tol)
            if ctx.per_voxel:
                g = gvox.to(ctx.sigma_dtype)
            else:
                g = torch.tensor(gtab[:ctx.n], dtype=ctx.sigma_dtype, device=ctx.sigma_device)
            return g, None, None, None, None

    return SPFDField


def __getattr__(name):
    if name == "SPFDField":
        fn = _autograd_function()
        globals()["SPFDField"] = fn
        return fn
    raise AttributeError(name)
