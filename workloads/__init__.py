"""Seeded synthetic inputs for the Co-Sim. SPFD Poisson solve.

This module produces *inputs only*: voxel tissue labels, a conductivity table
per label, and the source edge potentials a (line integrals of an analytic
magnetic vector potential along every grid edge).  It holds none of the
method's arithmetic (no conductance assembly, no gradient/divergence, no
solve, no post-processing), so both the CPU oracle and the HIP path can take
their inputs from here without sharing any code of the method.

Index conventions (shared interface of the oracle and the library):
  * voxel grid nx*ny*nz, voxel (i,j,k) -> i + nx*(j + ny*k), numpy shape (nz,ny,nx);
  * node grid (nx+1)*(ny+1)*(nz+1), node (i,j,k) -> i + Nx*(j + Ny*k), numpy
    shape (nz+1,ny+1,nx+1); node (i,j,k) sits at (i*hx, j*hy, k*hz) metres and
    voxel (i,j,k) spans nodes i..i+1, j..j+1, k..k+1;
  * edge potentials a[d][n] (d = 0,1,2 for x,y,z): line integral of A along the
    edge from node n to node n + e_d, in V*s (Wb); entries of edges that leave
    the grid are 0;
  * labels: 0 = air (sigma 0), tissue class t is label t+1.

The paper's voxel model ("Duke") and tissue tables are licensed and absent;
the phantoms below stand in for them with the paper's shapes and sizes: 2 mm
voxels, a ~1.8 m tall body with ~8.9 M unknowns, tens of tissues with
conductivities in the low-frequency tissue range (Sec. I, Sec. III.A).
The field frequency is 85 kHz (Sec. II.B).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MU0 = 4e-7 * math.pi            # H/m; both sides take a as given, so the exact value is immaterial
F_HZ = 85e3                     # field frequency of the charging system (Sec. II.B)
OMEGA = 2.0 * math.pi * F_HZ    # rad/s, omega = 2 pi f (Eq. (1))
SEED_BASE = 12879

# Radial scale of the body-shaped phantom, chosen once by bisection so that the
# number of body nodes is 8.9 M +- 0.5 % (the 2 mm "Duke" DOF count, Sec. I).
BODY_RADIAL_SCALE = 0.9755
# The same body on a 1 mm grid (500x300x1800 voxels), scale bisected to 69.73 M body nodes:
# the 1 mm count of the paper's model (69.8 M, Sec. III) within 0.5 %.
BODY_RADIAL_SCALE_1MM = 0.9734375


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    h: tuple                      # (hx, hy, hz) in metres
    labels: np.ndarray            # uint8 (nz, ny, nx); 0 = air
    sigma_table: np.ndarray       # float64 (n_labels,), sigma_table[0] = 0, S/m
    a: np.ndarray                 # float64 (nrhs, 3, nz+1, ny+1, nx+1) or (3, nz+1, ny+1, nx+1)
    omega: float = OMEGA
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nnodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    def sigma_voxel(self) -> np.ndarray:
        """Per-voxel conductivity (nz, ny, nx), float64."""
        return self.sigma_table[self.labels]


# --------------------------------------------------------------------------
# analytic sources: exact edge line integrals of A
# --------------------------------------------------------------------------

def _node_coords(n: int, h: float) -> np.ndarray:
    return np.arange(n + 1, dtype=np.float64) * h


def dipole_edge_potentials(nx, ny, nz, h, r0, m=1.0) -> np.ndarray:
    """Edge integrals of the vector potential of a point dipole m*z_hat at r0.

    A = mu0/(4 pi) * m x R / |R|^3 = mu0 m/(4 pi) * (-Y, X, 0)/R^3 with R = r - r0.
    Along an x-edge at fixed (Y, Z): int A_x dX = -(mu0 m/4pi) * Y * [X / ((Y^2+Z^2) R)],
    along a y-edge: int A_y dY = +(mu0 m/4pi) * X * [Y / ((X^2+Z^2) R)]; A_z = 0.
    An edge whose line passes through r0 gets 0.
    Returns (3, nz+1, ny+1, nx+1) float64.
    """
    hx, hy, hz = h
    c = MU0 * m / (4.0 * math.pi)
    X = _node_coords(nx, hx) - r0[0]
    Y = _node_coords(ny, hy) - r0[1]
    Z = _node_coords(nz, hz) - r0[2]
    a = np.zeros((3, nz + 1, ny + 1, nx + 1))
    Zk = Z[:, None, None]
    # x-edges: from X[i] to X[i+1], at (Y[j], Z[k])
    Yj = Y[None, :, None]
    rho2 = Yj * Yj + Zk * Zk                                  # (nz+1, ny+1, 1)
    Xi = X[None, None, :]
    R = np.sqrt(Xi * Xi + rho2)
    with np.errstate(divide="ignore", invalid="ignore"):
        F = Xi / (rho2 * R)
        ax = -c * Yj * (F[:, :, 1:] - F[:, :, :-1])
    ax = np.where(np.broadcast_to(rho2 > 0, ax.shape), ax, 0.0)
    a[0, :, :, :nx] = ax
    # y-edges: from Y[j] to Y[j+1], at (X[i], Z[k])
    Xi3 = X[None, None, :]
    rho2 = Xi3 * Xi3 + Zk * Zk                                # (nz+1, 1, nx+1)
    Yj3 = Y[None, :, None]
    R = np.sqrt(Yj3 * Yj3 + rho2)
    with np.errstate(divide="ignore", invalid="ignore"):
        F = Yj3 / (rho2 * R)
        ay = c * Xi3 * (F[:, 1:, :] - F[:, :-1, :])
    ay = np.where(np.broadcast_to(rho2 > 0, ay.shape), ay, 0.0)
    a[1, :, :ny, :] = ay
    return a


def _parallel_filament(u, d):
    """F(u) = u*asinh(u/d) - sqrt(u^2+d^2): double antiderivative of 1/sqrt(u^2+d^2)."""
    return u * np.arcsinh(u / d) - np.sqrt(u * u + d * d)


def rect_loop_edge_potentials(nx, ny, nz, h, centre, size, current=1.0) -> np.ndarray:
    """Edge integrals of A of a rectangular current loop in a plane z = const.

    The loop has corners centre +- size/2 (x and y), current I counter-clockwise
    seen from +z.  A straight segment from s1 to s2 along x at (ys, z0) gives
    A_x(r) = mu0 I/(4 pi) * int_{s1}^{s2} dx' / |r - r'|, so the line integral over an
    x-edge [e1, e2] at transverse distance d is mu0 I/(4 pi) times
    F(e2-s1) - F(e2-s2) - F(e1-s1) + F(e1-s2) (Neumann integral of two parallel
    filaments, closed form).  Segments along y enter a_y the same way; a_z = 0.
    Returns (3, nz+1, ny+1, nx+1) float64.
    """
    hx, hy, hz = h
    c = MU0 * current / (4.0 * math.pi)
    cx, cy, z0 = centre
    lx, ly = size
    xs = (cx - lx / 2, cx + lx / 2)
    ys = (cy - ly / 2, cy + ly / 2)
    X = _node_coords(nx, hx)
    Y = _node_coords(ny, hy)
    Z = _node_coords(nz, hz)
    a = np.zeros((3, nz + 1, ny + 1, nx + 1))
    # slabs of node planes keep the temporaries small on large grids (elementwise: same values)
    for k0 in range(0, nz + 1, 64):
        k1 = min(k0 + 64, nz + 1)
        dz = (Z[k0:k1] - z0)[:, None, None]
        # x-directed segments: at y = ys[0] current flows +x, at y = ys[1] flows -x
        for yseg, sgn in ((ys[0], 1.0), (ys[1], -1.0)):
            d = np.sqrt(dz * dz + ((Y - yseg) ** 2)[None, :, None])      # (planes, ny+1, 1)
            u = X[None, None, :]
            phi = _parallel_filament(u - xs[0], d) - _parallel_filament(u - xs[1], d)
            a[0, k0:k1, :, :nx] += sgn * c * (phi[:, :, 1:] - phi[:, :, :-1])
        # y-directed segments: at x = xs[1] current flows +y, at x = xs[0] flows -y
        for xseg, sgn in ((xs[1], 1.0), (xs[0], -1.0)):
            d = np.sqrt(dz * dz + ((X - xseg) ** 2)[None, None, :])      # (planes, 1, nx+1)
            u = Y[None, :, None]
            phi = _parallel_filament(u - ys[0], d) - _parallel_filament(u - ys[1], d)
            a[1, k0:k1, :ny, :] += sgn * c * (phi[:, 1:, :] - phi[:, :-1, :])
    return a


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------

def _voxel_centres(n):
    return np.arange(n, dtype=np.float64) + 0.5


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def homogeneous_ellipsoid(n_nodes=32, h=1e-3, semi=(12.0, 10.0, 14.0), sigma=0.2, dipole_depth=20.0):
    """Homogeneous ellipsoid in air, dipole m = 1 A m^2 along z below its centre.

    Node grid n_nodes^3 (voxels n_nodes-1 per axis), voxel size h; body =
    voxels whose centre lies inside the ellipsoid centred in the grid with the
    given semi-axes (in voxels).  The dipole sits dipole_depth voxels below the
    centre.
    """
    n = n_nodes - 1
    c = n / 2.0
    x = _voxel_centres(n)
    q = (((x - c) / semi[0]) ** 2)[None, None, :] + (((x - c) / semi[1]) ** 2)[None, :, None] \
        + (((x - c) / semi[2]) ** 2)[:, None, None]
    labels = (q <= 1.0).astype(np.uint8)
    table = np.array([0.0, sigma])
    r0 = (c * h, c * h, (c - dipole_depth) * h)
    a = dipole_edge_potentials(n, n, n, (h, h, h), r0)
    return Workload("ellipsoid32", n, n, n, (h, h, h), labels, table, a,
                    meta={"dipole": r0, "semi_axes_vox": semi})


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid_union(nx, ny, nz, rng, n_ell=60, n_classes=20, semi_range=(4.0, 24.0)):
    """Seeded "random growth" union of rotated ellipsoids (labels, sigma table).

    Draw order per ellipsoid e: (centre: parent index, 3 normals, radius fraction
    for e > 0), 3 semi-axes U[4,24] voxels, 3x3 normal matrix for the rotation,
    class U{0..n_classes-1}.  Afterwards the n_classes conductivities,
    log-uniform in [0.02, 2] S/m.  Ellipsoid 0 is centred in the box; each later
    centre lies inside the inner half of an earlier ellipsoid, so the union is
    connected.  Later ellipsoids overwrite earlier ones.
    """
    labels = np.zeros((nz, ny, nx), np.uint8)
    ells = []
    for e in range(n_ell):
        if e == 0:
            ctr = np.array([nx / 2.0, ny / 2.0, nz / 2.0])
        else:
            p = ells[int(rng.integers(0, e))]
            v = rng.normal(size=3)
            v /= max(np.linalg.norm(v), 1e-12)
            rad = 0.5 * rng.uniform() ** (1.0 / 3.0)
            ctr = p[0] + p[2] @ (v * rad * p[1])
            ctr = np.clip(ctr, 2.0, np.array([nx, ny, nz]) - 2.0)
        semi = rng.uniform(semi_range[0], semi_range[1], 3)
        rot = _random_rotation(rng)
        cls = int(rng.integers(0, n_classes))
        ells.append((ctr, semi, rot, cls))
    for ctr, semi, rot, cls in ells:
        r = float(semi.max()) + 1.0
        lo = np.maximum(np.floor(ctr - r).astype(int), 0)
        hi = np.minimum(np.ceil(ctr + r).astype(int) + 1, [nx, ny, nz])
        if np.any(hi <= lo):
            continue
        xs = np.arange(lo[0], hi[0]) + 0.5 - ctr[0]
        ys = np.arange(lo[1], hi[1]) + 0.5 - ctr[1]
        zs = np.arange(lo[2], hi[2]) + 0.5 - ctr[2]
        # body-frame coordinates: rot^T (p - ctr)
        q = np.zeros((len(zs), len(ys), len(xs)))
        for ax in range(3):
            comp = rot[0, ax] * xs[None, None, :] + rot[1, ax] * ys[None, :, None] + rot[2, ax] * zs[:, None, None]
            q += (comp / semi[ax]) ** 2
        sub = labels[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub[q <= 1.0] = cls + 1
    sig = _log_uniform(rng, 0.02, 2.0, n_classes)
    table = np.concatenate([[0.0], sig])
    return labels, table


def random_ellipsoid_phantom(nx=128, ny=96, nz=256, h=2e-3, seed=SEED_BASE + 1, n_ell=60,
                             semi_range=(4.0, 24.0), name="ellipsoids128x96x256"):
    """Heterogeneous phantom: union of seeded ellipsoids, 20 classes, 4 dipoles below.

    Dipoles: m = 1 A m^2 along z at (nx/2 +- 16, ny/2 +- 16, zmin - 10) voxels
    (zmin = lowest body voxel layer) plus U[-2,2] jitter per coordinate, drawn
    after the phantom in the order (-,-), (+,-), (-,+), (+,+).
    """
    rng = np.random.default_rng(seed)
    labels, table = ellipsoid_union(nx, ny, nz, rng, n_ell=n_ell, semi_range=semi_range)
    zmin = int(np.argmax(labels.reshape(nz, -1).max(axis=1) > 0))
    a = np.zeros((3, nz + 1, ny + 1, nx + 1))
    dipoles = []
    for sy in (-1, 1):
        for sx in (-1, 1):
            jit = rng.uniform(-2.0, 2.0, 3)
            pos = np.array([nx / 2 + 16 * sx, ny / 2 + 16 * sy, zmin - 10.0]) + jit
            r0 = tuple(pos * h)
            dipoles.append(r0)
            a += dipole_edge_potentials(nx, ny, nz, (h, h, h), r0)
    return Workload(name, nx, ny, nz, (h, h, h), labels, table, a,
                    meta={"dipoles": dipoles, "seed": seed})


# ---- body-shaped phantom -------------------------------------------------

def _body_shapes(s, refine=1):
    """Primitive shapes of the standing body (voxel units of 2 mm / refine, z up); s = radial scale."""
    shapes, bones = _body_shapes_2mm(s)
    if refine == 1:
        return shapes, bones

    def scaled(p):
        q = {}
        for k, v in p.items():
            q[k] = tuple(refine * x for x in v) if isinstance(v, tuple) else refine * v
        return q

    shapes = [(k, scaled(p)) for k, p in shapes]
    bones = [(k, scaled(p), r0, r1) for k, p, r0, r1 in bones]
    return shapes, bones


def _body_shapes_2mm(s):
    xc, yc = 125.0, 75.0
    shapes = [
        ("ellipsoid", dict(c=(xc, yc, 830.0), r=(40 * s, 50 * s, 55.0))),             # head
        ("cylinder", dict(c=(xc, yc), r=(28 * s, 28 * s), z=(760.0, 792.0))),         # neck
        ("cylinder", dict(c=(xc, yc), r=(75 * s, 55 * s), z=(430.0, 765.0))),         # torso
        ("ellipsoid", dict(c=(xc - 85 * s, yc, 740.0), r=(30 * s, 30 * s, 25.0))),    # shoulders
        ("ellipsoid", dict(c=(xc + 85 * s, yc, 740.0), r=(30 * s, 30 * s, 25.0))),
        ("capsule", dict(c=(xc - 99 * s, yc), r=22 * s, z=(450.0, 745.0))),           # arms
        ("capsule", dict(c=(xc + 99 * s, yc), r=22 * s, z=(450.0, 745.0))),
        ("capsule", dict(c=(xc - 40 * s, yc), r=35 * s, z=(5.0, 470.0))),             # legs
        ("capsule", dict(c=(xc + 40 * s, yc), r=35 * s, z=(5.0, 470.0))),
        ("ellipsoid", dict(c=(xc - 40 * s, yc - 25.0, 17.0), r=(25 * s, 45.0, 12.0))),  # feet
        ("ellipsoid", dict(c=(xc + 40 * s, yc - 25.0, 17.0), r=(25 * s, 45.0, 12.0))),
    ]
    bones = [  # (kind, params, inner, outer) shells in normalised radius
        ("ellipsoid", shapes[0][1], 0.80, 0.90),
        ("capsule", shapes[5][1], 0.25, 0.35),
        ("capsule", shapes[6][1], 0.25, 0.35),
        ("capsule", shapes[7][1], 0.25, 0.35),
        ("capsule", shapes[8][1], 0.25, 0.35),
    ]
    return shapes, bones


def _shape_radius(kind, p, x, y, z):
    """Normalised radius of a shape at voxel-centre coordinate arrays (<= 1 inside)."""
    if kind == "ellipsoid":
        return np.sqrt(((x - p["c"][0]) / p["r"][0]) ** 2 + ((y - p["c"][1]) / p["r"][1]) ** 2
                       + ((z - p["c"][2]) / p["r"][2]) ** 2)
    if kind == "cylinder":
        rr = np.sqrt(((x - p["c"][0]) / p["r"][0]) ** 2 + ((y - p["c"][1]) / p["r"][1]) ** 2)
        inside_z = (z >= p["z"][0]) & (z <= p["z"][1])
        return np.where(inside_z, rr, np.inf)
    if kind == "capsule":
        z0, z1 = p["z"][0] + p["r"], p["z"][1] - p["r"]
        zc = np.clip(z, z0, z1)
        return np.sqrt((x - p["c"][0]) ** 2 + (y - p["c"][1]) ** 2 + (z - zc) ** 2) / p["r"]
    raise ValueError(kind)


def _shape_bbox(kind, p, nx, ny, nz):
    if kind == "ellipsoid":
        lo = [p["c"][i] - p["r"][i] for i in range(3)]
        hi = [p["c"][i] + p["r"][i] for i in range(3)]
    elif kind == "cylinder":
        lo = [p["c"][0] - p["r"][0], p["c"][1] - p["r"][1], p["z"][0]]
        hi = [p["c"][0] + p["r"][0], p["c"][1] + p["r"][1], p["z"][1]]
    else:
        lo = [p["c"][0] - p["r"], p["c"][1] - p["r"], p["z"][0]]
        hi = [p["c"][0] + p["r"], p["c"][1] + p["r"], p["z"][1]]
    lo = [max(int(math.floor(v)) - 1, 0) for v in lo]
    hi = [min(int(math.ceil(v)) + 1, n) for v, n in zip(hi, (nx, ny, nz))]
    return lo, hi


def _paint(mask, kind, p, rmin, rmax):
    nz, ny, nx = mask.shape
    lo, hi = _shape_bbox(kind, p, nx, ny, nz)
    if any(h_ <= l_ for l_, h_ in zip(lo, hi)):
        return
    x = (np.arange(lo[0], hi[0]) + 0.5)[None, None, :]
    y = (np.arange(lo[1], hi[1]) + 0.5)[None, :, None]
    z = (np.arange(lo[2], hi[2]) + 0.5)[:, None, None]
    r = _shape_radius(kind, p, x, y, z)
    sel = (r <= rmax) & (r >= rmin)
    mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= sel


def body_mask(s=BODY_RADIAL_SCALE, shape=(900, 150, 250), refine=1):
    mask = np.zeros(shape, bool)
    shapes, _ = _body_shapes(s, refine)
    for kind, p in shapes:
        _paint(mask, kind, p, 0.0, 1.0)
    return mask


def count_body_nodes(mask: np.ndarray) -> int:
    """Number of grid nodes that are a corner of at least one body voxel."""
    nz, ny, nx = mask.shape
    touched = np.zeros((nz + 1, ny + 1, nx + 1), bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                touched[dz:dz + nz, dy:dy + ny, dx:dx + nx] |= mask
    return int(touched.sum())


def _skin(mask):
    inner = mask.copy()
    inner[1:, :, :] &= mask[:-1, :, :]
    inner[:-1, :, :] &= mask[1:, :, :]
    inner[:, 1:, :] &= mask[:, :-1, :]
    inner[:, :-1, :] &= mask[:, 1:, :]
    inner[:, :, 1:] &= mask[:, :, :-1]
    inner[:, :, :-1] &= mask[:, :, 1:]
    inner[0, :, :] = False
    inner[-1, :, :] = False
    inner[:, 0, :] = False
    inner[:, -1, :] = False
    inner[:, :, 0] = False
    inner[:, :, -1] = False
    return mask & ~inner


def body_phantom_labels(seed=SEED_BASE + 2, s=BODY_RADIAL_SCALE, n_sites=380, grid=(250, 150, 900), refine=1):
    """Body-shaped phantom labels and the 40-class sigma table.

    Classes: 0 skin (body voxels with an air 6-neighbour), 1 bone (2-voxel
    shells: skull at 0.8-0.9 of the head radii, cylinders at 0.25-0.35 of the
    limb radii), 2..39 Voronoi cells of n_sites seeded interior sites (class =
    site mod 38 + 2).  Draw order: site indices (without replacement among
    interior voxels in C order), then 40 conductivities in class order: skin
    log-U[0.02, 0.1], bone log-U[0.02, 0.05], others log-U[0.02, 2] S/m.
    """
    from scipy.spatial import cKDTree
    nx, ny, nz = grid
    rng = np.random.default_rng(seed)
    mask = body_mask(s, (nz, ny, nx), refine)
    skin = _skin(mask)
    bone = np.zeros_like(mask)
    _, bones = _body_shapes(s, refine)
    for kind, p, r0, r1 in bones:
        _paint(bone, kind, p, r0, r1)
    bone &= mask & ~skin
    interior = mask & ~skin & ~bone
    idx = np.flatnonzero(interior)
    sites = idx[rng.choice(idx.size, n_sites, replace=False)]
    sig = np.concatenate([_log_uniform(rng, 0.02, 0.1, 1), _log_uniform(rng, 0.02, 0.05, 1),
                          _log_uniform(rng, 0.02, 2.0, 38)])

    def coords(flat):
        k, rem = np.divmod(flat, nx * ny)
        j, i = np.divmod(rem, nx)
        return np.stack([i, j, k], axis=1).astype(np.float32)

    tree = cKDTree(coords(sites))
    _, nearest = tree.query(coords(idx), k=1, workers=-1)
    labels = np.zeros(mask.shape, np.uint8)
    flat = labels.reshape(-1)
    flat[idx] = (nearest % 38 + 2 + 1).astype(np.uint8)
    labels[bone] = 2
    labels[skin] = 1
    table = np.concatenate([[0.0], sig])
    return labels, table


def body_phantom(seed=SEED_BASE + 2, loop_offset=(0.0, 0.0), with_source=True):
    """Body-shaped 2 mm phantom, 250x150x900 voxels, ~8.9 M body nodes, 40 tissues.

    Source: rectangular loop 150x100 voxels (0.3 m x 0.2 m), I = 1 A, in the
    plane z = -20 voxels, centred at (125 + 60 + dx, 75 + dy) voxels.
    """
    nx, ny, nz = 250, 150, 900
    h = 2e-3
    labels, table = body_phantom_labels(seed)
    a = None
    if with_source:
        a = body_loop_source(loop_offset)
    return Workload("body250x150x900", nx, ny, nz, (h, h, h), labels, table, a,
                    meta={"seed": seed, "loop_offset": loop_offset})


def body_phantom_1mm(seed=SEED_BASE + 5, with_source=True):
    """The body phantom on a 1 mm grid: 500x300x1800 voxels, ~69.7 M body nodes, 40 tissues
    (shapes of the 2 mm phantom with coordinates doubled, radial scale BODY_RADIAL_SCALE_1MM, the
    same class rules and 380 Voronoi sites), and the same 0.3 m x 0.2 m loop 40 mm below the feet."""
    nx, ny, nz = 500, 300, 1800
    h = 1e-3
    labels, table = body_phantom_labels(seed, BODY_RADIAL_SCALE_1MM, 380, (nx, ny, nz), refine=2)
    a = None
    if with_source:
        a = rect_loop_edge_potentials(nx, ny, nz, (h, h, h), (370.0 * h, 150.0 * h, -40.0 * h),
                                      (300.0 * h, 200.0 * h))
    return Workload("body500x300x1800", nx, ny, nz, (h, h, h), labels, table, a, meta={"seed": seed})


def body_loop_source(offset=(0.0, 0.0), grid=(250, 150, 900), h=2e-3):
    nx, ny, nz = grid
    centre = ((125.0 + 60.0 + offset[0]) * h, (75.0 + offset[1]) * h, -20.0 * h)
    return rect_loop_edge_potentials(nx, ny, nz, (h, h, h), centre, (150 * h, 100 * h))


def multi_source_offsets(seed=SEED_BASE + 3, n=8):
    """8x8 coil offsets in whole voxels: dx in {-70,-50,...,70}, dy in {-35,-25,...,35},
    plus a jitter drawn from U{-2,...,2} per coordinate (row-major over dy, then dx)."""
    rng = np.random.default_rng(seed)
    dxs = np.linspace(-70.0, 70.0, n).round().astype(int)
    dys = np.linspace(-35.0, 35.0, n).round().astype(int)
    out = []
    for dy in dys:
        for dx in dxs:
            j = rng.integers(-2, 3, 2)
            out.append((int(dx + j[0]), int(dy + j[1])))
    return out


class ShiftedLoopSources:
    """Edge potentials of the body-phantom loop translated by whole voxels.

    The field of a coil moved by (dx, dy) voxels in its plane is the field of the
    unmoved coil translated by (dx, dy): a_dx,dy(i, j, k) = a_0(i - dx, j - dy, k).
    The unmoved field is computed once on a grid padded by the largest shift;
    each source is then a slice of it.
    """

    def __init__(self, offsets, grid=(250, 150, 900), h=2e-3):
        nx, ny, nz = grid
        self.grid = grid
        self.px = max(abs(o[0]) for o in offsets)
        self.py = max(abs(o[1]) for o in offsets)
        big = rect_loop_edge_potentials(nx + 2 * self.px, ny + 2 * self.py, nz, (h, h, h),
                                        ((125.0 + 60.0 + self.px) * h, (75.0 + self.py) * h, -20.0 * h),
                                        (150 * h, 100 * h))
        self.big = big
        self.offsets = offsets

    def source(self, idx):
        dx, dy = self.offsets[idx]
        nx, ny, nz = self.grid
        x0, y0 = self.px - dx, self.py - dy
        a = self.big[:, :, y0:y0 + ny + 1, x0:x0 + nx + 1].copy()
        a[0, :, :, nx] = 0.0     # edges that leave the grid
        a[1, :, ny, :] = 0.0
        return a


def uneven_phantom_sizes(n=16, lo=64, span=128):
    return [lo + int(round(span * i / (n - 1))) for i in range(n)]


def uneven_phantoms(n=16, seed=SEED_BASE + 4, h=2e-3):
    """n ellipsoid-union phantoms in cubes of 64^3 ... 192^3 voxels, each with 4 dipoles."""
    out = []
    for i, m in enumerate(uneven_phantom_sizes(n)):
        sc = m / 128.0
        out.append(random_ellipsoid_phantom(m, m, m, h, seed=seed + 100 * i, n_ell=max(8, int(40 * sc)),
                                            semi_range=(4.0 * max(sc, 0.75), 24.0 * max(sc, 0.75)),
                                            name=f"ellipsoids{m}"))
    return out


def tiny_random_phantom(nx, ny, nz, seed, fill=0.6, n_classes=3, h=(1e-3, 1.2e-3, 0.9e-3)):
    """Tiny random voxel phantom for brute-force tests (holes, several components)."""
    rng = np.random.default_rng(seed)
    labels = (rng.uniform(size=(nz, ny, nx)) < fill) * rng.integers(1, n_classes + 1, (nz, ny, nx))
    labels = labels.astype(np.uint8)
    table = np.concatenate([[0.0], _log_uniform(rng, 0.02, 2.0, n_classes)])
    a = rng.normal(size=(3, nz + 1, ny + 1, nx + 1)) * 1e-6
    a[0, :, :, nx] = 0.0
    a[1, :, ny, :] = 0.0
    a[2, nz, :, :] = 0.0
    return Workload(f"tiny{nx}x{ny}x{nz}", nx, ny, nz, h, labels, table, a, meta={"seed": seed})


# named configurations
def config(k: int):
    if k == 0:
        return homogeneous_ellipsoid()
    if k == 1:
        return random_ellipsoid_phantom()
    if k == 2:
        return body_phantom()
    raise ValueError(k)
