"""Pins of the seeded input generators (closed-form edge integrals, Stokes, sizes)."""
import math

import numpy as np
import pytest

import workloads as W
from tests import discrete as D

GL16 = np.polynomial.legendre.leggauss(16)


def _gl_line(f, p0, p1, n=16):
    x, wts = np.polynomial.legendre.leggauss(n)
    p0, p1 = np.asarray(p0, float), np.asarray(p1, float)
    t = 0.5 * (x + 1.0)
    pts = p0[None, :] + t[:, None] * (p1 - p0)[None, :]
    vals = f(pts)
    return 0.5 * np.sum(wts[:, None] * vals, axis=0) @ (p1 - p0)


def _dipole_A(r0, m=1.0):
    def f(p):
        R = p - np.asarray(r0)[None, :]
        r3 = np.linalg.norm(R, axis=1) ** 3
        return W.MU0 * m / (4 * math.pi) * np.stack([-R[:, 1], R[:, 0], 0 * R[:, 0]], axis=1) / r3[:, None]
    return f


def _dipole_B(r0, m=1.0):
    def f(p):
        R = p - np.asarray(r0)[None, :]
        r = np.linalg.norm(R, axis=1)
        Rh = R / r[:, None]
        mz = np.array([0.0, 0.0, m])
        return W.MU0 / (4 * math.pi) * (3 * (Rh @ mz)[:, None] * Rh - mz[None, :]) / r[:, None] ** 3
    return f


def _segment_A(p1, p2, I=1.0):
    p1, p2 = np.asarray(p1, float), np.asarray(p2, float)
    L = np.linalg.norm(p2 - p1)
    t = (p2 - p1) / L

    def f(p):
        R1 = np.linalg.norm(p - p1[None, :], axis=1)
        R2 = np.linalg.norm(p - p2[None, :], axis=1)
        return W.MU0 * I / (4 * math.pi) * np.log((R1 + R2 + L) / (R1 + R2 - L))[:, None] * t[None, :]
    return f


def _segment_B(p1, p2, I=1.0):
    """Biot-Savart field of a finite straight segment."""
    p1, p2 = np.asarray(p1, float), np.asarray(p2, float)
    L = np.linalg.norm(p2 - p1)
    t = (p2 - p1) / L

    def f(p):
        r1 = p - p1[None, :]
        r2 = p - p2[None, :]
        cr = np.cross(t[None, :], r1)
        d2 = np.sum(cr * cr, axis=1)
        br = r1 @ t / np.linalg.norm(r1, axis=1) - r2 @ t / np.linalg.norm(r2, axis=1)
        return W.MU0 * I / (4 * math.pi) * cr * (br / d2)[:, None]
    return f


def _loop_corners(centre, size):
    cx, cy, z0 = centre
    lx, ly = size
    return [(cx - lx / 2, cy - ly / 2, z0), (cx + lx / 2, cy - ly / 2, z0),
            (cx + lx / 2, cy + ly / 2, z0), (cx - lx / 2, cy + ly / 2, z0)]


def test_dipole_edge_integrals_vs_quadrature():
    nx, ny, nz, h = 6, 5, 4, (2e-3, 1.5e-3, 2.5e-3)
    r0 = (4e-3, 3.3e-3, -10e-3)
    a = W.dipole_edge_potentials(nx, ny, nz, h, r0)
    f = _dipole_A(r0)
    rng = np.random.default_rng(0)
    for _ in range(30):
        d = int(rng.integers(0, 2))
        i, j, k = int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz + 1))
        p0 = np.array([i * h[0], j * h[1], k * h[2]])
        p1 = p0.copy()
        p1[d] += h[d]
        ref = _gl_line(f, p0, p1)
        assert abs(a[d, k, j, i] - ref) <= 1e-12 * abs(ref) + 1e-22
    assert np.all(a[2] == 0)


def test_loop_edge_integrals_vs_quadrature():
    nx, ny, nz, h = 8, 7, 5, (2e-3, 2e-3, 2e-3)
    centre, size = (9e-3, 6e-3, -6e-3), (10e-3, 8e-3)
    a = W.rect_loop_edge_potentials(nx, ny, nz, h, centre, size)
    cs = _loop_corners(centre, size)
    segs = [_segment_A(cs[q], cs[(q + 1) % 4]) for q in range(4)]
    rng = np.random.default_rng(1)
    for _ in range(30):
        d = int(rng.integers(0, 2))
        i, j, k = int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz + 1))
        p0 = np.array([i * h[0], j * h[1], k * h[2]])
        p1 = p0.copy()
        p1[d] += h[d]
        ref = sum(_gl_line(s, p0, p1, n=32) for s in segs)
        assert abs(a[d, k, j, i] - ref) <= 1e-9 * abs(ref) + 1e-20, (d, i, j, k, a[d, k, j, i], ref)


def _facet_flux(Bf, d, i, j, k, h, n=8):
    x, wts = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (x + 1.0)
    ax = [q for q in range(3) if q != d]
    base = np.array([i * h[0], j * h[1], k * h[2]])
    pts = []
    ww = []
    for s, ws in zip(t, wts):
        for r, wr in zip(t, wts):
            p = base.copy()
            p[ax[0]] += s * h[ax[0]]
            p[ax[1]] += r * h[ax[1]]
            pts.append(p)
            ww.append(ws * wr * 0.25)
    B = Bf(np.array(pts))
    return float(np.sum(np.array(ww) * B[:, d]) * h[ax[0]] * h[ax[1]])


@pytest.mark.parametrize("source", ["dipole", "loop"])
def test_stokes_circulation_equals_flux(source):
    nx, ny, nz, h = 6, 6, 5, (2e-3, 2e-3, 2e-3)
    if source == "dipole":
        r0 = (5e-3, 7e-3, -8e-3)
        a = W.dipole_edge_potentials(nx, ny, nz, h, r0)
        Bf = _dipole_B(r0)
    else:
        centre, size = (6e-3, 5e-3, -4e-3), (8e-3, 6e-3)
        a = W.rect_loop_edge_potentials(nx, ny, nz, h, centre, size)
        cs = _loop_corners(centre, size)
        segs = [_segment_B(cs[q], cs[(q + 1) % 4]) for q in range(4)]
        Bf = lambda p: sum(s(p) for s in segs)  # noqa: E731
    circ = D.curl(a)
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = int(rng.integers(0, 3))
        i, j, k = int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))
        flux = _facet_flux(Bf, d, i, j, k, h, n=12)
        assert abs(circ[d, k, j, i] - flux) <= 1e-8 * abs(flux) + 1e-16 * 4e-6, (d, i, j, k, circ[d, k, j, i], flux)


def test_homogeneous_ellipsoid_size():
    w = W.config(0)
    assert (w.nx, w.ny, w.nz) == (31, 31, 31)
    assert int((w.labels > 0).sum()) == 6989
    assert W.count_body_nodes(w.labels > 0) == 8400
    assert w.sigma_table[1] == 0.2


def test_random_ellipsoids_reproducible():
    w1 = W.random_ellipsoid_phantom(40, 32, 48, seed=5, n_ell=10, semi_range=(3.0, 8.0))
    w2 = W.random_ellipsoid_phantom(40, 32, 48, seed=5, n_ell=10, semi_range=(3.0, 8.0))
    assert np.array_equal(w1.labels, w2.labels) and np.array_equal(w1.a, w2.a)
    assert np.all((w1.sigma_table[1:] >= 0.02) & (w1.sigma_table[1:] <= 2.0))


@pytest.mark.slow
def test_body_phantom_dof_count_and_tissues():
    labels, table = W.body_phantom_labels()
    n = W.count_body_nodes(labels > 0)
    assert abs(n - 8.9e6) <= 0.005 * 8.9e6, n
    assert len(table) == 41 and table[0] == 0
    assert 0.02 <= table[1] <= 0.1 and 0.02 <= table[2] <= 0.05
    assert np.all((table[3:] >= 0.02) & (table[3:] <= 2.0))
    counts = np.bincount(labels.ravel(), minlength=41)
    assert np.all(counts[1:] > 0)          # every tissue class present


def test_uneven_sizes():
    assert W.uneven_phantom_sizes() == [64, 73, 81, 90, 98, 107, 115, 124, 132, 141, 149, 158, 166, 175, 183, 192]


def test_shifted_loop_sources_are_translations():
    offs = [(3, -2), (-4, 1)]
    gen = W.ShiftedLoopSources(offs, grid=(40, 30, 20))
    h = 2e-3
    for k, (dx, dy) in enumerate(offs):
        a = gen.source(k)
        ref = W.rect_loop_edge_potentials(40, 30, 20, (h, h, h), ((125.0 + 60.0 + dx) * h, (75.0 + dy) * h, -20.0 * h),
                                          (150 * h, 100 * h))
        assert np.abs(a - ref).max() <= 1e-11 * np.abs(ref).max()


def test_multi_source_offsets():
    offs = W.multi_source_offsets()
    assert len(offs) == 64
    assert all(isinstance(v, int) for o in offs for v in o)
    assert max(abs(o[0]) for o in offs) <= 72 and max(abs(o[1]) for o in offs) <= 37


def test_body_phantom_1mm_dof_count():
    m = W.body_mask(W.BODY_RADIAL_SCALE_1MM, (1800, 300, 500), refine=2)
    n = W.count_body_nodes(m)
    assert abs(n - 69.8e6) <= 0.005 * 69.8e6, n
