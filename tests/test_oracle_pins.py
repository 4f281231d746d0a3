"""Pins of the CPU oracle against hand computation, closed forms, brute force and invariants.

Each test fixes the oracle to something other than itself:
  * single- and two-voxel systems written out by hand (assembly of M_kappa and Eq. (3));
  * a voxel-by-voxel "element" assembly (scatter of each voxel's 12 edges),
    a different route to G^T M G than the oracle's edge gather;
  * dense pseudo-inverse solves on tiny grids with holes and several components;
  * manufactured discrete solutions (exact Psi and exact u, since C G = 0);
  * the continuum solution of a homogeneous ellipsoid in a uniform B field (signs, scale, O(h));
  * invariants: conductivity scaling, source linearity, mirror symmetry, Thomson's principle,
    current continuity G^T M u = 0 (Eq. (1) with Eq. (3));
  * adjoint gradient against central finite differences and the Euler identity.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import discrete as D


def _cube_laplacian(wx, wy, wz):
    """Hand-built 8x8 matrix of one voxel: node (i,j,k) in {0,1}^3 -> i + 2j + 4k; nodes that
    differ in exactly one coordinate are joined by an edge of weight wx/wy/wz."""
    A = np.zeros((8, 8))
    for p in range(8):
        for q in range(8):
            diff = p ^ q
            if diff in (1, 2, 4):
                w = {1: wx, 2: wy, 4: wz}[diff]
                A[p, q] = -w
                A[p, p] += w
    return A


def test_single_voxel_system_by_hand():
    # sigma = 1, h = (1, 2, 4): x-edge conductance = 1/4 * hy*hz/hx = 2, y: 1/4*4/2 = 0.5, z: 1/4*2/4 = 0.125
    sig = np.ones((1, 1, 1))
    A, b, node_of, comp = oracle.dense_system(sig, (1.0, 2.0, 4.0), np.zeros((3, 2, 2, 2)))
    assert A.shape == (8, 8)
    assert list(node_of) == list(range(8))
    np.testing.assert_allclose(A, _cube_laplacian(2.0, 0.5, 0.125), rtol=0, atol=1e-15)
    M = oracle.edge_conductance(sig, (1.0, 2.0, 4.0))
    assert M[0, 0, 0, 0] == 2.0 and M[1, 0, 0, 0] == 0.5 and M[2, 0, 0, 0] == 0.125
    assert M[0, 0, 0, 1] == 0.0            # x-edge leaving the grid
    assert np.count_nonzero(M) == 12


def test_single_voxel_rhs_by_hand():
    # a = 1 on the x-edge from node 0 to node 1 only; M = 0.5 (sigma 2, h 1):
    # b = -G^T M a: node 0 (tail) gets +0.5, node 1 (head) gets -0.5
    sig = np.full((1, 1, 1), 2.0)
    a = np.zeros((3, 2, 2, 2))
    a[0, 0, 0, 0] = 1.0
    A, b, node_of, _ = oracle.dense_system(sig, (1.0, 1.0, 1.0), a)
    np.testing.assert_allclose(b, [0.5, -0.5, 0, 0, 0, 0, 0, 0], atol=1e-16)
    np.testing.assert_allclose(A, _cube_laplacian(0.5, 0.5, 0.5), atol=1e-16)


def test_two_voxels_shared_face_by_hand():
    # voxels 0 (sigma 1) and 1 (sigma 3) along x, h = 1: the 4 edges in the shared face
    # (y- and z-edges at i = 1) carry (1+3)/4 = 1; edges of voxel 0 only: 1/4; of voxel 1 only: 3/4
    sig = np.array([[[1.0, 3.0]]])
    M = oracle.edge_conductance(sig, (1.0, 1.0, 1.0))
    # y-edges at i = 1: nodes (1, 0, k), k = 0, 1; z-edges at i = 1: nodes (1, j, 0), j = 0, 1
    assert M[1, 0, 0, 1] == 1.0 and M[1, 1, 0, 1] == 1.0
    assert M[2, 0, 0, 1] == 1.0 and M[2, 0, 1, 1] == 1.0
    assert M[1, 0, 0, 0] == 0.25 and M[1, 0, 0, 2] == 0.75
    assert M[0, 0, 0, 0] == 0.25 and M[0, 0, 0, 1] == 0.75
    assert M[0, 1, 1, 1] == 0.75
    assert np.count_nonzero(M) == 20        # 12 + 12 - 4 shared


def _element_assembly(sig, h):
    """A = sum over voxels of sigma_v * (area/4/length) * (cube Laplacian of its 12 edges),
    mapped to global nodes by scatter; the independent route to G^T M G."""
    nz, ny, nx = sig.shape
    Nx, Ny, Nz = nx + 1, ny + 1, nz + 1
    nn = Nx * Ny * Nz
    A = np.zeros((nn, nn))
    geo = (h[1] * h[2] / h[0], h[0] * h[2] / h[1], h[0] * h[1] / h[2])
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                s = sig[k, j, i]
                if s == 0:
                    continue
                loc = _cube_laplacian(s * geo[0] / 4, s * geo[1] / 4, s * geo[2] / 4)
                nodes = [(i + (c & 1)) + Nx * ((j + ((c >> 1) & 1)) + Ny * (k + ((c >> 2) & 1))) for c in range(8)]
                for p in range(8):
                    for q in range(8):
                        A[nodes[p], nodes[q]] += loc[p, q]
    return A


@pytest.mark.parametrize("seed,shape", [(1, (3, 4, 2)), (2, (4, 3, 5)), (3, (5, 5, 4)), (4, (1, 6, 3))])
def test_element_assembly_matches(seed, shape):
    w = W.tiny_random_phantom(*shape, seed=seed)
    sig = w.sigma_voxel()
    A, b, node_of, _ = oracle.dense_system(sig, w.h, w.a)
    Afull = _element_assembly(sig, w.h)
    np.testing.assert_allclose(A, Afull[np.ix_(node_of, node_of)], rtol=1e-14, atol=1e-18)
    # the nodes that are not DOFs have empty rows in the element assembly
    others = np.setdiff1d(np.arange(Afull.shape[0]), node_of)
    assert np.all(Afull[others] == 0)
    # b = -G^T M a with M from the element view: M_e = -A_{tail,head}
    M = np.zeros_like(w.a)
    Nz, Ny, Nx = w.nz + 1, w.ny + 1, w.nx + 1
    step = (1, Nx, Nx * Ny)
    flatM = M.reshape(3, -1)
    for d in range(3):
        for n in range(Nx * Ny * Nz):
            m = n + step[d]
            i, j, k = n % Nx, (n // Nx) % Ny, n // (Nx * Ny)
            if (d == 0 and i == Nx - 1) or (d == 1 and j == Ny - 1) or (d == 2 and k == Nz - 1):
                continue
            flatM[d, n] = -Afull[n, m]
    bfull = -D.div_T(M * w.a).reshape(-1)
    np.testing.assert_allclose(b, bfull[node_of], rtol=1e-12, atol=1e-22)


@pytest.mark.parametrize("seed,shape,fill", [(5, (4, 4, 4), 0.5), (6, (6, 5, 4), 0.35), (7, (3, 6, 6), 0.7),
                                              (8, (6, 6, 6), 0.3)])
def test_solve_matches_dense_pinv(seed, shape, fill):
    w = W.tiny_random_phantom(*shape, seed=seed, fill=fill)
    sig = w.sigma_voxel()
    A, b, node_of, comp = oracle.dense_system(sig, w.h, w.a)
    x_ref = np.linalg.pinv(A) @ b           # minimum norm = mean-zero on every component
    psi, info = oracle.solve(sig, w.h, w.a, tol=1e-14, max_iter=100000)
    x = psi.reshape(-1)[node_of]
    assert info["ncomp"] == len(np.unique(comp))
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-10 * np.abs(x_ref).max())
    for c in np.unique(comp):
        assert abs(x[comp == c].sum()) <= 1e-12 * np.abs(x).sum()
    assert np.all(psi.reshape(-1)[np.setdiff1d(np.arange(psi.size), node_of)] == 0)


def test_several_components_counted():
    # sig is indexed (k, j, i); voxel (i,j,k) owns the nodes i..i+1, j..j+1, k..k+1
    sig = np.zeros((5, 5, 7))
    sig[1:3, 1:3, 0:2] = 1.0     # block A: nodes i 0..2, j 1..3, k 1..3
    sig[1:3, 1:3, 4:6] = 0.5     # block B: nodes i 4..6: no node shared with A
    sig[4, 4, 6] = 2.0           # single voxel: nodes i 6..7, j 4..5, k 4..5
    comp, nc = oracle.components(sig, (1e-3,) * 3)
    assert nc == 3
    sig[3, 3, 3] = 1.0           # nodes i 3..4, j 3..4, k 3..4: shares node (4,3,3) with B
    sig[3, 3, 1] = 1.0           # nodes i 1..2: shares (1..2,3,3) with A, nothing with (3,3,3)
    comp, nc = oracle.components(sig, (1e-3,) * 3)
    assert nc == 3
    sig[3, 3, 2] = 1.0           # nodes i 2..3: joins the voxels at i = 1 and i = 3, hence A and B
    comp, nc = oracle.components(sig, (1e-3,) * 3)
    assert nc == 2
    assert comp[3, 3, 4] == comp[2, 2, 1] != comp[5, 5, 7]


@pytest.mark.parametrize("cfg", ["ellipsoid", "hetero"])
def test_manufactured_solution(cfg):
    rng = np.random.default_rng(11)
    if cfg == "ellipsoid":
        w = W.homogeneous_ellipsoid(n_nodes=20, semi=(7.0, 6.0, 8.0))
    else:
        w = W.random_ellipsoid_phantom(24, 20, 28, seed=99, n_ell=6, semi_range=(3.0, 8.0))
    sig = w.sigma_voxel()
    body = sig > 0
    M = oracle.edge_conductance(sig, w.h)
    a, psi_star, u_exact = D.manufactured(M, body, rng)
    assert np.all(D.curl_T(np.zeros_like(a)) == 0)
    psi, info = oracle.solve(sig, w.h, a, tol=1e-13)
    comp, _ = oracle.components(sig, w.h)
    expect = D.project_mean_zero(psi_star, comp)
    err = np.abs(psi - expect).max() / np.abs(expect).max()
    assert err < 1e-9, err
    u, E = oracle.efield(sig, w.h, a, psi, w.omega)
    np.testing.assert_allclose(u, u_exact, rtol=0, atol=1e-8 * np.abs(u_exact).max())
    E_ref = D.voxel_emag_bruteforce(u_exact, body, w.h, w.omega)
    np.testing.assert_allclose(E, E_ref, rtol=1e-8, atol=1e-12 * E_ref.max())
    assert np.all(E[~body] == 0)


def test_gradient_source_gives_zero_field():
    # a = -G psi*: the whole source is a gauge, so u = 0 and psi = psi* (mean-zero)
    w = W.homogeneous_ellipsoid(n_nodes=16, semi=(6.0, 5.0, 7.0))
    sig = w.sigma_voxel()
    rng = np.random.default_rng(3)
    psi_star = rng.standard_normal((16, 16, 16)) * 1e-6
    a = -D.grad(psi_star)
    psi, info = oracle.solve(sig, w.h, a, tol=1e-14)
    comp, _ = oracle.components(sig, w.h)
    np.testing.assert_allclose(psi, D.project_mean_zero(psi_star, comp), atol=1e-9 * 1e-6)
    u, E = oracle.efield(sig, w.h, a, psi, w.omega)
    assert np.abs(u).max() < 1e-9 * np.abs(a).max()


def _ellipsoid_uniform_B(n_vox, semi_m=(0.012, 0.010, 0.014), B=1e-3):
    """Homogeneous ellipsoid in uniform B_z, symmetric gauge A = B/2 (-y, x, 0) about its centre."""
    L = 2 * max(semi_m) * 1.1
    h = L / n_vox
    c = n_vox / 2.0
    xc = (np.arange(n_vox) + 0.5 - c) * h
    q = (xc[None, None, :] / semi_m[0]) ** 2 + (xc[None, :, None] / semi_m[1]) ** 2 + (xc[:, None, None] / semi_m[2]) ** 2
    sig = np.where(q <= 1.0, 0.3, 0.0)
    xn = (np.arange(n_vox + 1) - c) * h
    a = np.zeros((3, n_vox + 1, n_vox + 1, n_vox + 1))
    # A_x = -B y/2 is constant along an x-edge, A_y = B x/2 along a y-edge
    a[0, :, :, :-1] = (-B / 2 * xn[None, :, None] * h) * np.ones((n_vox + 1, 1, n_vox))
    a[1, :, :-1, :] = (B / 2 * xn[None, None, :] * h) * np.ones((n_vox + 1, n_vox, 1))
    return sig, (h, h, h), a, xn, xc


def test_ellipsoid_uniform_field_continuum():
    ax_, by_ = 0.012, 0.010
    B = 1e-3
    kappa = B / 2 * (by_ ** 2 - ax_ ** 2) / (ax_ ** 2 + by_ ** 2)
    errs = []
    for n in (16, 32, 48):
        sig, h, a, xn, xc = _ellipsoid_uniform_B(n, B=B)
        psi, info = oracle.solve(sig, h, a, tol=1e-12)
        comp, _ = oracle.components(sig, h)
        ref = kappa * xn[None, None, :] * xn[None, :, None] * np.ones((n + 1, 1, 1))
        ref = D.project_mean_zero(ref, comp)
        dof = comp >= 0
        errs.append(np.sqrt(((psi - ref)[dof] ** 2).sum() / (ref[dof] ** 2).sum()))
        u, E = oracle.efield(sig, h, a, psi, 1.0)
        # field deep inside (normalised radius < 0.6) vs E = omega B/(a^2+b^2) (-a^2 y, b^2 x, 0)
        q = np.sqrt((xc[None, None, :] / ax_) ** 2 + (xc[None, :, None] / by_) ** 2 + (xc[:, None, None] / 0.014) ** 2)
        inner = q < 0.6
        Eref = B / (ax_ ** 2 + by_ ** 2) * np.sqrt((ax_ ** 2 * xc[None, :, None]) ** 2 + (by_ ** 2 * xc[None, None, :]) ** 2) \
            * np.ones((n, 1, 1))
        rel = np.sqrt(((E - Eref)[inner] ** 2).sum() / (Eref[inner] ** 2).sum())
        assert rel < 0.12, (n, rel)
    # first-order (staircase) convergence: the error falls at least like h
    assert errs[1] < errs[0] * 0.6 and errs[2] < errs[1] * 0.8 and errs[2] < 0.12, errs
    # sign and scale: psi follows kappa*x*y with kappa < 0 (b < a)
    assert kappa < 0
    c = float(np.sum(psi[dof] * ref[dof]) / np.sum(ref[dof] ** 2))
    assert 0.9 < c < 1.1, c


def test_conductivity_scaling_and_source_linearity():
    w = W.random_ellipsoid_phantom(20, 16, 24, seed=7, n_ell=5, semi_range=(3.0, 7.0))
    sig = w.sigma_voxel()
    psi, _ = oracle.solve(sig, w.h, w.a, tol=1e-13)
    psi2, _ = oracle.solve(sig * 37.0, w.h, w.a, tol=1e-13)
    psi3, _ = oracle.solve(sig, w.h, -2.5 * w.a, tol=1e-13)
    s = np.abs(psi).max()
    assert np.abs(psi2 - psi).max() < 1e-9 * s
    assert np.abs(psi3 + 2.5 * psi).max() < 1e-9 * s


def test_mirror_symmetry():
    # ellipsoid and dipole symmetric under x -> -x; A_x is even in x... (A_x = -c Y f(R)) so
    # a_x(-x) equals a_x(x) on mirrored edges while a_y flips sign: psi is odd in x.
    w = W.homogeneous_ellipsoid(n_nodes=20, semi=(7.0, 6.0, 8.0))
    sig = w.sigma_voxel()
    assert np.array_equal(sig, sig[:, :, ::-1])
    psi, _ = oracle.solve(sig, w.h, w.a, tol=1e-13)
    assert np.abs(psi + psi[:, :, ::-1]).max() < 1e-8 * np.abs(psi).max()
    u, E = oracle.efield(sig, w.h, w.a, psi, w.omega)
    np.testing.assert_allclose(E, E[:, :, ::-1], rtol=1e-7, atol=1e-10 * E.max())


def test_thomson_principle_and_continuity():
    w = W.random_ellipsoid_phantom(18, 16, 20, seed=5, n_ell=5, semi_range=(3.0, 7.0))
    sig = w.sigma_voxel()
    M = oracle.edge_conductance(sig, w.h)
    psi, _ = oracle.solve(sig, w.h, w.a, tol=1e-13)
    u, _ = oracle.efield(sig, w.h, w.a, psi, w.omega)
    comp, _ = oracle.components(sig, w.h)
    dof = comp >= 0
    # current continuity G^T M u = 0 (relative to G^T M a)
    cont = D.div_T(M * u)[dof]
    ref = D.div_T(M * w.a)[dof]
    assert np.linalg.norm(cont) < 1e-11 * np.linalg.norm(ref)
    # dissipated power u^T M u is minimal over a + G(psi + dpsi)
    P0 = np.sum(M * u * u)
    rng = np.random.default_rng(0)
    for _ in range(5):
        dpsi = rng.standard_normal(psi.shape) * 1e-3 * np.abs(psi).max()
        u2 = np.where(M > 0, w.a + D.grad(psi + dpsi), 0.0)
        assert np.sum(M * u2 * u2) > P0


def test_dipole_field_zero_in_air_and_continuity_c1():
    w = W.config(0)
    sig = w.sigma_voxel()
    psi, info = oracle.solve(sig, w.h, w.a, tol=1e-10)
    assert info["ndof"] == 8400 and info["ncomp"] == 1
    assert info["relres"] <= 1e-10 * 1.01
    u, E = oracle.efield(sig, w.h, w.a, psi, w.omega)
    assert np.all(E[sig == 0] == 0) and np.all(E[sig > 0] > 0)
    M = oracle.edge_conductance(sig, w.h)
    comp, _ = oracle.components(sig, w.h)
    cont = D.div_T(M * u)[comp >= 0]
    ref = D.div_T(M * w.a)[comp >= 0]
    assert np.linalg.norm(cont) <= 1.01e-10 * np.linalg.norm(ref)


# ---------------------------------------------------------------------------- adjoint
def _J_of(sig, h, a, omega, tol=1e-14):
    psi, _ = oracle.solve(sig, h, a, tol=tol, max_iter=200000)
    _, E = oracle.efield(sig, h, a, psi, omega)
    return oracle.pnorm_objective(E)[0], psi, E


def test_adjoint_against_finite_differences():
    w = W.tiny_random_phantom(5, 4, 6, seed=21, fill=0.8, n_classes=3)
    labels = w.labels
    table = w.sigma_table
    h = w.h
    J0, psi, E = _J_of(table[labels], h, w.a, w.omega)
    _, gE = oracle.pnorm_objective(E)
    gs, gt, info = oracle.adjoint(table[labels], h, w.a, psi, w.omega, gE, tol=1e-14,
                                  labels=labels, n_labels=len(table))
    assert info["relres"] < 1e-12
    for t in range(1, len(table)):
        if not np.any(labels == t):
            continue
        st = table[t]
        step = 1e-6 * st
        tp, tm = table.copy(), table.copy()
        tp[t] += step
        tm[t] -= step
        fd = (_J_of(tp[labels], h, w.a, w.omega)[0] - _J_of(tm[labels], h, w.a, w.omega)[0]) / (2 * step)
        assert abs(gt[t] - fd) <= 1e-5 * abs(fd) + 1e-9 * J0 / st, (t, gt[t], fd)
    # per voxel, on a few voxels
    sig = table[labels].copy()
    body = np.argwhere(sig > 0)
    for idx in body[:: max(1, len(body) // 6)]:
        k, j, i = idx
        step = 1e-6 * sig[k, j, i]
        sp, sm = sig.copy(), sig.copy()
        sp[k, j, i] += step
        sm[k, j, i] -= step
        fd = (_J_of(sp, h, w.a, w.omega)[0] - _J_of(sm, h, w.a, w.omega)[0]) / (2 * step)
        assert abs(gs[k, j, i] - fd) <= 1e-4 * abs(fd) + 1e-7 * J0 / sig[k, j, i], (idx, gs[k, j, i], fd)
    # Euler identity: J is invariant under sigma -> c sigma, so sum sigma_v dJ/dsigma_v = 0
    assert abs(np.sum(sig * gs)) <= 1e-9 * np.sum(np.abs(sig * gs))
    # per label = sum of per voxel
    for t in range(len(table)):
        assert abs(gt[t] - gs[labels == t].sum()) <= 1e-12 * (np.abs(gs).sum() + 1e-300)
    assert np.all(gs[sig == 0] == 0)


# ---------------------------------------------------------------------------- percentile (step 6)
def test_percentile_nearest_rank_by_hand():
    # 10 values 1..10 in scrambled order: rank ceil(0.99*10) = 10 -> 10; q = 0.5 -> rank 5 -> 5
    e = np.array([[[7.0, 2.0, 9.0, 1.0, 10.0, 3.0, 5.0, 8.0, 4.0, 6.0, 0.0]]])
    lab = np.array([[[1, 1, 2, 1, 2, 1, 1, 2, 1, 1, 0]]])
    sig = np.where(lab > 0, 0.3, 0.0)
    p99, per = oracle.percentile_nearest_rank(e, lab, sig, 0.99)
    assert p99 == 10.0
    p50, per50 = oracle.percentile_nearest_rank(e, lab, sig, 0.5)
    assert p50 == 5.0
    # label 2 holds 9, 10, 8 -> rank ceil(0.5*3) = 2 -> 9; label 1 holds 7,2,1,3,5,4,6 -> rank 4 -> 4
    assert per50[2] == 9.0 and per50[1] == 4.0 and np.isnan(per50[0])


def test_percentile_body_is_the_conducting_voxels():
    # Sec. III.A: only conducting voxels are modelled.  A labelled tissue with sigma = 0 is not body:
    # the same 10 values as above, but label 2 (values 9, 10, 8) is given sigma = 0 and the field 0 there
    # (as Eq. (1) leaves air voxels).  Body = 7,2,1,3,5,4,6 -> q = 0.99: rank 7 -> 7; q = 0.5: rank 4 -> 4.
    e = np.array([[[7.0, 2.0, 0.0, 1.0, 0.0, 3.0, 5.0, 0.0, 4.0, 6.0, 0.0]]])
    lab = np.array([[[1, 1, 2, 1, 2, 1, 1, 2, 1, 1, 0]]])
    sig = np.where(lab == 1, 0.3, 0.0)
    p99, per = oracle.percentile_nearest_rank(e, lab, sig, 0.99)
    assert p99 == 7.0 and per[1] == 7.0 and np.isnan(per[2]) and np.isnan(per[0])
    p50, _ = oracle.percentile_nearest_rank(e, lab, sig, 0.5)
    assert p50 == 4.0
    # a voxel of label 0 that conducts (per-voxel conductivities) is body and forms group 0
    sig2 = sig.copy()
    sig2[0, 0, 10] = 0.1
    e2 = e.copy()
    e2[0, 0, 10] = 11.0
    p, per = oracle.percentile_nearest_rank(e2, lab, sig2, 1.0)
    assert p == 11.0 and per[0] == 11.0


def test_percentile_matches_inverted_cdf():
    rng = np.random.default_rng(5)
    e = rng.lognormal(size=(7, 9, 11))
    lab = rng.integers(0, 4, size=e.shape)
    sig = np.where(lab > 0, 0.2, 0.0)
    sig[(lab == 3) & (rng.random(e.shape) < 0.3)] = 0.0   # some tissue voxels without conductivity
    e[sig == 0] = 0.0
    p, per = oracle.percentile_nearest_rank(e, lab, sig, 0.99)
    assert p == np.percentile(e[sig > 0], 99, method="inverted_cdf")
    for t in range(1, 4):
        assert per[t] == np.percentile(e[(lab == t) & (sig > 0)], 99, method="inverted_cdf")


def test_percentile_ties_and_extremes():
    # ties: values 1,1,2,2,2,3 -> rank ceil(0.5*6) = 3 -> 2; q = 1 -> maximum; q tiny -> minimum
    e = np.array([[[2.0, 1.0, 2.0, 3.0, 1.0, 2.0]]])
    lab = np.ones_like(e, dtype=np.uint8)
    sig = np.ones_like(e)
    assert oracle.percentile_nearest_rank(e, lab, sig, 0.5)[0] == 2.0
    assert oracle.percentile_nearest_rank(e, lab, sig, 1.0)[0] == 3.0
    assert oracle.percentile_nearest_rank(e, lab, sig, 1e-9)[0] == 1.0
    # brute force on random data: the result r satisfies #(v <= r) >= k and #(v < r) < k, k = ceil(q n)
    rng = np.random.default_rng(11)
    v = np.round(rng.random(997) * 50) / 7.0
    lab = np.ones((1, 1, v.size), np.uint8)
    sig = np.ones((1, 1, v.size))
    for q in (0.01, 0.37, 0.99, 1.0):
        r = oracle.percentile_nearest_rank(v.reshape(1, 1, -1), lab, sig, q)[0]
        k = int(np.ceil(q * v.size))
        assert np.sum(v <= r) >= k and np.sum(v < r) < k


# ---------------------------------------------------------------------------- residual of a given potential
# oracle.residual is the check applied at sizes the oracle cannot solve in test time; it must return
# ||b - A psi||_2 / ||b||_2 over the unknowns with b = -G^T M a (Eq. (3); the relative residual of
# Sec. II.A).  Pinned here to a hand value, the zero potential, exact manufactured answers, an
# independent element assembly and the solver's own true residual.
def test_residual_single_voxel_by_hand():
    # one voxel, sigma 2, h 1: every edge conducts 0.5; a = 1 on the x-edge 0 -> 1 gives b = (0.5, -0.5, 0, ...).
    # psi = 1 at node 0: A psi = column 0 of the cube Laplacian = (1.5, -0.5, -0.5, 0, -0.5, 0, 0, 0),
    # r = (-1, 0, 0.5, 0, 0.5, 0, 0, 0): ||r||^2 = 1.5, ||b||^2 = 0.5, ratio sqrt(3)
    sig = np.full((1, 1, 1), 2.0)
    a = np.zeros((3, 2, 2, 2))
    a[0, 0, 0, 0] = 1.0
    psi = np.zeros((2, 2, 2))
    psi[0, 0, 0] = 1.0
    rel, r = oracle.residual(sig, (1.0, 1.0, 1.0), a, psi, want_nodes=True)
    assert abs(rel - np.sqrt(3.0)) <= 1e-15
    np.testing.assert_array_equal(r.reshape(-1), [-1.0, 0.0, 0.5, 0.0, 0.5, 0.0, 0.0, 0.0])
    # a constant added to psi is in the null space: same residual
    assert abs(oracle.residual(sig, (1.0, 1.0, 1.0), a, psi + 7.0) - np.sqrt(3.0)) <= 1e-14


@pytest.mark.parametrize("seed,shape", [(21, (4, 3, 5)), (22, (6, 6, 4))])
def test_residual_of_zero_potential_is_one(seed, shape):
    w = W.tiny_random_phantom(*shape, seed=seed)
    rel = oracle.residual(w.sigma_voxel(), w.h, w.a, np.zeros((w.nz + 1, w.ny + 1, w.nx + 1)))
    assert abs(rel - 1.0) <= 1e-15


@pytest.mark.parametrize("cfg", ["ellipsoid", "hetero"])
def test_residual_of_manufactured_answer_vanishes(cfg):
    # a = -G psi* + M^-1 C^T W gives b = A psi* exactly (C G = 0), whatever constant psi* carries
    rng = np.random.default_rng(12)
    if cfg == "ellipsoid":
        w = W.homogeneous_ellipsoid(n_nodes=20, semi=(7.0, 6.0, 8.0))
    else:
        w = W.random_ellipsoid_phantom(24, 20, 28, seed=98, n_ell=6, semi_range=(3.0, 8.0))
    sig = w.sigma_voxel()
    M = oracle.edge_conductance(sig, w.h)
    a, psi_star, _ = D.manufactured(M, sig > 0, rng)
    comp, _ = oracle.components(sig, w.h)
    assert oracle.residual(sig, w.h, a, D.project_mean_zero(psi_star, comp)) <= 1e-13
    assert oracle.residual(sig, w.h, a, psi_star + 3e-6) <= 1e-13
    # a wrong potential is seen: psi* with one body node moved
    bad = psi_star.copy()
    k, j, i = np.argwhere(comp >= 0)[len(np.argwhere(comp >= 0)) // 2]
    bad[k, j, i] += 1e-6
    assert oracle.residual(sig, w.h, a, bad) > 1e-3


@pytest.mark.parametrize("seed,shape,fill", [(23, (4, 4, 4), 0.5), (24, (5, 3, 6), 0.35), (25, (3, 6, 4), 0.7)])
def test_residual_matches_independent_assembly(seed, shape, fill):
    # A from the voxel-by-voxel element scatter, b = -G^T M a with M read off that A: a different route
    # to b - A psi than the oracle's edge gather, on random potentials at every node (also off the body)
    w = W.tiny_random_phantom(*shape, seed=seed, fill=fill)
    sig = w.sigma_voxel()
    Afull = _element_assembly(sig, w.h)
    Nz, Ny, Nx = w.nz + 1, w.ny + 1, w.nx + 1
    dof = np.where(np.abs(Afull).sum(axis=1) > 0)[0]
    M = np.zeros_like(w.a)
    flatM = M.reshape(3, -1)
    step = (1, Nx, Nx * Ny)
    for d in range(3):
        for n in range(Nx * Ny * Nz):
            i, j, k = n % Nx, (n // Nx) % Ny, n // (Nx * Ny)
            if (d == 0 and i == Nx - 1) or (d == 1 and j == Ny - 1) or (d == 2 and k == Nz - 1):
                continue
            flatM[d, n] = -Afull[n, n + step[d]]
    bfull = -D.div_T(M * w.a).reshape(-1)
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal((Nz, Ny, Nx)) * 1e-3
    rfull = bfull - Afull @ psi.reshape(-1)
    expect = np.linalg.norm(rfull[dof]) / np.linalg.norm(bfull[dof])
    rel, r = oracle.residual(sig, w.h, w.a, psi, want_nodes=True)
    assert abs(rel - expect) <= 1e-12 * expect
    np.testing.assert_allclose(r.reshape(-1)[dof], rfull[dof], rtol=0, atol=1e-12 * np.abs(rfull).max())
    assert np.all(np.delete(r.reshape(-1), dof) == 0)


def test_residual_matches_the_solvers_true_residual():
    # a loose solve leaves a residual far above rounding: the relative residual the solve reports
    # (its own true residual at exit) and the residual of its returned potential agree
    w = W.random_ellipsoid_phantom(20, 18, 24, seed=97, n_ell=5, semi_range=(3.0, 7.0))
    sig = w.sigma_voxel()
    psi, info = oracle.solve(sig, w.h, w.a, tol=1e-6)
    assert 1e-8 < info["relres"] <= 1e-6
    assert abs(oracle.residual(sig, w.h, w.a, psi) - info["relres"]) <= 1e-9 * info["relres"]


# ---------------------------------------------------------------------------- tree-cotree gauge (Eq. (2))
def test_tree_cotree_single_voxel_uniform_bz():
    # one voxel in a uniform B_z: flux phi through both z-facets, none through the others
    phi = 3.0e-6
    f = np.zeros((3, 2, 2, 2))
    f[2, 0, 0, 0] = f[2, 1, 0, 0] = phi
    a = oracle.tree_cotree_potentials(f)
    assert a[0, 0, 1, 0] == -phi and a[0, 1, 1, 0] == -phi          # cotree x-edges at j = 1
    assert a[0, 0, 0, 0] == 0.0 and a[0, 1, 0, 0] == 0.0            # the line j = 0 (tree at k = 0)
    assert np.all(a[2] == 0.0) and np.all(a[1, 0] == 0.0)           # tree: z-edges, y-edges at k = 0
    assert np.array_equal(D.curl(a), f)


def _random_divfree_flux(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    a0 = rng.standard_normal((3, nz + 1, ny + 1, nx + 1))
    a0[0, :, :, nx] = 0.0
    a0[1, :, ny, :] = 0.0
    a0[2, nz, :, :] = 0.0
    return a0, D.curl(a0)


def test_tree_cotree_reproduces_fluxes_and_differs_by_a_gradient():
    a0, f = _random_divfree_flux((5, 6, 7), 21)
    a = oracle.tree_cotree_potentials(f)
    c = D.curl(a)
    assert np.abs(c - f).max() <= 1e-12 * np.abs(f).max()
    # tree edges are zero
    assert np.all(a[2] == 0.0) and np.all(a[1, 0] == 0.0) and np.all(a[0, 0, 0] == 0.0)
    # a - a0 = G phi: integrate the difference along the tree from node (0,0,0), then check every edge
    d = a - a0
    Nz, Ny, Nx = d.shape[1:]
    phi = np.zeros((Nz, Ny, Nx))
    for i in range(1, Nx):
        phi[0, 0, i] = phi[0, 0, i - 1] + d[0, 0, 0, i - 1]
    for j in range(1, Ny):
        phi[0, j, :] = phi[0, j - 1, :] + d[1, 0, j - 1, :]
    for k in range(1, Nz):
        phi[k] = phi[k - 1] + d[2, k - 1]
    g = np.zeros_like(d)
    g[0, :, :, :-1] = phi[:, :, 1:] - phi[:, :, :-1]
    g[1, :, :-1, :] = phi[:, 1:, :] - phi[:, :-1, :]
    g[2, :-1, :, :] = phi[1:] - phi[:-1]
    assert np.abs(g - d).max() <= 1e-11 * np.abs(d).max()


def test_tree_cotree_gauge_leaves_the_field_unchanged():
    # |E| from the tree-cotree potentials equals |E| from the analytic edge integrals (the
    # difference is a discrete gradient, absorbed by Psi)
    w = W.random_ellipsoid_phantom(14, 12, 16, seed=7, n_ell=6, semi_range=(2.0, 5.0))
    sig = w.sigma_voxel()
    a_tc = oracle.tree_cotree_potentials(D.curl(w.a))
    p0, _ = oracle.solve(sig, w.h, w.a, tol=1e-13)
    p1, _ = oracle.solve(sig, w.h, a_tc, tol=1e-13)
    _, e0 = oracle.efield(sig, w.h, w.a, p0, w.omega)
    _, e1 = oracle.efield(sig, w.h, a_tc, p1, w.omega)
    assert np.linalg.norm(e1 - e0) <= 1e-9 * np.linalg.norm(e0)
    assert np.linalg.norm(p1 - p0) > 1e-3 * np.linalg.norm(p0)   # the potentials themselves do differ
