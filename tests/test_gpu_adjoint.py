"""Adjoint conductivity gradient of J = (sum_v |E_v|^8)^(1/8) on the GPU.

Checked against the CPU oracle's adjoint (same forward potential), against
central finite differences through the autograd Function, and against the
Euler identity sum_v sigma_v dJ/dsigma_v = 0 (J is invariant under sigma -> c sigma).
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2010_12879_amd as P  # noqa: E402

DEV = torch.device("cuda:0")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _J(emag, p=8):
    return torch.linalg.vector_norm(emag.reshape(-1), ord=p)


@pytest.mark.parametrize("case", ["ellipsoid", "hetero"])
def test_adjoint_matches_oracle(case):
    print(f"case adjoint-vs-oracle {case}", flush=True)
    if case == "ellipsoid":
        w = W.config(0)
    else:
        w = W.random_ellipsoid_phantom(40, 32, 48, seed=17, n_ell=8, semi_range=(3.0, 9.0))
    s = P.Solver(_dev(w.labels), w.sigma_table, w.h, precision="fp64")
    a = _dev(w.a)
    psi, info = s.solve(a, tol=1e-13, max_iter=400)
    emag = s.efield(a, psi, w.omega)
    J, gE = oracle.pnorm_objective(emag.cpu().numpy())
    gvox, gtab, ainfo = s.adjoint(a, psi, w.omega, _dev(gE), tol=1e-13, max_iter=400)
    s.close()
    assert ainfo["status"] == "OK", ainfo
    psi_np = psi.cpu().numpy()
    gs_ref, gt_ref, oinfo = oracle.adjoint(w.sigma_voxel(), w.h, w.a, psi_np, w.omega, gE, tol=1e-13,
                                           labels=w.labels, n_labels=len(w.sigma_table))
    g = gvox.cpu().numpy()
    print(f"adjoint {case}: grad err {_rel(g, gs_ref):.2e}, its {ainfo['iterations']}", flush=True)
    assert _rel(g, gs_ref) <= 1e-7
    # per-label sums cancel (exactly 0 for a single tissue by the Euler identity): absolute scale = sum |g_v|
    np.testing.assert_allclose(gtab[:len(gt_ref)], gt_ref, rtol=1e-7, atol=1e-9 * np.abs(gs_ref).sum())
    # per label = sum of per voxel; air voxels have zero gradient
    for t in range(len(w.sigma_table)):
        assert abs(gtab[t] - g[w.labels == t].sum()) <= 1e-10 * np.abs(g).sum()
    assert np.all(g[w.sigma_voxel() == 0] == 0)
    # Euler identity
    sig = w.sigma_voxel()
    assert abs(np.sum(sig * g)) <= 1e-7 * np.sum(np.abs(sig * g))


def test_autograd_against_finite_differences():
    print("case adjoint-fd", flush=True)
    w = W.random_ellipsoid_phantom(48, 40, 56, seed=23, n_ell=10, semi_range=(3.0, 10.0))
    lab = _dev(w.labels)
    a = _dev(w.a)
    solver = P.Solver(lab, w.sigma_table, w.h, precision="fp64")
    sig = torch.tensor(w.sigma_table, dtype=torch.float64, requires_grad=True)
    emag = P.SPFDField.apply(sig, solver, a, w.omega, 1e-13)
    J = _J(emag)
    J.backward()
    grad = sig.grad.numpy().copy()

    def J_of(table):
        with torch.no_grad():
            e = P.SPFDField.apply(torch.tensor(table, dtype=torch.float64), solver, a, w.omega, 1e-13)
            return float(_J(e))

    present = [t for t in range(1, len(w.sigma_table)) if np.any(w.labels == t)]
    scale = max(abs(grad[t] * w.sigma_table[t]) for t in present)
    checked = 0
    for t in present:
        if abs(grad[t] * w.sigma_table[t]) < 1e-3 * scale:
            continue
        h = 1e-6 * w.sigma_table[t]
        tp, tm = w.sigma_table.copy(), w.sigma_table.copy()
        tp[t] += h
        tm[t] -= h
        fd = (J_of(tp) - J_of(tm)) / (2 * h)
        print(f"  tissue {t}: adjoint {grad[t]:.6e} fd {fd:.6e}", flush=True)
        assert abs(grad[t] - fd) <= 1e-4 * abs(fd), (t, grad[t], fd)
        checked += 1
    assert checked >= 3
    # the Euler identity on the table: J is scale-invariant in sigma
    assert abs(np.dot(grad[1:], w.sigma_table[1:])) <= 1e-6 * np.sum(np.abs(grad[1:] * w.sigma_table[1:]))
    solver.close()


def test_per_voxel_sigma_gradient():
    print("case adjoint-voxel", flush=True)
    w = W.random_ellipsoid_phantom(32, 28, 36, seed=29, n_ell=6, semi_range=(3.0, 8.0))
    sigv = _dev(w.sigma_voxel()).requires_grad_(True)
    solver = P.Solver(_dev(w.labels), sigv.detach(), w.h, precision="fp64")
    a = _dev(w.a)
    emag = P.SPFDField.apply(sigv, solver, a, w.omega, 1e-13)
    J = _J(emag)
    J.backward()
    g = sigv.grad.cpu().numpy()
    sv = w.sigma_voxel()
    body = np.argwhere(sv > 0)
    rng = np.random.default_rng(0)
    for idx in body[rng.choice(len(body), 5, replace=False)]:
        k, j, i = idx
        h = 1e-6 * sv[k, j, i]
        vals = []
        for sgn in (1, -1):
            s2 = sv.copy()
            s2[k, j, i] += sgn * h
            with torch.no_grad():
                e = P.SPFDField.apply(_dev(s2), solver, a, w.omega, 1e-13)
            vals.append(float(_J(e)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[k, j, i] - fd) <= 1e-3 * abs(fd) + 1e-6 * float(J) / sv[k, j, i], (idx, g[k, j, i], fd)
    solver.close()
