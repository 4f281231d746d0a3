"""Many right sides sharing one hierarchy: one launch per kernel covers the whole batch.

Each source keeps its own scalars, stop flag and partial sums, so a batched
solve must give bitwise the same potentials as solving each source alone.
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


def _sources(w, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        r0 = (rng.uniform(0.3, 0.7) * w.nx * w.h[0], rng.uniform(0.3, 0.7) * w.ny * w.h[1], -rng.uniform(5, 15) * w.h[2])
        out.append(W.dipole_edge_potentials(w.nx, w.ny, w.nz, w.h, r0))
    return np.stack(out)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_single_solves(prec):
    print(f"case batch-vs-single {prec}", flush=True)
    w = W.random_ellipsoid_phantom(48, 40, 64, seed=41, n_ell=12, semi_range=(3.0, 10.0))
    srcs = _sources(w, 6, 7)
    s = P.Solver(_dev(w.labels), w.sigma_table, w.h, precision=prec)
    psi_b, info_b = s.solve(_dev(srcs), tol=1e-11, max_iter=300)
    singles = []
    for i in range(len(srcs)):
        p1, i1 = s.solve(_dev(srcs[i]), tol=1e-11, max_iter=300)
        singles.append(p1)
        assert i1["iterations"] == info_b[i]["iterations"]
        assert torch.equal(p1, psi_b[i]), i
    s.close()
    # and each against the oracle
    for i in (0, len(srcs) - 1):
        ref, _ = oracle.solve(w.sigma_voxel(), w.h, srcs[i], tol=1e-12)
        err = np.linalg.norm(psi_b[i].cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= (1e-7 if prec == "fp64" else 1e-6), err


def test_batch_with_zero_source_and_uneven_convergence():
    print("case batch-uneven", flush=True)
    w = W.random_ellipsoid_phantom(32, 32, 40, seed=43, n_ell=8, semi_range=(3.0, 9.0))
    srcs = _sources(w, 3, 9)
    srcs[1] = 0.0                         # a zero source converges at once
    srcs[2] *= 1e6                        # very different scales
    s = P.Solver(_dev(w.labels), w.sigma_table, w.h, precision="mixed")
    psi, info = s.solve(_dev(srcs), tol=1e-10, max_iter=300)
    assert [i["status"] for i in info] == ["OK"] * 3
    assert float(psi[1].abs().max()) == 0.0 and info[1]["iterations"] == 0
    for i in (0, 2):
        rel = oracle.residual(w.sigma_voxel(), w.h, srcs[i], psi[i].cpu().numpy())
        assert rel <= 1e-10 * 1.01, (i, rel)
    s.close()


def test_solve_many_uneven_phantoms_equals_single():
    print("case solve-many", flush=True)
    sizes = [20, 28, 36, 44]
    solvers, srcs, ws = [], [], []
    for i, m in enumerate(sizes):
        w = W.random_ellipsoid_phantom(m, m, m, seed=200 + i, n_ell=6, semi_range=(3.0, 8.0), name=f"e{m}")
        ws.append(w)
        st = torch.cuda.Stream(DEV)
        solvers.append(P.Solver(_dev(w.labels), w.sigma_table, w.h, precision="mixed", stream=st))
        srcs.append(_dev(w.a))
    torch.cuda.synchronize()
    psis, infos = P.solve_many(solvers, srcs, tol=1e-11)
    assert all(i["status"] == "OK" for i in infos)
    for k, (s, w) in enumerate(zip(solvers, ws)):
        p1, i1 = s.solve(srcs[k], tol=1e-11)
        torch.cuda.synchronize()
        assert i1["iterations"] == infos[k]["iterations"]
        assert torch.equal(p1, psis[k]), k
        rel = oracle.residual(w.sigma_voxel(), w.h, w.a, psis[k].cpu().numpy())
        assert rel <= 1e-11 * 1.01
    for s in solvers:
        s.close()
