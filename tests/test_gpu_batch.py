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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_short_window_of_search_directions_same_bits(prec):
    """x is formed from a window of kept CG search directions, in step order: a window of 2 (x updated
    every second step, with right sides of a batch stopping at different steps, one at once) gives the
    same potentials bit for bit as the default window, and they meet the oracle's residual."""
    print(f"case window {prec}", flush=True)
    w = W.random_ellipsoid_phantom(32, 32, 40, seed=47, n_ell=8, semi_range=(3.0, 9.0))
    srcs = _sources(w, 4, 13)
    srcs[1] = 0.0                         # stops before its first step
    srcs[3] *= 1e-3
    res = {}
    for win in (0, 2, 6):
        s = P.Solver(_dev(w.labels), w.sigma_table, w.h, precision=prec, cg_window=win)
        res[win] = s.solve(_dev(srcs), tol=1e-11, max_iter=300)
        s.close()
    psi0, info0 = res[0]
    assert all(i["status"] == "OK" for i in info0)
    assert len({i["iterations"] for i in info0}) >= 2        # uneven stops within the batch
    for win in (2, 6):
        psi, info = res[win]
        assert [i["iterations"] for i in info] == [i["iterations"] for i in info0], win
        assert torch.equal(psi, psi0), win
    for i in (0, 2, 3):
        rel = oracle.residual(w.sigma_voxel(), w.h, srcs[i], psi0[i].cpu().numpy())
        assert rel <= 1e-11 * 1.01, (i, rel)
    with pytest.raises(RuntimeError):
        P.Solver(_dev(w.labels), w.sigma_table, w.h, precision=prec, cg_window=3)


def test_packed_models_short_window_same_bits():
    """Packed models (one CG per model, each with its own window counter) with a window of 2 against the
    default window: the same potentials bit for bit."""
    print("case packed window", flush=True)
    dims = [(24, 20, 28), (40, 32, 48), (17, 23, 9)]
    ws = [W.random_ellipsoid_phantom(nx, ny, nz, seed=310 + i, n_ell=5, semi_range=(2.5, 9.0), name=f"q{i}")
          for i, (nx, ny, nz) in enumerate(dims)]
    ws = [w for w in ws if np.any(w.sigma_voxel() > 0)]
    out = {}
    for win in (0, 2):
        ms = P.MultiSolver([_dev(w.labels) for w in ws], [w.sigma_table for w in ws], ws[0].h, precision="mixed",
                           cg_window=win)
        out[win] = ms.solve([_dev(w.a) for w in ws], tol=1e-11, max_iter=400)
        ms.close()
    assert out[0][1] == out[2][1]
    assert all(torch.equal(a, b) for a, b in zip(out[0][0], out[2][0]))


def _relmax(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_packed_models_against_oracle(prec):
    """Several voxel models of uneven size in one handle (packed along z, one hierarchy, every level
    kernel launched once for all of them, one CG per model): each potential against the oracle at the
    matching criterion 1e-12, and against the model solved alone."""
    print(f"case packed models {prec}", flush=True)
    dims = [(24, 20, 28), (40, 32, 48), (17, 23, 9), (33, 29, 37), (8, 8, 8)]
    ws = [W.random_ellipsoid_phantom(nx, ny, nz, seed=300 + i, n_ell=5, semi_range=(2.5, 9.0), name=f"p{i}")
          for i, (nx, ny, nz) in enumerate(dims)]
    ws = [w for w in ws if np.any(w.sigma_voxel() > 0)]
    assert len(ws) >= 4
    bar = {"fp64": 1e-7, "mixed": 1e-6}[prec]
    ms = P.MultiSolver([_dev(w.labels) for w in ws], [w.sigma_table for w in ws], ws[0].h, precision=prec)
    psis, infos = ms.solve([_dev(w.a) for w in ws], tol=1e-12, max_iter=400)
    # a second solve gives the same result bit for bit (replayed graphs, fixed reductions)
    psis2, infos2 = ms.solve([_dev(w.a) for w in ws], tol=1e-12, max_iter=400)
    assert infos == infos2 and all(torch.equal(a, b) for a, b in zip(psis, psis2))
    ms.close()
    for k, w in enumerate(ws):
        assert infos[k]["status"] == "OK" and infos[k]["rel_residual"] <= 1e-12, (k, infos[k])
        ref, oinfo = oracle.solve(w.sigma_voxel(), w.h, w.a, tol=1e-12)
        p = psis[k].cpu().numpy()
        print(f"packed {prec} model {k}: it={infos[k]['iterations']} err={_rel(p, ref):.2e}", flush=True)
        assert _rel(p, ref) <= bar and _relmax(p, ref) <= bar, k
        s = P.Solver(_dev(w.labels), w.sigma_table, w.h, precision=prec)
        p1, i1 = s.solve(_dev(w.a), tol=1e-12, max_iter=400)
        s.close()
        assert _rel(p, p1.cpu().numpy()) <= bar, k


def test_packed_uneven_phantoms():
    """The 16 phantoms of 64^3 ... 192^3 voxels in one handle, FP32 cycle: each model's residual by the
    oracle's own assembly at the benchmark's criterion, and each potential against its own single-model
    solve (both at 1e-12)."""
    print("case packed uneven phantoms", flush=True)
    ws = W.uneven_phantoms()
    ms = P.MultiSolver([_dev(w.labels) for w in ws], [w.sigma_table for w in ws], ws[0].h, precision="mixed")
    srcs = [_dev(w.a) for w in ws]
    psis, infos = ms.solve(srcs, tol=1e-8)
    for k, w in enumerate(ws):
        assert infos[k]["status"] == "OK"
        rel = oracle.residual(w.sigma_voxel(), w.h, w.a, psis[k].cpu().numpy())
        assert rel <= 1e-8 and abs(rel - infos[k]["rel_residual"]) <= 1e-6 * rel, (k, rel, infos[k])
    tight, _ = ms.solve(srcs, tol=1e-12, max_iter=400)
    ms.close()
    for k, w in enumerate(ws):
        s = P.Solver(_dev(w.labels), w.sigma_table, w.h, precision="mixed")
        p1, i1 = s.solve(srcs[k], tol=1e-12, max_iter=400)
        s.close()
        err = _rel(tight[k].cpu().numpy(), p1.cpu().numpy())
        print(f"packed uneven model {k} ({w.name}): it={infos[k]['iterations']} vs single {err:.2e}", flush=True)
        assert err <= 1e-6, k


def test_packed_models_errors():
    print("case packed errors", flush=True)
    ws = [W.random_ellipsoid_phantom(16, 16, 16, seed=400 + i, n_ell=4, semi_range=(2.5, 6.0)) for i in range(2)]
    h = P.spfd_create(0)
    try:
        P.spfd_set_geometry_many(h, [_dev(w.labels) for w in ws], *ws[0].h)
        with pytest.raises(P.SPFDError) as e:       # label 19 not covered by a two-entry table
            P.spfd_set_sigma_tables(h, [[0.0, 0.3], ws[1].sigma_table])
            P.spfd_build(h)
        assert e.value.status == 1
        P.spfd_set_sigma_tables(h, [w.sigma_table for w in ws])
        opts = P.AmgOptions()
        opts.no_split = 1
        with pytest.raises(P.SPFDError) as e:
            P.spfd_build(h, opts)
        assert e.value.status == 1
        P.spfd_build(h)
        emag = torch.zeros(1, dtype=torch.float64, device=DEV)
        with pytest.raises(P.SPFDError) as e:
            P.spfd_percentile(h, emag)
        assert e.value.status == 2
    finally:
        P.spfd_destroy(h)
