"""The allocation-free quantile entry point (spfd_percentile_noalloc) against the handle-based
spfd_percentile on the same |E|: two calls in a row through the C-ABI, the second on a smaller
voxel model (the shared work area keeps the first call's contents), plus a per-voxel conductivity
input.  Both are exact radix selections, so the values must be bit-identical."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2010_12879_amd as P  # noqa: E402

DEV = torch.device("cuda:0")


def _field(w):
    s = P.Solver(torch.from_numpy(w.labels).to(DEV), w.sigma_table, w.h, precision="mixed")
    a = torch.from_numpy(w.a).to(DEV)
    psi, info = s.solve(a, tol=1e-10)
    emag = s.efield(a, psi, w.omega)
    return s, emag


def _noalloc(w, emag, q, per_voxel=False):
    labels = torch.from_numpy(w.labels).to(DEV)
    table = torch.tensor(w.sigma_table, dtype=torch.float64, device=DEV)
    sv = torch.from_numpy(w.sigma_voxel()).to(DEV) if per_voxel else None
    out = torch.full((1 + len(w.sigma_table),), -1.0, dtype=torch.float64, device=DEV)
    stream = torch.cuda.current_stream(DEV)
    P.spfd_percentile_noalloc(labels, table, sv, emag.contiguous(), q, out, 0, stream.cuda_stream)
    stream.synchronize()
    return out.cpu().numpy()


def _same(x, y):
    return (np.isnan(x) and np.isnan(y)) or x == y


@pytest.mark.parametrize("q", [0.99, 0.5])
def test_noalloc_percentile_matches_handle_twice(q):
    print(f"case noalloc percentile q={q}", flush=True)
    big, small = W.config(1), W.config(0)
    for w in (big, small):       # second call: fewer voxels and labels than the first
        s, emag = _field(w)
        body, per = s.percentile(emag, q)
        s.close()
        got = _noalloc(w, emag, q)
        assert got[0] == body, (w.name, got[0], body)
        for t in range(len(w.sigma_table)):
            assert _same(got[1 + t], per[t]), (w.name, t, got[1 + t], per[t])
        # per-voxel conductivities give the same body set here
        got_v = _noalloc(w, emag, q, per_voxel=True)
        assert got_v[0] == body


def test_noalloc_percentile_rejects_oversize():
    print("case noalloc limits", flush=True)
    w = W.config(0)
    labels = torch.from_numpy(w.labels).to(DEV)
    emag = torch.zeros(w.labels.shape, dtype=torch.float64, device=DEV)
    table = torch.zeros(300, dtype=torch.float64, device=DEV)
    out = torch.zeros(301, dtype=torch.float64, device=DEV)
    with pytest.raises(P.SPFDError) as e:
        P.spfd_percentile_noalloc(labels, table, None, emag, 0.99, out)
    assert e.value.status == 1
    with pytest.raises(P.SPFDError) as e:
        P.spfd_percentile_noalloc(labels, table[:2], None, emag, 1.5, out)
    assert e.value.status == 1
