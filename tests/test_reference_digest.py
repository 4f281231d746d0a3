"""The digest that oracle/reference_runs.py writes for the full-size parity test, checked on a small
phantom against the oracle's own arrays: every stored figure is the quantity it names (sampled potential
at its flat node index, norms per component, |E| norm and nearest-rank percentiles over sigma > 0), and
the stored golden file has the shape the GPU test reads."""
import json
import os
import types

import numpy as np

import oracle
import oracle.reference_runs as R
import workloads as W


def test_digest_fields_match_the_oracle(tmp_path, monkeypatch):
    w = W.random_ellipsoid_phantom(24, 20, 28, seed=61, n_ell=6, semi_range=(2.5, 8.0), name="digest24")
    sig = w.sigma_voxel()
    psi, info = oracle.solve(sig, w.h, w.a, tol=1e-12)
    (tmp_path / "tests" / "golden").mkdir(parents=True)
    monkeypatch.setattr(R, "ROOT", str(tmp_path))
    monkeypatch.setattr(R, "STRIDE", 37)
    R.write_digest(w, psi, info, types.SimpleNamespace(tol=1e-12, threads=1), 0.0)
    d = json.load(open(tmp_path / "tests" / "golden" / "oracle_body_digest_1e-12.json"))
    comp, nc = oracle.components(sig, w.h)
    nodes = np.flatnonzero(comp.reshape(-1) >= 0)
    assert d["ndof"] == nodes.size == info["ndof"] and d["stride"] == 37
    idx = [i for i, _ in d["psi_sample"]]
    assert idx == list(nodes[::37])
    assert all(v == psi.reshape(-1)[i] for i, v in d["psi_sample"])
    assert d["psi_norm2"] == np.linalg.norm(psi) and d["psi_maxabs"] == np.abs(psi).max()
    assert len(d["components"]) == nc
    cf = comp.reshape(-1)
    for c, dc in enumerate(d["components"]):
        assert dc["nodes"] == int((cf == c).sum())
        assert dc["norm2"] == np.linalg.norm(psi.reshape(-1)[cf == c])
    assert abs(sum(dc["norm2"] ** 2 for dc in d["components"]) - d["psi_norm2"] ** 2) <= 1e-12 * d["psi_norm2"] ** 2
    _, emag = oracle.efield(sig, w.h, w.a, psi, w.omega)
    body = sig > 0
    assert d["emag_norm2_body"] == np.linalg.norm(emag[body])
    # nearest rank by brute force: the value v with #(e <= v) >= ceil(q n) > #(e < v)
    e = emag[body]
    v = d["emag_p99_body"]
    k = int(np.ceil(0.99 * e.size))
    assert (e <= v).sum() >= k > (e < v).sum()
    for t, vt in enumerate(d["emag_p99_per_label"]):
        et = emag[body & (w.labels == t)]
        if vt is None:
            assert et.size == 0
        else:
            kt = int(np.ceil(0.99 * et.size))
            assert (et <= vt).sum() >= kt > (et < vt).sum()


def test_stored_golden_digest_shape():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_body_digest_1e-12.json")
    d = json.load(open(path))
    w_name = "body250x150x900"
    assert d["workload"] == w_name and d["rel_tol"] == 1e-12 and d["relres"] <= 1e-11
    assert d["ndof"] == 8900766 and d["stride"] == R.STRIDE
    assert len(d["psi_sample"]) == (d["ndof"] + d["stride"] - 1) // d["stride"]
    idx = [i for i, _ in d["psi_sample"]]
    assert idx == sorted(idx) and len(set(idx)) == len(idx)
    assert max(abs(v) for _, v in d["psi_sample"]) <= d["psi_maxabs"]
    assert sum(c["nodes"] for c in d["components"]) == d["ndof"]
    assert len(d["emag_p99_per_label"]) == 41 and d["emag_p99_per_label"][0] is None
