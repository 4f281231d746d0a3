"""Record oracle reference figures that are too slow to recompute in a test.

Runs only the CPU oracle (no HIP code) and writes JSON under tests/golden/:
  oracle_body_1e-8.json: Jacobi-PCG iterations and times of the body-shaped
  2 mm phantom (250x150x900 voxels, ~8.9 M unknowns, rectangular-loop source)
  solved to relative residual 1e-8.  The benchmark scales its bounded CPU
  sample by this iteration count.

  oracle_body_digest_1e-12.json (--digest --tol 1e-12): a compact digest of the
  oracle's own solution of that system to relative residual 1e-12, for a
  full-size parity test: every STRIDE-th node of the conductor (flat index,
  potential), norms of the potential per connected component, and the voxel
  |E| of Eq. (1) by its 2-norm and nearest-rank 99th percentiles (whole body and
  per tissue).  At 1e-12 two solutions of Eq. (3) agree far below the bars the
  test applies; at 1e-8 they need not.

Usage: python -m oracle.reference_runs [--threads N] [--tol T] [--digest]
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    import oracle
    import workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--digest", action="store_true", help="write the solution digest instead of the timing record")
    args = ap.parse_args()
    w = workloads.config(2)
    t0 = time.time()
    psi, info = oracle.solve(w.sigma_voxel(), w.h, w.a, tol=args.tol, max_iter=1_000_000, nthreads=args.threads)
    if args.digest:
        return write_digest(w, psi, info, args, time.time() - t0)
    out = {
        "workload": w.name,
        "rel_tol": args.tol,
        "iterations": info["iterations"],
        "ndof": info["ndof"],
        "relres": info["relres"],
        "t_assemble_s": info["t_assemble"],
        "t_solve_s": info["t_solve"],
        "wall_s": time.time() - t0,
        "threads": args.threads,
        "host": platform.processor() or platform.machine(),
        "method": "oracle Jacobi-PCG (FP64, CSR), written by oracle/reference_runs.py",
    }
    path = os.path.join(ROOT, "tests", "golden", f"oracle_body_{args.tol:.0e}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


STRIDE = 4447   # nodes of the conductor between two samples (about 2,000 of the 8.9 M)


def write_digest(w, psi, info, args, wall):
    import numpy as np
    import oracle
    sig = w.sigma_voxel()
    comp, nc = oracle.components(sig, w.h)
    flat = comp.reshape(-1)
    nodes = np.flatnonzero(flat >= 0)
    pick = nodes[::STRIDE]
    pf = psi.reshape(-1)
    _, emag = oracle.efield(sig, w.h, w.a, psi, w.omega)
    p99, per = oracle.percentile_nearest_rank(emag, w.labels, sig, 0.99, n_labels=len(w.sigma_table))
    body = sig > 0
    out = {
        "workload": w.name,
        "rel_tol": args.tol,
        "iterations": info["iterations"],
        "relres": info["relres"],
        "ndof": int(nodes.size),
        "stride": STRIDE,
        "psi_sample": [[int(i), float(pf[i])] for i in pick],
        "psi_norm2": float(np.linalg.norm(pf)),
        "psi_maxabs": float(np.abs(pf).max()),
        "components": [{"nodes": int((flat == c).sum()), "norm2": float(np.linalg.norm(pf[flat == c]))}
                       for c in range(nc)],
        "emag_norm2_body": float(np.linalg.norm(emag[body])),
        "emag_p99_body": p99,
        "emag_p99_per_label": [None if np.isnan(v) else float(v) for v in per],
        "threads": args.threads,
        "wall_s": wall,
        "method": "oracle Jacobi-PCG (FP64, CSR) to the stated tolerance, digest written by oracle/reference_runs.py",
    }
    path = os.path.join(ROOT, "tests", "golden", f"oracle_body_digest_{args.tol:.0e}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(json.dumps({k: v for k, v in out.items() if k != "psi_sample"}))


if __name__ == "__main__":
    main()
