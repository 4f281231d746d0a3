"""Record oracle reference figures that are too slow to recompute in a test.

Runs only the CPU oracle (no HIP code) and writes JSON under tests/golden/:
  oracle_body_1e-8.json: Jacobi-PCG iterations and times of the body-shaped
  2 mm phantom (250x150x900 voxels, ~8.9 M unknowns, rectangular-loop source)
  solved to relative residual 1e-8.  The benchmark scales its bounded CPU
  sample by this iteration count.

Usage: python -m oracle.reference_runs [--threads N]
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
    args = ap.parse_args()
    w = workloads.config(2)
    t0 = time.time()
    psi, info = oracle.solve(w.sigma_voxel(), w.h, w.a, tol=args.tol, max_iter=1_000_000, nthreads=args.threads)
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


if __name__ == "__main__":
    main()
