#!/usr/bin/env python3
"""Benchmark of the Co-Sim. SPFD hot path on one MI355X.

Workload: the body-shaped 2 mm phantom (250x150x900 voxels, ~8.9 M unknowns,
40 tissues, rectangular-loop source at 85 kHz), inputs resident in HBM.
A step is one pass of the whole path on the GPU:
  conductances + multigrid hierarchy (spfd_set_sigma_table + spfd_build),
  right side b = -G^T M a (spfd_set_source),
  AMG-preconditioned CG to relative residual 1e-8 (spfd_solve),
  edge voltages and voxel-averaged |E| (spfd_efield).
The headline value is the solve time with the FP32 cycle inside FP64 CG;
the same steps are timed with the all-FP64 cycle for the speedup.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# finest-level kernel classes timed with events (one sampled CG iteration per solve);
# the dominant one (largest estimated share of the solve) carries the roofline figure
FINE_CLASSES = {0: "k_col_cg_step (outer CG: p = z + beta p, p.Ap)",
                1: "k_col_rupdate (r -= alpha A p, A p formed again; ||r||^2, FP32 copy of r)",
                2: "k_col_cheb_step + CG dot z.r (last post-smoothing step)",
                4: "k_col_cheb_first2 (first two Chebyshev steps, the pre-smoothing)",
                6: "k_col_resid_restrict (residual + restriction)",
                7: "k_col_cheb_step + prolongation (first post-smoothing step)"}
# rocprofv3 summaries under profiles/ (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE)
PROFILE_OF = {0: "k_col_cg_step", 1: "k_col_rupdate", 2: "k_col_cheb_step_dots", 4: "k_col_cheb_first2",
              6: "k_col_resid_restrict", 7: "k_col_cheb_step_prolong"}
KERNEL_SOURCES = ["paper_2010_12879_amd/csrc/kernels_col.hip", "paper_2010_12879_amd/csrc/kernels.hip",
                  "paper_2010_12879_amd/csrc/common.h", "paper_2010_12879_amd/csrc/kernels.h"]


def measured_traffic(name, workload):
    """HBM bytes per launch from the committed counter summary, or None when the summary is
    missing or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_{workload}.md")
    if not os.path.exists(path):
        return None, None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("    ") and not line.strip().startswith("rocprofv3"):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "hbm_bytes_per_launch" not in fields:
        return None, fields.get("median_duration_us")
    return float(fields["hbm_bytes_per_launch"]), fields.get("median_duration_us")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=150, help="oracle iterations in the bounded CPU sample")
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--no-batch", action="store_true", help="skip the multi-source and multi-phantom runs")
    ap.add_argument("--scale-1mm", action="store_true",
                    help="also solve the 1 mm body phantom (500x300x1800 voxels, ~69.7 M unknowns)")
    ap.add_argument("--no-cold", action="store_true", help="skip the cold-cache per-kernel timing")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint gradient and its finite differences")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the runs, copy a MIB-sized device buffer 3 times (a plain copy kernel of known "
                         "size, to scale hardware byte counters)")
    return ap.parse_args()


def copy_calibration(mib, torch):
    """Device-to-device copies of a known size: reads and writes mib MiB each."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t = []
    for _ in range(3):
        t0 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    return {"bytes_read": n * 8, "bytes_written": n * 8, "copies": 3,
            "best_gbs": 2 * n * 8 / min(t) / 1e9}


def run_precision(prec, w, lab, a, args, P, torch):
    dev = lab.device
    cur = torch.cuda.current_stream(dev)
    alloc = P.torch_allocator(dev, cur)    # the handle's device memory from PyTorch's caching allocator
    h = P.spfd_create(dev.index or 0, cur.cuda_stream, alloc)
    nx, ny, nz = w.nx, w.ny, w.nz
    P.spfd_set_geometry(h, nx, ny, nz, *w.h, lab)
    opts = P.AmgOptions(P.MIXED if prec == "mixed" else P.FP64, P.CYCLE_V, 0, 0, 0.0, 0.0)
    sopt = P.SolveOptions(args.tol, 500, 0)
    psi = torch.empty((nz + 1, ny + 1, nx + 1), dtype=torch.float64, device=dev)
    emag = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev)
    phases = {"setup": [], "rhs": [], "solve": [], "efield": [], "step": []}
    info = None

    def step(record):
        nonlocal info
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.spfd_set_sigma_table(h, list(w.sigma_table))
        P.spfd_build(h, opts)
        t1 = time.perf_counter()
        P.spfd_set_source(h, 0, a)
        t2 = time.perf_counter()
        st, inf = P.spfd_solve(h, sopt, psi, 1)
        t3 = time.perf_counter()
        P.spfd_efield(h, w.omega, a, psi, None, emag)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        if st != 0:
            raise RuntimeError(f"solve failed: {inf}")
        info = inf[0]
        if record:
            for k, v in (("setup", t1 - t0), ("rhs", t2 - t1), ("solve", t3 - t2), ("efield", t4 - t3),
                         ("step", t4 - t0)):
                phases[k].append(v)

    for _ in range(args.warmup):
        step(False)
    P.spfd_timing(h, sum(1 << k for k in FINE_CLASSES))
    for _ in range(args.steps):
        step(True)
    stats = {name: P.spfd_timing_get(h, k) for k, name in enumerate(P.KERNEL_CLASSES)}
    cold = None
    if not args.no_cold:
        # the same kernels with the caches flushed before every sampled launch (outside its events)
        P.spfd_timing(h, sum(1 << k for k in FINE_CLASSES) | P.TIMING_COLD)
        for _ in range(2):
            step(False)
        cold = {name: P.spfd_timing_get(h, k) for k, name in enumerate(P.KERNEL_CLASSES)}
        P.spfd_timing(h, 0)
    psi_out = psi.cpu().numpy()
    # the paper's own criterion (relative residual below 1e-12, Sec. II.A), same hierarchy
    tight = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st12, inf12 = P.spfd_solve(h, P.SolveOptions(1e-12, 500, 0), psi, 1)
        torch.cuda.synchronize()
        tight.append(time.perf_counter() - t0)
    tight_info = {"solve_ms_mean": mean(tight[1:]) * 1e3, "iterations": inf12[0]["iterations"],
                  "rel_residual": inf12[0]["rel_residual"], "status": inf12[0]["status"]}
    ndofs = P.spfd_get_info(h)
    ndofs["hierarchy"] = [P.spfd_level_info(h, lv) for lv in range(ndofs["n_levels"])]
    P.spfd_destroy(h)
    return phases, info, stats, ndofs, psi_out, emag, cold, tight_info


def mean(v):
    return sum(v) / len(v)


def std(v):
    m = mean(v)
    return (sum((x - m) ** 2 for x in v) / max(len(v) - 1, 1)) ** 0.5


def cpu_baseline(w, args, iters_full):
    """The oracle (FP64 Jacobi-PCG on CSR) on a bounded sample of the same solve."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    psi, info = oracle.solve(w.sigma_voxel(), w.h, w.a, tol=args.tol, max_iter=args.cpu_iters, nthreads=threads)
    wall = time.perf_counter() - t0
    per_it = info["t_solve"] / max(info["iterations"], 1)
    est = info["t_assemble"] + per_it * iters_full
    return {"value": est, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": (f"{info['iterations']} Jacobi-PCG iterations of the {info['ndof']}-unknown body solve "
                       f"({wall:.1f} s wall incl. assembly {info['t_assemble']:.1f} s), scaled to the "
                       f"{iters_full} iterations the oracle needs for rel. residual {args.tol:g}"),
            "s_per_iteration": per_it, "iterations_full": iters_full}


def batch_sources(w, lab, P, torch, args):
    """64 coil positions on an 8x8 offset grid sharing one hierarchy (batched solve)."""
    import workloads as W
    dev = lab.device
    offs = W.multi_source_offsets()
    t0 = time.perf_counter()
    gen = W.ShiftedLoopSources(offs)
    t_gen = time.perf_counter() - t0
    s = P.Solver(lab, w.sigma_table, w.h, precision="mixed")
    P.spfd_set_num_rhs(s.handle, len(offs))
    s.nrhs = len(offs)
    abuf = torch.empty((3, w.nz + 1, w.ny + 1, w.nx + 1), dtype=torch.float64, device=dev)
    for k in range(len(offs)):
        abuf.copy_(torch.from_numpy(gen.source(k)))
        P.spfd_set_source(s.handle, k, abuf)
    del gen
    psi = torch.empty((len(offs), w.nz + 1, w.ny + 1, w.nx + 1), dtype=torch.float64, device=dev)
    times, info = [], None
    for rep in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, info = P.spfd_solve(s.handle, P.SolveOptions(args.tol, 500, 0), psi, len(offs))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    its = [i["iterations"] for i in info]
    ok = all(i["status"] == "OK" for i in info)
    # the same sources one at a time through the same hierarchy, for comparison (first 8)
    P.spfd_set_num_rhs(s.handle, 1)
    s.nrhs = 1
    seq = []
    for k in range(8):
        gk = W.rect_loop_edge_potentials(w.nx, w.ny, w.nz, w.h, ((125.0 + 60.0 + offs[k][0]) * w.h[0],
                                         (75.0 + offs[k][1]) * w.h[1], -20.0 * w.h[2]), (150 * w.h[0], 100 * w.h[1]))
        abuf.copy_(torch.from_numpy(gk))
        P.spfd_set_source(s.handle, 0, abuf)
        torch.cuda.synchronize()
        t = time.perf_counter()
        P.spfd_solve(s.handle, P.SolveOptions(args.tol, 500, 0), psi[:1], 1)
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t)
    s.close()
    return {"workload": f"{w.name}, 64 coil positions (8x8 offsets), one hierarchy, mixed precision",
            "sources": len(offs), "batched_solve_s": min(times), "solves_per_s": len(offs) / min(times),
            "iterations_min": min(its), "iterations_max": max(its), "all_ok": ok,
            "sequential_solve_s_per_source": sum(seq) / len(seq),
            "batch_speedup_vs_sequential": (sum(seq) / len(seq)) * len(offs) / min(times),
            "source_generation_s": t_gen}


def scale_1mm(P, torch, args):
    """The same path at 1 mm: ~69.7 M unknowns on one GPU (the paper needed several GPUs, Sec. III)."""
    import oracle
    import workloads as W
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = W.body_phantom_1mm()
    t_gen = time.perf_counter() - t0
    print(f"# 1 mm inputs generated in {t_gen:.1f} s", file=sys.stderr, flush=True)
    lab = torch.from_numpy(w.labels).to(dev)
    a = torch.from_numpy(w.a).to(dev)
    out = {"workload": f"{w.name}: 1 mm body phantom, rectangular loop 0.3x0.2 m at 85 kHz", "generation_s": t_gen}
    psi_mixed = None
    for prec in ("mixed", "fp64"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        s = P.Solver(lab, w.sigma_table, w.h, precision=prec)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t
        s.solve(a, tol=args.tol)                        # warm-up (graph capture)
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            psi, info = s.solve(a, tol=args.tol)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        sinfo = s.info()
        out[prec] = {"solve_ms": min(times) * 1e3, "iterations": info["iterations"],
                     "rel_residual": info["rel_residual"], "status": info["status"], "build_ms": t_build * 1e3,
                     "levels": sinfo["n_levels"], "device_bytes": sinfo["device_bytes"]}
        out["n_dofs"] = sinfo["n_dofs"]
        if prec == "mixed":
            psi_mixed = psi.cpu().numpy()
        s.close()
        del psi
        print(f"# 1 mm {prec}: {out[prec]}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    out["oracle_rel_residual"] = oracle.residual(w.sigma_voxel(), w.h, w.a, psi_mixed)
    out["oracle_residual_s"] = time.perf_counter() - t
    out["mixed_vs_fp64_speedup"] = out["fp64"]["solve_ms"] / out["mixed"]["solve_ms"]
    return out


def fgmres_compare(w, lab, a, P, torch, args):
    """The paper's outer solver (flexible GMRES(30)) against the CG (standard beta, the default, and the
    flexible beta), same FP32 cycle and criterion."""
    s = P.Solver(lab, w.sigma_table, w.h, precision="mixed")
    out = {}
    for name, method, flexible in (("cg", "cg", False), ("cg_flexible", "cg", True), ("fgmres", "fgmres", False)):
        s.solve(a, tol=args.tol, method=method, flexible=flexible)   # warm-up (allocates the basis)
        times, info = [], None
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = s.solve(a, tol=args.tol, method=method, flexible=flexible)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        out[name] = {"solve_ms": min(times) * 1e3, "iterations": info["iterations"],
                     "rel_residual": info["rel_residual"]}
    s.close()
    out["restart"] = 30
    out["fgmres_vs_cg_time"] = out["fgmres"]["solve_ms"] / out["cg"]["solve_ms"]
    return out


def stream_ceiling(torch, P):
    """Best STREAM triad over three 1 GiB float64 arrays (HBM, far beyond the Infinity Cache), GB/s."""
    n = (1 << 30) // 8
    bufs = [torch.ones(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    torch.cuda.synchronize()
    g = P.spfd_stream_triad(bufs[0], bufs[1], bufs[2], reps=5, stream=torch.cuda.current_stream().cuda_stream)
    del bufs
    torch.cuda.empty_cache()
    return g


def adjoint_block(w, lab, a, P, torch):
    """Gradient of J = (sum over body voxels of |E|^8)^(1/8) with respect to the 40 tissue conductivities
    on the benchmark phantom: forward solve, E-field and adjoint solve (FP64 cycle, same hierarchy), timed;
    then central finite differences (h = 1e-6 sigma_t, two rebuilt hierarchies and solves per tissue) on
    all tissues."""
    tol = 1e-13
    s = P.Solver(lab, w.sigma_table, w.h, precision="fp64")

    def J_of(emag):
        return torch.linalg.vector_norm(emag.reshape(-1), ord=8)

    # warm-up of the whole timed block (graph capture; the first torch reduction and power load their kernels)
    p0, _ = s.solve(a, tol=tol)
    e0 = s.efield(a, p0, w.omega)
    J0 = J_of(e0)
    _ = (e0 / J0) ** 7
    del p0, e0, J0, _
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi, info = s.solve(a, tol=tol)
    emag = s.efield(a, psi, w.omega)
    J = J_of(emag)
    gE = (emag / J) ** 7                                  # dJ/d|E_v| (0 in air, where |E| = 0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gvox, gtab, ainfo = s.adjoint(a, psi, w.omega, gE, tol=tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad = gtab[:len(w.sigma_table)]
    fd = []
    base = list(w.sigma_table)
    t3 = time.perf_counter()
    for t in range(1, len(base)):
        hstep = 1e-6 * base[t]
        vals = []
        for sgn in (1.0, -1.0):
            tab = list(base)
            tab[t] += sgn * hstep
            s.set_sigma(tab)
            p_, _ = s.solve(a, tol=tol)
            vals.append(float(J_of(s.efield(a, p_, w.omega))))
        fd.append((vals[0] - vals[1]) / (2 * hstep))
    t4 = time.perf_counter()
    s.close()
    scale = max(abs(grad[t] * base[t]) for t in range(1, len(base)))
    errs = []
    for t in range(1, len(base)):
        if abs(grad[t] * base[t]) >= 1e-3 * scale:
            errs.append(abs(grad[t] - fd[t - 1]) / abs(fd[t - 1]))
    euler = sum(grad[t] * base[t] for t in range(1, len(base))) / sum(abs(grad[t] * base[t]) for t in range(1, len(base)))
    return {"workload": f"{w.name}, J = 8-norm of voxel |E| over the body, 40 tissue conductivities",
            "tol": tol, "forward_solve_and_efield_ms": (t1 - t0) * 1e3, "adjoint_solve_ms": (t2 - t1) * 1e3,
            "forward_iterations": info["iterations"], "adjoint_iterations": ainfo["iterations"],
            "adjoint_status": ainfo["status"], "J": float(J),
            "fd_tissues": len(base) - 1, "fd_compared": len(errs), "fd_max_rel_err": max(errs) if errs else None,
            "fd_median_rel_err": sorted(errs)[len(errs) // 2] if errs else None,
            "fd_s": t4 - t3, "euler_identity_rel": euler}


def batch_phantoms(P, torch, args):
    """16 phantoms of 64^3 ... 192^3 voxels: packed into one handle (one hierarchy, every level kernel
    launched once for all models, one CG per model), against the same phantoms in separate handles
    stepped in lockstep on their own streams, and one after the other."""
    import workloads as W
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    ws = W.uneven_phantoms()
    t_gen = time.perf_counter() - t0
    labs = [torch.from_numpy(w.labels).to(dev) for w in ws]
    srcs = [torch.from_numpy(w.a).to(dev) for w in ws]
    # packed
    torch.cuda.synchronize()
    t = time.perf_counter()
    ms = P.MultiSolver(labs, [w.sigma_table for w in ws], ws[0].h, precision="mixed")
    torch.cuda.synchronize()
    t_build_packed = time.perf_counter() - t
    ms.set_sources(srcs)
    ms.solve(tol=args.tol)                                 # warm-up (graph capture)
    packed = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, pinfo = ms.solve(tol=args.tol)
        torch.cuda.synchronize()
        packed.append(time.perf_counter() - t)
    pdofs = ms.info()["n_dofs"]
    ms.close()
    # separate handles
    solvers = []
    for lab, w in zip(labs, ws):
        st = torch.cuda.Stream(dev)
        solvers.append(P.Solver(lab, w.sigma_table, w.h, precision="mixed", stream=st))
    dofs = sum(s.info()["n_dofs"] for s in solvers)
    P.solve_many(solvers, srcs, tol=args.tol)            # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    psis, infos = P.solve_many(solvers, srcs, tol=args.tol)
    torch.cuda.synchronize()
    t_many = time.perf_counter() - t
    t = time.perf_counter()
    for s_, a_ in zip(solvers, srcs):
        s_.solve(a_, tol=args.tol)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    for s_ in solvers:
        s_.close()
    t_packed = min(packed)
    return {"workload": "16 ellipsoid-union phantoms, cubes of 64^3 ... 192^3 voxels at 2 mm, 4 dipoles each",
            "phantoms": len(ws), "unknowns_total": dofs, "packed_unknowns": pdofs,
            "packed_solve_s": t_packed, "packed_build_s": t_build_packed,
            "packed_iterations": [i["iterations"] for i in pinfo],
            "packed_all_ok": all(i["status"] == "OK" for i in pinfo),
            "lockstep_solve_s": t_many, "sequential_solve_s": t_seq,
            "packed_speedup_vs_lockstep": t_many / t_packed, "packed_speedup_vs_sequential": t_seq / t_packed,
            "lockstep_speedup": t_seq / t_many, "all_ok": all(i["status"] == "OK" for i in infos),
            "iterations": [i["iterations"] for i in infos], "generation_s": t_gen}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2010_12879_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(2)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = W.config(2)
    lab = torch.from_numpy(w.labels).to(dev)
    a = torch.from_numpy(w.a).to(dev).contiguous()
    t_gen = time.perf_counter() - t0
    print(f"# inputs generated in {t_gen:.1f} s", file=sys.stderr, flush=True)

    res = {}
    for prec in args.precisions.split(","):
        res[prec] = run_precision(prec, w, lab, a, args, P, torch)
        ph, info, stats, ninfo = res[prec][:4]
        print(f"# {prec}: solve {mean(ph['solve'])*1e3:.2f} ms, {info['iterations']} it, "
              f"relres {info['rel_residual']:.2e}", file=sys.stderr, flush=True)

    head = "mixed" if "mixed" in res else list(res)[0]
    ph, info, stats, ninfo, psi_head, _, cold, tight = res[head]
    solve_s = mean(ph["solve"])
    # algorithmic HBM bytes of the solve: every kernel class except setup/rhs/efield, per step
    solve_bytes = sum(v["bytes"] for k, v in stats.items() if k not in ("rhs", "efield")) / args.steps
    kernels = {}
    for k, desc in FINE_CLASSES.items():
        v = stats[P.KERNEL_CLASSES[k]]
        if v["timed_launches"] == 0 or v["timed_ms"] <= 0:
            continue
        avg_ms = v["timed_ms"] / v["timed_launches"]
        kernels[desc] = {"avg_us": avg_ms * 1e3, "launches_per_solve": v["launches"] / args.steps,
                         "est_ms_per_solve": avg_ms * v["launches"] / args.steps,
                         "algorithmic_gbs": v["timed_bytes"] / (v["timed_ms"] * 1e-3) / 1e9,
                         "bytes_per_launch": v["timed_bytes"] / v["timed_launches"]}
    if cold:
        for k, desc in FINE_CLASSES.items():
            v = cold[P.KERNEL_CLASSES[k]]
            if desc in kernels and v["timed_launches"] > 0 and v["timed_ms"] > 0:
                c_us = v["timed_ms"] / v["timed_launches"] * 1e3
                kernels[desc]["avg_us_cold"] = c_us
                kernels[desc]["algorithmic_gbs_cold"] = v["timed_bytes"] / (v["timed_ms"] * 1e-3) / 1e9
    ceiling = stream_ceiling(torch, P)
    for d in kernels.values():
        d["frac_of_peak"] = d["algorithmic_gbs"] / HBM_PEAK_GBS
        d["frac_of_stream"] = d["algorithmic_gbs"] / ceiling if ceiling else None
        if "algorithmic_gbs_cold" in d:
            d["frac_of_peak_cold"] = d["algorithmic_gbs_cold"] / HBM_PEAK_GBS
    dom = max(kernels, key=lambda d: kernels[d]["est_ms_per_solve"]) if kernels else None
    achieved = kernels[dom]["algorithmic_gbs"] if dom else None
    dom_class = next((k for k, d in FINE_CLASSES.items() if d == dom), None)
    traffic, prof_us = measured_traffic(PROFILE_OF[dom_class], w.name) if dom_class is not None else (None, None)

    # independent check of the headline solution with the oracle's own assembly
    import oracle
    oracle_relres = oracle.residual(w.sigma_voxel(), w.h, w.a, psi_head)

    out = {
        "metric": "AMG-PCG solve time @8.9M DOF to 1e-8 rel res; HBM GB/s; mixed vs FP64 speedup",
        "value": solve_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mean(ph["step"]) * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64 CG (x, r, A p, dots; search directions p stored in f32), f32 cycle (f16 weights on coarse level 1), "
                  "f64 coarsest" if head == "mixed"
                  else "f64"),
        "data": "synthetic",
        "config": {"workload": f"{w.name}: 2 mm body phantom, {ninfo['n_dofs']} unknowns, 40 tissues, "
                               f"rectangular loop 0.3x0.2 m at 85 kHz",
                   "rel_tol": args.tol, "precision": head, "levels": ninfo["n_levels"]},
        "solve_ms_mean": solve_s * 1e3,
        "solve_ms_std": std(ph["solve"]) * 1e3,
        "iterations": info["iterations"],
        "rel_residual": info["rel_residual"],
        "oracle_rel_residual": oracle_relres,
        "setup_ms": mean(ph["setup"]) * 1e3,
        "rhs_ms": mean(ph["rhs"]) * 1e3,
        "efield_ms": mean(ph["efield"]) * 1e3,
        "solve_hbm_gbs": solve_bytes / solve_s / 1e9,
        "device_bytes": ninfo["device_bytes"],
        "hierarchy": ninfo["hierarchy"],
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "traffic_gbs": traffic / (kernels[dom]["avg_us"] * 1e-6) / 1e9 if traffic else None,
                     "rocprof_median_us": float(prof_us) if prof_us else None,
                     "avg_us": kernels[dom]["avg_us"] if dom else None,
                     "algorithmic_bytes_per_launch": kernels[dom]["bytes_per_launch"] if dom else None,
                     "stream_triad_gbs": ceiling,
                     "frac_of_stream": achieved / ceiling if (achieved and ceiling) else None,
                     "avg_us_cold": kernels[dom].get("avg_us_cold") if dom else None,
                     "frac_cold": kernels[dom].get("frac_of_peak_cold") if dom else None},
        "solve_1e-12": {"mixed" if head == "mixed" else head: tight},
        "finest_level_kernels": kernels,
    }
    if "fp64" in res and head != "fp64":
        ph64, info64, _, _, psi64, _, _, tight64 = res["fp64"]
        out["fp64_solve_ms_mean"] = mean(ph64["solve"]) * 1e3
        out["fp64_iterations"] = info64["iterations"]
        out["mixed_vs_fp64_speedup"] = mean(ph64["solve"]) / solve_s
        import numpy as np
        out["mixed_vs_fp64_rel_diff"] = float(np.linalg.norm(psi_head - psi64) / np.linalg.norm(psi64))
        out["solve_1e-12"]["fp64"] = tight64
        out["solve_1e-12"]["mixed_vs_fp64_speedup"] = tight64["solve_ms_mean"] / tight["solve_ms_mean"]
    if not args.no_adjoint:
        out["adjoint"] = adjoint_block(w, lab, a, P, torch)
        print(f"# adjoint: {out['adjoint']['adjoint_solve_ms']:.1f} ms, fd max rel err "
              f"{out['adjoint']['fd_max_rel_err']:.2e}", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["fgmres_vs_cg"] = fgmres_compare(w, lab, a, P, torch, args)
        print(f"# fgmres: {out['fgmres_vs_cg']['fgmres']}", file=sys.stderr, flush=True)
        out["batch_sources"] = batch_sources(w, lab, P, torch, args)
        print(f"# batch sources: {out['batch_sources']['batched_solve_s']:.3f} s", file=sys.stderr, flush=True)
        out["batch_phantoms"] = batch_phantoms(P, torch, args)
        print(f"# batch phantoms: packed {out['batch_phantoms']['packed_solve_s']*1e3:.2f} ms, lockstep "
              f"{out['batch_phantoms']['lockstep_solve_s']*1e3:.2f} ms", file=sys.stderr, flush=True)
    if args.scale_1mm:
        out["scale_1mm"] = scale_1mm(P, torch, args)
    if args.copy_calibration:
        out["copy_calibration"] = copy_calibration(args.copy_calibration, torch)
    if not args.no_cpu_baseline:
        gold = os.path.join(ROOT, "tests", "golden", f"oracle_body_{args.tol:.0e}.json")
        iters_full = json.load(open(gold))["iterations"] if os.path.exists(gold) else None
        if iters_full:
            out["cpu_baseline"] = cpu_baseline(w, args, iters_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
