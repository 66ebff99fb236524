#!/usr/bin/env python3
"""Benchmark: pressure solves per second on one MI355X.

Workload (default): the 128^3 unit cube with two parallel plates tilted 17
degrees about x and a 0.3-cell gap between them, second-order VEM pressure,
pure Neumann walls, 16 successive right-hand sides from seeded smooth
velocity fields (32 Fourier modes, |k| <= 8, amplitude ~1/|k|).  Each solve
runs the mixed-precision MG-PCG (FP32 V-cycle, FP64 outer CG) to a true
relative residual of 1e-8.

One step = the 16-solve sequence.  Setup (grid construction, hierarchy,
Galerkin products, coarsest factorisation) is outside the timed region; the
inputs are resident in device memory before timing starts.

Also reported: the finest-level fused Chebyshev kernel's average launch time
(HIP events on the solve stream, every launch of the timed region) against
the HBM roofline, and the FP64 oracle's CPU time on a bounded sample.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_cheb_plates128_traffic.json")
# iteration cap of the benchmark's solves (the thin sheet needs several hundred)
MAXIT = 2000
# the stencil kernel, its epilogue and view, and the host code that lays the
# lattice tiles out
LAYOUT_SOURCES = [os.path.join(ROOT, "paper_2607_17725_amd", "csrc", f)
                  for f in ("sell.hip", "epilogues.hpp", "kernels.hpp", "setup_host.cpp")]


def layout_hash():
    """sha256 over the kernel, data-layout and option-default sources the counter figures depend on."""
    import hashlib
    h = hashlib.sha256()
    for f in LAYOUT_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when they were taken on other kernel or layout sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != layout_hash() or rec.get("workload") != workload:
        return None
    return rec.get("traffic_bytes_per_launch")


def host_description():
    """CPU model, logical CPUs and RAM of the machine the baseline runs on."""
    model, ram = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_bytes": ram}


def cpu_baseline(name, N, target, seconds=20.0):
    """The oracle's FP64 MG-PCG on a reduced instance of the workload, on one core.

    The oracle runs the same algorithm on the same kind of hierarchy (V(1,1)
    degree-5 Chebyshev, dense coarsest solve, flexible PCG) with SciPy CSR
    matvecs, whose cost is proportional to the stored nonzeros of the
    hierarchy.  Its measured time per PCG iteration at N is scaled by the
    ratio of hierarchy nonzeros (sum over levels of nnz(A_l) + 2 nnz(P_l))
    and multiplied by the GPU's measured iteration count at the full size:
    an extrapolation, stated as such in the sample field.
    """
    code = f"""
import json, os, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
import synth
from oracle.problem import Problem
w = synth.get_config({name!r}, N={N})
pb = Problem(w)
n = pb.K.shape[0]
u = synth.fourier_field(pb.vertices, w.field_seed).ravel()
b = pb.rhs(u)
mg = pb.mg
work = sum(A.nnz for A in mg.A) + 2 * sum(P.nnz for P in mg.P)
t0 = time.perf_counter(); k = 0; its = []
while True:
    p, it, hist = pb.solve_mgpcg(b=b, tol=w.tol)
    its.append(it); k += 1
    if time.perf_counter() - t0 > {seconds}:
        break
dt = (time.perf_counter() - t0) / k
print(json.dumps({{"n_dof": int(n), "s_per_solve": dt, "iterations": its[0], "solves": k, "work": int(work)}}))
"""
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[v] = "1"
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        log("cpu baseline failed: " + out.stderr[-2000:])
        return None
    r = json.loads(out.stdout.strip().splitlines()[-1])
    s_iter = r["s_per_solve"] / max(r["iterations"], 1)
    s_solve = s_iter * (target["work"] / r["work"]) * target["iterations"]
    host = host_description()
    return {
        "value": 1.0 / s_solve,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle FP64 MG-PCG on the same geometry at N={N} ({r['n_dof']} DOFs, {r['iterations']} "
                   f"iterations to tol 1e-8, {r['s_per_solve']:.3f} s/solve over {r['solves']} solves, "
                   f"{s_iter * 1e3:.1f} ms/iteration on one core); extrapolated to the full workload by the "
                   f"hierarchy nonzeros ({target['work']:.4g} / {r['work']:.4g}) times the GPU's "
                   f"{target['iterations']} iterations"),
        "iterations_sample": r["iterations"],
        "iterations_full": target["iterations"],
        "host": host,
    }


def time_smoke_step(grid, hier, w, stream):
    """One simulation step of Algorithm 1 with eight particles per background
    cell, each phase timed on its own (synchronised), after one untimed step."""
    import numpy as np
    import torch
    import synth
    from paper_2607_17725_amd import fvem
    x, u, rho, temp = synth.seeded_particles(w.N, seed=0)
    tr = fvem.Transport(grid, stream=stream)
    X = torch.as_tensor(x, device="cuda")
    ghost = (tr.locate(X) < 0).to(torch.uint8)
    g = ghost.cpu().numpy().astype(bool)
    u[g], rho[g], temp[g] = 0.0, 0.0, 0.0
    U, R, Tm = (torch.as_tensor(np.ascontiguousarray(a), device="cuda") for a in (u, rho, temp))
    dt, a_flip, alpha, beta = 0.01, 0.95, 0.5, 2.0
    fvem.smoke_step(hier, tr, X.clone(), U.clone(), R, Tm, ghost, dt, a_flip, alpha, beta)
    torch.cuda.synchronize()
    ms = {}

    def timed(name, fn):
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ms[name] = (time.perf_counter() - t0) * 1e3
        return r

    f = torch.cat([U, R[:, None], Tm[:, None]], dim=1).contiguous()
    fv = timed("p2g", lambda: tr.p2g(X, f))
    u_grid = fv[:, :3].contiguous().view(-1)
    u_forced = timed("buoyancy", lambda: tr.buoyancy(fv, alpha, beta, dt))
    s_new, st = timed("projection", lambda: hier.project_velocity(u_forced, tol=w.tol))
    s_old = timed("pi1", lambda: hier.apply(fvem.OP_PI1, u_grid))
    timed("g2p", lambda: tr.g2p(X, ghost, U, s_new, s_old, a_flip))
    _, n_sub = timed("advect", lambda: tr.advect(X, ghost, s_new, dt))
    out = {"particles": int(len(x)), "ghosts": int(g.sum()), "dt": dt, "substeps": n_sub,
           "projection_iterations": st["iterations"], "ms": ms, "ms_total": sum(ms.values())}
    log(f"smoke step: {len(x)} particles, " + ", ".join(f"{k} {v:.2f} ms" for k, v in ms.items()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--N", type=int, default=None, help="background resolution override")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the untimed-for-value comparisons (plain FP64 MG-PCG, adjoint solves)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-N", type=int, default=16)
    ap.add_argument("--rhs", type=int, default=16, help="right-hand sides per step (profiling runs use fewer)")
    ap.add_argument("--max-templates", type=int, default=0,
                    help="value templates per operator (0: library default, <0: none)")
    ap.add_argument("--small-level-rows", type=int, default=0,
                    help="levels up to this many rows use the row-split SpMV (0: library default, <0: never)")
    ap.add_argument("--lattice-min", type=float, default=0.0,
                    help="smallest share of stencil rows for the lattice layout of a level (0: library default)")
    ap.add_argument("--prolongation", choices=["diffusion-free", "naive"], default="diffusion-free",
                    help="naive: the Sec. 4 ablation, with coarse operators from general sparse products")
    ap.add_argument("--smoke-step", action="store_true",
                    help="also time one simulation step (P2G, buoyancy, projection, G2P, advection) of 8 particles "
                         "per background cell")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB buffer 3 times (reference kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("FVEM_VERBOSE", "1")   # setup progress lines on stderr
    import numpy as np
    import torch
    import synth
    from paper_2607_17725_amd import fvem

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = synth.get_config(args.config, N=args.N)
    V, F = w.mesh()
    log(f"workload {w.name}: N={w.N} k={w.k} levels={w.levels} triangles={len(F)}")
    t0 = time.perf_counter()
    naive = args.prolongation == "naive"
    grid = fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top, naive_prolongation=naive)
    t_grid = time.perf_counter() - t0
    log(f"grid built in {t_grid:.1f} s: {grid.n_dof} DOFs, {grid.n_vert} vertices, {grid.n_trees} cut cells")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    hier = fvem.Hierarchy(grid, stream=stream, small_level_rows=args.small_level_rows,
                          max_templates=args.max_templates, galerkin_general=naive,
                          lattice_min_fraction=args.lattice_min)
    torch.cuda.synchronize()
    t_hier = time.perf_counter() - t0
    n0 = hier.n_dof
    stor = hier.level_storage(0)
    nnz0 = stor["nnz"]
    log(f"hierarchy built in {t_hier:.1f} s: {hier.n_levels} levels, nnz(K)={nnz0}, "
        f"device memory {hier.device_bytes / 2**30:.1f} GiB")

    if args.copy_calibration:
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 3 copies of 1 GiB done")
    seeds = w.rhs_seeds()[:args.rhs]
    U = [torch.as_tensor(synth.fourier_field(grid.vertices, s).ravel(), device="cuda") for s in seeds]
    p = torch.empty(n0, dtype=torch.float64, device="cuda")
    prec = fvem.PREC_MIXED if args.precision == "mixed" else fvem.PREC_FP64
    torch.cuda.synchronize()

    def step(profile):
        st_all = []
        for u in U:
            _, st = hier.solve(u, out=p, tol=w.tol, precision=prec, profile=profile, maxit=MAXIT)
            st_all.append(st)
        return st_all

    for i in range(args.warmup):
        st = step(False)
        log(f"warmup step {i}: iterations {[s['iterations'] for s in st]}")
    # the timed steps time every V-cycle with HIP events (profile level 2:
    # the V-cycles still replay as graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats += step(2)
        log(f"timed step {i} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = len(U) * args.steps
    value = solves / dt
    its = [s["iterations"] for s in stats]
    res = [s["rel_residual"] for s in stats]
    # per-launch times of the finest Chebyshev step come from an untimed pass
    # over the first right-hand sides with every finest-level launch timed
    # (profile level 1, V-cycles kernel by kernel)
    kstats = []
    for u in U[:min(len(U), 2)]:
        kstats.append(hier.solve(u, out=p, tol=w.tol, precision=prec, profile=1, maxit=MAXIT)[1])
    ms_k = sum(s["ms_fine_smoother"] for s in kstats)
    n_k = sum(s["n_fine_smoother"] for s in kstats)
    avg_ms = ms_k / max(n_k, 1)
    # the lattice stencil launch inside each finest Chebyshev step: the
    # dominant kernel when the finest operator has stencil rows
    ms_s = sum(s["ms_fine_stencil"] for s in kstats)
    n_s = sum(s["n_fine_stencil"] for s in kstats)
    st0 = hier.level_stencil(0)
    # algorithmic bytes of one stencil launch: five FP32 vector streams per
    # stencil row (x, b, d read; d, x_out written; D^-1 is the class's) and a
    # tile id plus 8 mask words per tile; the class tables and halo re-reads
    # of x are cache traffic and are not counted
    st_bytes = 20 * st0["rows"] + 68 * st0["tiles"]
    st_ms = ms_s / max(n_s, 1)
    st_gbs = st_bytes / (st_ms * 1e-3) / 1e9 if n_s else 0.0
    # whole V-cycles (all levels, transfers and the coarsest solve), timed
    # with HIP events around each application of the preconditioner
    ms_v = sum(s["ms_vcycle"] for s in stats)
    n_v = sum(s["n_vcycle"] for s in stats)
    avg_v = ms_v / max(n_v, 1)
    vbytes = hier.vcycle_bytes(prec)
    v_gbs = vbytes / (avg_v * 1e-3) / 1e9
    # algorithmic bytes of one finest Chebyshev step: the stored operator once
    # (a 16-bit column code per nonzero of coded slices plus their block
    # tables, an int32 column per nonzero elsewhere; an FP32 value per
    # nonzero of rows that store values; an int32 template id per row that
    # reads a shared value template) and six FP32 vector streams per row (x,
    # b, D^-1, d read; d, x_out written; stencil rows take D^-1 from their
    # class); slice padding, the cache-resident template table and cache
    # misses are not counted
    matrix_bytes = hier.level_bytes(0, fvem.PREC_MIXED)
    bytes_per_launch = matrix_bytes + 24 * n0 - 4 * st0["rows"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    log(f"{solves} solves in {dt:.2f} s: {value:.3f} solves/s, iterations {min(its)}-{max(its)}, "
        f"max residual {max(res):.2e}; fine Chebyshev step {avg_ms:.3f} ms avg over {n_k} launches "
        f"= {achieved:.0f} GB/s (stencil launch {st_ms:.3f} ms = {st_gbs:.0f} GB/s); "
        f"V-cycle {avg_v:.3f} ms avg over {n_v} = {v_gbs:.0f} GB/s "
        f"({vbytes / 1e9:.3f} GB)")

    extra = {}
    if not args.no_reference:
        # beside the value: the same right-hand sides through the plain FP64
        # MG-PCG, and the adjoint solve (B^T K^+ of a seeded pressure
        # sensitivity) in the benchmark's precision, both to the same tolerance
        prec_save = prec
        prec = fvem.PREC_FP64
        hier.solve(U[0], out=p, tol=w.tol, precision=prec, maxit=MAXIT)   # untimed: captures the FP64 graphs
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st64 = step(False)
        torch.cuda.synchronize()
        d64 = time.perf_counter() - t1
        prec = prec_save
        extra["fp64_reference"] = {"solves_per_s": len(U) / d64,
                                   "iterations": [s["iterations"] for s in st64],
                                   "max_rel_residual": max(s["rel_residual"] for s in st64)}
        log(f"FP64 reference: {len(U) / d64:.3f} solves/s")
        # error of the mixed-precision pressure against the FP64 one on the
        # first right-hand sides (untimed), at the benchmark tolerance and, for
        # cache-resident sizes, also at 1e-10
        tols = [w.tol] + ([1e-10] if n0 <= 2_000_000 and w.tol > 1e-10 else [])
        p64 = torch.empty_like(p)
        errs = []
        for tol in tols:
            for u in U[:2]:
                _, sm = hier.solve(u, out=p, tol=tol, precision=fvem.PREC_MIXED, maxit=MAXIT)
                _, sd = hier.solve(u, out=p64, tol=tol, precision=fvem.PREC_FP64, maxit=MAXIT)
                rel = float(torch.linalg.vector_norm(p - p64) / torch.linalg.vector_norm(p64))
                errs.append({"tol": tol, "iterations_mixed": sm["iterations"], "iterations_fp64": sd["iterations"],
                             "rel_l2_mixed_vs_fp64": rel})
                log(f"tol {tol:g}: mixed {sm['iterations']} its, FP64 {sd['iterations']} its, "
                    f"|p_mixed - p_fp64| / |p_fp64| = {rel:.2e}")
        extra["fp64_reference"]["error_table"] = errs
        G = [torch.as_tensor(np.random.default_rng(500 + k).standard_normal(n0), device="cuda")
             for k in range(len(U))]
        gu = torch.empty(3 * grid.n_vert, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sta = [hier.solve_adjoint(gp, out=gu, tol=w.tol, precision=prec, maxit=MAXIT)[1] for gp in G]
        torch.cuda.synchronize()
        dad = time.perf_counter() - t1
        extra["adjoint"] = {"solves_per_s": len(G) / dad, "iterations": [s["iterations"] for s in sta],
                            "max_rel_residual": max(s["rel_residual"] for s in sta),
                            "input": "N(0,1) pressure sensitivities, seeds 500+"}
        log(f"adjoint: {len(G) / dad:.3f} solves/s")

    if args.smoke_step:
        extra["smoke_step"] = time_smoke_step(grid, hier, w, stream)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle at N={args.cpu_N}")
        work = sum(hier.level_storage(l)["nnz"] for l in range(hier.n_levels)) + \
            2 * sum(hier.transfer_nnz(l) for l in range(hier.n_levels - 1))
        cpu = cpu_baseline(args.config, args.cpu_N, {"work": work, "iterations": max(its)})

    line = {
        "metric": "pressure solves/s to 1e-8 rel. residual @128^3 VEM; V-cycle HBM GB/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == fvem.PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: {w.description}; {len(U)} RHS per step, "
                         f"tol {w.tol}, {args.precision} precision, {args.prolongation} prolongation"),
            "N": w.N, "k": w.k, "levels": hier.n_levels, "n_dof": n0, "nnz_K": nnz0,
            "rhs_per_step": len(U), "iterations": [min(its), max(its)],
            "level_nnz": [hier.level_storage(l)["nnz"] for l in range(hier.n_levels)],
            "level_templated_rows": [hier.level_storage(l)["rows_templated"] for l in range(hier.n_levels)],
            "level_rows": [hier.level_rows(l) for l in range(hier.n_levels)],
            "stencil_level0": hier.level_stencil(0),
            "device_memory": hier.memory_breakdown(),
            "max_rel_residual": max(res), "setup_s": t_grid + t_hier,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("stencil_kernel<float, float, EpiCheb<float>>: the lattice stencil rows of the finest "
                       "Chebyshev step (FP32, x staged in LDS by class, fused update)"),
            "achieved": st_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": st_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(f"{w.name}@{w.N}"),
            "avg_launch_ms": st_ms,
            "launches": n_s,
            "algorithmic_bytes_per_launch": st_bytes,
            "stencil": st0,
            "fine_step": {"kernels": "stencil launch + sliced-ELLPACK launch for the other rows",
                          "avg_ms": avg_ms, "launches": n_k, "algorithmic_bytes": bytes_per_launch,
                          "achieved": achieved, "storage": stor},
        },
        "cpu_baseline": cpu,
        "vcycle_hbm": {
            "achieved": v_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": v_gbs / HBM_PEAK_GBS,
            "avg_ms": avg_v, "count": n_v, "algorithmic_bytes": vbytes,
            "level_bytes": [hier.level_bytes(l, prec) for l in range(hier.n_levels)],
            "transfer_bytes": [hier.transfer_storage(l, prec) for l in range(hier.n_levels - 1)],
        },
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
