"""Benchmark of the dense OMM CG path on one MI355X.

Workload (default): 1000 atoms on a 10x10x10 lattice (a = 3.0 bohr, r_c = 8 bohr), 13 orbitals
per atom -> N = 13000 basis orbitals, M = 2000 Wannier functions, eta = 0, tau = 10, synthetic
finite-range S/T/H (seeded). A "step" is one CG line search (gradient, preconditioning,
Polak-Ribiere direction, operator products, projections, quartic coefficients + line minimum,
updates + energy + stopping test); inputs are resident in HBM before the timed region.

Prints ONE JSON line: the headline value is mixed-precision (BF16x3 MFMA, FP64 reductions)
line searches per second; it also carries the FP64 rate, time to a converged energy for both,
the roofline of the dominant kernel and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "OMM CG iters/sec + time-to-converged E (1e-8 rel) vs FP64, N=13000 M=2000"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
WORKLOADS = {
    "c3": "1000-atom 13-orbital finite-range basis (10x10x10, a=3.0, rc=8): N=13000, M=2000, eta=0, tau=10",
    "c2": "512-atom 4-orbital finite-range basis (8x8x8, a=2.5, rc=6): N=2048, M=384, eta=0.5, tau=10",
    "c5": "1024-atom 4-orbital finite-range basis (16x8x8, a=2.5, rc=6): N=4096, M=768, eta=0.5, tau=10",
    "c1": "32-atom 4-orbital finite-range basis (4x4x2, a=2.5, rc=6): N=128, M=24, eta=0.5, tau=10",
    "c4": "64 independent 4-orbital systems, 64-512 atoms (N=256..2048, M=round(3N/16)), "
          "eta=0.5, tau=10, FP32 MFMA grouped launches + hipGraph; cold solve then warm start "
          "after H += 1e-3 sym(N(0,1))",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def reference_energy(name, s):
    """Closed-form minimum stored by tests/golden/make_golden.py, if it matches these inputs."""
    f = ROOT / "tests" / "golden" / f"{name}_reference.json"
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    tr, sm = float(np.real(np.trace(s.H))), float(np.real(np.sum(s.S)))
    if abs(d["trace_H"] - tr) > 1e-9 * abs(d["trace_H"]) or \
            abs(d["sum_S"] - sm) > 1e-9 * abs(d["sum_S"]):
        return None
    return float(d["E_min"])


def measured_traffic(workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None when the GEMM sources changed since the counters were taken."""
    import hashlib

    f = ROOT / "profiles" / f"traffic_{workload}_{precision}.json"
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    h = hashlib.sha256()
    for src in d["gemm_sources"]:
        h.update((ROOT / src).read_bytes())
    if h.hexdigest()[:16] != d["gemm_sources_sha256_16"]:
        return None
    return d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]


def time_iterations(OMM, torch, dev, s, prec, steps, warmup, prof_steps, refine=False, resync=20,
                    flavour="dense", sparse=False):
    solver = OMM(s.N, s.M, precision=prec, refine=refine, resync=resync, flavour=flavour,
                 sparse=sparse)
    solver.set_HS(dev["H"], dev["S"], dev["T"])
    t0 = time.perf_counter()
    solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)  # setup only
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    solver.iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.iterate(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = None
    if prof_steps > 0:
        solver.set_profiling(True)
        solver.iterate(prof_steps)
        torch.cuda.synchronize()
        stages, n = solver.stage_times()
        stages = {k: v / max(n, 1) for k, v in stages.items()}
        solver.set_profiling(False)
    solver.close()
    return wall, setup_s, stages


def time_to_converged(OMM, torch, dev, s, prec, E_ref, target, max_iter, resync, flavour="dense",
                      sparse=False):
    """Wall time from omm_minimize entry (P already built) to the first FP64-exact energy within
    `target` of the closed-form minimum E_ref. The run proceeds in chunks of `resync` line
    searches (omm_iterate) and stops at the first chunk that reaches the target."""
    mixed = prec != "fp64"
    solver = OMM(s.N, s.M, precision=prec, refine=True, resync=resync, flavour=flavour,
                 sparse=sparse)
    solver.set_HS(dev["H"], dev["S"], dev["T"])
    t0 = time.perf_counter()
    solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)  # builds P (or L)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    log_every = max(1, 200 // resync)
    t0 = time.perf_counter()
    solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)  # setup: a2 from C0
    done, hit, err, chunks = 0, None, float("inf"), 0
    while done < max_iter:
        solver.iterate(resync, tol=0.0)
        done += resync
        chunks += 1
        E = solver.checkpoints()[1][-1] if mixed else solver.energy_trace()[-1]
        err = abs(E - E_ref) / abs(E_ref)
        if chunks % log_every == 0:
            log(f"  {prec}: {done} line searches, rel err {err:.3e}, {time.perf_counter() - t0:.1f}s")
        if err <= target:
            hit = done
            break
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    solver.close()
    out = {"precision": prec + ("+fp64-state" if mixed else ""), "target": target,
           "line_searches": hit, "time_to_target_s": total if hit else None,
           "rel_err_at_stop": err, "first_call_with_precon_s": t_first,
           "checked_every": resync}
    if mixed:
        out["resync_every"] = resync
    return out


def complex_bench(args, torch):
    """Complex Hermitian problems (k-points) through OMMComplex / OMMBatchComplex: the 1024-atom
    16x8x8 lattice (4 orbitals per atom) made periodic along x at k = 0.3 (complex N = 4096,
    M = 768; real embedding 8192 x 1536), BF16-scheme and FP64 rates and time to 1e-8 of the
    closed form; and a batch of four k-points of the 512-atom 8x8x8 lattice (complex N = 2048,
    M = 384; FP32 grouped launches) solved to tol 1e-10."""
    from paper_1312_1549_amd import OMMBatchComplex, OMMComplex
    from synth import bloch_system, complex_start_coefficients

    k = 0.3
    log(f"complex: generating c5 at k={k}")
    s = bloch_system("c5", k, 0)
    C0 = complex_start_coefficients(s.S, s.M, 1)
    out = {"workload": f"1024-atom lattice (16x8x8, a=2.5, rc=6) periodic along x, k={k}: complex "
                       f"N={s.N}, M={s.M} (real embedding {2 * s.N} x {2 * s.M})",
           "eta": s.eta, "tau": s.tau}

    def solver_for(prec):
        sol = OMMComplex(s.N, s.M, precision=prec, refine=True, resync=args.resync)
        sol.set_HS(s.H, s.S, s.T)
        sol.minimize(C0, eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)
        torch.cuda.synchronize()
        return sol

    for prec, steps in (("bf16x3", args.steps), ("fp64", max(3, args.steps // 4))):
        sol = solver_for(prec)
        sol.iterate(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.iterate(steps)
        torch.cuda.synchronize()
        out[f"{prec}_iters_per_s"] = steps / (time.perf_counter() - t0)
        sol.close()
        log(f"complex {prec}: {out[prec + '_iters_per_s']:.2f} iters/s")
    E_ref = reference_energy("c5_k0.3", s)
    if E_ref is not None and not args.no_converge:
        conv = {}
        for prec in ("bf16x3", "fp64"):
            sol = solver_for(prec)
            t0 = time.perf_counter()
            sol.minimize(C0, eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)
            done, hit, err = 0, None, float("inf")
            while done < args.max_iter:
                sol.iterate(args.resync, tol=0.0)
                done += args.resync
                E = sol.checkpoints()[1][-1] if prec != "fp64" else sol.energy_trace()[-1]
                err = abs(E - E_ref) / abs(E_ref)
                if err <= 1e-8:
                    hit = done
                    break
            torch.cuda.synchronize()
            conv[prec] = {"line_searches": hit, "time_to_target_s": time.perf_counter() - t0 if hit
                          else None, "rel_err_at_stop": err, "checked_every": args.resync}
            sol.close()
            log(f"complex {prec}: 1e-8 after {hit} line searches")
        conv["E_ref"] = E_ref
        out["time_to_converged_1e-8"] = conv
    # a k-point batch: four k-points of the 8x8x8 lattice solved together
    ks = (0.0, 0.1, 0.2, 0.3)
    log("complex: k-point batch, 8x8x8 lattice x 4 k-points")
    systems = [bloch_system("c2", kk, 0) for kk in ks]
    b = OMMBatchComplex([x.N for x in systems], [x.M for x in systems])
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
    C0s = [complex_start_coefficients(x.S, x.M, 10 + i) for i, x in enumerate(systems)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.minimize(C0s, [x.eta for x in systems], [x.tau for x in systems], 1e-10, 5000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    its = b.iterations()
    out["kpoint_batch"] = {"workload": f"512-atom lattice (8x8x8, a=2.5, rc=6) periodic along x, "
                                       f"complex N=2048, M=384, at k = {list(ks)}",
                           "line_searches": int(its.sum()), "wall_s": wall,
                           "line_searches_per_s": float(its.sum()) / wall,
                           "precision": "fp32 products, fp64 reductions"}
    b.close()
    return out


def cpu_baseline(s, C0, iters):
    from oracle import omm as oracle

    try:
        from threadpoolctl import threadpool_info

        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    P = oracle.preconditioner(s.S, s.T, s.tau)  # setup, not timed
    stamps = []
    oracle.minimize(s.H, s.S, s.T, C0, s.eta, s.tau, 0.0, iters, P=P, use_given_P=True,
                    callback=lambda k, E: stamps.append(time.perf_counter()))
    per = (stamps[-1] - stamps[0]) / iters
    return {"value": 1.0 / per, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{iters} FP64 line searches of the NumPy oracle on the same N={s.N}, "
                      f"M={s.M} inputs after its untimed setup (P inverse, initial products); "
                      f"host BLAS threads={threads}, os.cpu_count()={os.cpu_count()}"}


def summarize_rocprof(trace_csv, top=12):
    """Per (kernel, grid) launch statistics from a rocprofv3 --kernel-trace CSV."""
    import csv
    from collections import defaultdict

    groups = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        name = r["Kernel_Name"]
        grid = (r.get("Grid_Size_X") or r.get("Grid_Size"), r.get("Grid_Size_Y"), r.get("Grid_Size_Z"))
        groups[(name, grid)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in groups.values())
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]
    out = [f"{'calls':>6} {'avg_us':>10} {'share':>7}  grid(x,y,z)  kernel"]
    for (name, grid), d in rows:
        short = name.replace("omm::gemm_detail::", "").replace("omm::", "")
        short = short.replace("(anonymous namespace)::", "").split("(")[0]
        out.append(f"{len(d):>6} {sum(d) / len(d) / 1e3:>10.1f} {100 * sum(d) / total:>6.2f}%  "
                   f"{','.join(str(g) for g in grid)}  {short}")
    return "\n".join(out)


def batched_bench(args):
    """Batched systems: cold solve to tol 1e-10, then an SCF-like warm start."""
    import torch
    from paper_1312_1549_amd import OMMBatch, flops_per_iteration
    from synth import batched_systems, perturb_hamiltonian, start_coefficients

    log("generating 64 systems")
    systems = batched_systems(count=64)
    C0s = [start_coefficients(x.S, x.M, 1000 + i) for i, x in enumerate(systems)]
    b = OMMBatch([x.N for x in systems], [x.M for x in systems])
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
    etas, taus = [x.eta for x in systems], [x.tau for x in systems]
    b.minimize(C0s, etas, taus, 1e-10, 10)  # warm-up: setup, autotune, graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = b.minimize(C0s, etas, taus, 1e-10, 5000)
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
    it = b.iterations()
    flops = sum(int(k) * flops_per_iteration(x.N, x.M) for k, x in zip(it, systems))
    log(f"cold: {cold:.2f}s, {int(it.sum())} line searches, max {int(it.max())}")
    Cs = [b.get_C(i) for i in range(len(systems))]
    for i, x in enumerate(systems):
        b.set_HS(i, perturb_hamiltonian(x.H, 200 + i), x.S, x.T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.minimize(Cs, etas, taus, 1e-10, 5000)
    torch.cuda.synchronize()
    warm = time.perf_counter() - t0
    itw = b.iterations()
    return {
        "metric": "batched OMM CG line searches/sec (64 systems, N=256..2048)",
        "value": float(it.sum()) / cold, "unit": "line searches/s", "n_gpus": 1,
        "steps": int(it.max()), "warmup": 10, "ms_per_step": 1e3 * cold / max(1, int(it.max())),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic", "config": {"workload": WORKLOADS["c4"]},
        "systems_per_s": len(systems) / cold, "algorithmic_tflops": flops / cold / 1e12,
        "cold_s": cold, "cold_line_searches_total": int(it.sum()), "status": int(st),
        "warm_s": warm, "warm_line_searches_total": int(itw.sum()),
        "warm_line_searches_max": int(itw.max()),
    }


def copy_kernel(nbytes):
    """A plain device copy of a known size (reads and writes `nbytes` each): the calibration
    kernel for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    b = a.clone()
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "check": float(b[-1])}))


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "--summarize-rocprof":
        print(summarize_rocprof(sys.argv[2]))
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--copy-kernel":
        copy_kernel(int(sys.argv[2]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=80)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-converge", action="store_true", help="skip time-to-converged runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison rate")
    ap.add_argument("--no-cholesky", action="store_true",
                    help="skip the Cholesky-reduced flavour's rate and time to converged")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the block-sparse operator products' rate and time to converged")
    ap.add_argument("--no-complex", action="store_true",
                    help="skip the complex Hermitian (k-point) rates and time to converged")
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--resync", type=int, default=80)
    ap.add_argument("--cpu-iters", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "c4":
        print(json.dumps(batched_bench(args)), flush=True)
        return

    import torch
    from paper_1312_1549_amd import OMM, flops_per_iteration
    from synth import config_system, start_coefficients

    log(f"generating {args.workload}")
    s = config_system(args.workload, 0)
    C0 = start_coefficients(s.S, s.M, 1)
    log(f"N={s.N} M={s.M} generated")
    dev = {k: torch.from_numpy(v).cuda() for k, v in (("H", s.H), ("S", s.S), ("T", s.T), ("C0", C0))}
    torch.cuda.synchronize()

    flops = flops_per_iteration(s.N, s.M, preconditioned=s.tau > 0)
    prof_steps = min(args.steps, 10)
    mixed = args.precision != "fp64"
    log(f"timing {args.precision}: warmup {args.warmup}, steps {args.steps}")
    wall, setup_s, stages = time_iterations(OMM, torch, dev, s, args.precision, args.steps,
                                            args.warmup, prof_steps, refine=mixed,
                                            resync=args.resync)
    ips = args.steps / wall
    log(f"{args.precision}: {ips:.3f} iters/s ({1e3 * wall / args.steps:.2f} ms/iter)")
    pure = None
    if mixed:
        wp, _, stp = time_iterations(OMM, torch, dev, s, args.precision, args.steps, 2, 0)
        pure = args.steps / wp
        log(f"{args.precision} with FP32 state, no resync: {pure:.3f} iters/s")

    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        log("timing fp64")
        w64, _, st64 = time_iterations(OMM, torch, dev, s, "fp64", max(3, args.steps // 4), 1, 3)
        fp64 = {"iters_per_s": max(3, args.steps // 4) / w64, "stages_ms": st64}
        log(f"fp64: {fp64['iters_per_s']:.3f} iters/s")

    chol = None
    if not args.no_cholesky and mixed:
        log(f"timing the Cholesky-reduced flavour ({args.precision})")
        wc, setup_c, stc = time_iterations(OMM, torch, dev, s, args.precision, args.steps,
                                           args.warmup, prof_steps, refine=True,
                                           resync=args.resync, flavour="cholesky")
        chol = {"iters_per_s": args.steps / wc, "setup_s": setup_c, "stages_ms": stc,
                "note": "Cholesky-reduced flavour: S = L L^T once, no S or P products per line "
                        "search; its iterates are those of P = S^-1 (tau = inf), not of tau = "
                        f"{s.tau}"}
        log(f"cholesky: {chol['iters_per_s']:.3f} iters/s, setup {setup_c:.2f} s")

    sparse = None
    if not args.no_sparse and args.precision == "bf16x3":
        log("timing block-sparse operator products (bf16x3)")
        wsp, _, stsp = time_iterations(OMM, torch, dev, s, args.precision, args.steps, args.warmup,
                                       prof_steps, refine=True, resync=args.resync, sparse=True)
        sparse = {"iters_per_s": args.steps / wsp, "stages_ms": stsp,
                  "note": "[HD|SD] over the non-zero 32-deep K blocks of each 256-column tile of Hs "
                          "and S only; same iterates as the dense products (bitwise, same tile)"}
        log(f"sparse products: {sparse['iters_per_s']:.3f} iters/s")

    op_ms = stages["operator_products"]
    op_flops = 2 * 2.0 * s.M * s.N * s.N
    achieved = op_flops / (op_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(args.workload, args.precision),
                "kernel": f"[HD|SD] = D [Hs|S] ({args.precision}), {op_ms:.3f} ms/launch, "
                          f"{op_flops:.4g} algorithmic flops/launch"}
    if args.precision == "bf16x3":
        # the search direction is bf16-exact, so each product is two bf16 MFMA passes
        # (D_hi B_lo + D_hi B_hi): MFMA work is twice the algorithmic flops
        roofline["hardware_frac"] = 2 * achieved / peak

    result = {
        "metric": METRIC, "value": ips, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "N": s.N, "M": s.M, "eta": s.eta,
                   "tau": s.tau, "seed": 0, "c0_seed": 1},
        "algorithmic_tflops": flops * ips / 1e12,
        "scheme": (f"{args.precision} MFMA products, FP64 CG state and reductions, FP64 "
                   f"resynchronization every {args.resync} line searches" if mixed else
                   "FP64 MFMA products and FP64 reductions"),
        "setup_s": setup_s,
        "stages_ms": stages,
        "roofline": roofline,
    }
    if pure:
        result["fp32_state_no_resync_iters_per_s"] = pure
    if chol:
        result["cholesky_flavour"] = chol
    if sparse:
        result["sparse_operator_products"] = sparse
    if fp64:
        result["fp64_iters_per_s"] = fp64["iters_per_s"]
        result["fp64_stages_ms"] = fp64["stages_ms"]
        result["speedup_vs_fp64_per_iter"] = ips / fp64["iters_per_s"]

    if not args.no_converge:
        E_ref = reference_energy(args.workload, s)
        if E_ref is None:
            log("no stored closed-form energy for these inputs: skipping time-to-converged")
        else:
            conv = {}
            log("time to converged: fp64 (1e-8)")
            conv["fp64_1e-8"] = time_to_converged(OMM, torch, dev, s, "fp64", E_ref, 1e-8,
                                                  args.max_iter, args.resync)
            if args.precision != "fp64":
                log(f"time to converged: {args.precision} with FP64 state (1e-8)")
                conv[args.precision + "_1e-8"] = time_to_converged(
                    OMM, torch, dev, s, args.precision, E_ref, 1e-8, args.max_iter, args.resync)
                a = conv["fp64_1e-8"].get("time_to_target_s")
                b = conv[args.precision + "_1e-8"].get("time_to_target_s")
                if a and b:
                    conv["mixed_speedup_1e-8"] = a / b
                if sparse:
                    log(f"time to converged: block-sparse operator products, {args.precision} (1e-8)")
                    sparse["time_to_converged_1e-8"] = time_to_converged(
                        OMM, torch, dev, s, args.precision, E_ref, 1e-8, args.max_iter,
                        args.resync, sparse=True)
                if chol:
                    log(f"time to converged: Cholesky-reduced flavour, {args.precision} (1e-8)")
                    chol["time_to_converged_1e-8"] = time_to_converged(
                        OMM, torch, dev, s, args.precision, E_ref, 1e-8, 2 * args.max_iter,
                        args.resync, flavour="cholesky")
            conv["E_ref"] = E_ref
            result["time_to_converged"] = conv

    if not args.no_complex and args.workload == "c3":
        result["complex_kpoints"] = complex_bench(args, torch)

    if not args.no_cpu_baseline:
        log(f"cpu baseline: {args.cpu_iters} oracle iterations")
        result["cpu_baseline"] = cpu_baseline(s, C0, args.cpu_iters)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
