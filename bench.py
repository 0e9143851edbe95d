"""Benchmark of the dense OMM CG path on one MI355X.

Workload (default): 1000 atoms on a 10x10x10 lattice (a = 3.0 bohr, r_c = 8 bohr), 13 orbitals
per atom -> N = 13000 basis orbitals, M = 2000 Wannier functions, eta = 0, tau = 10, synthetic
finite-range S/T/H (seeded); inputs are resident in HBM before the timed region.

A "step" is one pass over every stage of the path. In the mixed-precision scheme (the default)
that is one resynchronization period: `--resync` (80) CG line searches (gradient,
preconditioning, Polak-Ribiere direction, operator products, projections, quartic coefficients +
line minimum, updates + energy) with bf16 MFMA products on the FP64 state, closed by the FP64
recomputation of the state from C that the scheme performs every `--resync` line searches. The
timed window therefore always holds whole periods, and `value` (line searches per second)
includes each resynchronization's full cost. With `--precision fp64` or `fp32` a step is one
line search.

Prints ONE JSON line: the headline value, the FP64 and FP32 rates, time to a converged energy for
the mixed scheme and FP64, the roofline of the dominant kernel, the batched workload (64 systems)
at the mixed-precision bar, and the CPU oracle timed on a bounded sample.
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
                    flavour="dense", sparse=False, per_step=1, step_walls=None):
    """Wall time of `steps` steps of `per_step` line searches each, after `warmup` steps. With the
    mixed scheme (refine) per_step is the resynchronization interval, so the window holds whole
    periods; the run restarts from C0 after the warm-up (setup outside the window) and the
    window's resynchronizations are counted from the scheme's checkpoints. With `step_walls` (a
    list) the window runs step by step, each step's wall time appended (same line searches: the
    resynchronization schedule counts across calls)."""
    solver = OMM(s.N, s.M, precision=prec, refine=refine, resync=resync, flavour=flavour,
                 sparse=sparse)
    solver.set_HS(dev["H"], dev["S"], dev["T"])
    t0 = time.perf_counter()
    solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)  # setup only
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    # at least two untimed line searches: the first two of a phase tune every GEMM shape
    solver.iterate(max(warmup * per_step, 2))
    solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=0)  # restart from C0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if step_walls is None:
        solver.iterate(steps * per_step)
    else:
        for _ in range(steps):
            ts = time.perf_counter()
            solver.iterate(per_step)
            torch.cuda.synchronize()
            step_walls.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    resyncs = None
    if prec == "bf16x3" and refine:
        resyncs = len(solver.checkpoints()[0]) - 1  # the first checkpoint is the start
    stages = None
    if prof_steps > 0:
        solver.set_profiling(True)
        solver.iterate(prof_steps)
        torch.cuda.synchronize()
        stages, n = solver.stage_times()
        stages = {k: v / max(n, 1) for k, v in stages.items()}
        solver.set_profiling(False)
    solver.close()
    return wall, setup_s, stages, resyncs


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


def c2_grid_bench(args, torch):
    """The 2048-orbital workload (N = 2048, M = 384) over the shift x preconditioner grid
    eta in {0, 0.5} x tau in {1, 10, 100}, per precision: line searches to the stopping rule,
    wall time from omm_minimize entry (P built and tiles tuned by an untimed first call), rate,
    and the error against the closed form of each eta (tests/golden/c2_reference.json). FP64 and
    FP32 products with FP64 refinement run to tol 1e-12, the BF16 scheme on an FP64 state to
    tol 1e-10 at its resynchronizations."""
    from paper_1312_1549_amd import OMM
    from synth import config_system, start_coefficients

    s = config_system("c2", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    ref = json.loads((ROOT / "tests" / "golden" / "c2_reference.json").read_text())
    E_ref = ref.get("E_min_by_eta", {}) if ref.get("trace_H") and abs(
        ref["trace_H"] - float(np.trace(s.H))) <= 1e-9 * abs(ref["trace_H"]) else {}
    dev = {k: torch.from_numpy(v).cuda() for k, v in (("H", s.H), ("S", s.S), ("T", s.T),
                                                      ("C0", C0))}
    rows = []
    for prec, refine, tol in (("fp64", False, 1e-12), ("fp32", True, 1e-12),
                              ("bf16x3", True, 1e-10)):
        for eta in (0.0, 0.5):
            for tau in (1.0, 10.0, 100.0):
                solver = OMM(s.N, s.M, precision=prec, refine=refine, resync=args.resync)
                solver.set_HS(dev["H"], dev["S"], dev["T"])
                solver.minimize(dev["C0"], eta=eta, tau=tau, tol=0.0, max_iter=2)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = solver.minimize(dev["C0"], eta=eta, tau=tau, tol=tol, max_iter=6000)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                it = int(solver.stats()[0])
                E = solver.energy()
                row = {"precision": prec + ("+fp64" if refine else ""), "eta": eta, "tau": tau,
                       "tol": tol, "status": int(st), "line_searches": it, "s": wall,
                       "iters_per_s": it / wall, "E": E}
                if str(eta) in E_ref:
                    row["rel_err_vs_closed_form"] = abs(E - E_ref[str(eta)]) / abs(E_ref[str(eta)])
                rows.append(row)
                solver.close()
                log(f"c2 grid {row['precision']} eta={eta} tau={tau}: {it} line searches, "
                    f"{wall:.2f}s, rel err {row.get('rel_err_vs_closed_form', float('nan')):.2e}")
    return {"workload": WORKLOADS["c2"].split(", eta")[0] + ", eta in {0, 0.5} x tau in {1, 10, 100}",
            "runs": rows}


def autograd_bench(args, torch):
    """The differentiable energy on the 1024-atom workload (N = 4096, M = 768): E = min_C of the
    functional through omm_energy (FP32 products with FP64 refinement to tol 1e-12), then
    E.backward() (dE/dH = the density matrix, dE/dS = minus the energy-density matrix minus eta
    times it). Forward and backward wall times after an untimed warm-up call (preconditioner,
    tiles), the error against the closed form (tests/golden/c5_reference.json), and at the
    minimum Tr(dE/dH S) = 2 M (S_W = I)."""
    from paper_1312_1549_amd import OMM, omm_energy
    from synth import config_system, start_coefficients

    s = config_system("c5", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    E_ref = reference_energy("c5", s)
    H = torch.from_numpy(s.H).cuda().requires_grad_(True)
    S = torch.from_numpy(s.S).cuda().requires_grad_(True)
    T, C0d = torch.from_numpy(s.T).cuda(), torch.from_numpy(C0).cuda()
    solver = OMM(s.N, s.M, precision="fp32", refine=True)
    omm_energy(H, S, T, C0d, s.eta, s.tau, 1e-6, 200, solver).backward()
    torch.cuda.synchronize()
    H.grad = None
    S.grad = None
    t0 = time.perf_counter()
    E = omm_energy(H, S, T, C0d, s.eta, s.tau, 1e-12, 6000, solver)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    E.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    tr = float((H.grad * S.detach()).sum())
    out = {"workload": WORKLOADS["c5"] + ", fp32 products + fp64 refinement, tol 1e-12",
           "forward_s": t_fwd, "backward_s": t_bwd, "line_searches": int(solver.stats()[0]),
           "trace_dEdH_S_rel_err": abs(tr - 2 * s.M) / (2 * s.M)}
    if E_ref is not None:
        out["rel_err_vs_closed_form"] = abs(float(E.detach()) - E_ref) / abs(E_ref)
    solver.close()
    log(f"autograd c5: forward {t_fwd:.2f}s ({out['line_searches']} line searches), backward "
        f"{1e3 * t_bwd:.1f} ms, rel err {out.get('rel_err_vs_closed_form', float('nan')):.2e}")
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

    # bf16 scheme: whole resynchronization periods, FP64: 20 line searches; after 2 untimed
    # line searches (they tune the GEMM tiles), so the bf16 window holds one resynchronization
    # per period
    for prec, steps in (("bf16x3", max(2, args.steps // 4) * args.resync), ("fp64", 20)):
        sol = solver_for(prec)
        sol.iterate(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.iterate(steps)
        torch.cuda.synchronize()
        out[f"{prec}_iters_per_s"] = steps / (time.perf_counter() - t0)
        out[f"{prec}_line_searches_timed"] = steps
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


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


def _oracle_rate(oracle, s, C0, P, warm, iters):
    """Line searches per second of the oracle over `iters` line searches after `warm` (setup and
    the warm-up outside the window)."""
    stamps = []
    oracle.minimize(s.H, s.S, s.T, C0, s.eta, s.tau, 0.0, warm + iters, P=P, use_given_P=True,
                    callback=lambda k, E: stamps.append(time.perf_counter()))
    return iters / (stamps[warm + iters] - stamps[warm])


def cpu_baseline(s, C0, iters, warm, closed_form=False):
    """The CPU oracle on the host cores: the bench workload on all BLAS threads, plus the
    2048-orbital workload on all threads and on one (a single-threaded line search of the bench
    workload would take about a minute), and optionally LAPACK's closed form of the bench
    workload (the exact-energy baseline)."""
    from oracle import brute, omm as oracle
    from synth import config_system, start_coefficients

    threads = _blas_threads()
    P = oracle.preconditioner(s.S, s.T, s.tau)  # setup, not timed
    rate = _oracle_rate(oracle, s, C0, P, warm, iters)
    out = {"value": rate, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{iters} FP64 line searches of the NumPy oracle on the same N={s.N}, M={s.M} "
                     f"inputs after {warm} untimed warm-up line searches and its untimed setup (P "
                     f"inverse, initial products); host BLAS threads={threads}, "
                     f"os.cpu_count()={os.cpu_count()}"}
    del P
    c2 = config_system("c2", 0)
    C02 = start_coefficients(c2.S, c2.M, 1)
    P2 = oracle.preconditioner(c2.S, c2.T, c2.tau)
    out["workload_2048"] = {"workload": WORKLOADS["c2"],
                            "all_threads_iters_per_s": _oracle_rate(oracle, c2, C02, P2, 1, 4)}
    try:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            out["workload_2048"]["one_thread_iters_per_s"] = _oracle_rate(oracle, c2, C02, P2, 1, 4)
    except Exception as e:  # threadpoolctl missing: no single-thread figure
        out["workload_2048"]["one_thread_error"] = str(e)
    if closed_form:
        t0 = time.perf_counter()
        w = brute.generalized_eigh_lapack(s.H, s.S, s.M + 1)[0]
        out["closed_form_s"] = time.perf_counter() - t0
        out["closed_form_E"] = brute.closed_form_energy(w, s.M, s.eta)
        out["closed_form_note"] = ("LAPACK generalized symmetric-definite eigensolver, lowest "
                                   "M + 1 eigenvalues, all BLAS threads")
    return out


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


def batched_bench(args, standalone=False):
    """Batched systems (64, N = 256..2048): FP32 grouped phase to 1e-9 then the FP64 grouped
    phase to tol 1e-12, cold, then an SCF-like warm start after H += 1e-3 sym(N(0,1)); the
    energies against the closed forms stored by tests/golden/make_golden.py (when they match the
    generated inputs)."""
    import torch
    from paper_1312_1549_amd import OMMBatch, flops_per_iteration
    from synth import batched_systems, perturb_hamiltonian, start_coefficients

    t0 = time.perf_counter()
    log("batched: generating 64 systems")
    systems = batched_systems(count=64)
    C0s = [start_coefficients(x.S, x.M, 1000 + i) for i, x in enumerate(systems)]
    gen_s = time.perf_counter() - t0
    ref = None
    f = ROOT / "tests" / "golden" / "c4_reference.json"
    if f.exists():
        rows = json.loads(f.read_text())["systems"]
        if len(rows) == len(systems) and all(
                r["N"] == x.N and abs(r["trace_H"] - float(np.trace(x.H))) <= 1e-9 * abs(r["trace_H"])
                for r, x in zip(rows, systems)):
            ref = rows
    tol = 1e-12
    b = OMMBatch([x.N for x in systems], [x.M for x in systems], precision="fp32", refine=True)
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
    etas, taus = [x.eta for x in systems], [x.tau for x in systems]
    b.minimize(C0s, etas, taus, tol, 10)  # warm-up: setup, autotune, graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = b.minimize(C0s, etas, taus, tol, 5000)
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
    it32, it64 = b.phase_iterations()
    it = it32 + it64
    E = b.energies()
    flops = sum(int(k) * flops_per_iteration(x.N, x.M) for k, x in zip(it, systems))
    log(f"batched cold: {cold:.2f}s, {int(it.sum())} line searches ({int(it32.sum())} fp32 + "
        f"{int(it64.sum())} fp64)")
    out = {"workload": WORKLOADS["c4"], "precision": "fp32 grouped phase to 1e-9, then fp64 "
           "grouped phase to tol 1e-12 (fp64 reductions throughout)",
           "line_searches_per_s": float(it.sum()) / cold, "systems_per_s": len(systems) / cold,
           "algorithmic_tflops": flops / cold / 1e12, "cold_s": cold, "status": int(st),
           "cold_line_searches": {"fp32": int(it32.sum()), "fp64": int(it64.sum()),
                                  "max_per_system": int(it.max())},
           "generation_s": gen_s}
    if ref is not None:
        err = np.abs(E - np.array([r["E_min"] for r in ref])) / np.abs([r["E_min"] for r in ref])
        out["max_rel_err_vs_closed_form"] = float(err.max())
    Cs = [b.get_C(i) for i in range(len(systems))]
    for i, x in enumerate(systems):
        b.set_HS(i, perturb_hamiltonian(x.H, 200 + i), x.S, x.T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stw = b.minimize(Cs, etas, taus, tol, 5000)
    torch.cuda.synchronize()
    warm = time.perf_counter() - t0
    w32, w64 = b.phase_iterations()
    out.update({"warm_s": warm, "warm_status": int(stw),
                "warm_line_searches": {"fp32": int(w32.sum()), "fp64": int(w64.sum()),
                                       "max_per_system": int((w32 + w64).max())}})
    if ref is not None:
        Ew = b.energies()
        refw = np.array([r["E_min_warm"] for r in ref])
        out["warm_max_rel_err_vs_closed_form"] = float((np.abs(Ew - refw) / np.abs(refw)).max())
    b.close()
    log(f"batched warm: {warm:.2f}s; max rel err cold {out.get('max_rel_err_vs_closed_form')} "
        f"warm {out.get('warm_max_rel_err_vs_closed_form')}")
    if not standalone:
        return out
    return {
        "metric": "batched OMM CG line searches/sec (64 systems, N=256..2048)",
        "value": out["line_searches_per_s"], "unit": "line searches/s", "n_gpus": 1,
        "steps": int(it.max()), "warmup": 10, "ms_per_step": 1e3 * cold / max(1, int(it.max())),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64",
        "data": "synthetic", "config": {"workload": WORKLOADS["c4"]}, "batched": out,
    }


def summarize_pmc(csv_path, kernel_substr):
    """Per-dispatch counter values of the kernels whose name contains `kernel_substr`, from a
    rocprofv3 --pmc counter_collection CSV: one line per counter with the mean and the values."""
    import csv
    from collections import defaultdict

    vals = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if kernel_substr not in r["Kernel_Name"]:
            continue
        vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = []
    for k, v in sorted(vals.items()):
        out.append(f"{k}: dispatches {len(v)}, mean {sum(v) / len(v):.6g}, values "
                   + ", ".join(f"{x:.6g}" for x in v[:8]))
    return "\n".join(out)


def copy_kernel(nbytes):
    """A plain device copy of a known size (reads and writes `nbytes` each): the calibration
    kernel for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    b = a.clone()
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "check": float(b[-1])}))


def vendor_gemm(reps=20):
    """Context for the GEMM rooflines: the rate of the vendor BF16 GEMM (torch.matmul on
    hipBLASLt) on the single-pass shapes of the N=13000, M=2000 line search (random bf16 operands,
    FP32 accumulation). Not part of the method's path; it shows what a tuned library reaches on
    these shapes against the 2.5 PFLOP/s dense peak."""
    import torch

    torch.manual_seed(0)
    out = []
    shapes = [("[HD|SD], PG: one pass", 2000, 13000, 13000),
              ("gradient: one pass", 2000, 13000, 4000),
              ("projections: one pass", 2000, 2000, 13000),
              ("square reference", 8192, 8192, 8192)]
    for name, m, n, k in shapes:
        a = torch.randn(m, k, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(k, n, device="cuda", dtype=torch.bfloat16)
        for _ in range(3):
            c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
        out.append({"shape": name, "m": m, "n": n, "k": k, "ms": round(ms, 4),
                    "tflops": round(tf, 1), "frac": round(tf / 2500.0, 3)})
        del a, b, c
    print(json.dumps({"vendor_bf16_gemm": out}))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--vendor-gemm":
        vendor_gemm()
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--summarize-rocprof":
        print(summarize_rocprof(sys.argv[2]))
        return
    if len(sys.argv) > 3 and sys.argv[1] == "--summarize-pmc":
        print(summarize_pmc(sys.argv[2], sys.argv[3]))
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--copy-kernel":
        copy_kernel(int(sys.argv[2]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps (mixed scheme: resynchronization periods of --resync line "
                         "searches each; fp64/fp32: line searches)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-converge", action="store_true", help="skip time-to-converged runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-closed-form", action="store_true",
                    help="also time LAPACK's closed form of the workload on the host")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison rate")
    ap.add_argument("--no-cholesky", action="store_true",
                    help="skip the Cholesky-reduced flavour's rate and time to converged")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the block-sparse operator products' rate and time to converged")
    ap.add_argument("--no-complex", action="store_true",
                    help="skip the complex Hermitian (k-point) rates and time to converged")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-system batch")
    ap.add_argument("--no-c2-grid", action="store_true",
                    help="skip the eta x tau grid of the 2048-orbital workload")
    ap.add_argument("--no-autograd", action="store_true",
                    help="skip the differentiable energy on the 4096-orbital workload")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline scheme only (profiling runs): implies every --no-* "
                         "flag and skips the side rates and the latency workload")
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--resync", type=int, default=80)
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--cpu-warmup", type=int, default=2)
    args = ap.parse_args()
    if args.only_headline:
        for flag in ("no_converge", "no_cpu_baseline", "no_fp64", "no_cholesky", "no_sparse",
                     "no_complex", "no_batched", "no_c2_grid", "no_autograd"):
            setattr(args, flag, True)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "c4":
        print(json.dumps(batched_bench(args, standalone=True)), flush=True)
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
    prof_steps = 10
    mixed = args.precision == "bf16x3"
    R = args.resync if mixed else 1  # line searches per step
    side = max(2, args.steps // 4)   # steps of the flavours timed beside the headline
    log(f"timing {args.precision}: warmup {args.warmup}, steps {args.steps} x {R} line searches")
    step_walls = []
    wall, setup_s, stages, resyncs = time_iterations(
        OMM, torch, dev, s, args.precision, args.steps, args.warmup, prof_steps, refine=mixed,
        resync=args.resync, per_step=R, step_walls=step_walls)
    ips = args.steps * R / wall
    step_rates = sorted(R / w for w in step_walls)
    log(f"{args.precision}: {ips:.3f} iters/s ({1e3 * wall / (args.steps * R):.3f} ms/line search,"
        f" {resyncs} resynchronizations in the window)")
    rates = {}
    if mixed and not args.only_headline:
        wp, _, _, _ = time_iterations(OMM, torch, dev, s, "bf16x3", 80, 2, 0)
        rates["bf16_fp32_state_no_resync_iters_per_s"] = 80 / wp
        log(f"bf16 products with an FP32 state, no resync: {rates['bf16_fp32_state_no_resync_iters_per_s']:.3f} iters/s")
    if args.precision != "fp32" and not args.only_headline:
        w32, _, st32, _ = time_iterations(OMM, torch, dev, s, "fp32", 40, 2, 3)
        rates["fp32_iters_per_s"] = 40 / w32
        rates["fp32_stages_ms"] = st32
        log(f"fp32 products: {rates['fp32_iters_per_s']:.3f} iters/s")

    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        log("timing fp64")
        w64, _, st64, _ = time_iterations(OMM, torch, dev, s, "fp64", 20, 1, 3)
        fp64 = {"iters_per_s": 20 / w64, "stages_ms": st64}
        log(f"fp64: {fp64['iters_per_s']:.3f} iters/s")

    chol = None
    if not args.no_cholesky and mixed:
        log(f"timing the Cholesky-reduced flavour ({args.precision})")
        wc, setup_c, stc, _ = time_iterations(OMM, torch, dev, s, args.precision, side, 1,
                                              prof_steps, refine=True, resync=args.resync,
                                              flavour="cholesky", per_step=R)
        chol = {"iters_per_s": side * R / wc, "setup_s": setup_c, "stages_ms": stc,
                "steps": side, "line_searches_per_step": R,
                "note": "Cholesky-reduced flavour: S = L L^T once, no S or P products per line "
                        "search; its iterates are those of P = S^-1 (tau = inf), not of tau = "
                        f"{s.tau}"}
        log(f"cholesky: {chol['iters_per_s']:.3f} iters/s, setup {setup_c:.2f} s")

    sparse = None
    if not args.no_sparse and mixed:
        log("timing block-sparse operator products (bf16x3)")
        wsp, _, stsp, _ = time_iterations(OMM, torch, dev, s, args.precision, side, 1, prof_steps,
                                          refine=True, resync=args.resync, sparse=True, per_step=R)
        sparse = {"iters_per_s": side * R / wsp, "stages_ms": stsp, "steps": side,
                  "line_searches_per_step": R,
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
    if mixed:
        # the search direction is bf16-exact, so each product is two bf16 MFMA passes
        # (D_hi B_lo + D_hi B_hi): MFMA work is twice the algorithmic flops
        roofline["hardware_frac"] = 2 * achieved / peak

    result = {
        "metric": METRIC, "value": ips, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if mixed else args.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "N": s.N, "M": s.M, "eta": s.eta,
                   "tau": s.tau, "seed": 0, "c0_seed": 1},
        "line_searches_per_step": R, "line_searches_timed": args.steps * R,
        "algorithmic_tflops": flops * ips / 1e12,
        "scheme": ("bf16 MFMA products with FP32 accumulation (3 passes for the gradient, 2 for "
                   "every product with the bf16-rounded direction D~, 1 for PG = G~ P~), FP64 CG "
                   "state, FP64 reductions and line search, FP64 recomputation of the state from "
                   f"C every {args.resync} line searches (one per step)" if mixed else
                   f"{args.precision} MFMA products and FP64 reductions"),
        "setup_s": setup_s,
        "stages_ms": stages,
        "roofline": roofline,
    }
    if mixed:
        result["resyncs_in_window"] = resyncs
    # spread of the window: the rate of each step (one resynchronization period in the BF16
    # scheme), median, lowest and highest
    result["step_rates"] = {"median": step_rates[len(step_rates) // 2], "min": step_rates[0],
                            "max": step_rates[-1], "unit": "iters/s", "steps": len(step_rates)}
    result.update(rates)
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
            if mixed:
                log(f"time to converged: {args.precision} with FP64 state (1e-8)")
                conv["bf16_1e-8"] = time_to_converged(
                    OMM, torch, dev, s, args.precision, E_ref, 1e-8, args.max_iter, args.resync)
                a = conv["fp64_1e-8"].get("time_to_target_s")
                b = conv["bf16_1e-8"].get("time_to_target_s")
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

    if args.workload == "c3" and not args.only_headline:
        log("c1 latency: fp64 line searches on the 128-orbital workload")
        c1 = config_system("c1", 0)
        C01 = start_coefficients(c1.S, c1.M, 1)
        d1 = {k: torch.from_numpy(v).cuda() for k, v in (("H", c1.H), ("S", c1.S), ("T", c1.T),
                                                          ("C0", C01))}
        wl, _, _, _ = time_iterations(OMM, torch, d1, c1, "fp64", 100, 20, 0)
        result["c1_fp64_us_per_iter"] = 1e6 * wl / 100
        result["c1_workload"] = WORKLOADS["c1"]
        log(f"c1 fp64: {result['c1_fp64_us_per_iter']:.1f} us per line search")

    if not args.no_complex and args.workload == "c3":
        result["complex_kpoints"] = complex_bench(args, torch)
    if not args.no_c2_grid and args.workload == "c3":
        log("c2 grid: eta x tau on the 2048-orbital workload")
        result["c2_grid"] = c2_grid_bench(args, torch)
    if not args.no_autograd and args.workload == "c3":
        log("autograd: forward and backward on the 4096-orbital workload")
        result["autograd_c5"] = autograd_bench(args, torch)

    if not args.no_batched and args.workload == "c3":
        result["batched"] = batched_bench(args)

    if not args.no_cpu_baseline:
        log(f"cpu baseline: {args.cpu_warmup} + {args.cpu_iters} oracle line searches")
        result["cpu_baseline"] = cpu_baseline(s, C0, args.cpu_iters, args.cpu_warmup,
                                              closed_form=args.cpu_closed_form)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
