#!/usr/bin/env python
"""Benchmark of the DD-FGMRES solver on one MI355X.

One step = one full solve of A u = f to outer relative residual 1e-6 (FGMRES from a
zero guess, preconditioned by the batched inexact subdomain solves), with the
right-hand side already resident in device memory.  The default workload is
k = 200, 20 points per wavelength (N = 637, 404,496 unknowns), 16 x 16 subdomains
with widths perturbed by +-25%, three seeded Gaussian sources, inner tolerance 1e-2.

`value` is whole-job throughput in subdomain solves per second of the chosen form
(complex64 subdomain Krylov work, FP64 coarse solves and outer FGMRES, outer steps
replayed from a captured hipGraph, autotuned launch configuration); `ms_per_step` is its
time to solution.  The plain form (complex128 subdomain Krylov work as one batched launch
per GMRES stage with the inner loop on the host, no persistent kernel, outer steps launched
one by one) is timed beside it, and `fused_fp64` times the complex128 subdomain GMRES inside
the fused kernel (steps one by one), separating the gain of fusion from that of precision.
`kernels` gives, for the batched subdomain-solve kernel and the two basis sweeps of the
outer delayed-CGS2 Arnoldi, algorithmic bytes (counted per launch by the
library) over durations from HIP events recorded on the library's stream around each
kernel, in one more solve of the same handle and inputs with the steps launched one
by one right after the timed solves (HIP cannot time events inside graph replays);
`roofline` is the one with the largest total time.  The CPU baseline is the oracle timed on a
bounded sample of the same workload (its first outer iterations).  `direct_local_solves`
times the same solve with exact subdomain solves (FP64 block factorisation of every local matrix, the
direct-solve baseline of the paper's experiments) for comparison; `learned_guess` times the
chosen form with the trained BF16 guess network attached (its output offered to every
subdomain GMRES, kept only when it lowers the deflated residual); `two_level` times the
two-level method (a global coarse space added to the chosen form, the extension the
paper proposes in its conclusions).  `tol_sweep` repeats the solve on the medium workload
(k = 100, N = 160, 8 x 8) at inner tolerances 1e-1, 1e-2 and 1e-4 in the chosen and the
complex128 forms, with the stored oracle counts beside them, and `large_inner_tol` the
headline workload's chosen form at inner tolerances 1e-3 and 1e-4; `restart_study` runs the
one-level chosen form with restarted FGMRES (restart 100, 300, 1000, 2000); `xlarge` solves the
largest one-GPU configuration (k = 400, N = 1274, 32 x 32 perturbed blocks, eight
right-hand sides) with the two-level method as two unrestarted batches of four, in the
chosen, complex128 and exact-local-solve forms.  `--xlarge-batches` runs only that leg, and
`--breakeven` only a study of the one-level method over uniform P x P partitions of the
headline grid (P = 12 ... 32), inexact against exact subdomain solves.
Progress goes to stderr; stdout carries the one result line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def progress(msg: str):
    """Progress on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)
METRIC = "DD-FGMRES time-to-solution (rel res 1e-6) & subdomain solves/s, chosen vs plain"


# Sources of the kernels whose HBM counters profiles/large_solve_hbm_traffic.md records.
TRAFFIC_SOURCES = ["inner_kernels.hip", "outer_kernels.hip", "kernels.hpp", "coarse.hpp", "stencil.hpp", "outer.hpp",
                   "common.hpp"]


def sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(ROOT, "paper_2103_17081_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def recorded_traffic():
    """Calibrated HBM bytes per dispatch from the committed counter summary, if the sources
    of the profiled kernels are unchanged since the counters were taken (else {})."""
    path = os.path.join(ROOT, "profiles", "large_solve_hbm_traffic.md")
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    if "```json" not in text:
        return {}
    block = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if block.get("sources") != TRAFFIC_SOURCES or block.get("sources_sha256") != sources_sha256():
        return {}
    return block["traffic_bytes_per_dispatch"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--no-plain", action="store_true", help="skip the all-FP64 comparison solve")
    ap.add_argument("--no-guess", action="store_true", help="skip the solve with the learned initial guess")
    ap.add_argument("--xlarge-batches", action="store_true",
                    help="only: the k = 400 grid's eight right-hand sides with the two-level method (M = N/2), "
                         "as two unrestarted batches of four, chosen form and exact local solves")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the comparison with exact (FP64 block-factorised) subdomain solves")
    ap.add_argument("--no-two-level", action="store_true",
                    help="skip the two-level solve (global coarse space of --coarse-intervals per edge)")
    ap.add_argument("--coarse-intervals", type=int, default=0,
                    help="coarse intervals per edge of the two-level leg (0: N / 2, i.e. H = 2h)")
    ap.add_argument("--two-level-only", action="store_true",
                    help="run only the two-level leg and print it (profiling of the coarse correction)")
    ap.add_argument("--no-tol-sweep", action="store_true",
                    help="skip the inner-tolerance study on the medium workload (1e-1, 1e-2, 1e-4)")
    ap.add_argument("--no-restart", action="store_true",
                    help="skip the restarted-FGMRES study (restart 100, 300, 1000, 2000) of the one-level solve")
    ap.add_argument("--no-xlarge", action="store_true",
                    help="skip the k = 400 eight-right-hand-side leg (two-level, batches of four)")
    ap.add_argument("--breakeven", action="store_true",
                    help="only: the one-level method on the k = 200 grid over uniform P x P partitions, inexact "
                         "(chosen form) against exact subdomain solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-outer", type=int, default=40, help="outer iterations of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="before the solve, copy a 1 GiB buffer 3 times (reference kernel for HBM counters)")
    return ap.parse_args()


def make_solver(w, precision: int, local_solver: str = "deflated", coarse_intervals: int = 0,
                inner_launch: str = "fused", **kw):
    from paper_2103_17081_amd.binding import Solver
    kw.setdefault("inner_tol", w.inner_tol)
    kw.setdefault("outer_maxit", 4000)
    return Solver(w.k, n_intervals=w.n, cuts_x=w.cuts_x, cuts_y=w.cuts_y, overlap=w.overlap,
                  inner_precision=precision, outer_tol=w.outer_tol, local_solver=local_solver,
                  coarse_intervals=coarse_intervals, inner_launch=inner_launch,
                  use_graph=inner_launch == "fused", **kw)


def describe(w) -> str:
    """Workload line: grid, partition (with the width perturbation and its seed), sources."""
    from paper_2103_17081_amd import inputs
    px, py = len(w.cuts_x) - 1, len(w.cuts_y) - 1
    uniform = (list(w.cuts_x) == list(inputs.uniform_cuts(w.n, px))
               and list(w.cuts_y) == list(inputs.uniform_cuts(w.n, py)))
    part = (f"{px}x{py} uniform" if uniform else
            f"{px}x{py} with widths perturbed by +-25% (seed {inputs.SEED_BASE}, x then y)")
    src = {"small": "unit point source at (0.5, 0.5)",
           "medium": f"point source + 3 Gaussians (seed {inputs.SEED_BASE} + rhs)",
           "large": f"3 Gaussians (seed {inputs.SEED_BASE} + rhs)",
           "xlarge": f"3 Gaussians + a seeded point source per rhs (seed {inputs.SEED_BASE} + rhs)"}[w.name]
    return (f"{w.name}: k={w.k:g}, N={w.n} ({w.ndof} dofs), {w.nsub} subdomains ({part}, overlap {w.overlap}), "
            f"{src}, inner tol {w.inner_tol:g}, outer tol {w.outer_tol:g}")


def default_coarse_intervals(w) -> int:
    """M = N / 2: coarse spacing H = 2h, the coarsening of the subdomain deflation (Sec. 2)."""
    return max(2, w.n // 2)


def true_relres(torch, solver, f, u):
    r = f - solver.op_global_apply(u)
    return float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(f))


def timed_solves(torch, solver, f, steps: int, warmup: int):
    for _ in range(warmup):
        solver.solve(f)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        u, st = solver.solve(f)
        stats.append(st)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, u, stats


def cpu_baseline(w, outer: int):
    """The oracle (complex128, scipy) on the first `outer` outer iterations of the workload."""
    import numpy as np
    from oracle import schwarz
    threads = os.environ.get("OMP_NUM_THREADS") or os.environ.get("OPENBLAS_NUM_THREADS")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    t0 = time.perf_counter()
    _, st = S.solve(w.rhs[0], mode="deflated", inner_tol=w.inner_tol, outer_maxit=outer)
    dt = time.perf_counter() - t0
    cores = int(threads) if threads and threads.isdigit() else (os.cpu_count() or 1)
    return {"value": st.subdomain_solves / dt, "unit": "subdomain solves/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {st.outer_iters} outer FGMRES iterations of workload '{w.name}' "
                      f"({st.subdomain_solves} subdomain solves, avg {st.avg_inner:.1f} inner its) "
                      f"in {dt:.1f} s; a per-step rate over those iterations (not a time to solution: the "
                      f"oracle's full solve of this workload takes hours); setup excluded; "
                      f"BLAS threads {threads or 'default'}"}


GUESS_WEIGHTS = os.path.join(ROOT, "paper_2103_17081_amd", "weights", "guess_t64.ddnet")


def guess_leg(torch, w, f, t_zero: float):
    """The chosen form with the learned initial guess attached (the trained BF16 network's
    output offered to every subdomain GMRES, kept only when it lowers the deflated
    residual); t_zero (s) is the zero-guess chosen form's time to solution."""
    from paper_2103_17081_amd.guess import load_net
    s = make_solver(w, 32)
    s.autotune(None)
    net = load_net(GUESS_WEIGHTS, max_batch=s.nsub * s.nrhs)
    s.set_guess(net)
    tg, ug, sg = timed_solves(torch, s, f, 1, 1)
    s.set_graph(False)
    _, gi = s.solve(f)
    torch.cuda.synchronize()
    last = sg[-1]
    out = {"weights": os.path.relpath(GUESS_WEIGHTS, ROOT), "time_to_solution_s": tg,
           "outer_iters": last["outer_iters"],
           "avg_inner_iters": last["inner_iters_total"] / max(last["subdomain_solves"], 1),
           "guesses_accepted_frac": last["guesses_accepted"] / max(last["subdomain_solves"], 1),
           "true_relres": true_relres(torch, s, f, ug), "status": last["status"],
           "ms_per_step_guess": gi["ms_guess"] / max(gi["timed_steps"], 1),
           "ms_per_step_inner": gi["ms_inner"] / max(gi["timed_steps"], 1),
           "speedup_vs_zero_guess": t_zero / tg}
    s.set_guess(None)
    s.close()
    net.close()
    return out


def xlarge_batches(torch, batch: int = 4, maxit: int = 1000):
    """The largest one-GPU configuration (k = 400, N = 1274, 32 x 32 blocks, eight right-hand
    sides) with the two-level method, M = N/2.  Unrestarted FGMRES keeps 2 x 26 MB of FP64
    bases per right-hand side and column, so the eight are solved as batches of `batch`."""
    import numpy as np
    from paper_2103_17081_amd import inputs
    from paper_2103_17081_amd.binding import Solver
    w = inputs.workload("xlarge", 8)
    F_all = torch.from_numpy(np.stack(w.rhs)).to("cuda")
    out = {"workload": describe(w) + ", 8 right-hand sides",
           "method": "two-level (global coarse space, M = N/2) in every form: the one-level outer count grows "
                     "with the subdomain count and eight unrestarted one-level bases do not fit in memory",
           "coarse_intervals": default_coarse_intervals(w), "batch": batch, "outer_maxit": maxit}
    for form, prec, local in (("chosen", 32, "deflated"), ("fused_fp64", 64, "deflated"),
                              ("exact_local_solves", 64, "direct")):
        tot, runs = 0.0, []
        for b0 in range(0, len(w.rhs), batch):
            F = F_all[b0:b0 + batch].contiguous()
            s = Solver(w.k, n_intervals=w.n, cuts_x=w.cuts_x, cuts_y=w.cuts_y, overlap=w.overlap,
                       inner_precision=prec, inner_tol=w.inner_tol, outer_tol=w.outer_tol, outer_maxit=maxit,
                       nrhs=batch, coarse_intervals=default_coarse_intervals(w), local_solver=local)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, st = s.solve(F)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            R = F - torch.stack([s.op_global_apply(U[q].contiguous()) for q in range(batch)])
            rels = (torch.linalg.vector_norm(R, dim=1) / torch.linalg.vector_norm(F, dim=1)).tolist()
            rel = max(rels)
            s.close()
            del U, R
            torch.cuda.empty_cache()
            tot += dt
            runs.append({"rhs": [b0, b0 + batch], "time_to_solution_s": dt, "outer_iters": st["outer_iters"],
                         "true_relres_max": rel, "true_relres_per_rhs": rels, "status": st["status"],
                         "avg_inner_iters": st["inner_iters_total"] / max(st["subdomain_solves"], 1)})
            progress(f"xlarge {form} rhs {b0}..{b0 + batch - 1}: {dt:.1f} s, {st['outer_iters']} outer")
        out[form] = {"time_to_solution_s": tot, "batches": runs}
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_counts.json")


def tol_sweep_leg(torch, tols=(0.1, 0.01, 1e-4)):
    """Inner-tolerance study on the medium workload (k = 100, N = 160, 8 x 8): per tolerance,
    the chosen form (complex64 inner, autotuned, graph replay) and the complex128 inner form
    (fused kernel), their time to solution, outer count and average inner count, the stored
    oracle count (tests/golden/oracle_counts.json, written by the oracle), and the
    FP32-vs-FP64 difference of one preconditioner application on a seeded residual."""
    import numpy as np
    from paper_2103_17081_amd import inputs
    w = inputs.workload("medium")
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    rng = np.random.default_rng(72)
    r = torch.from_numpy(rng.standard_normal(w.ndof) + 1j * rng.standard_normal(w.ndof)).to("cuda")
    gold = json.load(open(GOLDEN))["medium"] if os.path.exists(GOLDEN) else {}
    rows = []
    for tol in tols:
        row = {"inner_tol": tol}
        z = {}
        for form, prec in (("chosen_fp32", 32), ("fused_fp64", 64)):
            s = make_solver(w, prec, inner_tol=tol, outer_maxit=3000)
            if prec == 32:
                s.autotune(None)
            t, u, st = timed_solves(torch, s, f, 1, 1)
            z[form] = s.apply_preconditioner(r)
            row[form] = {"time_to_solution_s": t, "outer_iters": st[-1]["outer_iters"],
                         "avg_inner_iters": st[-1]["inner_iters_total"] / max(st[-1]["subdomain_solves"], 1),
                         "true_relres": true_relres(torch, s, f, u), "status": st[-1]["status"]}
            s.close()
        row["z_rel_diff_fp32_vs_fp64"] = float(torch.linalg.vector_norm(z["chosen_fp32"] - z["fused_fp64"])
                                               / torch.linalg.vector_norm(z["fused_fp64"]))
        g = gold if gold.get("inner_tol") == tol else gold.get("tol_sweep", {}).get(f"{tol:g}")
        if g:
            row["oracle_outer_iters"] = g["outer_iters"]
            row["oracle_avg_inner_iters"] = g["inner_iters"] / g["subdomain_solves"]
        rows.append(row)
    return {"workload": describe(w), "rows": rows}


def large_tol_leg(torch, w, f, tols=(1e-3, 1e-4)):
    """The one-level chosen form on the headline workload at tighter inner tolerances: the
    outer orthogonalisation grows with the square of the outer count, so fewer, dearer outer
    steps can shorten the solve."""
    rows = []
    for tol in tols:
        s = make_solver(w, 32, inner_tol=tol)
        s.autotune(None)
        t, u, st = timed_solves(torch, s, f, 1, 0)
        rows.append({"inner_tol": tol, "time_to_solution_s": t, "outer_iters": st[-1]["outer_iters"],
                     "avg_inner_iters": st[-1]["inner_iters_total"] / max(st[-1]["subdomain_solves"], 1),
                     "true_relres": true_relres(torch, s, f, u), "status": st[-1]["status"]})
        s.close()
    return rows


def restart_leg(torch, w, f, restarts=(100, 300, 1000, 2000), maxit=6000):
    """The one-level chosen form with restarted FGMRES: outer count, time to solution, and
    the orthogonalisation share of an instrumented solve (steps launched one by one)."""
    rows = []
    for m in restarts:
        s = make_solver(w, 32, outer_restart=m, outer_maxit=maxit)
        s.autotune(None)
        t, u, st = timed_solves(torch, s, f, 1, 0)
        s.set_graph(False)
        _, inst = s.solve(f, check=False)
        torch.cuda.synchronize()
        rows.append({"restart": m, "time_to_solution_s": t, "outer_iters": st[-1]["outer_iters"],
                     "status": st[-1]["status"], "true_relres": true_relres(torch, s, f, u),
                     "orth_share_instrumented": inst["ms_orth"] / max(inst["ms_steps"], 1e-9),
                     "ms_per_step_instrumented": inst["ms_steps"] / max(inst["precond_applies"], 1)})
        s.close()
    return rows


def apply_ms(torch, solver, j: int, reps: int = 5) -> float:
    """Median duration (HIP events on torch's stream) of one preconditioner application to
    outer basis vector j of the solver's last solve."""
    r = solver.outer_basis(j).contiguous()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        solver.apply_preconditioner(r)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


def breakeven_leg(torch, w, f, parts=(12, 16, 20, 24, 32), maxit=4000):
    """The one-level method on the headline grid over uniform P x P partitions, inexact
    subdomain solves (chosen form) against exact ones: time to solution and time per
    preconditioner application as the subdomains shrink, i.e. where the inexact solves
    start to pay (the wall-clock question the paper leaves open, Sec. 4)."""
    import dataclasses
    from paper_2103_17081_amd import inputs
    rows = []
    for P in parts:
        cuts = inputs.uniform_cuts(w.n, P)
        wp = dataclasses.replace(w, cuts_x=cuts, cuts_y=cuts)
        row = {"subdomains": f"{P}x{P}", "widest_block_cells": int(max(cuts[1:] - cuts[:-1]))}
        for form, prec, local in (("inexact_c64", 32, "deflated"), ("exact", 64, "direct")):
            progress(f"break-even {P}x{P} {form}")
            s = make_solver(wp, prec, local, outer_maxit=maxit)
            s.autotune(None)
            t, u, st = timed_solves(torch, s, f, 1, 1)
            last = st[-1]
            entry = {"time_to_solution_s": t, "outer_iters": last["outer_iters"], "status": last["status"],
                     "true_relres": true_relres(torch, s, f, u),
                     "ms_per_apply_basis_300": apply_ms(torch, s, min(300, last["outer_iters"] - 1))}
            if local == "deflated":
                entry["avg_inner_iters"] = last["inner_iters_total"] / max(last["subdomain_solves"], 1)
            row[form] = entry
            s.close()
        rows.append(row)
    return rows


def two_level_leg(torch, w, f, M: int, t_one_level=None, direct: bool = True):
    """The two-level method (global coarse space of M intervals per edge) in the chosen
    form, and with exact subdomain solves; t_one_level (s) gives the speedups."""
    t0 = time.perf_counter()
    two = make_solver(w, 32, coarse_intervals=M)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    two.autotune(None)
    t2, u2, s2 = timed_solves(torch, two, f, 1, 1)
    two.set_graph(False)
    _, ti = two.solve(f)
    torch.cuda.synchronize()
    ap2 = max(ti["precond_applies"], 1)
    ms_c = ti["ms_coarse"] / ap2
    ach = ti["coarse_bytes"] / (ms_c * 1e-3) / 1e9 if ms_c > 0 else 0.0
    out = {
        "coarse_intervals": M, "coarse_unknowns": two.nglobal_coarse, "setup_s": t_setup,
        "time_to_solution_s": t2, "outer_iters": s2[-1]["outer_iters"],
        "precond_applies": s2[-1]["precond_applies"],
        "subdomain_solves_per_s": s2[-1]["subdomain_solves"] / t2,
        "avg_inner_iters": s2[-1]["inner_iters_total"] / max(s2[-1]["subdomain_solves"], 1),
        "true_relres": true_relres(torch, two, f, u2), "status": s2[-1]["status"],
        "speedup_vs_one_level": t_one_level / t2 if t_one_level else None,
        "coarse_correction": {"ms_per_apply": ms_c, "solve_bytes": ti["coarse_bytes"],
                              "achieved_GBs_vs_solve_bytes": ach, "frac_of_hbm_peak": ach / HBM_PEAK_GBS},
        "ms_phase_instrumented_solve": {"coarse": ti["ms_coarse"], "inner": ti["ms_inner"],
                                        "spmv": ti["ms_spmv"], "orth": ti["ms_orth"],
                                        "all_steps": ti["ms_steps"]}}
    two.close()
    if direct:
        twod = make_solver(w, 64, "direct", coarse_intervals=M)
        t3, u3, s3 = timed_solves(torch, twod, f, 1, 1)
        out["with_direct_local_solves"] = {
            "time_to_solution_s": t3, "outer_iters": s3[-1]["outer_iters"],
            "true_relres": true_relres(torch, twod, f, u3), "status": s3[-1]["status"],
            "speedup_vs_one_level": t_one_level / t3 if t_one_level else None}
        twod.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}): the solver has no multi-GPU path",
              file=sys.stderr)
        return 2
    import torch
    from paper_2103_17081_amd import inputs

    w = inputs.workload(args.workload)
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.xlarge_batches:
        print(json.dumps({"xlarge_batches": xlarge_batches(torch)}), flush=True)
        return 0
    if args.breakeven:
        print(json.dumps({"breakeven": breakeven_leg(torch, w, f)}), flush=True)
        return 0
    if args.two_level_only:
        M = args.coarse_intervals or default_coarse_intervals(w)
        print(json.dumps({"two_level": two_level_leg(torch, w, f, M, direct=not args.no_direct)}), flush=True)
        return 0
    progress("chosen form")
    chosen = make_solver(w, 32)
    tune_report = chosen.autotune(None)      # launch configuration measured on this problem (set-up)
    t, u, stats = timed_solves(torch, chosen, f, args.steps, args.warmup)
    last = stats[-1]
    relres = true_relres(torch, chosen, f, u)
    solves = sum(s["subdomain_solves"] for s in stats)
    # Per-kernel durations: the same handle and inputs, outer steps launched one by one
    # with HIP events around every kernel (events cannot be timed inside graph replays).
    chosen.set_graph(False)
    torch.cuda.synchronize()
    _, inst = chosen.solve(f)
    torch.cuda.synchronize()
    chosen.set_graph(True)
    stats_k = [inst]
    launches = inst["precond_applies"]
    traffic = recorded_traffic() if args.workload == "large" else {}
    kernels = []
    for name, ms_key, b_key in (("inner_solve_kernel<float, 512>", "ms_inner", "inner_bytes"),
                                ("dots2_kernel", "ms_dots", "dots_bytes"),
                                ("dcgs2_update_kernel", "ms_update", "update_bytes")):
        ms = sum(s[ms_key] for s in stats_k)
        by = sum(s[b_key] for s in stats_k)
        ach = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        kernels.append({"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "traffic": traffic.get(name), "launches": launches,
                        "total_ms": ms, "avg_launch_ms": ms / max(launches, 1),
                        "bytes_per_launch": by / max(launches, 1)})
    dom = max(kernels, key=lambda k: k["total_ms"])
    out = {
        "metric": METRIC,
        "value": solves / t,
        "unit": "subdomain solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": describe(w) + ", no restart",
                   "form": "chosen (complex64 inner, FP64 coarse LU and outer FGMRES)"},
        "chosen": {"time_to_solution_s": t / args.steps, "outer_iters": last["outer_iters"],
                   "precond_applies": last["precond_applies"],
                   "avg_inner_iters": last["inner_iters_total"] / max(last["subdomain_solves"], 1),
                   "true_relres": relres, "status": last["status"],
                   "graph_replays": last["graph_replays"], "ms_outer_steps": last["ms_steps"],
                   "autotune": tune_report.split("\n")[0],
                   "ms_phase_instrumented_solve": {"inner": inst["ms_inner"], "spmv": inst["ms_spmv"],
                                                   "orth": inst["ms_orth"], "dots": inst["ms_dots"],
                                                   "bookkeeping": inst["ms_other"], "update": inst["ms_update"],
                                                   "all_steps": inst["ms_steps"]}},
        "roofline": dom,
        "kernels": kernels,
    }
    chosen.close()
    if not args.no_plain:
        # plain: complex128 subdomain Krylov work as one batched launch per GMRES stage (all
        # subdomains per launch) with the inner loop on the host, no persistent kernel, outer
        # steps launched one by one (no graph replay)
        progress("plain form")
        plain = make_solver(w, 64, inner_launch="multi")
        tp, up, sp = timed_solves(torch, plain, f, 1, 1)
        out["plain"] = {"time_to_solution_s": tp, "outer_iters": sp[-1]["outer_iters"],
                        "subdomain_solves_per_s": sp[-1]["subdomain_solves"] / tp,
                        "avg_inner_iters": sp[-1]["inner_iters_total"] / max(sp[-1]["subdomain_solves"], 1),
                        "true_relres": true_relres(torch, plain, f, up), "status": sp[-1]["status"],
                        "graph_replays": sp[-1]["graph_replays"], "ms_inner": sp[-1]["ms_inner"],
                        "form": "complex128 inner, one batched launch per GMRES stage, host-driven inner "
                                "loop, steps launched one by one"}
        out["chosen_speedup_vs_plain"] = tp / (t / args.steps)
        plain.close()
        # the same complex128 subdomain GMRES inside the fused batched kernel (steps one by
        # one, default launch configuration): separates the fusion from the precision
        fused = make_solver(w, 64)
        fused.set_graph(False)
        tq, uq, sq = timed_solves(torch, fused, f, 1, 0)
        out["fused_fp64"] = {"time_to_solution_s": tq, "outer_iters": sq[-1]["outer_iters"],
                             "true_relres": true_relres(torch, fused, f, uq), "status": sq[-1]["status"],
                             "ms_inner": sq[-1]["ms_inner"],
                             "form": "complex128 inner in the fused batched kernel, steps launched one by one"}
        fused.close()
    if not args.no_direct:
        # the paper's direct-solve baseline: exact FP64 subdomain solves (block factorisation of each B_j)
        progress("exact local solves")
        direct = make_solver(w, 64, "direct")
        td, ud, sd = timed_solves(torch, direct, f, 1, 1)
        direct.set_graph(False)
        _, di = direct.solve(f)
        torch.cuda.synchronize()
        out["direct_local_solves"] = {
            "time_to_solution_s": td, "outer_iters": sd[-1]["outer_iters"],
            "subdomain_solves_per_s": sd[-1]["subdomain_solves"] / td,
            "true_relres": true_relres(torch, direct, f, ud), "status": sd[-1]["status"],
            "ms_per_precond_apply": di["ms_inner"] / max(di["precond_applies"], 1),
            "algorithmic_GB_per_apply": di["inner_bytes"] / max(di["precond_applies"], 1) / 1e9}
        direct.close()
    if not args.no_guess:
        progress("learned guess")
        out["learned_guess"] = guess_leg(torch, w, f, t / args.steps)
    if not args.no_two_level:
        progress("two-level")
        out["two_level"] = two_level_leg(torch, w, f, args.coarse_intervals or default_coarse_intervals(w),
                                         t / args.steps)
    if not args.no_tol_sweep:
        progress("inner-tolerance sweep")
        out["tol_sweep"] = tol_sweep_leg(torch)
    if not args.no_tol_sweep and args.workload == "large":
        progress("inner-tolerance study on the headline workload")
        out["large_inner_tol"] = large_tol_leg(torch, w, f)
    if not args.no_restart and args.workload == "large":
        progress("restart study")
        out["restart_study"] = restart_leg(torch, w, f)
    if not args.no_xlarge and args.workload == "large":
        progress("xlarge")
        out["xlarge"] = xlarge_batches(torch)
    if not args.no_cpu:
        progress("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_outer)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
