"""Write tests/golden/oracle_counts.json from the oracle alone.

Usage: python tests/golden/make_golden.py small [medium] [large]
       python tests/golden/make_golden.py --tol-sweep medium 0.1 0.0001
       python tests/golden/make_golden.py --spread-tol medium 0.1 16 [AMP]
       python tests/golden/make_golden.py --spread small [medium]
       python tests/golden/make_golden.py --direct small [medium] [large]
       python tests/golden/make_golden.py --two-level small:16 [medium:80]
       python tests/golden/make_golden.py --paper-two-level
       python tests/golden/make_golden.py --paper-tables [workers]
       python tests/golden/make_golden.py --recycling small [medium]

For each named workload (paper_2103_17081_amd.inputs.workload) and its first right-hand
side, runs the oracle's outer FGMRES with impedance (ORAS) local matrices, linear
deflation and deflated-GMRES subdomain solves at the workload's inner tolerance, and
records the outer count, total inner iterations, subdomain solves and the true relative
residual.  Existing entries for other workloads are kept.  --direct records, under
"direct", the same run with exact (sparse LU) subdomain solves.  --two-level NAME:M
records, under "two_level" -> "M", the oracle's two-level method (global coarse space of
M coarse intervals per edge) with deflated-GMRES and with exact subdomain solves.
--paper-two-level writes paper_mesh_two_level.json: the paper's variant in its mesh mode
(Dirichlet local matrices, Bezier deflation, k = 20 and 40 at 10 points per wavelength,
N = 4, 9, 16, 25) without and with the global coarse space (M = n/2), and the two-level
counts' spread under coarse solutions perturbed by 1e-12 relative.
--recycling writes recycling_study.json: the one-level solve with the subdomain GMRES
solves recycling across outer iterations (oracle/recycling.py, GCRO-DR) for recycle
spaces of k = 5, 10 (and 20 on small) harmonic Ritz vectors updated after every solve, and k = 5 kept
from the first solve: outer count, average inner count, and the mean over applications of
the largest subdomain iteration count (what bounds a batched launch).
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import schwarz  # noqa: E402
from paper_2103_17081_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "oracle_counts.json")


EPS32 = 2.0 ** -24   # complex64 unit roundoff


def store(path, update):
    """Apply update(data) to the JSON file at path, re-read under an exclusive lock just
    before writing, so that oracle runs started side by side keep each other's entries."""
    import fcntl
    with open(path + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        data = json.load(open(path)) if os.path.exists(path) else {}
        update(data)
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    return data


def spread(name, seeds=8, tol=None, amp=1.0):
    """Outer counts of the oracle when its subdomain solves are perturbed at FP32 level.

    Mode "round": local right-hand sides and local solutions rounded to complex64.
    Mode "noise": local solutions multiplied by (1 + amp * EPS32 * xi), xi complex normal,
    seeded.  Each run is the oracle's FGMRES with the oracle's deflated-GMRES solves.
    amp > 1 models subdomain solves whose whole Krylov process runs in complex64: their
    results differ from the complex128 ones by a few unit roundoffs, not by one rounding.
    """
    import numpy as np
    from oracle import krylov
    w = inputs.workload(name)
    tol = w.inner_tol if tol is None else tol
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    r32 = lambda x: x.astype(np.complex64).astype(np.complex128)

    def run(post, pre=lambda f: f):
        def apply(r):
            us = []
            for s, f in zip(S.subs, S.local_rhs(r)):
                u, _, _ = s.deflated_gmres(pre(f), tol, 100)
                us.append(post(u))
            return S.scatter(us)
        return krylov.fgmres(lambda v: S.A @ v, apply, w.rhs[0], rtol=w.outer_tol, maxit=5000).iters

    counts = {"round": run(r32, r32)}
    noise = []
    for sd in range(seeds):
        rng = np.random.default_rng(1000 + sd)
        noise.append(run(lambda u: u * (1 + amp * EPS32 * (rng.standard_normal(u.size) +
                                                             1j * rng.standard_normal(u.size)))))
    counts["noise"] = noise
    allc = [counts["round"]] + noise
    counts["min"], counts["max"] = min(allc), max(allc)
    return counts


def solve_with_progress(S, w, inner_tol, label, every=50):
    """The oracle's outer FGMRES (as Schwarz.solve runs it) with a progress line every
    `every` preconditioner applications, for runs that take hours."""
    import numpy as np
    from oracle import krylov
    st = schwarz.SolveStats()
    count = [0]
    t0 = time.time()

    def precond(v):
        count[0] += 1
        if count[0] % every == 0:
            print(f"{label}: {count[0]} applications, {time.time() - t0:.0f} s", flush=True)
        return S.apply(v, "deflated", inner_tol, 200, st)

    f = w.rhs[0]
    res = krylov.fgmres(lambda v: S.A @ v, precond, f, rtol=w.outer_tol, maxit=5000)
    st.outer_iters = res.iters
    st.converged = res.converged
    st.history = res.history
    st.true_relres = float(np.linalg.norm(f - S.A @ res.x) / np.linalg.norm(f))
    return st


def main(names):
    for name in names:
        w = inputs.workload(name)
        S = schwarz.Schwarz(schwarz.problem_from_workload(w))
        t = time.time()
        st = solve_with_progress(S, w, w.inner_tol, name)
        entry = {
            "outer_iters": st.outer_iters,
            "inner_iters": st.inner_iters,
            "subdomain_solves": st.subdomain_solves,
            "true_relres": st.true_relres,
            "inner_tol": w.inner_tol,
            "outer_tol": w.outer_tol,
            "oracle_seconds": round(time.time() - t, 1),
        }
        # other keys of the entry (direct, two-level, spreads) are kept
        store(OUT, lambda d: d.setdefault(name, {}).update(entry))
        print(name, entry, flush=True)


def tol_sweep(name, tols):
    """The workload's one-level solve at other inner tolerances (the inner-tolerance study of
    Sec. 3, Tables 2-4), with the spread of outer counts under FP32-level perturbations of
    the subdomain solves at each tolerance; stored under entry["tol_sweep"][tol]."""
    w = inputs.workload(name)
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    for tol in tols:
        t = time.time()
        st = solve_with_progress(S, w, tol, f"{name} tol {tol:g}")
        entry = {"outer_iters": st.outer_iters, "inner_iters": st.inner_iters,
                 "subdomain_solves": st.subdomain_solves, "true_relres": st.true_relres,
                 "inner_tol": tol, "outer_tol": w.outer_tol, "oracle_seconds": round(time.time() - t, 1)}
        entry["fp32_perturbed_outer"] = spread(name, 2, tol)
        key = f"{tol:g}"
        store(OUT, lambda d: d.setdefault(name, {}).setdefault("tol_sweep", {}).update({key: entry}))
        print(name, key, entry, flush=True)


def direct(names):
    for name in names:
        w = inputs.workload(name)
        S = schwarz.Schwarz(schwarz.problem_from_workload(w))
        t = time.time()
        _, st = S.solve(w.rhs[0], mode="direct", outer_maxit=5000)
        entry = {"outer_iters": st.outer_iters, "true_relres": st.true_relres,
                 "oracle_seconds": round(time.time() - t, 1)}
        store(OUT, lambda d: d.setdefault(name, {}).update({"direct": entry}))
        print(name, entry, flush=True)


def perturbed_two_level(T, w, seeds=4, eps=1e-12):
    """Outer counts of the oracle's two-level method when every coarse solution is
    multiplied by (1 + eps xi), xi standard normal (seeded): the spread that coarse solves
    accurate to ~1e-12 relative, instead of the sparse LU's ~1e-16, can cause."""
    import numpy as np
    exact = T.coarse.coarse_solve
    out = {}
    for mode in ("deflated", "direct"):
        counts = []
        for sd in range(seeds):
            rng = np.random.default_rng(2000 + sd)
            T.coarse.coarse_solve = lambda t, r=rng: (lambda y: y * (1 + eps * r.standard_normal(y.size)))(exact(t))
            _, st = T.solve(w.rhs[0], mode=mode, inner_tol=w.inner_tol, outer_maxit=5000)
            counts.append(st.outer_iters)
        out[mode] = counts
    T.coarse.coarse_solve = exact
    return out


def two_level(specs):
    from oracle import coarse_space
    for spec in specs:
        name, m = spec.split(":")
        w = inputs.workload(name)
        T = coarse_space.TwoLevel(schwarz.Schwarz(schwarz.problem_from_workload(w)), int(m))
        t = time.time()
        _, st = T.solve(w.rhs[0], mode="deflated", inner_tol=w.inner_tol, outer_maxit=5000)
        _, sd = T.solve(w.rhs[0], mode="direct", outer_maxit=5000)
        entry = {
            "outer_iters": st.outer_iters, "inner_iters": st.inner_iters, "subdomain_solves": st.subdomain_solves,
            "true_relres": st.true_relres, "direct_outer_iters": sd.outer_iters,
            "oracle_seconds": round(time.time() - t, 1)}
        if name == "small":
            entry["coarse_perturbed_outer"] = perturbed_two_level(T, w)
        store(OUT, lambda d: d.setdefault(name, {}).setdefault("two_level", {}).update({m: entry}))
        print(name, m, entry, flush=True)


def paper_two_level():
    import numpy as np
    from oracle import coarse_space
    rows = []
    for k, nglob in ((20, 30), (40, 60)):
        n = nglob + 1
        f = inputs.point_source(n)
        for N in (4, 9, 16, 25):
            P = int(round(N ** 0.5))
            cuts = inputs.uniform_cuts(n, P)
            S = schwarz.Schwarz(schwarz.Problem(float(k), n, cuts, cuts, 1, "dirichlet", "bezier"))
            _, s1 = S.solve(f, mode="deflated", inner_tol=1e-2)
            T = coarse_space.TwoLevel(S, n // 2)
            _, s2 = T.solve(f, mode="deflated", inner_tol=1e-2)
            exact = T.coarse.coarse_solve
            spread = []
            for sd in range(4):
                rng = np.random.default_rng(3000 + sd)
                T.coarse.coarse_solve = lambda t, r=rng: (lambda y: y * (1 + 1e-12 * r.standard_normal(y.size)))(exact(t))
                _, sp_ = T.solve(f, mode="deflated", inner_tol=1e-2)
                spread.append(sp_.outer_iters)
            T.coarse.coarse_solve = exact
            rows.append({"k": k, "n_glob": nglob, "N": N, "M": n // 2, "one_level": s1.outer_iters,
                         "two_level": s2.outer_iters, "two_level_perturbed": spread})
            print(rows[-1], flush=True)
    with open(os.path.join(HERE, "paper_mesh_two_level.json"), "w") as fh:
        json.dump({"source": "oracle (tests/golden/make_golden.py --paper-two-level)", "rows": rows}, fh, indent=1)


def _paper_cell(args):
    """One (k, ppwl, N) cell of the paper's Tables 1-4 in its own setting (Dirichlet local
    matrices, Bezier deflation, n_glob interior nodes per edge, point source at the centre):
    outer counts and average inner counts with direct subdomain solves and with deflated
    GMRES at inner tolerances 1e-10, 1e-5 and 1e-2; plus the no-recovery diagnostic, the
    1e-10 run with the local solution taken as the deflated system's x (no recovery)."""
    import numpy as np
    from oracle import krylov
    k, ppwl, N = args
    nglob = int(round(1.5 * k)) if ppwl == 10 else 3 * k
    n = nglob + 1
    P = int(round(N ** 0.5))
    cuts = inputs.uniform_cuts(n, P)
    f = inputs.point_source(n)
    S = schwarz.Schwarz(schwarz.Problem(float(k), n, cuts, cuts, 1, "dirichlet", "bezier"))
    cell = {"k": k, "ppwl": ppwl, "n_glob": nglob, "N": N}
    t0 = time.time()
    _, st = S.solve(f, mode="direct", outer_maxit=3000)
    cell["direct"] = {"outer": st.outer_iters, "relres": st.true_relres}
    for tol in (1e-10, 1e-5, 1e-2):
        _, st = S.solve(f, mode="deflated", inner_tol=tol, inner_maxit=300, outer_maxit=3000)
        cell[f"{tol:g}"] = {"outer": st.outer_iters, "avg_inner": st.avg_inner, "relres": st.true_relres}
    # no recovery: the subdomain "solution" is x of P B x = P f
    stats = schwarz.SolveStats()

    def apply_x(r):
        us = []
        for sd, fj in zip(S.subs, S.local_rhs(r)):
            d = sd.defl
            Pf = d.P(fj)
            ref = np.linalg.norm(Pf)
            if ref == 0.0:
                us.append(np.zeros_like(fj))
                continue
            res = krylov.gmres(d.PB, Pf, rtol=1e-10, maxit=300, ref_norm=ref)
            stats.inner_iters += res.iters
            stats.subdomain_solves += 1
            us.append(res.x)
        return S.scatter(us)

    res = krylov.fgmres(lambda v: S.A @ v, apply_x, f, rtol=1e-6, maxit=3000)
    cell["no_recovery_1e-10"] = {"outer": res.iters, "converged": bool(res.converged),
                                 "avg_inner": stats.avg_inner}
    cell["seconds"] = round(time.time() - t0, 1)
    print(json.dumps(cell), flush=True)
    return cell


def recycling_study(names):
    import numpy as np
    from oracle import recycling
    path = os.path.join(HERE, "recycling_study.json")
    for name in names:
        w = inputs.workload(name)
        S = schwarz.Schwarz(schwarz.problem_from_workload(w))
        rows = []
        configs = ((0, True), (5, False), (5, True), (10, True))
        if name == "small":
            configs += ((20, True),)   # 20 vectors cost seconds per solve in this dense oracle
        for k, update in configs:
            t0 = time.time()
            R = recycling.RecyclingSchwarz(S, k, update)
            _, st = R.solve(w.rhs[0], inner_tol=w.inner_tol, outer_maxit=3000)
            row = {"k": k, "update": update, "outer_iters": st.outer_iters, "avg_inner": st.avg_inner,
                   "mean_max_inner_per_apply": float(np.mean(R.max_per_apply)),
                   "true_relres": st.true_relres, "converged": st.converged,
                   "oracle_seconds": round(time.time() - t0, 1)}
            rows.append(row)
            print(name, json.dumps(row), flush=True)
            store(path, lambda d: d.update({name: {"inner_tol": w.inner_tol, "rows": list(rows),
                                                    "source": "oracle (tests/golden/make_golden.py --recycling)"}}))


def paper_tables(workers=4):
    """tests/golden/paper_mesh_tables.json: _paper_cell over k = 20, 40, ppwl = 10, 20,
    N = 4, 9, 16, 25 (a process per cell)."""
    import multiprocessing as mp
    cells = [(k, ppwl, N) for k in (20, 40) for ppwl in (10, 20) for N in (4, 9, 16, 25)]
    with mp.get_context("fork").Pool(workers) as pool:
        rows = pool.map(_paper_cell, cells, chunksize=1)
    with open(os.path.join(HERE, "paper_mesh_tables.json"), "w") as fh:
        json.dump({"source": "oracle (tests/golden/make_golden.py --paper-tables)",
                   "setting": "Dirichlet local matrices, Bezier deflation, n_glob = 1.5 k (10 ppwl) or 3 k "
                              "(20 ppwl) interior nodes per edge, uniform N = P^2 subdomains with one "
                              "appended element layer, unit point source at the centre, outer FGMRES "
                              "rtol 1e-6 without restart, inner GMRES without restart (max 300)",
                   "rows": rows}, fh, indent=1)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--paper-two-level":
        paper_two_level()
    elif args and args[0] == "--paper-tables":
        paper_tables(int(args[1]) if len(args) > 1 else 4)
    elif args and args[0] == "--recycling":
        recycling_study(args[1:] or ["small"])
    elif args and args[0] == "--two-level":
        two_level(args[1:] or ["small:16"])
    elif args and args[0] == "--direct":
        direct(args[1:] or ["small"])
    elif args and args[0] == "--spread":
        for name in args[1:] or ["small"]:
            sp = spread(name, 8 if name == "small" else 2)
            store(OUT, lambda d: d.setdefault(name, {}).update({"fp32_perturbed_outer": sp}))
            print(name, sp, flush=True)
    elif args and args[0] == "--spread-tol":
        # --spread-tol NAME TOL SEEDS [AMP]: the FP32-perturbation spread of the outer count at
        # one inner tolerance, stored beside that tolerance's golden (the workload's own
        # tolerance at the entry's top level, others under tol_sweep).  With AMP (noise of AMP
        # unit roundoffs) the counts are added under "noise_amp<AMP>" and min/max cover all runs.
        name, tol, seeds = args[1], float(args[2]), int(args[3])
        amp = float(args[4]) if len(args) > 4 else 1.0
        sp = spread(name, seeds, tol, amp)
        key = f"{tol:g}"

        def merge(old):
            if amp == 1.0 or not old:
                return sp
            new = dict(old)
            new[f"noise_amp{amp:g}"] = sp["noise"]
            new["min"], new["max"] = min(old["min"], sp["min"]), max(old["max"], sp["max"])
            return new

        def put(d):
            e = d.setdefault(name, {})
            if e.get("inner_tol") == tol:
                e["fp32_perturbed_outer"] = merge(e.get("fp32_perturbed_outer"))
            else:
                t = e.setdefault("tol_sweep", {}).setdefault(key, {})
                t["fp32_perturbed_outer"] = merge(t.get("fp32_perturbed_outer"))
        store(OUT, put)
        print(name, key, sp, flush=True)
    elif args and args[0] == "--tol-sweep":
        tol_sweep(args[1], [float(t) for t in args[2:]])
    else:
        main(args or ["small"])
