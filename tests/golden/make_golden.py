"""Write tests/golden/oracle_counts.json from the oracle alone.

Usage: python tests/golden/make_golden.py small [medium] [large]

For each named workload (paper_2103_17081_amd.inputs.workload) and its first right-hand
side, runs the oracle's outer FGMRES with impedance (ORAS) local matrices, linear
deflation and deflated-GMRES subdomain solves at the workload's inner tolerance, and
records the outer count, total inner iterations, subdomain solves and the true relative
residual.  Existing entries for other workloads are kept.
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


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names:
        w = inputs.workload(name)
        S = schwarz.Schwarz(schwarz.problem_from_workload(w))
        t = time.time()
        _, st = S.solve(w.rhs[0], mode="deflated", inner_tol=w.inner_tol, outer_maxit=5000)
        data[name] = {
            "outer_iters": st.outer_iters,
            "inner_iters": st.inner_iters,
            "subdomain_solves": st.subdomain_solves,
            "true_relres": st.true_relres,
            "inner_tol": w.inner_tol,
            "outer_tol": w.outer_tol,
            "oracle_seconds": round(time.time() - t, 1),
        }
        print(name, data[name], flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["small"])
