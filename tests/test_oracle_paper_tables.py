"""The paper's own experiments (Sec. 3, Tables 1-4) in its own setting -- Dirichlet local
matrices (eq. 3), quadratic Bezier deflation (Sec. 2), n_glob = 1.5 k (10 points per
wavelength) or 3 k (20) interior nodes per edge, uniform sqrt(N) x sqrt(N) splits with one
appended element layer, unit point source at the centre -- run by the oracle for k = 20,
40 and N = 4, 9, 16, 25 (tests/golden/paper_mesh_tables.json, written by
tests/golden/make_golden.py --paper-tables).

The paper's exact counts depend on settings it does not state (PETSc/FreeFem defaults:
restarts, orthogonalisation, partition of unity, mesh diagonal), so exact parity with its
tables is not asserted ("parity unpinned").  Asserted instead:
* the trends the tables show robustly: outer counts grow with k at fixed N and ppwl, and
  from N = 4 to N = 25; average inner counts fall as the inner tolerance loosens
  (1e-10 > 1e-5 > 1e-2, Tables 2-4); a loose inner tolerance costs outer iterations
  (1e-2 >= direct - 2);
* exact inner solves reproduce the direct counts: the 1e-10 runs are within 3 of Table 1's
  analogue (with the recovery step the inner tolerance bounds the true local residual);
* the no-recovery diagnostic: taking the deflated system's x as the local solution (no
  recovery step) does not reproduce the paper's modest 1e-10 excess over its direct counts --
  FGMRES needs over ten times the iterations or does not converge in 3000;
* the oracle's direct counts lie within [0.7, 1.5] times the paper's Table 1 values, cell
  by cell (a band, stated here, not a parity claim);
* the golden file is the oracle's: one cell is recomputed here.
"""

import json
import os

import pytest

from oracle import schwarz
from paper_2103_17081_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_mesh_tables.json")
NS = [4, 9, 16, 25]
# Sec. 3, Table 1: outer FGMRES iterations with direct subdomain solves, keyed (k, ppwl)
TABLE1 = {(20, 10): [20, 27, 48, 45], (40, 10): [31, 60, 85, 101],
          (20, 20): [20, 40, 42, 59], (40, 20): [37, 66, 89, 115]}


@pytest.fixture(scope="module")
def rows():
    with open(GOLDEN) as fh:
        data = json.load(fh)["rows"]
    assert len(data) == 16
    return {(r["k"], r["ppwl"], r["N"]): r for r in data}


def test_every_run_converged(rows):
    for r in rows.values():
        for mode in ("direct", "1e-10", "1e-05", "0.01"):
            assert r[mode]["relres"] <= 1e-6, (r["k"], r["ppwl"], r["N"], mode)


def test_outer_counts_grow_with_k_and_subdomains(rows):
    for ppwl in (10, 20):
        for N in NS:
            for mode in ("direct", "1e-10", "1e-05", "0.01"):
                assert rows[(40, ppwl, N)][mode]["outer"] > rows[(20, ppwl, N)][mode]["outer"]
        for k in (20, 40):
            for mode in ("direct", "1e-10", "1e-05", "0.01"):
                assert rows[(k, ppwl, 25)][mode]["outer"] > rows[(k, ppwl, 4)][mode]["outer"]


def test_inner_counts_fall_as_tolerance_loosens(rows):
    for r in rows.values():
        a10, a5, a2 = r["1e-10"]["avg_inner"], r["1e-05"]["avg_inner"], r["0.01"]["avg_inner"]
        assert a10 > a5 > a2 > 1.0
        # each loosening by five orders of magnitude roughly halves the inner count here
        assert a10 > 1.5 * a5 and a5 > 1.5 * a2


def test_loose_inner_tolerance_costs_outer_iterations(rows):
    for r in rows.values():
        assert r["0.01"]["outer"] >= r["direct"]["outer"] - 2
        assert r["1e-05"]["outer"] >= r["direct"]["outer"] - 2


def test_tight_inner_tolerance_reproduces_direct_counts(rows):
    for r in rows.values():
        assert abs(r["1e-10"]["outer"] - r["direct"]["outer"]) <= 3, (r["k"], r["ppwl"], r["N"])


def test_no_recovery_does_not_explain_the_paper_excess(rows):
    for r in rows.values():
        nr = r["no_recovery_1e-10"]
        assert (not nr["converged"]) or nr["outer"] >= 10 * r["1e-10"]["outer"], (r["k"], r["ppwl"], r["N"])


def test_direct_counts_within_band_of_table1(rows):
    for (k, ppwl), paper in TABLE1.items():
        for N, p in zip(NS, paper):
            ours = rows[(k, ppwl, N)]["direct"]["outer"]
            assert 0.7 * p <= ours <= 1.5 * p, (k, ppwl, N, ours, p)


def test_golden_cell_is_the_oracle(rows):
    """k = 20, 10 ppwl, N = 4, recomputed: direct and inner tolerance 1e-2."""
    r = rows[(20, 10, 4)]
    n = r["n_glob"] + 1
    cuts = inputs.uniform_cuts(n, 2)
    S = schwarz.Schwarz(schwarz.Problem(20.0, n, cuts, cuts, 1, "dirichlet", "bezier"))
    f = inputs.point_source(n)
    _, d = S.solve(f, mode="direct", outer_maxit=3000)
    _, st = S.solve(f, mode="deflated", inner_tol=1e-2, inner_maxit=300, outer_maxit=3000)
    assert d.outer_iters == r["direct"]["outer"]
    assert st.outer_iters == r["0.01"]["outer"]
    assert st.avg_inner == pytest.approx(r["0.01"]["avg_inner"], rel=1e-12)
