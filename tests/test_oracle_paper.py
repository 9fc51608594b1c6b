"""The oracle reproduces the numbers the paper prints (Section 5 tables).

The integers (dimension of the GenEO coarse space, rank of A_-) must match
exactly; condition numbers (Lanczos estimates from the PCG coefficients)
within 3 %; iteration counts, counted with the preconditioned residual norm
as PETSc's CG does by default, within 2.
"""
import json
import os

import numpy as np
import pytest

import awg_problems as P
from awg_problems import configs as C
from oracle import awg_oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
LAYERS = {"THREE": C.THREE_LAYERS, "NINE": C.NINE_LAYERS}


def _x0(kwargs, tau):
    kw = dict(kwargs)
    if "layers" in kw:
        kw["layers"] = LAYERS[kw["layers"]]
    return P.paper_x0(tau=tau, **kw)


def _check(w, case, st=None):
    st = st or O.setup(w.A, w.subs, w.tau)
    assert st.n_minus == case["n_minus"]
    assert st.n0 == case["n0"]
    res = O.pcg(w.A, w.b, st.apply, tol=1e-10, norm="preconditioned", maxit=200)
    assert res.converged
    lmin, lmax = res.lanczos_extremes()
    assert abs(lmax / lmin - case["kappa"]) <= 0.03 * case["kappa"]
    assert abs(res.iters - case["it"]) <= 2
    if "lmin" in case:
        assert abs(lmin - case["lmin"]) <= 0.05
        assert abs(lmax - case["lmax"]) <= 0.05 * case["lmax"]
    return st


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_paper_table_rows(case):
    w = _x0(case["kwargs"], case["tau"])
    assert w.A.shape[0] == 8064          # stated size of the test problem
    st = _check(w, case)
    if case["name"] == "six_layers":
        cs = GOLD["central_subdomain"]
        assert st.split[4].nneg == cs["kernel"]
        assert st.Y[4].shape[1] == cs["selected"]


T1 = GOLD["table1_awg_variants"]


@pytest.fixture(scope="module")
def six_layers():
    w = P.paper_x0(tau=0.1)
    return w, O.setup(w.A, w.subs, w.tau)


@pytest.mark.parametrize("row", T1["rows"], ids=[f"{r['coarse2']}-{r['h2']}" for r in T1["rows"]])
def test_paper_table1_awg_variants(six_layers, row):
    """The eight AWG rows of Table 1: H3,ad and H3,hyb, each with
    H^NN_hyb(0.1), H^AS_hyb(0.1, 10), H^AS_{+,hyb}(10) and H^AS_{+,ad}(10) as
    H2, on the six-layer problem."""
    w, st = six_layers
    assert st.n0 == T1["n0"] and st.n_minus == T1["n_minus"]
    h2 = st.h2(row["h2"])
    ap = (lambda r: st.apply(r, h2=h2)) if row["coarse2"] == "ad" else (lambda r: st.apply_hyb(r, h2=h2))
    res = O.pcg(w.A, w.b, ap, tol=1e-10, norm="preconditioned", maxit=200)
    assert res.converged
    lmin, lmax = res.lanczos_extremes()
    assert abs(lmax / lmin - row["kappa"]) <= 0.03 * row["kappa"]
    assert abs(res.iters - row["it"]) <= 2
    assert abs(lmin - row["lmin"]) <= 0.05 * max(1.0, row["lmin"])
    assert abs(lmax - row["lmax"]) <= 0.05 * row["lmax"]


T4 = GOLD["table4_w_rtol"]


@pytest.mark.parametrize("row", [r for r in T4["rows"] if r["w_rtol"] <= 1e-2], ids=lambda r: f"rtol{r['w_rtol']:g}")
def test_paper_table4_w_tolerance(row):
    """W from PCG with H2 stopped at w_rtol (Table 4): up to 1e-2 kappa and
    the iteration count are those of the exact W.  Looser rows are not
    compared: the paper's W solves stop on the preconditioned residual norm,
    these on ||r||_2, and at 0.05 and beyond the two stop at different
    iterates."""
    w = P.paper_x0(tau=0.1)
    st = O.setup(w.A, w.subs, w.tau, w_solver="pcg", w_rtol=row["w_rtol"])
    assert st.n0 == T4["n0"] and st.n_minus == T4["n_minus"]
    res = O.pcg(w.A, w.b, st.apply, tol=1e-10, norm="preconditioned", maxit=200)
    assert res.converged
    lmin, lmax = res.lanczos_extremes()
    assert abs(lmax / lmin - row["kappa"]) <= 0.03 * row["kappa"]
    assert abs(res.iters - row["it"]) <= 2


def test_paper_table4_nu04_exact_w():
    """Table 4, nu = 0.4, with W to 1e-10: #V0, n_-, kappa and iterations.
    The 1e-2 row is not compared: there the paper's W solves (preconditioned
    norm) and these (||r||_2) stop at different iterates."""
    g = GOLD["table4_nu04"]
    row = g["rows"][0]
    w = P.paper_x0(tau=g["tau"], **g["kwargs"])
    st = O.setup(w.A, w.subs, w.tau, w_solver="pcg", w_rtol=row["w_rtol"])
    assert st.n0 == g["n0"] and st.n_minus == g["n_minus"]
    res = O.pcg(w.A, w.b, st.apply, tol=1e-10, norm="preconditioned", maxit=200)
    assert res.converged
    lmin, lmax = res.lanczos_extremes()
    assert abs(lmax / lmin - row["kappa"]) <= 0.03 * row["kappa"]
    assert abs(res.iters - row["it"]) <= 2


@pytest.mark.parametrize("i", range(5))
def test_paper_long_domain(i):
    g = GOLD["long_domain"]
    N = g["N"][i]
    w = P.paper_long(N)
    case = dict(n_minus=g["n_minus"][i], n0=g["n0"][i], kappa=g["kappa"][i], it=g["it"][i])
    _check(w, case)


def test_paper_problem_unpreconditioned_count_recorded():
    """With the plain ||r_k||/||b|| test used by this repository the same
    solve takes more iterations; record that it still converges with the
    same true residual level."""
    w = P.paper_x0()
    st = O.setup(w.A, w.subs, w.tau)
    res = O.pcg(w.A, w.b, st.apply, tol=1e-10)
    # the recursive residual reaches 1e-10; the true residual stalls near the
    # rounding floor of b - A x (about 6e-10 here), so the restarts from the
    # true residual run out and the solve reports non-convergence honestly
    assert min(res.res_hist) <= 1e-10 and res.rel_res_true <= 2e-9
    assert res.iters >= 26 and res.restarts <= 5
    assert np.isfinite(res.rel_res_true)
    res8 = O.pcg(w.A, w.b, st.apply, tol=1e-8)
    assert res8.converged and res8.restarts == 0 and res8.rel_res_true <= 1e-8
