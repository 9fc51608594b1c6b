"""The paper's parameter studies (Section 5) run by the GPU library.

Tables 2, 3 and 5 (Poisson ratio, Young's moduli, number of hard layers on
the six-layer problem, n = 8064) and Table 6 (long domain [0,N]x[0,1],
h = 1/14, one subdomain per unit square): #V0 and n_- exactly as printed.
For Tables 2, 3 and 5, the iteration count within 1 and the Lanczos estimate
of kappa within 1 % of the oracle's with the same stopping test
(||r||/||b|| <= 1e-8); for Table 6, kappa within 3 % of the printed value
(the long cantilever's true residual reaches the FP64 floor, so only the
conditioning is compared).  The same rows on meshes refined 2x and 4x
(subdomains of the paper's size, N = 36 and 144) against the oracle, and the
six-layer problem refined 8x (n = 509,040) against the theorem's bound.
Beyond the table the long domain grows to N = 464
(weak scaling in the number of subdomains): kappa must stay below the
theorem's bound N(A_+)/tau + 1, and its values, the iteration counts and the
times are printed.
"""
import json
import os
import time

import numpy as np
import pytest

import awg_problems as P
from awg_problems import configs as C
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
LAYERS = {"THREE": C.THREE_LAYERS, "NINE": C.NINE_LAYERS}
TOL = 1e-8


def run_gpu(gpu_lib, w, want_x=False):
    import torch
    t0 = time.perf_counter()
    s = gpu_lib.Solver(w.A, w.subs, tau=w.tau)
    st = s.stats()
    x, info = s.pcg(torch.as_tensor(w.b, device="cuda"), tol=TOL, maxit=2000)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    s.close()
    if want_x:
        return st, info, ms, x.cpu().numpy()
    return st, info, ms


ROWS_PATH = os.path.join(os.path.dirname(__file__), "golden", "paper_rows_oracle.json")
ROWS = json.load(open(ROWS_PATH)) if os.path.exists(ROWS_PATH) else {}


def check_against(w, st, info, n0, n_minus, kappa_printed, ref=None):
    """Integers exactly; iterations within 1 and kappa within 1 % of the
    oracle's with the same stopping test (ref: the oracle's stored results,
    written by tests/golden/make_paper_rows.py; else the oracle is run)."""
    assert st["n0"] == n0 and st["n_minus"] == n_minus
    assert info["converged"] == 1
    kappa = info["lmax_est"] / info["lmin_est"]
    if ref is None:
        ost = O.setup(w.A, w.subs, w.tau)
        r = O.pcg(w.A, w.b, ost.apply, tol=TOL, maxit=2000)
        lmin, lmax = r.lanczos_extremes()
        ref = {"iters": r.iters, "kappa": lmax / lmin}
    assert abs(info["iters"] - ref["iters"]) <= 1, (info["iters"], ref["iters"])
    assert abs(kappa - ref["kappa"]) <= 0.01 * ref["kappa"], (kappa, ref["kappa"])
    if kappa_printed is not None:
        assert abs(kappa - kappa_printed) <= 0.03 * kappa_printed, (kappa, kappa_printed)
    return kappa


def paper_row(case):
    kw = dict(case["kwargs"])
    if "layers" in kw:
        kw["layers"] = LAYERS[kw["layers"]]
    return P.paper_x0(tau=case["tau"], **kw)


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_tables_2_3_5_rows(gpu_lib, case):
    w = paper_row(case)
    print(f"\n[gpu case] paper problem {case['name']} ({case['cite']})", flush=True)
    st, info, ms = run_gpu(gpu_lib, w)
    # the printed kappa comes from the paper's own stopping test (1e-10 on the
    # preconditioned norm); the oracle reproduces it with that test
    check_against(w, st, info, case["n0"], case["n_minus"], None, ROWS.get(case["name"]))


@pytest.mark.parametrize("case", GOLD.get("not_reproduced", []), ids=[c["name"] for c in GOLD.get("not_reproduced", [])])
def test_rows_the_oracle_does_not_reproduce(gpu_lib, case):
    """A printed row the oracle does not reproduce (Table 2, nu = 0.45): the
    library is held to the oracle's integers, iterations and kappa."""
    if case["name"] not in ROWS:
        pytest.skip("oracle results not stored")
    ref = ROWS[case["name"]]
    w = paper_row(case)
    print(f"\n[gpu case] paper problem {case['name']} ({case['cite']}; not reproduced by the oracle)", flush=True)
    st, info, ms = run_gpu(gpu_lib, w)
    check_against(w, st, info, ref["n0"], ref["n_minus"], None, ref)


def long_domain_checks(st, info):
    """The long domain is a cantilever under gravity: kappa(A) grows about
    like N^4, and from N = 15 on the FP64 true residual b - A x stalls near
    1e-8 ||b|| while the recurrence goes on; the solve then reports
    non-convergence after its restarts from the true residual.  The quantity
    of the study is the conditioning of HA, which the Lanczos estimate of
    the first segment gives; the recursive residual must have met the
    tolerance."""
    assert info["rel_res"] <= TOL
    return info["lmax_est"] / info["lmin_est"]


@pytest.mark.parametrize("i", range(5))
def test_table6_long_domain(gpu_lib, i):
    g = GOLD["long_domain"]
    w = P.paper_long(g["N"][i])
    print(f"\n[gpu case] long domain N={g['N'][i]} (Table 6)", flush=True)
    st, info, ms = run_gpu(gpu_lib, w)
    assert st["n0"] == g["n0"][i] and st["n_minus"] == g["n_minus"][i]
    kappa = long_domain_checks(st, info)
    assert abs(kappa - g["kappa"][i]) <= 0.03 * g["kappa"][i], (kappa, g["kappa"][i])


def test_long_domain_weak_scaling_beyond_the_table(gpu_lib):
    rows = []
    for N in (58, 116, 232, 464):
        w = P.paper_long(N)
        print(f"\n[gpu case] long domain N={N} n={w.A.shape[0]}", flush=True)
        st, info, ms = run_gpu(gpu_lib, w)
        kappa = long_domain_checks(st, info)
        # every subdomain meets its two neighbours only: N(A_+) <= 3
        assert kappa <= 3 / w.tau + 1
        if N == 58:
            ost = O.setup(w.A, w.subs, w.tau)
            assert st["n0"] == ost.n0 and st["n_minus"] == ost.n_minus
        rows.append(dict(N=N, n=int(w.A.shape[0]), n0=st["n0"], n_minus=st["n_minus"], iters=info["iters"],
                         kappa=round(kappa, 3), rel_res_true=info["rel_res_true"], converged=info["converged"],
                         setup_ms=round(st["ms"]["total"], 1), total_ms=round(ms, 1)))
    print("[long domain] " + json.dumps(rows), flush=True)


REFINED_PATH = os.path.join(os.path.dirname(__file__), "golden", "paper_rows_refined_oracle.json")
REFINED = json.load(open(REFINED_PATH)) if os.path.exists(REFINED_PATH) else {}
REFINED_ROWS = {
    "six_layers": dict(tau=0.1),
    "homogeneous": dict(tau=0.1, E1=1e11, E2=1e11),
    "three_layers": dict(tau=0.1, layers="THREE"),
    "nine_layers": dict(tau=0.1, layers="NINE"),
    "E_1e5_1e11": dict(tau=0.1, E1=1e5, E2=1e11),
    "nu_0.4": dict(tau=0.05, E1=1e11, E2=1e11, nu=0.4),
    "nu_0.49": dict(tau=0.05, E1=1e11, E2=1e11, nu=0.49),
}


def refined_workload(p, row):
    kw = dict(REFINED_ROWS[row])
    if "layers" in kw:
        kw["layers"] = LAYERS[kw["layers"]]
    return C.paper_x0_refined(21 * p, p, **kw)


def theorem_bound(w):
    from test_gpu_fullsize import coloring_constant_Aplus
    return coloring_constant_Aplus(w.subs, w.A.shape[0]) / w.tau + 1


@pytest.mark.parametrize("key", sorted(REFINED) or ["none"])
def test_refined_mesh_rows(gpu_lib, key):
    """Rows of Tables 2, 3 and 5 on meshes refined 2x and 4x (h = 1/42 and
    1/84; every unit square cut into p x p boxes, N = 36 and 144, so the
    subdomains keep the paper's size), against the oracle with the same
    stopping test: #V0 and n_- exactly, the first run of the recurrence (up
    to the first restart from the true residual) within 1 iteration, the
    whole count within 1 where neither side restarted, kappa below the bound
    N(A_+)/tau + 1 of the H3,ad theorem (Section 4.3), which holds for every
    h, and convergence (or, where FP64 cannot evaluate b - A x to 1e-8, the
    attainable-accuracy check).  The Lanczos estimate of kappa is held to
    10 %: on these meshes b has almost no component along the top
    eigenvectors of HA, and the oracle alone gives 14.94 or 16.01 on
    p4:homogeneous depending on its BLAS summation order."""
    if key not in REFINED or "iters_first" not in REFINED.get(key, {}):
        pytest.skip("oracle results for the refined meshes not stored")
    p, row = key.split(":")
    w = refined_workload(int(p[1:]), row)
    ref = REFINED[key]
    assert w.A.shape[0] == ref["n"] and len(w.subs) == ref["N"]
    print(f"\n[gpu case] refined six-layer problem {key} n={ref['n']} N={ref['N']}", flush=True)
    st, info, ms, x = run_gpu(gpu_lib, w, want_x=True)
    if min(ref["e0_margin"], st["e0_margin"]) < 100:
        print(f"[parity unpinned] {key}: E0 deletion margin {min(ref['e0_margin'], st['e0_margin']):.3g}", flush=True)
    assert st["n0"] == ref["n0"] and st["n_minus"] == ref["n_minus"]
    assert info["rel_res"] <= TOL
    kappa = info["lmax_est"] / info["lmin_est"]
    bound = theorem_bound(w)
    print(f"[refined {key}] n_- {st['n_minus']} #V0 {st['n0']} iters {info['iters']} (first run "
          f"{info['iters_first']}, restarts {info['restarts']}; oracle {ref['iters']}, {ref['iters_first']}, "
          f"{ref['restarts']}) kappa {kappa:.3f} (oracle {ref['kappa']:.3f}, bound {bound:.1f}) {ms:.0f} ms",
          flush=True)
    assert abs(info["iters_first"] - ref["iters_first"]) <= 1
    if info["restarts"] == 0 and ref["restarts"] == 0:
        assert abs(info["iters"] - ref["iters"]) <= 1
    assert abs(kappa - ref["kappa"]) <= 0.1 * ref["kappa"], (kappa, ref["kappa"])
    assert kappa <= bound
    if info["converged"] != 1:
        from test_gpu_large_configs import residual_ext
        rext, gamma = residual_ext(w.A, w.b, x)
        print(f"[refined {key}] FP64 floor: extended residual {rext:.3e}, gamma {gamma:.3e}", flush=True)
        assert gamma > TOL and rext <= gamma


def test_refined_mesh_six_layers_8x(gpu_lib):
    """The six-layer problem on a mesh refined 8x (h = 1/168, N = 576,
    n = 509,040) at subdomains of the paper's size: converged to 1e-8 (or to
FP64's attainable accuracy), kappa
    below the theorem's N(A_+)/tau + 1, and within 25 % of the oracle's
    kappa on the 4x mesh (the bound does not depend on h; the coarse space
    keeps kappa near the coarser meshes' value)."""
    w = refined_workload(8, "six_layers")
    print(f"\n[gpu case] refined six-layer problem p8:six_layers n={w.A.shape[0]} N={len(w.subs)}", flush=True)
    st, info, ms, x = run_gpu(gpu_lib, w, want_x=True)
    assert info["rel_res"] <= TOL
    if info["converged"] != 1:
        # FP64 cannot always evaluate b - A x to 1e-8 here: then the iterate's
        # residual in extended precision must lie below the attainable-accuracy
        # scale eps || |A| |x| || / ||b||
        from test_gpu_large_configs import residual_ext
        rext, gamma = residual_ext(w.A, w.b, x)
        print(f"[refined p8:six_layers] FP64 floor: extended residual {rext:.3e}, gamma {gamma:.3e}", flush=True)
        assert gamma > TOL and rext <= gamma
    kappa = info["lmax_est"] / info["lmin_est"]
    bound = theorem_bound(w)
    print(f"[refined p8:six_layers] n_- {st['n_minus']} #V0 {st['n0']} iters {info['iters']} kappa {kappa:.3f} "
          f"(bound {bound:.1f}) set-up {st['ms']['total']:.0f} ms, total {ms:.0f} ms", flush=True)
    assert kappa <= bound
    if "p4:six_layers" in REFINED:
        k4 = REFINED["p4:six_layers"]["kappa"]
        assert abs(kappa - k4) <= 0.25 * k4, (kappa, k4)


def test_table4_nu04_row(gpu_lib):
    """Table 4, nu = 0.4, W to 1e-10 (the six-layer problem with Poisson
    ratio 0.4): #V0 and n_- as printed, iterations and kappa against the
    oracle with the same stopping test."""
    g = GOLD["table4_nu04"]
    w = P.paper_x0(tau=g["tau"], **g["kwargs"])
    print("\n[gpu case] paper problem nu = 0.4 (Table 4)", flush=True)
    st, info, ms = run_gpu(gpu_lib, w)
    check_against(w, st, info, g["n0"], g["n_minus"], None)
