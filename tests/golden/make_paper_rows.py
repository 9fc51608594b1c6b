"""Write tests/golden/paper_rows_oracle.json: the FP64 oracle on every row of
the paper's parameter studies on its own 2D elasticity problem (Tables 2, 3
and 5, n = 8064), with the stopping test the GPU tests use.

Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_paper_rows.py

For each row: n_-, #V0, the iteration count and the Lanczos estimate of
kappa of PCG from x0 = 0 stopped at ||r||/||b|| <= 1e-8 (the GPU tests
compare the library with these), and the same with the paper's stopping test
(1e-10 on the preconditioned norm), for the comparison with the printed values.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import awg_problems as P  # noqa: E402
from awg_problems import configs as C  # noqa: E402
from oracle import awg_oracle as O  # noqa: E402

LAYERS = {"THREE": C.THREE_LAYERS, "NINE": C.NINE_LAYERS}


def rows():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
    return gold["cases"] + gold.get("not_reproduced", [])


def main():
    out = {}
    for case in rows():
        kw = dict(case["kwargs"])
        if "layers" in kw:
            kw["layers"] = LAYERS[kw["layers"]]
        w = P.paper_x0(tau=case["tau"], **kw)
        st = O.setup(w.A, w.subs, w.tau)
        r8 = O.pcg(w.A, w.b, st.apply, tol=1e-8, maxit=2000)
        lmin, lmax = r8.lanczos_extremes()
        rp = O.pcg(w.A, w.b, st.apply, tol=1e-10, norm="preconditioned", maxit=2000)
        pmin, pmax = rp.lanczos_extremes()
        out[case["name"]] = {"n_minus": st.n_minus, "n0": st.n0, "iters": r8.iters, "kappa": lmax / lmin,
                             "iters_paper_test": rp.iters, "kappa_paper_test": pmax / pmin}
        print(case["name"], out[case["name"]], flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "paper_rows_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
