"""Write tests/golden/paper_rows_refined_oracle.json: the FP64 oracle on rows
of the paper's parameter studies (Tables 2, 3 and 5) for its six-layer
elasticity problem on refined meshes, with the stopping test the GPU tests
use (||r||/||b|| <= 1e-8, x0 = 0).

Mesh h = 1/(21 p) with every unit square cut into p x p box subdomains that
share only their interface nodes (N = 9 p^2): the subdomains keep the size of
the paper's own mesh (h = 1/21, N = 9, n = 8064) while n and N grow by p^2.

Calls only the oracle and the input generators.  Run from the repository
root (about 25 minutes):
    python tests/golden/make_refined_rows.py
BLAS runs single-threaded: its summation order changes the rounding, and on
these rows the Lanczos estimate of kappa depends on it (b has almost no
component along the top eigenvectors of HA, so whether a run finds them is
decided by rounding: 14.94 with one thread, 16.01 with four on
p4:homogeneous); with one thread the stored values are reproducible.
Recorded per row: the integers, the iteration count, the restarts from the
true residual and the length of the first run of the recurrence (whose
coefficients give the kappa estimate).
"""
import json
import os
import sys
import time

for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from awg_problems import configs as C  # noqa: E402
from oracle import awg_oracle as O  # noqa: E402

# (p, row name) pairs; the rows take their parameters from the paper's tables
MESHES = (2, 4)
ROWS = {
    "six_layers": dict(tau=0.1),
    "homogeneous": dict(tau=0.1, E1=1e11, E2=1e11),
    "three_layers": dict(tau=0.1, layers="THREE"),
    "nine_layers": dict(tau=0.1, layers="NINE"),
    "E_1e5_1e11": dict(tau=0.1, E1=1e5, E2=1e11),
    "nu_0.4": dict(tau=0.05, E1=1e11, E2=1e11, nu=0.4),
    "nu_0.49": dict(tau=0.05, E1=1e11, E2=1e11, nu=0.49),
}
LAYERS = {"THREE": C.THREE_LAYERS, "NINE": C.NINE_LAYERS}
# the oracle's dense W of this row (n = 127,512 by n_- of about 7,000, with its
# right-hand sides and solves) needs more host memory than 64 GB
SKIP = {"p4:nu_0.49"}
OUT = os.path.join(ROOT, "tests", "golden", "paper_rows_refined_oracle.json")


def workload(p, row):
    kw = dict(ROWS[row])
    if "layers" in kw:
        kw["layers"] = LAYERS[kw["layers"]]
    return C.paper_x0_refined(21 * p, p, **kw)


def main():
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for p in MESHES:
        for row in ROWS:
            key = f"p{p}:{row}"
            if (key in out and "iters_first" in out[key]) or key in SKIP:
                continue
            t0 = time.perf_counter()
            w = workload(p, row)
            # 2D: a sparse LU of A_+ builds W exactly at every size here
            st = O.setup(w.A, w.subs, w.tau, w_solver="direct")
            r = O.pcg(w.A, w.b, st.apply, tol=1e-8, maxit=2000)
            lmin, lmax = r.lanczos_extremes()
            s = O.stats(st)
            out[key] = {"n": s["n"], "N": s["N"], "n_minus": int(s["n_minus"]), "n0": int(s["n0"]),
                        "iters": int(r.iters), "restarts": int(r.restarts), "iters_first": len(r.alphas),
                        "kappa": float(lmax / lmin), "converged": bool(r.converged),
                        "rel_res_true": float(r.rel_res_true), "e0_margin": float(s["e0_margin"]),
                        "ew_margin": float(s["ew_margin"])}
            print(key, out[key], f"{time.perf_counter() - t0:.0f} s", flush=True)
            with open(OUT, "w") as f:
                json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
