"""Write tests/golden/<workload>.json (and <workload>_x.npy with --full): the
FP64 oracle on the large synthetic workloads.

Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_large.py diff3d_64 --full
    python tests/golden/make_large.py q1_2d_512_rcb
    python tests/golden/make_large.py elast3d_40

Without --full the oracle stops after E0 (Theorem on H^NN_hyb, Section 3.4):
the integers that define the coarse spaces (k_s, strictly negative counts,
m_s, n_-, n0, the deleted coarse vectors and the deletion margins) do not
need W, whose dense n x n_- form does not fit in memory for the two largest
workloads.  With --full the oracle also builds W (sparse LU of A and the
Woodbury identity, exact), runs PCG and stores the whole iterate.  The wall
time of every oracle phase is recorded (the CPU baseline of the benchmark).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import awg_problems as P  # noqa: E402
from oracle import awg_oracle as O  # noqa: E402

WORKLOADS = {
    "q1_2d_512_rcb": lambda: P.q1_2d(m=512, seed=2, partition="rcb", nparts=256, delta=2),
    "elast3d_40": lambda: P.configs.elast3d(40),
    "diff3d_64": lambda: P.configs.diff3d_grf(65, seed=2000),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--full", action="store_true")
    args = ap.parse_args()
    t0 = time.perf_counter()
    w = WORKLOADS[args.workload]()
    t_gen = time.perf_counter() - t0
    print(f"{args.workload}: n={w.A.shape[0]} nnz={w.A.nnz} N={len(w.subs)} (generated in {t_gen:.1f} s)",
          flush=True)
    tm = {}
    if args.full:
        # progress of the W solves (one line per block of columns; the oracle's
        # arithmetic is untouched)
        inner = O.pcg_multi

        def pcg_multi_logged(*a, **k):
            t0 = time.perf_counter()
            X, its = inner(*a, **k)
            print(f"  W block of {a[2].shape[1]} columns: iterations max {int(its.max())}, "
                  f"{time.perf_counter() - t0:.0f} s", flush=True)
            return X, its

        O.pcg_multi = pcg_multi_logged
    st = O.setup(w.A, w.subs, w.tau, stop_after=None if args.full else "coarse0", timings=tm)
    s = O.stats(st)
    nm = sum(sp_.nstrict for sp_ in st.split)
    out = {
        "workload": w.name, "tau": w.tau, "tol": w.tol, "n": int(w.A.shape[0]), "nnz": int(w.A.nnz),
        "N": len(w.subs), "n_minus": int(nm), "n0": s["n0"], "n0_rank": s["n0_rank"],
        "k_s": s["k_s"], "kstrict_s": s["kstrict_s"], "m_s": s["m_s"],
        "e0_margin": s["e0_margin"],
        "threads": len(os.sched_getaffinity(0)),
    }
    print(f"  n_minus={nm} n0={s['n0']} rank {s['n0_rank']} e0_margin={s['e0_margin']:.3g} {tm}", flush=True)
    if args.full:
        t0 = time.perf_counter()
        res = O.pcg(w.A, w.b, st.apply, tol=w.tol, maxit=1000)
        tm["pcg"] = time.perf_counter() - t0
        lmin, lmax = res.lanczos_extremes()
        out.update({
            "n_minus_rank": s["n_minus_rank"], "ew_margin": s["ew_margin"],
            "w_solver": st.w_info.get("solver"), "w_iters_max": st.w_info.get("iters_max"),
            "iters": res.iters, "converged": bool(res.converged), "restarts": res.restarts,
            "rel_res_true": res.rel_res_true, "lmin": lmin, "lmax": lmax,
            "x_norm": float(np.linalg.norm(res.x)),
            "note": ("oracle: W by sparse LU of A + Woodbury identity (exact)" if st.w_info.get("solver") == "direct"
                     else "oracle: W by PCG with H2 on every column to rtol 1e-13")
                    + "; PCG x0 = 0, ||r||/||b|| <= tol",
        })
        np.save(os.path.join(ROOT, "tests", "golden", f"{args.workload}_x.npy"), res.x)
        print(f"  iters={res.iters} true={res.rel_res_true:.2e} restarts={res.restarts}", flush=True)
    out["oracle_seconds"] = {k: round(v, 2) for k, v in tm.items()}
    with open(os.path.join(ROOT, "tests", "golden", f"{args.workload}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
