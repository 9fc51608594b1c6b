"""Write tests/golden/q1_2d_256.json and q1_2d_256_x.npy: the FP64 oracle on
the full 2D Q1 256 x 256 workload (the whole PCG iterate x as .npy).

Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_q1_2d_256.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import awg_problems as P  # noqa: E402
from oracle import awg_oracle as O  # noqa: E402


def main():
    w = P.q1_2d(256)
    st = O.setup(w.A, w.subs, w.tau)
    res = O.pcg(w.A, w.b, st.apply, tol=w.tol)
    lmin, lmax = res.lanczos_extremes()
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(w.A.shape[0], 256, replace=False))
    s = O.stats(st)
    out = {
        "workload": w.name, "tau": w.tau, "tol": w.tol, "n": int(w.A.shape[0]),
        "n_minus": s["n_minus"], "n0": s["n0"], "k_s": s["k_s"], "kstrict_s": s["kstrict_s"], "m_s": s["m_s"],
        "iters": res.iters, "rel_res_true": res.rel_res_true, "lmin": lmin, "lmax": lmax,
        "x_norm": float(np.linalg.norm(res.x)), "x_idx": idx.tolist(), "x_val": res.x[idx].tolist(),
        "e0_margin": s["e0_margin"], "ew_margin": s["ew_margin"],
        "n0_rank": s["n0_rank"], "n_minus_rank": s["n_minus_rank"],
        "note": "oracle: W by sparse LU of A + Woodbury identity (exact), PCG x0 = 0, ||r||/||b|| <= tol",
    }
    np.save(os.path.join(ROOT, "tests", "golden", "q1_2d_256_x.npy"), res.x)
    with open(os.path.join(ROOT, "tests", "golden", "q1_2d_256.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
