"""Write tests/golden/q1_2d_256_as_hyb.json and q1_2d_256_as_hyb_x.npy: the FP64
oracle on the full 2D Q1 256 x 256 workload with H2 = H^AS_hyb(tau, 1/tau)
(Theorem on H^AS_hyb, Section 3.4) inside H3,ad (the whole iterate as .npy).

Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_q1_2d_256_as_hyb.py
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
    c = st._as_hyb_space()
    h2 = st.h2("as_hyb")
    res = O.pcg(w.A, w.b, lambda r: st.apply(r, h2=h2), tol=w.tol)
    lmin, lmax = res.lanczos_extremes()
    E = c["E0"]
    sc = np.sqrt(np.diag(E))
    ev = np.linalg.eigvalsh(E / sc[:, None] / sc[None, :])
    k = c["Z"].shape[1]
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(w.A.shape[0], 256, replace=False))
    out = {
        "workload": w.name, "h2": "as_hyb", "coarse2": "ad", "tau": w.tau, "tol": w.tol, "n": int(w.A.shape[0]),
        "n_minus": st.n_minus, "n0": int(c["R0T"].shape[1]), "m_s": [int(Y.shape[1]) for Y in c["Y"]],
        "n0_deflated": int(k + (c["R0T"].shape[1] - c["keep"].size)),
        "cond_E0_scaled_deflated": float(ev[-1] / ev[k]),
        "deflation_margin": float(min(1e-10 / max(ev[k - 1], 1e-300), ev[k] / 1e-10)) if k else float(ev[0] / 1e-10),
        "iters": res.iters, "rel_res_true": res.rel_res_true, "lmin": lmin, "lmax": lmax,
        "x_norm": float(np.linalg.norm(res.x)), "x_idx": idx.tolist(), "x_val": res.x[idx].tolist(),
        "note": "oracle: W exact (sparse LU + Woodbury); E0 pseudo-inverse deflating the eigenvectors of the "
                "Jacobi-scaled E0 below 1e-10; PCG x0 = 0, ||r||/||b|| <= tol",
    }
    np.save(os.path.join(ROOT, "tests", "golden", "q1_2d_256_as_hyb_x.npy"), res.x)
    with open(os.path.join(ROOT, "tests", "golden", "q1_2d_256_as_hyb.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
