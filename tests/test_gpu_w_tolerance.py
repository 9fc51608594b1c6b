"""Loose tolerances for the W solves (Section 5, Table 4: the relative
residual of the PCG solves for W = A_+^-1 V_- hardly changes the condition
number of H3,ad A down to 1e-2, and only mildly at 1e-1).

Through the C ABI, for each tolerance: every column of the exported W (its
solves preconditioned by H^AS_+,ad, the default) meets its stopping test
against the oracle's assembled A_+ and the GPU's own V_- (the
recursive residual that the GPU tests differs from the true one by at most a
few eps * cond(A_+)); the outer PCG still converges to its tolerance.  On the
paper's own problem, down to 1e-2 kappa stays that of its table."""
import numpy as np
import pytest

import awg_problems as P
from awg_problems import partition as part
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
RTOLS = [1e-10, 1e-6, 1e-2, 1e-1]


def cases():
    return {
        "fd5_32": P.fd5_32(),
        "elast_x0_small": P.paper_x0(hinv=6, L=2),
        "q1_2d_32_rcb": P.q1_2d(m=32, partition="rcb", nparts=6, delta=1),
    }


CASES = cases()


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, gpu_lib):
    import torch
    name = request.param
    w = CASES[name]
    st = O.setup(w.A, w.subs, w.tau)
    b = torch.as_tensor(w.b, device="cuda")
    runs = {}
    for rt in RTOLS:
        print(f"\n[gpu case] {name} w_rtol={rt:g} n={w.A.shape[0]} N={len(w.subs)}", flush=True)
        s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_rtol=rt)
        W = s.export("W").reshape(w.A.shape[0], -1)
        Vg = gpu_rhs(w, s)
        _, info = s.pcg(b, tol=w.tol)
        runs[rt] = (W, Vg, info, s.stats())
        s.close()
    return name, w, st, runs


def gpu_rhs(w, s):
    """The right-hand sides of the GPU's W: its own strictly negative
    eigenvectors of every B^s, prolongated (eigenvectors are fixed only up to
    sign, and up to rotation within clustered eigenvalues, so the oracle's
    V_- columns need not be the GPU's; A_+ does not depend on that choice)."""
    st = s.stats()
    V = s.export("V_minus")
    n = w.A.shape[0]
    cols = []
    o = 0
    for idx, k, ks in zip(w.subs, st["k_s"], st["kstrict_s"]):
        blk = V[o:o + len(idx) * k].reshape(k, len(idx)).T      # n_s x k_s column-major
        o += len(idx) * k
        for j in range(ks):
            c = np.zeros(n)
            c[idx] = blk[:, j]
            cols.append(c)
    return np.stack(cols, axis=1) if cols else np.zeros((n, 0))


def test_w_columns_meet_the_tolerance(case):
    name, w, st, runs = case
    Ap = O.assemble_A_plus(st).toarray()
    ev = np.linalg.eigvalsh(Ap)
    kap = ev[-1] / ev[0]
    for rt, (W, Vg, info, stats) in runs.items():
        assert W.shape == Vg.shape == st.Vg.shape, (name, rt)
        nv = np.linalg.norm(Vg, axis=0)
        res = np.linalg.norm(Ap @ W - Vg, axis=0) / nv
        bound = rt + 100 * EPS * kap
        assert res.max() <= bound, (name, rt, res.max(), bound)
        # a looser tolerance never takes more iterations
        if rt > RTOLS[0]:
            assert stats["w_iters"] <= runs[RTOLS[0]][3]["w_iters"]


def test_pcg_converges_at_every_tolerance(case):
    name, w, st, runs = case
    for rt, (W, Vg, info, stats) in runs.items():
        assert info["converged"] == 1, (name, rt)
        assert info["rel_res_true"] <= 2 * w.tol, (name, rt, info["rel_res_true"])


def test_paper_table4_on_gpu(gpu_lib):
    """Table 4 (nu = 0.3) on the paper's six-layer problem: W to 1e-2 leaves
    kappa within 3 % of the printed 9.0 (as W to 1e-10 does), and the
    iteration count within 1 of the oracle's with W from its own PCG at the
    same tolerance and the same stopping test (||r||/||b|| <= 1e-8)."""
    import json
    import os
    import torch
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")) as f:
        T4 = json.load(f)["table4_w_rtol"]
    w = P.paper_x0(tau=0.1)
    b = torch.as_tensor(w.b, device="cuda")
    for row in T4["rows"]:
        if row["w_rtol"] > 1e-2:
            continue
        print(f"\n[gpu case] six-layer problem, w_rtol={row['w_rtol']:g}", flush=True)
        # the W solves preconditioned by H2 itself, as the table's were (at a
        # loose tolerance W depends on the preconditioner of its solves)
        s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_rtol=row["w_rtol"], w_h2="nn_hyb")
        st = s.stats()
        assert st["n0"] == T4["n0"] and st["n_minus"] == T4["n_minus"]
        _, info = s.pcg(b, tol=1e-8, maxit=500)
        s.close()
        assert info["converged"] == 1
        kappa = info["lmax_est"] / info["lmin_est"]
        assert abs(kappa - row["kappa"]) <= 0.03 * row["kappa"], (row, kappa)
        ost = O.setup(w.A, w.subs, w.tau, w_solver="pcg", w_rtol=row["w_rtol"])
        ref = O.pcg(w.A, w.b, ost.apply, tol=1e-8, maxit=500)
        assert abs(info["iters"] - ref.iters) <= 1, (row, info["iters"], ref.iters)
