"""The other two second-coarse-space preconditioners on the GPU (options
coarse2 = "inex", "hyb"; Section 4) against the oracle's H3,inex and H3,hyb,
through the C ABI: H r to the tolerance derived from the conditioning of the
operators (as for H3,ad), the PCG iterate to 1e-10 relative and the iteration
count within 1, and the kept second-coarse columns."""
import numpy as np
import pytest

import awg_problems as P
from awg_problems import partition as part
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def cases():
    rng = np.random.default_rng(7)
    kc = np.where(rng.random((17, 17)) < 0.3, 1e3, 1.0)
    fd16 = P.fd5_diffusion(16, kc)
    return {
        "fd5_32": P.fd5_32(),
        "fd16_uneven": P.configs.Workload(fd16, part.box_subdomains(fd16, (3, 2), 1), 0.1, 1e-8, "fd16"),
        "elast_x0_small": P.paper_x0(hinv=6, L=2),
        "q1_2d_32_rcb": P.q1_2d(m=32, partition="rcb", nparts=6, delta=1),
    }


CASES = cases()


def h_rtol(st, variant):
    """10 eps max(cond(A^s_+) on its range, cond(E0), cond of the second
    coarse matrix: C for inex, W^T A W for hyb), floor 1e-10."""
    kap = max(sp_.L_plus.max() / sp_.L_plus.min() for sp_ in st.split)
    if st.n0:
        kap = max(kap, np.linalg.cond(st.E0[np.ix_(st.E0_keep, st.E0_keep)]))
    if st.n_minus:
        M = st.C[np.ix_(st.C_keep, st.C_keep)] if variant == "inex" else st.EW[np.ix_(st.EW_keep, st.EW_keep)]
        kap = max(kap, np.linalg.cond(M))
    return max(1e-10, 10.0 * EPS * kap)


@pytest.fixture(scope="module", params=[(c, v) for c in sorted(CASES) for v in ("inex", "hyb")],
                ids=lambda p: f"{p[0]}-{p[1]}")
def trio(request, gpu_lib):
    name, variant = request.param
    w = CASES[name]
    print(f"\n[gpu case] {name} coarse2={variant} n={w.A.shape[0]} N={len(w.subs)}", flush=True)
    st = O.setup(w.A, w.subs, w.tau)
    solver = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_rtol=1e-12, coarse2=variant)
    yield w, st, solver, variant
    solver.close()


def oracle_apply(st, variant):
    return st.apply_inex if variant == "inex" else st.apply_hyb


def test_stats_and_kept_columns(trio):
    w, st, solver, variant = trio
    s = solver.stats()
    assert s["coarse2"] == {"inex": 1, "hyb": 2}[variant]
    assert s["n_minus"] == st.n_minus
    keep = st.C_keep if variant == "inex" else st.EW_keep
    assert s["nminus_dropped"] == st.n_minus - keep.size


def test_apply_matches_oracle(trio):
    import torch
    w, st, solver, variant = trio
    rng = np.random.default_rng(5)
    ap = oracle_apply(st, variant)
    for _ in range(3):
        r = rng.standard_normal(w.A.shape[0])
        z = solver.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
        zr = ap(r)
        assert np.linalg.norm(z - zr) <= h_rtol(st, variant) * np.linalg.norm(zr)


def test_pcg_matches_oracle(trio):
    import torch
    w, st, solver, variant = trio
    b = torch.as_tensor(w.b, device="cuda")
    x, info = solver.pcg(b, tol=w.tol, maxit=500)
    ref = O.pcg(w.A, w.b, oracle_apply(st, variant), tol=w.tol)
    assert info["converged"] == 1 and ref.converged
    assert abs(info["iters"] - ref.iters) <= 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    assert info["rel_res_true"] <= 2 * w.tol


def test_rejects_unknown_variant(gpu_lib):
    from paper_2106_10913_amd.awg import AWGError
    w = CASES["fd5_32"]
    with pytest.raises(ValueError):
        gpu_lib.Solver(w.A, w.subs, tau=w.tau, coarse2="exact")
