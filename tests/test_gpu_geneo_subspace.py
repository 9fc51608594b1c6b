"""Iterative (subspace) GenEO solver on the GPU against the oracle's dense
generalized eigensolves, through the C ABI.

The subspace solver must select exactly the oracle's modes (same m_s per
subdomain, so the same n0), reproduce their eigenvalues to the Ritz residual
and span the same coarse space; the resulting PCG must behave like the dense
path.  Forced failures (iteration cap 1, block of one column) must fall back to
the dense solver and give its result.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import awg_problems as P
from awg_problems import partition as part
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu


def cases():
    rng = np.random.default_rng(7)
    kc = np.where(rng.random((17, 17)) < 0.3, 1e3, 1.0)
    fd16 = P.fd5_diffusion(16, kc)
    return {
        "fd5_32": P.fd5_32(),
        "fd16_uneven": P.configs.Workload(fd16, part.box_subdomains(fd16, (3, 2), 1), 0.1, 1e-8, "fd16"),
        "elast_x0_small": P.paper_x0(hinv=6, L=2),
        "q1_2d_32_rcb": P.q1_2d(m=32, partition="rcb", nparts=6, delta=1),
        "q1_2d_48_rcb": P.q1_2d(m=48, partition="rcb", nparts=12, delta=2),
    }


CASES = cases()


@pytest.fixture(scope="module", params=sorted(CASES))
def trio(request, gpu_lib):
    w = CASES[request.param]
    print(f"\n[gpu case] subspace GenEO {request.param} n={w.A.shape[0]} N={len(w.subs)}", flush=True)
    st = O.setup(w.A, w.subs, w.tau)
    sub = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_rtol=1e-12, geneo="subspace")
    yield w, st, sub
    sub.close()


def test_selects_the_oracle_modes(trio):
    w, st, sub = trio
    s = sub.stats()
    assert s["geneo_solver"] == 1
    assert s["eig_fallbacks"] == 0
    assert s["m_s"] == [Y.shape[1] for Y in st.Y]
    assert s["n0"] == st.n0 and s["n_minus"] == st.n_minus
    assert min(s["eig_iters"]) >= 1
    ge = sub.export("geneo_eigs")
    gref = np.concatenate([lam[:Y.shape[1]] for lam, Y in zip(st.geneo_lam, st.Y)])
    assert np.max(np.abs(ge - gref), initial=0.0) <= 1e-8


def test_spans_the_oracle_coarse_space(trio):
    w, st, sub = trio
    Yg = sub.export("Y")
    off = 0
    for s_, Yr in enumerate(st.Y):
        n, m = Yr.shape
        Ys = Yg[off:off + n * m].reshape(m, n).T
        off += n * m
        if m == 0:
            continue
        ang = sl.subspace_angles(Ys, Yr)
        assert np.max(ang) <= 1e-7, (s_, np.max(ang))


def test_pcg_matches_dense_path(trio, gpu_lib):
    import torch
    w, st, sub = trio
    b = torch.as_tensor(w.b, device="cuda")
    x, info = sub.pcg(b, tol=w.tol, maxit=500)
    ref = O.pcg(w.A, w.b, st.apply, tol=w.tol)
    assert info["converged"] == 1 and abs(info["iters"] - ref.iters) <= 1
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    print(f"[parity] subspace GenEO: ||x - x_o|| / ||x_o|| = {err:.3e}", flush=True)
    assert err <= 1e-10
    assert info["rel_res_true"] <= 2 * w.tol


@pytest.mark.parametrize("kw", [dict(eig_maxit=1), dict(eig_block=1)])
def test_forced_fallback_gives_dense_result(gpu_lib, kw):
    """An iteration cap of 1 leaves subdomains unconverged; a block of one
    column saturates wherever a non-kernel mode lies below tau.  Both must
    hand over to the dense solver."""
    import torch
    w = CASES["q1_2d_32_rcb"]
    print(f"\n[gpu case] forced fallback {kw}", flush=True)
    dense = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_rtol=1e-12)
    sub = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_rtol=1e-12, geneo="subspace", **kw)
    try:
        sd, ss = dense.stats(), sub.stats()
        assert ss["eig_fallbacks"] > 0
        assert ss["m_s"] == sd["m_s"] and ss["n0"] == sd["n0"]
        b = torch.as_tensor(w.b, device="cuda")
        xd, idn = dense.pcg(b, tol=w.tol)
        xs, isb = sub.pcg(b, tol=w.tol)
        assert idn["iters"] == isb["iters"]
        assert torch.equal(xd, xs)
    finally:
        dense.close()
        sub.close()
