"""H3,ad with H2 = H^AS_hyb(tau, 1/tau) on the full 2D Q1 256^2 workload
(64 subdomains) against the oracle's values stored in
tests/golden/q1_2d_256_as_hyb.json by tests/golden/make_q1_2d_256_as_hyb.py
(oracle only).

On this workload the union of the two pencils' vectors has one near-null
combination across subdomains (Jacobi-scaled E0 eigenvalue 2e-14): both
sides deflate it.  Checked: the coarse dimensions and the deflated count
exactly, the iteration count within 1, the Lanczos estimates within 1e-3,
and 256 sampled entries of the iterate within 10 eps cond(deflated scaled E0)
of the oracle's (the accuracy to which either side can apply E0^+)."""
import json
import os

import numpy as np
import pytest

import awg_problems as P

pytestmark = pytest.mark.gpu

GOLD_PATH = os.path.join(os.path.dirname(__file__), "golden", "q1_2d_256_as_hyb.json")
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def run(gpu_lib):
    import torch
    gold = json.load(open(GOLD_PATH))
    w = P.q1_2d(256)
    print(f"\n[gpu case] q1_2d 256^2, 64 subdomains, h2=as_hyb n={w.A.shape[0]}", flush=True)
    solver = gpu_lib.Solver(w.A, w.subs, tau=w.tau, h2="as_hyb")
    st = solver.stats()
    x, info = solver.pcg(torch.as_tensor(w.b, device="cuda"), tol=w.tol, maxit=1000)
    solver.close()
    return gold, w, st, x.cpu().numpy(), info


def test_coarse_sizes_and_deflation(run):
    gold, w, st, x, info = run
    assert st["n_minus"] == gold["n_minus"] and st["n0"] == gold["n0"]
    assert st["m_s"] == gold["m_s"]
    assert st["n0_dropped"] == gold["n0_deflated"]


def test_pcg_iterate_and_count(run):
    gold, w, st, x, info = run
    assert info["converged"] == 1
    assert abs(info["iters"] - gold["iters"]) <= 1
    assert abs(info["lmax_est"] - gold["lmax"]) <= 1e-3 * gold["lmax"]
    assert abs(info["lmin_est"] - gold["lmin"]) <= 1e-3 * gold["lmin"]
    bar = max(1e-10, 10 * EPS * gold["cond_E0_scaled_deflated"])
    xs = x[np.array(gold["x_idx"])]
    assert np.max(np.abs(xs - np.array(gold["x_val"]))) <= bar * gold["x_norm"]
    assert info["rel_res_true"] <= 2 * w.tol
