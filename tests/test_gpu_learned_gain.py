"""What the trained warm-start network gains over the random start.

The network is trained on the GPU by the library's own kernels, on the GenEO
modes the method computes for 3D Q1 diffusion with log-normal coefficients
(Gaussian random fields, correlation length 4-16 cells) on 32^3 dofs with
4^3 box subdomains of 8^3 nodes (the subdomain size of the 64^3 workload),
then compared with the random start on unseen seeds.  The refined modes must
give the same coarse space (m_s, n0) and the same PCG behaviour; the report
is printed and the gain in eigensolver iterations must be positive.
"""
import json

import numpy as np
import pytest

import awg_problems as P

pytestmark = pytest.mark.gpu


def test_learned_start_gain(gpu_lib):
    import torch
    from paper_2106_10913_amd import learned
    print("\n[gpu case] learned gain: collecting 24 training fields", flush=True)
    train = [P.configs.diff3d_grf(m_cells=33, seed=1000 + i, boxes=(4, 4, 4)) for i in range(24)]
    data = learned.collect(train, n_targets=4)
    net = gpu_lib.MLP(gpu_lib.MLP_FEATURES, 256, 3, 8, seed=0)
    print("[gpu case] learned gain: training", flush=True)
    hist = learned.train(net, data, steps=250, fields_per_step=4, lr=1e-3)
    assert np.mean(hist[-20:]) < 0.5 * hist[0]
    rep = {"cold": [], "learned": []}
    for i in range(10):
        w = P.configs.diff3d_grf(m_cells=33, seed=2000 + i, boxes=(4, 4, 4))
        b = torch.as_tensor(w.b, device="cuda")
        for mode in ("cold", "learned"):
            s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, geneo="subspace", coords=w.coords,
                               eig_init=net if mode == "learned" else None)
            st = s.stats()
            _, info = s.pcg(b, tol=w.tol)
            rep[mode].append(dict(it_max=max(st["eig_iters"]), it_mean=float(np.mean(st["eig_iters"])),
                                  fallbacks=st["eig_fallbacks"], geneo_ms=st["ms"]["geneo"],
                                  setup_ms=st["ms"]["total"], m_s=st["m_s"], pcg_iters=info["iters"],
                                  kappa=info["lmax_est"] / info["lmin_est"]))
            s.close()
    net.close()
    summary = {mode: {k: float(np.mean([r[k] for r in rows])) for k in
                      ("it_max", "it_mean", "fallbacks", "geneo_ms", "setup_ms", "pcg_iters", "kappa")}
               for mode, rows in rep.items()}
    print("[learned gain] " + json.dumps(summary), flush=True)
    for c, l in zip(rep["cold"], rep["learned"]):
        assert c["m_s"] == l["m_s"]
        assert l["fallbacks"] <= c["fallbacks"]
        assert abs(c["pcg_iters"] - l["pcg_iters"]) <= 1
        assert abs(c["kappa"] - l["kappa"]) <= 0.02 * c["kappa"]
    assert summary["learned"]["it_mean"] < summary["cold"]["it_mean"]
    assert summary["learned"]["it_max"] <= summary["cold"]["it_max"]
