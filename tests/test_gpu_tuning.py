"""The autotuner changes time only: every launch variant it may pick (GEMM
tiles, skinny and gathered GEMMs, SpMM kernels and row groups, explicit or
in-place restriction, the FP32 local-product forms) computes the same bits, so
a solve with the tuner off (variant 0 everywhere) and on gives the same
iterate, bit for bit, and the same counts."""
import numpy as np
import pytest

import awg_problems as P

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tuned_variants_do_not_change_results(gpu_lib, prec):
    import torch
    w = P.q1_2d(m=48, partition="rcb", nparts=12, delta=2)
    b = torch.as_tensor(w.b, device="cuda")
    out = []
    try:
        for tuned in (False, True):
            gpu_lib.autotune(tuned)
            s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec=prec)
            st = s.stats()
            x, info = s.pcg(b, tol=w.tol)
            out.append((x.cpu().numpy(), info["iters"], st["w_iters"], st["n0"], st["n_minus"]))
            s.close()
    finally:
        gpu_lib.autotune(True)
    (x0, *c0), (x1, *c1) = out
    assert c0 == c1
    assert np.array_equal(x0, x1)
