"""Compaction of the converged columns in the multi-column PCG that builds W
(Remark 2, Section 4.4): as columns meet their stopping test they are written
to W and the active ones move to narrower multi-vectors.  Every kernel of the
W solves computes each column independently of the others and of its
position, so W, the iteration counts and the final iterate must be the same
bit for bit with the compaction on and off.  Cases with enough columns for
the compaction to trigger (at least 128 converged while others still run):
the paper's six-layer problem with nu = 0.49 (n_- = 357) and Q1 diffusion on
128 x 128 elements with 8 x 8 boxes."""
import numpy as np
import pytest

import awg_problems as P
from awg_problems import configs as C

pytestmark = pytest.mark.gpu

CASES = {
    "paper_nu_0.49": lambda: P.paper_x0(tau=0.05, E1=1e11, E2=1e11, nu=0.49),
    "q1_2d_128": lambda: P.q1_2d(m=128, boxes=(8, 8)),
}


@pytest.mark.parametrize("prec", ["f64", "f16x3"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_w_compaction_is_bit_identical(gpu_lib, name, prec):
    import torch
    w = CASES[name]()
    b = torch.as_tensor(w.b, device="cuda")
    out = {}
    try:
        for on in (False, True):
            print(f"\n[gpu case] W compaction {'on' if on else 'off'}: {name} {prec} n={w.A.shape[0]}", flush=True)
            gpu_lib.w_compaction(on)
            s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec=prec)
            st = s.stats()
            Wm = s.export("W")
            x, info = s.pcg(b, tol=w.tol)
            out[on] = (st, Wm, x.cpu().numpy(), info)
            s.close()
    finally:
        gpu_lib.w_compaction(True)
    (s0, W0, x0, i0), (s1, W1, x1, i1) = out[False], out[True]
    print(f"[w compaction] {name} {prec}: n_- {s1['n_minus']}, compactions {s1['w_compactions']}, "
          f"W iterations {s1['w_iters']} (mean {s1['w_iters_mean']:.2f})", flush=True)
    assert s0["w_compactions"] == 0 and s1["w_compactions"] >= 1
    assert s0["w_iters"] == s1["w_iters"] and s0["w_iters_mean"] == s1["w_iters_mean"]
    assert np.array_equal(W0, W1)
    assert i0["iters"] == i1["iters"]
    assert np.array_equal(x0, x1)
