"""The preconditioner of the PCG solves that build W = A_+^-1 V_- (Remark 2,
Section 4.4): H2 = H^NN_hyb(tau) itself, or H^AS_+,ad(1/tau) / H^AS_+,hyb(1/tau)
(Theorem on H^AS_+,hyb/ad, Section 3.4), which share R0 and E0 with
H^NN_hyb(tau).  W is the same operator to the tolerance of its solves, so
with every choice the outer PCG (always H3,ad with H2 = H^NN_hyb) must give
the oracle's iterate to 1e-10 and its iteration count within 1 (the bar of
the FP64 parity tests), and every W column its stopping test against the
oracle's assembled A_+ (test_gpu_w_tolerance covers the default)."""
import numpy as np
import pytest

import awg_problems as P
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu

def cases():
    out = {"elast_x0_small": P.paper_x0(hinv=6, L=2),
           "q1_2d_32_rcb": P.q1_2d(m=32, partition="rcb", nparts=6, delta=1)}
    return out


@pytest.mark.parametrize("w_h2", ["nn_hyb", "asp_hyb", "asp_ad"])
@pytest.mark.parametrize("name", sorted(cases()))
def test_w_preconditioner_keeps_parity(gpu_lib, name, w_h2):
    import torch
    w = cases()[name]
    print(f"\n[gpu case] W solves with {w_h2}: {name} n={w.A.shape[0]}", flush=True)
    st = O.setup(w.A, w.subs, w.tau)
    ref = O.pcg(w.A, w.b, st.apply, tol=w.tol)
    s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, w_h2=w_h2)
    stats = s.stats()
    x, info = s.pcg(torch.as_tensor(w.b, device="cuda"), tol=w.tol)
    s.close()
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    print(f"[w preconditioner] {name} {w_h2}: W iterations {stats['w_iters']} (mean "
          f"{stats['w_iters_mean']:.2f}); ||x - x_o|| / ||x_o|| = {err:.3e}, iterations {info['iters']} "
          f"(oracle {ref.iters})", flush=True)
    assert stats["w_h2"] == {"nn_hyb": 0, "asp_hyb": 1, "asp_ad": 2}[w_h2]
    assert info["converged"] == 1
    assert abs(info["iters"] - ref.iters) <= 1
    assert err <= 1e-10
