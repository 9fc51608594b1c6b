"""Reduced-precision local operators (local_prec = f32, f16x3): the
eigen-setup stays FP64, so the coarse spaces are identical; the local
products run in FP32 (FP32 GEMM in the W solves, FP32 GEMV in PCG) or, for
f16x3, the multi-column local products of the W solves on split FP16
operands.  Judged, for every choice of H2, by the true final residual and
the iteration increase over the FP64 form of the same preconditioner, in
the W solves and in PCG (no element-wise parity: the operator itself differs
by the rounding)."""
import numpy as np
import pytest

import awg_problems as P

pytestmark = pytest.mark.gpu

CASES = {"fd5_32": P.fd5_32, "q1_2d_64": lambda: P.q1_2d(m=64, boxes=(2, 2))}


# every choice of H2: the FP32 copy of its local operators is made where
# each of them is formed
H2S = ["nn_hyb", "asp_hyb", "asp_ad", "as_hyb"]


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
@pytest.mark.parametrize("h2", H2S)
@pytest.mark.parametrize("name", sorted(CASES))
def test_f32_local_converges(gpu_lib, name, h2, prec):
    import torch
    w = CASES[name]()
    print(f"\n[gpu case] {prec} {name} h2={h2} n={w.A.shape[0]}", flush=True)
    b = torch.as_tensor(w.b, device="cuda")
    s64 = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec="f64", h2=h2)
    s32 = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec=prec, h2=h2)
    st64, st32 = s64.stats(), s32.stats()
    assert st32["n_minus"] == st64["n_minus"] and st32["n0"] == st64["n0"]
    assert st32["w_iters"] <= st64["w_iters"] + 3
    x64, i64 = s64.pcg(b, tol=w.tol)
    x32, i32 = s32.pcg(b, tol=w.tol)
    assert i32["converged"] == 1
    assert i32["rel_res_true"] <= 2 * w.tol
    assert i32["iters"] <= i64["iters"] + 3
    r = torch.as_tensor(np.random.default_rng(0).standard_normal(w.A.shape[0]), device="cuda")
    z64, z32 = s64.apply(r), s32.apply(r)
    rel = (torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64)).item()
    assert rel <= 1e-3
    s64.close()
    s32.close()


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_reduced_forms_with_subspace_geneo(gpu_lib, name, prec):
    """The fast forms' configuration: subspace GenEO, so the W solves' H^AS_+
    local operators come from the FP32 Cholesky and inverse of M_B^s on the
    matrix cores (FP64 for the subdomains it does not suit)."""
    import torch
    w = CASES[name]()
    print(f"\n[gpu case] {prec} subspace GenEO {name} n={w.A.shape[0]}", flush=True)
    b = torch.as_tensor(w.b, device="cuda")
    s64 = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec="f64", geneo="subspace")
    sr = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec=prec, geneo="subspace")
    st64, st = s64.stats(), sr.stats()
    assert st["n_minus"] == st64["n_minus"] and st["n0"] == st64["n0"]
    assert st["w_factor_fallbacks"] >= 0 and st64["w_factor_fallbacks"] == -1
    assert st["w_iters"] <= st64["w_iters"] + 3
    _, i64 = s64.pcg(b, tol=w.tol)
    _, ir = sr.pcg(b, tol=w.tol)
    print(f"[fp32 factor] {name} {prec}: FP64 fallbacks {st['w_factor_fallbacks']} of {len(w.subs)}, "
          f"W iterations {st['w_iters']} (FP64 {st64['w_iters']}), PCG {ir['iters']} (FP64 {i64['iters']})",
          flush=True)
    assert ir["converged"] == 1 and ir["rel_res_true"] <= 2 * w.tol
    assert ir["iters"] <= i64["iters"] + 3
    s64.close()
    sr.close()
