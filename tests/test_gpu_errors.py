"""Error codes and degenerate cases of the C ABI on the GPU (all forced from
host inputs; no kernel is made to fault)."""
import numpy as np
import pytest
import scipy.sparse as sp

import awg_problems as P
from awg_problems import partition as part
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu


def base():
    w = P.fd5_32()
    return w.A.copy(), [s.copy() for s in w.subs], w


def code_of(gpu_lib, A, subs, **kw):
    try:
        s = gpu_lib.Solver(A, subs, **kw)
    except gpu_lib.AWGError as e:
        return e.code
    s.close()
    return 0


def test_valid_after_errors(gpu_lib):
    A, subs, w = base()
    assert code_of(gpu_lib, A, subs[:-1]) == -3          # coverage gap
    assert code_of(gpu_lib, A, subs) == 0                # a fresh setup still works


def test_partition_errors(gpu_lib):
    A, subs, _ = base()
    bad = list(subs)
    bad[1] = bad[1][::-1].copy()
    assert code_of(gpu_lib, A, bad) == -3                # unsorted
    bad = list(subs)
    bad[2] = np.concatenate([bad[2], bad[2][-1:]])
    assert code_of(gpu_lib, A, bad) == -3                # duplicate
    bad = list(subs)
    bad[0] = np.concatenate([bad[0], [A.shape[0]]])
    assert code_of(gpu_lib, A, bad) == -3                # out of range
    bad = list(subs) + [np.zeros(0, dtype=np.int64)]
    assert code_of(gpu_lib, A, bad) == -3                # empty subdomain


def test_min_overlap_violation(gpu_lib):
    prob = P.fd5_diffusion(8, np.ones((9, 9)))
    G, kept = part.node_graph_of_A(prob)
    parts = part.box_parts(prob.node_xyz[kept], (2, 2))
    subs0 = part.nodes_to_dofs(prob, kept, part.extend_by_layers(G, parts, 4, 0))
    assert code_of(gpu_lib, prob.A, subs0) == -4


def test_matrix_errors(gpu_lib):
    A, subs, _ = base()
    Au = A.tolil()
    Au[0, 1] += 1.0
    assert code_of(gpu_lib, Au.tocsr(), subs) == -2      # not symmetric
    An = A.copy()
    An.data[5] = np.nan
    assert code_of(gpu_lib, An, subs) == -9              # NaN
    assert code_of(gpu_lib, A, subs, tau=0.0) == -1
    assert code_of(gpu_lib, A, subs, tau=1.0) == -1


def test_indefinite_matrix_reports_not_spd(gpu_lib):
    """A symmetric but indefinite A is caught by a Cholesky breakdown or by
    p^T A p <= 0 in PCG."""
    import torch
    A, subs, w = base()
    Ai = (A - 3.5 * sp.identity(A.shape[0], format="csr")).tocsr()
    Ai.sort_indices()
    try:
        s = gpu_lib.Solver(Ai, subs)
    except gpu_lib.AWGError as e:
        assert e.code in (-5, -6)
        return
    with pytest.raises(gpu_lib.AWGError) as ei:
        s.pcg(torch.as_tensor(w.b, device="cuda"), tol=1e-8)
    assert ei.value.code == -5
    s.close()


def test_single_subdomain_is_direct(gpu_lib):
    """N = 1: B^1 = A is spd, no coarse space, H = A^{-1}: one iteration."""
    import torch
    A, _, w = base()
    s = gpu_lib.Solver(A, [np.arange(A.shape[0])])
    st = s.stats()
    assert st["n_minus"] == 0 and st["n0"] == 0
    x, info = s.pcg(torch.as_tensor(w.b, device="cuda"), tol=1e-10)
    assert info["iters"] == 1
    xr = np.linalg.solve(A.toarray(), w.b)
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
    s.close()


def test_tiny_subdomains(gpu_lib):
    """Subdomains of 1 and 2 dofs next to ordinary ones (1x1 and 2x2 local
    eigenproblems) against the oracle."""
    import torch
    A, subs, w = base()
    subs = subs + [np.array([100]), np.array([200, 201])]
    st = O.setup(A, subs, 0.1)
    s = gpu_lib.Solver(A, subs)
    g = s.stats()
    assert g["k_s"] == [sp_.nneg for sp_ in st.split] and g["m_s"] == [Y.shape[1] for Y in st.Y]
    x, info = s.pcg(torch.as_tensor(w.b, device="cuda"), tol=1e-8)
    ref = O.pcg(A, w.b, st.apply, tol=1e-8)
    assert abs(info["iters"] - ref.iters) <= 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    s.close()


def test_not_converged_warning_and_zero_rhs(gpu_lib):
    import torch
    A, subs, w = base()
    s = gpu_lib.Solver(A, subs)
    x, info = s.pcg(torch.as_tensor(w.b, device="cuda"), tol=1e-14, maxit=2)
    assert info["status"] == "AWG_NOT_CONVERGED" and info["iters"] == 2
    x0, info0 = s.pcg(torch.zeros(A.shape[0], dtype=torch.float64, device="cuda"), tol=1e-8)
    assert info0["iters"] == 0 and torch.count_nonzero(x0).item() == 0
    z = s.apply(torch.zeros(A.shape[0], dtype=torch.float64, device="cuda"))
    assert torch.count_nonzero(z).item() == 0
    s.close()
