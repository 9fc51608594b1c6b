"""Pins of the FP64 oracle against mathematics fixed by the paper.

Every check here is independent of the oracle's own formulas: brute-force
counting, assembled dense matrices, textbook identities (Woodbury, projector
algebra), theorem bounds, special cases with a known answer.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import awg_problems as P
from awg_problems import partition as part
from oracle import awg_oracle as O


def small_fd(seed=3, nint=12, boxes=(3, 3), delta=1, contrast=1e3):
    rng = np.random.default_rng(seed)
    kc = np.where(rng.random((nint + 1, nint + 1)) < 0.3, contrast, 1.0)
    prob = P.fd5_diffusion(nint, kc)
    return prob.A, part.box_subdomains(prob, boxes, delta), prob.b


def small_elast(hinv=4, L=2):
    w = P.paper_x0(hinv=hinv, L=L)
    return w.A, w.subs, w.b


def random_spd(seed, n=60, nparts=5, delta=1):
    """Random sparse SPD matrix (weighted graph Laplacian + positive diagonal)
    with random parts grown by ``delta`` graph layers."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    d = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    adj = (d < 0.04) & ~np.eye(n, dtype=bool)
    adj = adj | adj.T
    Wt = np.triu(rng.uniform(0.1, 10.0, (n, n)) * adj, 1)
    Wt = Wt + Wt.T
    L = np.diag(Wt.sum(1)) - Wt + np.diag(rng.uniform(0.01, 1.0, n))
    A = sp.csr_matrix(L)
    A.sort_indices()
    parts = rng.integers(0, nparts, n)
    parts[:nparts] = np.arange(nparts)
    G = (A != 0).astype(np.float64)
    subs = part.extend_by_layers(G, parts, nparts, delta)
    return A, [np.asarray(s, dtype=np.int64) for s in subs]


CASES = [small_fd, small_elast, lambda: random_spd(11) + (None,), lambda: random_spd(12, 80, 7) + (None,)]


@pytest.fixture(scope="module", params=range(len(CASES)))
def case(request):
    A, subs, b = CASES[request.param]()
    st = O.setup(A, subs, 0.1)
    return A, subs, st


# ----------------------------------------------------------------------------
def test_pair_multiplicity_bruteforce(case):
    """M_mu counts, for each nonzero, the subdomains holding both indices (Section 3.1)."""
    A, subs, st = case
    Ac = A.tocoo()
    sets = [set(s.tolist()) for s in subs]
    csr = A.tocsr()
    for k in range(0, csr.nnz, max(1, csr.nnz // 400)):
        i = np.searchsorted(csr.indptr, k, side="right") - 1
        j = csr.indices[k]
        brute = sum(1 for S in sets if i in S and j in S)
        assert st.cnt[k] == brute
    del Ac


def test_splitting_sums_to_A(case):
    """sum_s R^sT B^s R^s = A (Theorem after the definition of B^s, Section 3.1)."""
    A, subs, st = case
    n = A.shape[0]
    S = np.zeros((n, n))
    for idx in subs:
        S[np.ix_(idx, idx)] += O.local_block(st.B, idx)
    Ad = A.toarray()
    assert np.max(np.abs(S - Ad)) <= 4e-16 * np.max(np.abs(Ad)) * 4


def test_A_plus_minus_properties(case):
    """A = A_+ - A_-, A_- spsd, A_+ spd, rank(A_-) <= sum n_s - n (Section 3.2, 4.1)."""
    A, subs, st = case
    n = A.shape[0]
    Ap = O.assemble_A_plus(st).toarray()
    Am = np.zeros((n, n))
    for idx, s_ in zip(subs, st.split):
        Am[np.ix_(idx, idx)] += s_.A_minus()
    Ad = A.toarray()
    scale = np.max(np.abs(Ad))
    assert np.max(np.abs(Ap - Am - Ad)) <= 1e-12 * scale
    em = np.linalg.eigvalsh(Am)
    ep = np.linalg.eigvalsh(Ap)
    assert em.min() >= -1e-12 * scale
    assert ep.min() > 0
    rank = int(np.count_nonzero(em > 1e-10 * scale))
    assert rank <= sum(len(s) for s in subs) - n
    # the implicit action used everywhere else agrees with the assembled A_+
    x = np.random.default_rng(0).standard_normal(n)
    assert np.allclose(st.A_plus_mv(x), Ap @ x, rtol=1e-12, atol=1e-12 * scale * np.abs(x).max())


def test_woodbury_identity(case):
    """A^{-1} = A_+^{-1} + A_+^{-1} V_- (L_-^{-1} - V_-^T A_+^{-1} V_-)^{-1} V_-^T A_+^{-1}
    with A_- = V_- L_- V_-^T its diagonalisation without the null part (Section 4.1)."""
    A, subs, st = case
    n = A.shape[0]
    Ap = O.assemble_A_plus(st).toarray()
    Am = Ap - A.toarray()
    lam, V = np.linalg.eigh(Am)
    keep = lam > 1e-9 * np.abs(lam).max()
    Vm, Lm = V[:, keep], lam[keep]
    Api = np.linalg.inv(Ap)
    C = np.diag(1.0 / Lm) - Vm.T @ Api @ Vm
    wood = Api + Api @ Vm @ np.linalg.solve(C, Vm.T @ Api)
    Ainv = np.linalg.inv(A.toarray())
    assert np.linalg.norm(wood - Ainv) <= 1e-8 * np.linalg.norm(Ainv)
    del n


def test_range_of_W(case):
    """range(A_+^{-1} V_-) = range(A^{-1} V_-) (Lemma, Section 4.3)."""
    A, subs, st = case
    if st.n_minus == 0:
        pytest.skip("no strictly negative local eigenvalue")
    W2 = np.linalg.solve(A.toarray(), st.Vg)
    ang = sla.subspace_angles(st.W, W2)
    assert ang.max() < 1e-8


def test_Pi3_projector(case):
    """Pi_3 is an A-orthogonal projector, A_- Pi_3 = 0, Pi_3 W = 0 (Theorem, Section 4.3)."""
    A, subs, st = case
    if st.n_minus == 0:
        pytest.skip("no strictly negative local eigenvalue")
    n = A.shape[0]
    Ad = A.toarray()
    W = st.W
    Pi3 = np.eye(n) - W @ np.linalg.solve(W.T @ Ad @ W, W.T @ Ad)
    assert np.linalg.norm(Pi3 @ Pi3 - Pi3) <= 1e-8 * np.linalg.norm(Pi3)
    APi = Ad @ Pi3
    assert np.linalg.norm(APi - APi.T) <= 1e-8 * np.linalg.norm(APi)
    Am = O.assemble_A_plus(st).toarray() - Ad
    assert np.linalg.norm(Am @ Pi3) <= 1e-8 * np.linalg.norm(Am) * np.linalg.norm(Pi3)
    assert np.linalg.norm(Pi3 @ W) <= 1e-8 * np.linalg.norm(W)


def test_local_pseudo_inverse_forms(case):
    """(A^s_+)^dagger three ways: numpy pinv; P B^dagger P with P = I - V_- V_-^T
    (Remark 3, Section 4.4); and K^{-1} - c^{-1} V_- V_-^T with
    K = A^s_+ + c V_- V_-^T (the factorisation the GPU uses)."""
    A, subs, st = case
    for s_, idx in zip(st.split, subs):
        G = s_.A_plus_pinv()
        Bs = O.local_block(st.B, idx)
        Ap = s_.A_plus()
        ref = np.linalg.pinv(Ap, rcond=1e-10, hermitian=True)
        nrm = np.linalg.norm(ref)
        assert np.linalg.norm(G - ref) <= 1e-8 * nrm
        Pm = np.eye(len(idx)) - s_.V_minus @ s_.V_minus.T
        if s_.nneg == s_.nstrict:        # B^s nonsingular: P B^{-1} P
            assert np.linalg.norm(Pm @ np.linalg.inv(Bs) @ Pm - G) <= 1e-8 * nrm
        c = float(np.mean(np.diag(Bs)))
        K = Bs + (s_.V_minus * (c - s_.L_minus)) @ s_.V_minus.T
        GK = np.linalg.inv(K) - s_.V_minus @ s_.V_minus.T / c
        assert np.linalg.norm(GK - G) <= 1e-8 * nrm


def test_geneo_selection_independent(case):
    """GenEO count and kernel (Definition of Y_L and the remark on the kernels,
    Section 3.4): the kernel of M_A is D^s V^s_- of dimension n^s_-, and the
    number of eigenvalues below tau agrees with an independent dense solve of
    M_B^{-1} M_A (nonsymmetric eigenvalues)."""
    A, subs, st = case
    Ap = O.assemble_A_plus(st)
    for s, idx in enumerate(subs):
        s_ = st.split[s]
        Dinv = 1.0 / st.Ds[s]
        MA = Dinv[:, None] * s_.A_plus() * Dinv[None, :]
        MB = O.local_block(Ap, idx)             # R^s A_+ R^sT from the assembled A_+
        ev = np.sort(np.linalg.eigvals(np.linalg.solve(MB, MA)).real)
        assert int(np.count_nonzero(ev < st.tau)) == st.Y[s].shape[1]
        # kernel: D^s V^s_- is annihilated by M_A
        if s_.nneg:
            K = st.Ds[s][:, None] * s_.V_minus
            assert np.linalg.norm(MA @ K) <= 1e-8 * np.linalg.norm(MA) * np.linalg.norm(K)
        # Y^s is M_B-orthonormal and spans eigenvectors
        Y = st.Y[s]
        if Y.shape[1]:
            assert np.allclose(Y.T @ MB @ Y, np.eye(Y.shape[1]), atol=1e-8)
            lam = st.geneo_lam[s][:Y.shape[1]]
            res = MA @ Y - (MB @ Y) * lam
            assert np.linalg.norm(res) <= 1e-7 * np.linalg.norm(MA)


def test_H_spd_and_spectral_bound(case):
    """H is spd and the spectrum of HA lies in [1, N(A_+)/tau + 1] (Theorem on
    H^NN_hyb, Section 3.4, and the H3,ad bound, Section 4.3); H2 A_+ lies in
    [1, N(A_+)/tau]."""
    A, subs, st = case
    n = A.shape[0]
    H = O.dense_operator(st.apply, n)
    assert np.linalg.norm(H - H.T) <= 1e-9 * np.linalg.norm(H)
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0
    Ap = O.assemble_A_plus(st)
    ncol = O.coloring_constant(subs, Ap)
    ev = O.spectrum_HA(0.5 * (H + H.T), A.toarray())
    assert ev.min() >= 1 - 1e-8
    assert ev.max() <= ncol / st.tau + 1 + 1e-8
    H2 = O.dense_operator(st.H2, n)
    ev2 = O.spectrum_HA(0.5 * (H2 + H2.T), Ap.toarray())
    assert ev2.min() >= 1 - 1e-8
    assert ev2.max() <= ncol / st.tau + 1e-8


def test_basis_invariance(case):
    """H depends on range(R0^T) and range(W) only (Assumption on V0, Section 2.3;
    Definition of Pi_3 and H3, Section 4.3)."""
    A, subs, st = case
    rng = np.random.default_rng(5)
    r = rng.standard_normal(A.shape[0])
    z = st.apply(r)
    import copy
    st2 = copy.copy(st)
    R0T = st.R0T.toarray()
    M0 = np.eye(R0T.shape[1]) + 0.3 * rng.standard_normal((R0T.shape[1],) * 2)
    R0T2 = R0T @ M0
    st2.R0T = sp.csr_matrix(R0T2)
    E0 = R0T2.T @ st.A_plus_mv(R0T2)
    st2.E0_keep = np.arange(R0T2.shape[1])
    st2.E0_cho = sla.cho_factor(0.5 * (E0 + E0.T), lower=True)
    if st.n_minus:
        Mw = np.eye(st.n_minus) + 0.3 * rng.standard_normal((st.n_minus,) * 2)
        st2.W = st.W @ Mw
        EW = st2.W.T @ (A @ st2.W)
        st2.EW_keep = np.arange(st.n_minus)
        st2.EW_cho = sla.cho_factor(0.5 * (EW + EW.T), lower=True)
    z2 = st2.apply(r)
    assert np.linalg.norm(z2 - z) <= 1e-8 * np.linalg.norm(z)


# ----------------------------------------------------------------------------
# special cases with a known answer
# ----------------------------------------------------------------------------
def test_single_subdomain_is_exact():
    """N = 1, Omega^1 = all dofs: B^1 = A is spd, so n_- = 0 and GenEO keeps
    nothing; H = H^NN = A^{-1} and PCG converges in one iteration."""
    A, _, b = small_fd()
    n = A.shape[0]
    st = O.setup(A, [np.arange(n)], 0.1)
    assert st.n_minus == 0 and st.n0 == 0
    H = O.dense_operator(st.apply, n)
    assert np.linalg.norm(H - np.linalg.inv(A.toarray())) <= 1e-9 * np.linalg.norm(H)
    res = O.pcg(A, b, st.apply, tol=1e-10)
    assert res.iters == 1


def test_spd_local_blocks_give_no_second_space():
    """A diagonally dominant 1D chain with single-node overlaps: every B^s is
    spd, A_+ = A and W is empty, so H = H2."""
    n = 31
    main = np.full(n, 4.0)
    off = np.full(n - 1, -1.0)
    A = sp.diags([off, main, off], [-1, 0, 1]).tocsr()
    A.sort_indices()
    subs = [np.arange(0, 11), np.arange(10, 21), np.arange(20, 31)]
    st = O.setup(A, subs, 0.1)
    assert all(s_.nneg == 0 for s_ in st.split)
    assert st.n_minus == 0
    r = np.random.default_rng(1).standard_normal(n)
    assert np.allclose(st.apply(r), st.H2(r))


def test_tau_to_zero_keeps_only_kernels():
    """As tau -> 0 the GenEO space reduces to the kernels D^s V^s_-, so
    #V0 = sum_s n^s_- (remark on the kernels, Section 3.4), and n_- does not
    depend on tau."""
    A, subs, _ = small_elast()
    st_small = O.setup(A, subs, 1e-9)
    st = O.setup(A, subs, 0.1)
    assert st_small.n0 == sum(s_.nneg for s_ in st_small.split)
    assert st_small.n_minus == st.n_minus
    assert st.n0 >= st_small.n0


def test_pcg_matches_direct_solve():
    """The PCG recurrence converges to A^{-1} b within the tolerance."""
    A, subs, b = small_fd()
    st = O.setup(A, subs, 0.1)
    res = O.pcg(A, b, st.apply, tol=1e-12)
    x = np.linalg.solve(A.toarray(), b)
    assert res.converged
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)
    assert res.rel_res_true <= 1e-11


def test_invalid_inputs_rejected():
    A, subs, _ = small_fd()
    with pytest.raises(O.OracleError):
        O.setup(A, subs[:-1], 0.1)                      # coverage gap
    bad = list(subs)
    bad[0] = bad[0][::-1].copy()
    with pytest.raises(O.OracleError):
        O.setup(A, bad, 0.1)                           # unsorted
    with pytest.raises(O.OracleError):
        O.setup(A, subs, 1.5)                          # tau outside (0, 1)
    # boxes without overlap violate the minimal-overlap assumption
    prob = P.fd5_diffusion(8, np.ones((9, 9)))
    G, kept = part.node_graph_of_A(prob)
    parts = part.box_parts(prob.node_xyz[kept], (2, 2))
    subs0 = part.nodes_to_dofs(prob, kept, part.extend_by_layers(G, parts, 4, 0))
    with pytest.raises(O.OracleError):
        O.setup(prob.A, subs0, 0.1)
    Au = prob.A.tolil()
    Au[0, 1] += 1.0
    with pytest.raises(O.OracleError):
        O.setup(Au.tocsr(), part.box_subdomains(prob, (2, 2), 1), 0.1)


def test_lanczos_extremes_match_dense_spectrum():
    A, subs, b = small_fd()
    st = O.setup(A, subs, 0.1)
    res = O.pcg(A, b, st.apply, tol=1e-14, maxit=500)
    H = O.dense_operator(st.apply, A.shape[0])
    ev = O.spectrum_HA(0.5 * (H + H.T), A.toarray())
    lmin, lmax = res.lanczos_extremes()
    assert abs(lmax - ev.max()) <= 1e-3 * ev.max()
    assert abs(lmin - ev.min()) <= 1e-3 * ev.min()


def test_W_by_pcg_matches_direct():
    """W from PCG on A_+ preconditioned by H2 (Remark 2, Section 4.4) spans the
    same space as the direct solve, so H is the same operator."""
    A, subs, _ = small_elast(hinv=6, L=2)
    st_d = O.setup(A, subs, 0.1, w_solver="direct")
    st_p = O.setup(A, subs, 0.1, w_solver="pcg", w_rtol=1e-13)
    assert st_p.w_info["iters_max"] < 60
    ang = sla.subspace_angles(st_d.W, st_p.W)
    assert ang.max() < 1e-9
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    zd, zp = st_d.apply(r), st_p.apply(r)
    assert np.linalg.norm(zd - zp) <= 1e-9 * np.linalg.norm(zd)


def test_woodbury_direct_W_matches_dense():
    """The large-n direct path (sparse LU of A plus the Woodbury identity)
    gives the same W as a dense Cholesky solve with the assembled A_+."""
    A, subs, _ = small_elast(hinv=6, L=2)
    st = O.setup(A, subs, 0.1)
    Ap = O.assemble_A_plus(st).toarray()
    Wd = np.linalg.solve(Ap, st.Vg)
    n_saved = st.A.shape
    import scipy.sparse.linalg as spla
    lu = spla.splu(st.A.tocsc())
    X = lu.solve(st.Vg)
    c = np.concatenate([-s_.lam[:s_.nstrict] for s_ in st.split if s_.nstrict])
    cap = np.diag(1.0 / c) + st.Vg.T @ X
    Ww = X - X @ np.linalg.solve(cap, st.Vg.T @ X)
    assert np.linalg.norm(Ww - Wd) <= 1e-9 * np.linalg.norm(Wd)
    del n_saved


# ----------------------------------------------------------------------------
# dependent coarse vectors (reading of the basis assumption, Section 2)
# ----------------------------------------------------------------------------
def test_gram_keep_drops_exactly_the_dependent_columns():
    rng = np.random.default_rng(8)
    a, b, c = rng.standard_normal((3, 40))
    X = np.stack([a, b, a + b, c, 2.0 * a, b - c, rng.standard_normal(40)], axis=1)
    keep = O.gram_keep(X.T @ X)
    assert keep.tolist() == [0, 1, 3, 6]
    # independent columns: nothing deleted
    Y = rng.standard_normal((30, 12))
    assert O.gram_keep(Y.T @ Y).tolist() == list(range(12))


def test_gram_keep_projection_is_the_projector_onto_the_span():
    rng = np.random.default_rng(9)
    B = rng.standard_normal((50, 6))
    X = np.concatenate([B, B @ rng.standard_normal((6, 4))], axis=1)[:, rng.permutation(10)]
    Mh = rng.standard_normal((50, 50))
    M = Mh @ Mh.T + 50 * np.eye(50)                 # the inner product of the Gram matrix
    keep = O.gram_keep(X.T @ M @ X)
    assert keep.size == 6
    Xk = X[:, keep]
    Pk = Xk @ np.linalg.solve(Xk.T @ M @ Xk, Xk.T @ M)
    Q, _ = np.linalg.qr(B)
    # M-orthogonal projector onto span(B): B (B^T M B)^{-1} B^T M
    Pr = B @ np.linalg.solve(B.T @ M @ B, B.T @ M)
    assert np.max(np.abs(Pk - Pr)) <= 1e-9


# ----------------------------------------------------------------------------
# coloring constant (Definition of the coloring constant, Section 2.2)
# ----------------------------------------------------------------------------
def _conflicts_bruteforce(subs, M):
    """s ~ t when M has a nonzero (i, j) with i in Omega^s and j in Omega^t,
    by looping over the entries of the dense M."""
    Md = M.toarray() != 0
    N = len(subs)
    C = np.zeros((N, N), dtype=bool)
    for s in range(N):
        for t in range(N):
            if s != t:
                C[s, t] = bool(Md[np.ix_(subs[s], subs[t])].any())
    return C


@pytest.mark.parametrize("mk", [small_fd, lambda: random_spd(11) + (None,)])
def test_coloring_is_valid(mk):
    """No two conflicting subdomains share a color, for the pattern of A and
    of A_+ (the matrices whose coloring constants enter the bounds)."""
    A, subs, _ = mk()
    subs = [np.asarray(s) for s in subs]
    st = O.setup(A, subs, 0.1)
    for M in (A, O.assemble_A_plus(st)):
        col = O.conflict_coloring(subs, M)
        C = _conflicts_bruteforce(subs, M)
        s, t = np.nonzero(C)
        assert np.all(col[s] != col[t])
        assert O.coloring_constant(subs, M) == col.max() + 1


def test_coloring_constant_of_box_partitions():
    """Known counts.  A 1D chain split into consecutive blocks overlapping in
    one node: each block meets only its two neighbours, so 2 colors.  The 5-point
    Laplacian on a grid split into 4 x 4 boxes extended by one layer: boxes
    conflict with their 8 neighbours (a king's graph, which contains K4), so
    at least 4 colors, and the greedy coloring in row-major order uses exactly 4."""
    n = 41
    A1 = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    subs1 = [np.arange(10 * k, min(10 * k + 11, n)) for k in range(4)]
    assert O.coloring_constant(subs1, A1) == 2
    prob = P.fd5_diffusion(16, np.ones((17, 17)))
    subs2 = [np.asarray(s) for s in part.box_subdomains(prob, (4, 4), 1)]
    C = _conflicts_bruteforce(subs2, prob.A)
    # the conflict graph is the king's graph of the 4 x 4 box layout
    for s in range(16):
        for t in range(16):
            if s != t:
                king = max(abs(s // 4 - t // 4), abs(s % 4 - t % 4)) == 1
                assert C[s, t] == king
    assert O.coloring_constant(subs2, prob.A) == 4


# ----------------------------------------------------------------------------
# PCG: restart from the true residual (reading of the stopping rule)
# ----------------------------------------------------------------------------
def _drift_case(seed, span):
    """Diagonally scaled 1D Laplacian S K S (entries of S spread over 10^span):
    Jacobi-preconditioned PCG converges in ~150 iterations while the recursive
    residual drifts away from b - A x by rounding."""
    rng = np.random.default_rng(seed)
    n = 200
    K = sp.diags([-np.ones(n - 1), 2.05 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).toarray()
    S = 10 ** rng.uniform(0, span, n)
    A = (S[:, None] * K) * S[None, :]
    b = rng.standard_normal(n)
    d = 1.0 / np.diag(A)
    return A, b, (lambda v: d * v)


def _true_res_extended(A, b, x):
    """||b - A x|| / ||b|| evaluated in 80-bit extended precision."""
    Al, bl, xl = (np.asarray(v, dtype=np.longdouble) for v in (A, b, x))
    return float(np.linalg.norm((bl - Al @ xl).astype(np.float64)) / np.linalg.norm(b))


def test_pcg_restart_recovers_the_true_residual():
    """The recursive residual meets tol while b - A x does not; without the
    restart PCG stops there unconverged, with it one restart from the true
    residual reaches tol, checked against the residual of the returned x in
    extended precision and against a direct solve."""
    A, b, M = _drift_case(36, 8)
    tol = 1e-8
    r0 = O.pcg(A, b, M, tol=tol, maxit=2000, max_restarts=0)
    assert r0.res_hist[-1] <= tol and not r0.converged
    assert _true_res_extended(A, b, r0.x) > tol
    r = O.pcg(A, b, M, tol=tol, maxit=2000)
    assert r.restarts >= 1 and r.converged
    assert r.iters > r0.iters
    assert _true_res_extended(A, b, r.x) <= tol
    assert abs(_true_res_extended(A, b, r.x) - r.rel_res_true) <= 0.05 * r.rel_res_true
    xd = np.linalg.solve(A, b)
    # same solution: A (x - x_direct) is small relative to b
    assert np.linalg.norm(A @ (r.x - xd)) <= 2 * tol * np.linalg.norm(b)


def test_pcg_restart_cap_reports_non_convergence():
    """Where b - A x cannot reach tol in FP64 (scaling spread 10^10), the
    restarts stop at the cap and PCG reports non-convergence with the
    residual of the returned iterate."""
    A, b, M = _drift_case(36, 10)
    r = O.pcg(A, b, M, tol=1e-8, maxit=2000, max_restarts=3)
    assert r.restarts == 3 and not r.converged
    tr = _true_res_extended(A, b, r.x)
    assert tr > 1e-8
    assert abs(tr - r.rel_res_true) <= 0.05 * tr


# ----------------------------------------------------------------------------
# the direct W of the oracle above n = 4000 (sparse LU of A + Woodbury)
# ----------------------------------------------------------------------------
def test_direct_W_large_branch_matches_assembled_A_plus():
    """O.setup's W for n > 4000 comes from solve_A_plus_direct's Woodbury
    branch on a sparse LU of A; it equals the dense solve with A_+ assembled
    from the local A^s_+ = V_+ L_+ V_+^T (a different route to the same
    matrix), column by column."""
    w = P.q1_2d(64)
    assert w.A.shape[0] > 4000
    st = O.setup(w.A, w.subs, w.tau)
    assert st.w_info["solver"] == "direct" and st.n_minus > 0
    Ap = O.assemble_A_plus(st).toarray()
    Wd = sla.cho_solve(sla.cho_factor(Ap, lower=True), st.Vg)
    # backward error of each column with the assembled A_+ (independent of
    # the conditioning), then the forward error within the first-order bound
    # 10 eps kappa(A_+) of two backward-stable solves (kappa ~ 2.4e7 here)
    nA = np.linalg.norm(Ap, 2)
    back = np.linalg.norm(Ap @ st.W - st.Vg, axis=0) / (nA * np.linalg.norm(st.W, axis=0))
    assert back.max() <= 1e-11
    ev = np.linalg.eigvalsh(Ap)
    kappa = ev[-1] / ev[0]
    err = np.linalg.norm(st.W - Wd, axis=0) / np.linalg.norm(Wd, axis=0)
    assert err.max() <= 10 * np.finfo(float).eps * kappa


# ----------------------------------------------------------------------------
# margin of the deletion of dependent coarse vectors (D2 / D4 readings)
# ----------------------------------------------------------------------------
def test_deletion_margin():
    """Pivots of gram_keep are the squared relative distances of each column
    from the span of the kept earlier ones; the margin is the factor to the
    threshold of the closest decision."""
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, 30))
    e = np.linalg.qr(np.stack([a, b, rng.standard_normal(30)], axis=1))[0][:, 2]   # unit, orthogonal to a, b
    for eps in (1e-2, 1e-4, 1e-6):
        c = a + b + eps * np.linalg.norm(a + b) * e       # distance eps * |a + b| from span(a, b)
        X = np.stack([a, b, c], axis=1)
        E = X.T @ X
        keep, piv = O.gram_keep(E, return_pivots=True)
        p2 = eps ** 2 / (1 + eps ** 2)                    # squared sine of the angle to span(a, b)
        assert abs(piv[2] - p2) <= 1e-5 * p2 + 1e-14            # cancellation: absolute error ~ eps
        if p2 > 1e-10:
            assert keep.tolist() == [0, 1, 2]
            assert np.isclose(O.deletion_margin(piv, keep), min(p2 / 1e-10, piv[:2].min() / 1e-10), rtol=1e-4)
        else:
            assert keep.tolist() == [0, 1]
            assert np.isclose(O.deletion_margin(piv, keep), 1e-10 / piv[2], rtol=1e-12)
    X = np.stack([a, b, a - 2 * b], axis=1)
    keep, piv = O.gram_keep(X.T @ X, return_pivots=True)
    assert keep.tolist() == [0, 1]
    assert O.deletion_margin(piv, keep) >= 1e3
