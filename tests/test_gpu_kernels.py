"""Batched dense building blocks (include/awg_dense.h) against numpy FP64.

Sizes are chosen to span several 64x64 tiles, 32-wide Cholesky panels and
64-row triangular-solve blocks, with ragged tails.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def to_dev(M):
    """numpy (batch, rows, cols) -> torch (batch, cols, rows) = column-major blocks."""
    import torch
    return torch.as_tensor(np.ascontiguousarray(M.transpose(0, 2, 1)), device="cuda")


def from_dev(T):
    return T.cpu().numpy().transpose(0, 2, 1)


def spd(rng, batch, n, cond=1e3):
    out = np.empty((batch, n, n))
    for b in range(batch):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        ev = np.logspace(0, np.log10(cond), n)
        out[b] = (Q * ev) @ Q.T
        out[b] = 0.5 * (out[b] + out[b].T)
    return out


@pytest.mark.parametrize("tA", [False, True])
@pytest.mark.parametrize("tB", [False, True])
@pytest.mark.parametrize("mnk", [(100, 70, 37), (64, 64, 16), (1, 130, 5), (131, 1, 200), (7, 9, 1),
                                 (300, 260, 70), (128, 128, 16), (257, 129, 33), (130, 700, 3)])
def test_gemm(gpu_lib, tA, tB, mnk):
    m, n, k = mnk
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    batch = 3
    A = rng.standard_normal((batch, k, m) if tA else (batch, m, k))
    B = rng.standard_normal((batch, n, k) if tB else (batch, k, n))
    C = rng.standard_normal((batch, m, n))
    ref = np.stack([(-0.5) * ((A[b].T if tA else A[b]) @ (B[b].T if tB else B[b])) + 2.0 * C[b]
                    for b in range(batch)])
    Cd = to_dev(C)
    gpu_lib.dense_gemm(to_dev(A), to_dev(B), Cd, alpha=-0.5, beta=2.0, transA=tA, transB=tB)
    out = from_dev(Cd)
    assert np.max(np.abs(out - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * k


@pytest.mark.parametrize("mnk", [(300, 30, 200), (130, 64, 2100), (257, 17, 33), (64, 100, 70), (1, 5, 3),
                                 (200, 1, 129), (150, 40, 16), (129, 33, 48)])
def test_gemm_variants_bit_identical(gpu_lib, mnk):
    """Every launch variant the autotuner may pick (64x64 and 128x128 tiles,
    4 or 8 wavefronts, the LDS-free skinny kernel) gives the same bits, for
    plain and row-gathered A operands (k > 2048 exercises the gathered index
    reads beyond the LDS table); the gathered form equals the product with
    the explicitly gathered matrix, bit for bit."""
    import torch
    m, n, k = mnk
    rng = np.random.default_rng(m + 31 * n + 7 * k)
    batch = 3
    rows = 2 * k + 5
    X = rng.standard_normal((rows, m))
    idx = rng.integers(0, rows, size=(batch, k)).astype(np.int32)
    B = rng.standard_normal((batch, k, n))
    C0 = rng.standard_normal((batch, m, n))
    Xd = torch.as_tensor(X, device="cuda")
    Id = torch.as_tensor(idx, device="cuda")
    Ag = np.stack([X[idx[b]].T for b in range(batch)])          # (batch, m, k)
    ref = np.stack([-0.5 * (Ag[b] @ B[b]) + 2.0 * C0[b] for b in range(batch)])
    outs = []
    for v in range(6):
        for gathered in (False, True):
            Cd = to_dev(C0)
            if gathered:
                gpu_lib.dense_gemm_ex(Xd, to_dev(B), Cd, alpha=-0.5, beta=2.0, variant=v, arows=Id)
            else:
                gpu_lib.dense_gemm_ex(to_dev(Ag), to_dev(B), Cd, alpha=-0.5, beta=2.0, variant=v)
            outs.append(from_dev(Cd))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.max(np.abs(outs[0] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * k
    # transposed operands: variant 3 falls back to the 8-wavefront tiles
    for tA, tB in [(True, False), (False, True), (True, True)]:
        A = rng.standard_normal((batch, k, m) if tA else (batch, m, k))
        Bt = rng.standard_normal((batch, n, k) if tB else (batch, k, n))
        res = []
        for v in range(6):
            Cd = to_dev(C0)
            gpu_lib.dense_gemm_ex(to_dev(A), to_dev(Bt), Cd, alpha=1.0, beta=0.0, transA=tA, transB=tB, variant=v)
            res.append(from_dev(Cd))
        for o in res[1:]:
            assert np.array_equal(o, res[0])


def test_gemm_ex_rejects_bad_arguments(gpu_lib):
    import torch
    from paper_2106_10913_amd.awg import AWGError
    A = torch.zeros((1, 4, 4), dtype=torch.float64, device="cuda")
    idx = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    for kw in [dict(variant=6), dict(variant=-2), dict(transA=True, arows=idx)]:
        with pytest.raises(AWGError):
            gpu_lib.dense_gemm_ex(A, A, A.clone(), **kw)


@pytest.mark.parametrize("ncols", [1, 5, 130, 257])
def test_local_product_f16x3(gpu_lib, ncols):
    """Split-FP16 local products against numpy FP64, element by element within
    the error bound of the arithmetic: the split x = hi + lo keeps 22
    significant bits (|x - hi - lo| <= 2^-22 |x|), the dropped lo.lo term is
    below 2^-22 |p x|, and FP32 sums of k terms add at most k 2^-24 of the
    sum of magnitudes; values that the scaling sends below the FP16
    subnormal range (2^-38 of the column's largest) are lost.  Sizes cover
    fewer than 8 rows, whole and ragged groups of 8, several 128 tiles; the
    columns span 60 decades, with one column of zeros.  The bound counts the
    lost values of both operands (below 2^-38 of the column's or the
    matrix's largest magnitude)."""
    import torch
    rng = np.random.default_rng(ncols)
    sizes = [1, 7, 8, 9, 100, 129, 300]
    rows = sum(sizes)
    X = rng.standard_normal((rows, ncols)) * 10.0 ** rng.uniform(-30, 30, ncols)
    if ncols > 1:
        X[:, 1] = 0.0
    Ps = [rng.standard_normal((k, k)) * 10.0 ** rng.uniform(-20, 20) for k in sizes]
    Pflat = np.concatenate([p.T.reshape(-1) for p in Ps])      # column-major blocks
    Xd = torch.as_tensor(X, device="cuda")
    Pd = torch.as_tensor(Pflat, device="cuda")
    Yd = torch.full_like(Xd, float("nan"))
    gpu_lib.dense_local_product_f16x3(sizes, Xd, Pd, Yd)
    Y = Yd.cpu().numpy()
    colmax = np.abs(X).max(axis=0)
    o = 0
    rel = []
    for k, p in zip(sizes, Ps):
        Xb = X[o:o + k]
        ref = p.T @ Xb
        mag = np.abs(p).T @ np.abs(Xb)
        bound = ((2.0 ** -20 + k * 2.0 ** -24) * mag
                 + 2.0 ** -36 * (np.abs(p).sum(axis=0)[:, None] * colmax
                                 + np.abs(p).max() * np.abs(Xb).sum(axis=0)[None, :]))
        err = np.abs(Y[o:o + k] - ref)
        assert np.all(err <= bound), (k, float((err / np.maximum(bound, 1e-300)).max()))
        nz = mag > 0
        rel.append((err[nz] / mag[nz]).max(initial=0.0))
        o += k
    assert not np.isnan(Y).any()
    print(f"\n[f16x3 local product] ncols={ncols} max err / sum|terms| = {max(rel):.2e}", flush=True)


def test_local_product_f16x3_rejects_bad_arguments(gpu_lib):
    import torch
    X = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    P = torch.zeros(16, dtype=torch.float64, device="cuda")
    from paper_2106_10913_amd.awg import AWGError
    with pytest.raises(AWGError):
        gpu_lib.dense_local_product_f16x3([4, 0], X, P, X)


def test_spd_inverse_f32(gpu_lib):
    """FP32 Cholesky inverses on the matrix cores against numpy FP64, on
    ragged sizes (one panel, panel and substitution-block boundaries, several
    tiles): relative Frobenius error within 20 sqrt(n) kappa 2^-24, the
    pivot ratio squared never above kappa, and a block that is not positive
    definite flagged while the others are unaffected."""
    import torch
    rng = np.random.default_rng(7)
    sizes = [1, 5, 31, 32, 33, 64, 65, 100, 257, 300]
    cond = 1e3
    blocks = [spd(rng, 1, k, cond)[0] for k in sizes]
    bad = rng.standard_normal((40, 40))
    blocks.append(0.5 * (bad + bad.T))                    # indefinite
    sizes = sizes + [40]
    flat = np.concatenate([b.T.reshape(-1) for b in blocks])
    A = torch.as_tensor(flat, device="cuda")
    Ai = torch.full_like(A, float("nan"))
    info, ratio = gpu_lib.dense_spd_inverse_f32(sizes, A, Ai)
    out = Ai.cpu().numpy()
    o = 0
    worst = 0.0
    for b, (k, M) in enumerate(zip(sizes, blocks)):
        if b == len(sizes) - 1:
            assert info[b] != 0
            break
        assert info[b] == 0
        G = out[o:o + k * k].reshape(k, k).T
        ref = np.linalg.inv(M)
        kap = np.linalg.cond(M)
        err = np.linalg.norm(G - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        assert err <= 20 * np.sqrt(k) * kap * 2.0 ** -24, (k, err)
        assert ratio[b] ** 2 <= kap * (1 + 1e-3)
        o += k * k
    print(f"\n[spd inverse f32] worst relative error {worst:.2e} at kappa {cond:g}", flush=True)


@pytest.mark.parametrize("n", [1, 31, 33, 64, 100, 257])
def test_potrf(gpu_lib, n):
    rng = np.random.default_rng(n)
    M = spd(rng, 2, n)
    Ad = to_dev(M)
    info = gpu_lib.dense_potrf(Ad)
    assert np.all(info == 0)
    L = np.tril(from_dev(Ad))
    for b in range(2):
        ref = np.linalg.cholesky(M[b])
        assert np.max(np.abs(L[b] - ref)) <= 1e-12 * np.max(np.abs(ref)) * n


def test_potrf_reports_breakdown(gpu_lib):
    rng = np.random.default_rng(1)
    M = spd(rng, 2, 80)
    M[1, 50, 50] = -1e6                      # indefinite second block
    info = gpu_lib.dense_potrf(to_dev(M))
    assert info[0] == 0 and 1 <= info[1] <= 51


@pytest.mark.parametrize("n,nrhs", [(100, 37), (64, 64), (130, 1), (65, 200)])
@pytest.mark.parametrize("trans", [False, True])
def test_trsm(gpu_lib, n, nrhs, trans):
    rng = np.random.default_rng(n + nrhs)
    L = np.tril(rng.standard_normal((2, n, n))) + 4.0 * np.eye(n)
    B = rng.standard_normal((2, n, nrhs))
    Bd = to_dev(B)
    gpu_lib.dense_trsm(to_dev(L), Bd, trans=trans)
    X = from_dev(Bd)
    for b in range(2):
        ref = np.linalg.solve(L[b].T if trans else L[b], B[b])
        assert np.max(np.abs(X[b] - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


# 700 and 900: more than 64 tiles of 64 x 64 in the trailing matrix, so each
# workgroup of the symmetric product walks several tiles
@pytest.mark.parametrize("n", [1, 2, 3, 40, 97, 200, 700, 900])
def test_low_eigs_against_eigh(gpu_lib, n):
    rng = np.random.default_rng(n)
    batch = 3
    M = np.empty((batch, n, n))
    for b in range(batch):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        ev = rng.uniform(-1.0, 4.0, n)
        if n >= 40:
            ev[:6] = -0.5                     # a repeated negative eigenvalue
            ev[6:9] = [1e-9, -1e-9, 0.0]      # a tight cluster at zero
        M[b] = (Q * ev) @ Q.T
        M[b] = 0.5 * (M[b] + M[b].T)
    thr = 0.25
    maxk = n
    cnt, lam, Z = gpu_lib.dense_low_eigs(to_dev(M), thr, maxk)
    lam = lam.cpu().numpy()
    Z = Z.cpu().numpy()                       # (batch, k, n): row j = eigenvector j
    for b in range(batch):
        ev, V = np.linalg.eigh(M[b])
        k = int(np.count_nonzero(ev < thr))
        assert cnt[b] == k
        assert np.max(np.abs(lam[b, :k] - ev[:k]), initial=0.0) <= 1e-12 * np.abs(ev).max() * n
        Zb = Z[b, :k].T
        assert np.max(np.abs(Zb.T @ Zb - np.eye(k)), initial=0.0) <= 1e-10
        res = M[b] @ Zb - Zb * lam[b, :k]
        assert np.max(np.abs(res), initial=0.0) <= 1e-10 * np.abs(ev).max()
        # same invariant subspace as LAPACK
        Pg = Zb @ Zb.T
        Pr = V[:, :k] @ V[:, :k].T
        assert np.max(np.abs(Pg - Pr), initial=0.0) <= 1e-8


@pytest.mark.parametrize("vector", [False, True])
@pytest.mark.parametrize("b", [2, 17, 64, 130, 300])
def test_csr_spmm_variants_bit_identical(gpu_lib, b, vector):
    """Every SpMM launch variant (and the autotuned one) gives the same bits,
    within rounding of the exact product; beta != 0 accumulates.  vector: 3
    dofs per node with a shared column pattern, plus rows of a different
    pattern and a dense block at the end; the grouped kernels run on the
    union patterns of consecutive rows, with zeros where a row has no entry."""
    import torch
    import scipy.sparse as sp
    import awg_problems as P
    A = P.q1_2d(m=24, partition="rcb", nparts=4, delta=1).A.tocsr()
    if vector:
        A = sp.kron(A, np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 1.0], [0.5, 1.0, 5.0]])).tocsr()
        # and a dense 150 x 150 block (long groups)
        D = np.random.default_rng(3).standard_normal((150, 150)) + 200 * np.eye(150)
        A = sp.block_diag([A, sp.random(7, 7, density=0.5, random_state=1) + 10 * sp.eye(7), sp.csr_matrix(D)]).tocsr()
    A.sort_indices()
    n = A.shape[0]
    rng = np.random.default_rng(b)
    X = rng.standard_normal((n, b))
    Y0 = rng.standard_normal((n, b))
    rp = torch.as_tensor(A.indptr.astype(np.int64), device="cuda")
    ci = torch.as_tensor(A.indices.astype(np.int32), device="cuda")
    va = torch.as_tensor(A.data, device="cuda")
    Xd = torch.as_tensor(X, device="cuda")
    ref = -0.5 * (A @ X) + 2.0 * Y0
    outs = []
    for v in [-1] + list(range(11)):
        Yd = torch.as_tensor(Y0, device="cuda")
        gpu_lib.csr_spmm(rp, ci, va, Xd, Yd, alpha=-0.5, beta=2.0, variant=v)
        outs.append(Yd.cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.max(np.abs(outs[0] - ref)) <= 1e-13 * np.max(np.abs(ref))
    # first tuned call with beta = 0 measures the variants on this shape
    Yd = torch.empty((n, b), dtype=torch.float64, device="cuda")
    gpu_lib.csr_spmm(rp, ci, va, Xd, Yd, alpha=1.0, beta=0.0, variant=-1)
    assert np.max(np.abs(Yd.cpu().numpy() - A @ X)) <= 1e-13 * np.max(np.abs(A @ X))
    rep = gpu_lib.tune_report()
    key = f"spmm:n={n}:nnz={A.nnz}:b={b}:grouped=1"
    # 11 variants measured: the row groups were built for the two grouped
    # variants (both matrices group: node dofs, neighbouring rows)
    nv = 11
    assert key in rep and 0 <= rep[key]["variant"] < nv and len(rep[key]["us"]) == nv
