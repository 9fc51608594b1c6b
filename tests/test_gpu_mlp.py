"""Warm-start network kernels (include/awg_mlp.h) against the FP64 oracle of
the network and its loss (oracle/mlp_oracle.py), and the per-dof features
against a NumPy recomputation from their definitions."""
import numpy as np
import pytest
import scipy.sparse as sp

import awg_problems as P
from awg_problems import partition as part
from oracle import mlp_oracle as M
from oracle import awg_oracle as O

pytestmark = pytest.mark.gpu


def batch(rng, sizes, cols, F=12):
    rows = int(sum(sizes))
    X = rng.standard_normal((rows, F)).astype(np.float32)
    row_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    targets, flat, off = [], [], [0]
    for n, m in zip(sizes, cols):
        T = rng.standard_normal((n, m)).astype(np.float32) if m else None
        targets.append(None if T is None else T.astype(np.float64))
        flat.append(np.zeros(0, np.float32) if T is None else T.T.ravel())   # column-major
        off.append(off[-1] + n * m)
    return X, row_ptr, targets, np.concatenate(flat), np.array(off[:-1], np.int64), np.array(cols, np.int32)


def dev(a):
    import torch
    return torch.as_tensor(a, device="cuda")


@pytest.mark.parametrize("width,hidden,p", [(256, 3, 8), (32, 2, 3), (64, 1, 16)])
def test_gradients_match_oracle(gpu_lib, width, hidden, p):
    rng = np.random.default_rng(width + p)
    net = gpu_lib.MLP(12, width, hidden, p, seed=5)
    dims = M.layer_dims(12, width, p, hidden)
    params = M.init_params(dims, rng)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    vec = M.flatten(params).astype(np.float32)
    net.set_params(vec)
    assert np.array_equal(net.get_params(), vec)
    sizes, cols = [70, 0, 131, 64, 9], [3, 2, 5, 1, 2]
    cols[1] = 0
    X, row_ptr, targets, T, toff, tcols = batch(rng, sizes, cols)
    ridge = 1e-3
    loss = net.loss_grad(dev(X), dev(row_ptr), dev(toff), dev(tcols), dev(T), ridge)
    g = net.get_grads().astype(np.float64)
    Lr, gref = M.loss_and_grad(M.unflatten(vec.astype(np.float64), dims), X.astype(np.float64), row_ptr, targets,
                               ridge)
    gr = M.flatten(gref)
    assert abs(loss - Lr) <= 1e-4 * abs(Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    # per layer as well (small layers must not hide behind large ones)
    o = 0
    for l in range(1, len(dims)):
        nw = dims[l] * dims[l - 1] + dims[l]
        assert np.linalg.norm(g[o:o + nw] - gr[o:o + nw]) <= 1e-4 * np.linalg.norm(gr[o:o + nw]) + 1e-12
        o += nw
    net.close()


@pytest.mark.parametrize("rows", [1, 63, 64, 65, 1000])
def test_forward_fp32_and_bf16(gpu_lib, rows):
    rng = np.random.default_rng(rows)
    net = gpu_lib.MLP(12, 256, 3, 8, seed=3)
    dims = M.layer_dims(12, 256, 8, 3)
    vec = net.get_params().astype(np.float64)
    X = rng.standard_normal((rows, 12)).astype(np.float32)
    ref, _ = M.forward(M.unflatten(vec, dims), X.astype(np.float64))
    y32 = net.forward(dev(X), bf16=False).cpu().numpy()
    y16 = net.forward(dev(X), bf16=True).cpu().numpy()
    scale = np.linalg.norm(ref)
    assert np.linalg.norm(y32 - ref) <= 1e-5 * scale
    # bf16 weights and activations: 8 significant bits per operand
    assert np.linalg.norm(y16 - ref) <= 3e-2 * scale
    net.close()


def test_training_reduces_the_loss(gpu_lib):
    """Targets that a linear function of the inputs spans exactly."""
    rng = np.random.default_rng(11)
    net = gpu_lib.MLP(12, 64, 2, 4, seed=1)
    sizes = [80] * 6
    X = rng.standard_normal((480, 12)).astype(np.float32)
    row_ptr = np.arange(0, 481, 80, dtype=np.int64)
    Tl, off = [], []
    for s in range(6):
        Xs = X[row_ptr[s]:row_ptr[s + 1]]
        T = Xs[:, :3] @ rng.standard_normal((3, 2)).astype(np.float32)
        off.append(sum(t.size for t in Tl))
        Tl.append(T.T.ravel())
    args = (dev(X), dev(row_ptr), dev(np.array(off, np.int64)), dev(np.full(6, 2, np.int32)), dev(np.concatenate(Tl)))
    first = net.loss_grad(*args, ridge=1e-4)
    for _ in range(300):
        net.loss_grad(*args, ridge=1e-4)
        net.adam_step(lr=3e-3)
    last = net.loss_grad(*args, ridge=1e-4)
    assert last < 0.1 * first, (first, last)
    net.close()


def test_create_rejects_bad_shapes(gpu_lib):
    from paper_2106_10913_amd.awg import AWGError
    for kw in [dict(in_features=0), dict(width=24), dict(width=512), dict(out_channels=17), dict(hidden_layers=0)]:
        with pytest.raises(AWGError):
            gpu_lib.MLP(**kw)


def _depth(A, idx):
    """Graph distance to the outside of the subdomain, capped at 4 (BFS)."""
    inside = np.zeros(A.shape[0], bool)
    inside[idx] = True
    d = np.full(A.shape[0], 4.0)
    A = A.tocsr()
    frontier = []
    for g in idx:
        nb = A.indices[A.indptr[g]:A.indptr[g + 1]]
        if np.any(~inside[nb[nb != g]]):
            d[g] = 0.0
            frontier.append(g)
    for level in range(1, 4):
        nxt = []
        for g in frontier:
            for j in A.indices[A.indptr[g]:A.indptr[g + 1]]:
                if inside[j] and d[j] > level:
                    d[j] = level
                    nxt.append(j)
        frontier = nxt
    return d[idx]


def test_features_follow_their_definitions(gpu_lib):
    w = P.q1_2d(m=32, partition="rcb", nparts=6, delta=1)
    coords = w.coords
    solver = gpu_lib.Solver(w.A, w.subs, tau=w.tau, geneo="subspace", coords=coords)
    f = solver.export("mlp_features").reshape(-1, 12)
    A = w.A.tocsr()
    ld = np.log10(np.abs(A.diagonal()))
    mult = O.multiplicity(A.shape[0], w.subs)
    V = solver.export("V_minus")
    ks = solver.stats()["k_s"]
    voff = 0
    r = 0
    for s, idx in enumerate(w.subs):
        n = len(idx)
        fs = f[r:r + n]
        r += n
        np.testing.assert_allclose(fs[:, 3], (ld[idx] - ld[idx].mean()) / 4, atol=1e-5)
        np.testing.assert_allclose(fs[:, 4], (ld[idx] - ld.mean()) / 4, atol=1e-5)
        np.testing.assert_allclose(fs[:, 8], 1.0 / mult[idx], rtol=1e-6)
        np.testing.assert_array_equal(fs[:, 9], _depth(A, idx) / 4)
        Vs = V[voff:voff + n * ks[s]].reshape(ks[s], n).T
        voff += n * ks[s]
        lev = ((Vs / mult[idx][:, None]) ** 2).sum(axis=1) * n / max(1, ks[s]) if ks[s] else np.zeros(n)
        np.testing.assert_allclose(fs[:, 10], lev, rtol=1e-4, atol=1e-6)
        for i in range(0, n, 37):
            g = idx[i]
            nb = A.indices[A.indptr[g]:A.indptr[g + 1]]
            vals = A.data[A.indptr[g]:A.indptr[g + 1]]
            keep = nb != g
            assert abs(fs[i, 5] - (max(ld[g], ld[nb[keep]].max()) - ld[g]) / 4) <= 1e-5
            assert abs(fs[i, 6] - (min(ld[g], ld[nb[keep]].min()) - ld[g]) / 4) <= 1e-5
            assert abs(fs[i, 7] - (np.log10(np.abs(vals[keep])).mean() - ld[g]) / 4) <= 1e-5
        xy = coords[idx]
        lo, hi = xy.min(axis=0), xy.max(axis=0)
        np.testing.assert_allclose(fs[:, :2], 2 * (xy - lo) / (hi - lo) - 1, atol=1e-6)
        assert np.all(fs[:, 2] == 0)
    assert r == f.shape[0]
    solver.close()


def test_learned_start_selects_the_same_modes(gpu_lib):
    w = P.q1_2d(m=48, partition="rcb", nparts=12, delta=2)
    net = gpu_lib.MLP(12, 256, 3, 8, seed=2)       # untrained: the eigensolver must still get it right
    dense = gpu_lib.Solver(w.A, w.subs, tau=w.tau)
    learned = gpu_lib.Solver(w.A, w.subs, tau=w.tau, geneo="subspace", eig_init=net)
    sd, sl = dense.stats(), learned.stats()
    assert sl["eig_learned"] == 1 and sl["eig_fallbacks"] == 0
    assert sl["m_s"] == sd["m_s"] and sl["n0"] == sd["n0"]
    import torch
    b = torch.as_tensor(w.b, device="cuda")
    _, i1 = dense.pcg(b, tol=w.tol)
    _, i2 = learned.pcg(b, tol=w.tol)
    assert abs(i1["iters"] - i2["iters"]) <= 1
    for o in (dense, learned, net):
        o.close()
