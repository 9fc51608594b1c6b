"""Pins of the FP64 network/loss oracle against closed forms, invariances and
central finite differences (no GPU)."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_subspace_loss_closed_forms():
    rng = np.random.default_rng(0)
    # targets inside the predicted span: zero loss without ridge
    P = rng.standard_normal((30, 4))
    T = P @ rng.standard_normal((4, 3))
    g, dP = M.subspace_loss(P, T, 0.0)
    assert g <= 1e-24 and np.max(np.abs(dP)) <= 1e-12
    # one column each: 1 - cos^2 of the angle between p and t
    p = rng.standard_normal((25, 1))
    t = rng.standard_normal((25, 1))
    g, _ = M.subspace_loss(p, t, 0.0)
    c = (p[:, 0] @ t[:, 0]) ** 2 / ((p[:, 0] @ p[:, 0]) * (t[:, 0] @ t[:, 0]))
    assert abs(g - (1.0 - c)) <= 1e-14
    # orthogonal targets: nothing explained
    Q, _ = np.linalg.qr(rng.standard_normal((20, 5)))
    g, _ = M.subspace_loss(Q[:, :3], Q[:, 3:], 0.0)
    assert abs(g - 1.0) <= 1e-14


@pytest.mark.parametrize("ridge", [0.0, 1e-3])
def test_subspace_loss_rotation_invariant_and_bounded(ridge):
    rng = np.random.default_rng(1)
    P = rng.standard_normal((40, 6))
    T = rng.standard_normal((40, 2))
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    g1, _ = M.subspace_loss(P, T, ridge)
    g2, _ = M.subspace_loss(P @ Q, T, ridge)
    g3, _ = M.subspace_loss(P, T @ np.linalg.qr(rng.standard_normal((2, 2)))[0], ridge)
    assert abs(g1 - g2) <= 1e-13 and abs(g1 - g3) <= 1e-13
    assert 0.0 <= g1 <= 1.0


@pytest.mark.parametrize("ridge", [0.0, 1e-2])
def test_subspace_loss_gradient_by_finite_differences(ridge):
    rng = np.random.default_rng(2)
    P = rng.standard_normal((12, 3))
    T = rng.standard_normal((12, 2))
    _, dP = M.subspace_loss(P, T, ridge)
    h = 1e-6
    fd = np.zeros_like(P)
    for i in range(P.shape[0]):
        for j in range(P.shape[1]):
            Pp, Pm = P.copy(), P.copy()
            Pp[i, j] += h
            Pm[i, j] -= h
            fd[i, j] = (M.subspace_loss(Pp, T, ridge)[0] - M.subspace_loss(Pm, T, ridge)[0]) / (2 * h)
    assert np.max(np.abs(fd - dP)) <= 1e-7 * max(1.0, np.max(np.abs(dP)))


def test_network_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    dims = M.layer_dims(4, 6, 3, hidden=3)
    params = M.init_params(dims, rng)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    X = rng.standard_normal((17, 4))
    row_ptr = [0, 9, 17]
    targets = [rng.standard_normal((9, 2)), rng.standard_normal((8, 1))]
    ridge = 1e-3
    L, grads = M.loss_and_grad(params, X, row_ptr, targets, ridge)
    vec = M.flatten(params)
    gvec = M.flatten(grads)
    h = 1e-6
    fd = np.zeros_like(vec)
    for k in range(vec.size):
        vp, vm = vec.copy(), vec.copy()
        vp[k] += h
        vm[k] -= h
        fd[k] = (M.loss_and_grad(M.unflatten(vp, dims), X, row_ptr, targets, ridge)[0]
                 - M.loss_and_grad(M.unflatten(vm, dims), X, row_ptr, targets, ridge)[0]) / (2 * h)
    assert np.max(np.abs(fd - gvec)) <= 1e-7 * max(1.0, np.max(np.abs(gvec)))


def test_flatten_layout_round_trip():
    rng = np.random.default_rng(4)
    dims = M.layer_dims(5, 8, 2, hidden=2)
    params = M.init_params(dims, rng)
    vec = M.flatten(params)
    assert vec.size == sum(dims[l] * dims[l - 1] + dims[l] for l in range(1, len(dims)))
    back = M.unflatten(vec, dims)
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)
