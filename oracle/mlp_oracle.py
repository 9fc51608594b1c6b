"""FP64 CPU oracle of the learned warm start's network and training loss.

TEST INFRASTRUCTURE ONLY: imported by the test-suite; never by the GPU
library, with which it shares no code.  Used to check the GPU's FP32
gradients.

The paper has no learned component; this is the network that predicts a
starting block for the local GenEO eigensolves (their modes are defined in the
Theorem on H^NN_hyb, Section 3.4).  Definitions:

* Per-dof multilayer perceptron with layer sizes d_0 = F, d_1 .. d_{L-1} = H,
  d_L = p.  Layer l has W_l (d_l x d_{l-1}) and b_l (d_l).  For an input row
  x:  h_0 = x,  h_l = tanh(h_{l-1} W_l^T + b_l) for l < L,
  output o = h_{L-1} W_L^T + b_L.
* For one subdomain with predicted block P (n_s x p, the outputs of its dofs)
  and target modes T (n_s x m), the rotation-invariant subspace loss
      g(P) = min_C ||T - P C||_F^2 + eps ||C||_F^2,   eps = ridge * n_s,
  normalised by ||T||_F^2.  The minimiser is C = (P^T P + eps I)^{-1} P^T T;
  with R = T - P C the gradient is dg/dP = -2 R C^T (the minimisation over C
  contributes nothing at the minimiser: variable projection, Golub and Pereyra,
  SIAM J. Numer. Anal. 10 (1973)).
* The batch loss is the mean of the normalised subdomain losses.
"""
from __future__ import annotations

import numpy as np


def layer_dims(F: int, H: int, p: int, hidden: int = 3):
    return [F] + [H] * hidden + [p]


def init_params(dims, rng):
    """Glorot-uniform weights, zero biases (any init is fine for the checks)."""
    ps = []
    for l in range(1, len(dims)):
        a = np.sqrt(6.0 / (dims[l] + dims[l - 1]))
        ps.append((rng.uniform(-a, a, (dims[l], dims[l - 1])), np.zeros(dims[l])))
    return ps


def flatten(params) -> np.ndarray:
    """W_1, b_1, W_2, b_2, ... with every W_l row-major (d_l x d_{l-1})."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(vec: np.ndarray, dims):
    out, o = [], 0
    for l in range(1, len(dims)):
        nw = dims[l] * dims[l - 1]
        W = vec[o:o + nw].reshape(dims[l], dims[l - 1])
        o += nw
        b = vec[o:o + dims[l]]
        o += dims[l]
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


def forward(params, X: np.ndarray):
    """Outputs (rows x p) and the hidden activations h_0 .. h_{L-1}."""
    hs = [np.asarray(X, dtype=np.float64)]
    for l, (W, b) in enumerate(params):
        z = hs[-1] @ W.T + b
        if l < len(params) - 1:
            hs.append(np.tanh(z))
        else:
            return z, hs
    raise AssertionError


def subspace_loss(P: np.ndarray, T: np.ndarray, ridge: float):
    """Normalised loss of one subdomain and its gradient with respect to P."""
    n, p = P.shape
    eps = ridge * n
    C = np.linalg.solve(P.T @ P + eps * np.eye(p), P.T @ T)
    R = T - P @ C
    tt = np.sum(T * T)
    g = (np.sum(R * R) + eps * np.sum(C * C)) / tt
    dP = -2.0 * (R @ C.T) / tt
    return g, dP


def batch_loss(O: np.ndarray, row_ptr, targets, ridge: float):
    """Mean subdomain loss over the subdomains with targets, and dL/dO."""
    dO = np.zeros_like(O)
    tot, cnt = 0.0, 0
    for s, T in enumerate(targets):
        if T is None or T.shape[1] == 0:
            continue
        r0, r1 = row_ptr[s], row_ptr[s + 1]
        g, dP = subspace_loss(O[r0:r1], T, ridge)
        tot += g
        dO[r0:r1] += dP
        cnt += 1
    if cnt == 0:
        return 0.0, dO
    return tot / cnt, dO / cnt


def backward(params, hs, dO):
    """Gradients (dW_l, db_l) of a loss with output gradient dO (backpropagation)."""
    grads = [None] * len(params)
    d = dO
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (d.T @ hs[l], d.sum(axis=0))
        if l > 0:
            d = (d @ W) * (1.0 - hs[l] ** 2)
    return grads


def loss_and_grad(params, X, row_ptr, targets, ridge: float):
    O, hs = forward(params, X)
    L, dO = batch_loss(O, row_ptr, targets, ridge)
    return L, backward(params, hs, dO)
