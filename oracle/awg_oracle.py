"""FP64 CPU oracle of PCG preconditioned by the additive AWG preconditioner.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  The GPU library
never calls it, and it shares no code with the GPU library.

What it computes (Gouarin & Spillane, "Fully algebraic domain decomposition
preconditioners with adaptive spectral bounds"):

    H = H3,ad = H2 + W (W^T A W)^{-1} W^T           (Definition of Pi_3 / H3, Section 4.3)
    H2 = H^NN_hyb(tau)                               (Theorem for H^NN with GenEO, Section 3.4)
       = Pi H^NN Pi^T + R0^T E0^{-1} R0,  E0 = R0 A_+ R0^T,
         Pi = I - R0^T E0^{-1} R0 A_+
    H^NN = sum_s R^sT D^s (A^s_+)^dagger D^s R^s      (Definition of H^NN, Section 3.3)

and the other choices: H3,inex and H3,hyb (Section 4) for the second coarse
space, and for H2 the AS forms H^AS_{+,hyb}(tau_flat) and H^AS_{+,ad}(tau_flat)
(Theorem on H^AS_{+,hyb/ad}, Section 3.4), H^AS_+ = sum_s R^sT (R^s A_+ R^sT)^{-1} R^s,
on the same coarse space with tau_flat = 1/tau, and H^AS_hyb(tau_sharp, tau_flat)
(Theorem on H^AS_hyb, Section 3.4) with local blocks R^s A R^sT and the
two-pencil coarse space, tau_sharp = tau and tau_flat = 1/tau.

The steps follow the paper's order and notation.  Dense LAPACK (numpy /
scipy) is used for every local and coarse problem; no iterative
eigensolver is involved.  Readings where the paper is silent:

* zero eigenvalues of B^s (Remark after the A_+ theorem, Section 3.2): an
  eigenvalue lambda counts as non-positive when lambda <= eps0 * max|lambda|,
  eps0 = 1e-12 by default; only strictly negative ones (lambda < -eps0 *
  max|lambda|) give columns of the second coarse space (Remark 1, Section 4.4).
* GenEO selection is the strict lambda < tau of the Y_L definition (Section 3.4).
* PCG starts from x0 = 0 and stops at the first k with ||r_k||_2 / ||b||_2 <= tol
  on the recursively updated residual; the iteration count is the number
  of products A p.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class OracleError(ValueError):
    """Invalid input for the method (not a bug in the oracle)."""


# ---------------------------------------------------------------------------
# Section 2: subdomains, restriction, partition of unity, coloring
# ---------------------------------------------------------------------------
def check_inputs(A: sp.csr_matrix, subs) -> None:
    """Validate A and the index sets (Definition of a partition and Assumption
    of minimal overlap, Section 2.1).  Raises OracleError."""
    n = A.shape[0]
    if A.shape[0] != A.shape[1]:
        raise OracleError("A is not square")
    if abs(A - A.T).max() if A.nnz else 0.0:
        raise OracleError("A is not symmetric")
    covered = np.zeros(n, dtype=bool)
    for s, idx in enumerate(subs):
        idx = np.asarray(idx)
        if idx.size == 0:
            raise OracleError(f"subdomain {s} is empty")
        if idx.min() < 0 or idx.max() >= n:
            raise OracleError(f"subdomain {s} has an index out of range")
        if np.any(np.diff(idx) <= 0):
            raise OracleError(f"subdomain {s} is not sorted and unique")
        covered[idx] = True
    if not covered.all():
        raise OracleError("the subdomains do not cover [0, n)")
    cnt = pair_multiplicity(A, subs)
    if np.any(cnt == 0):
        raise OracleError("minimal overlap assumption violated")


def multiplicity(n: int, subs) -> np.ndarray:
    """Diagonal of sum_t R^tT R^t: number of subdomains holding each dof (Section 2.2)."""
    m = np.zeros(n, dtype=np.int64)
    for idx in subs:
        m[idx] += 1
    return m


def partition_of_unity(n: int, subs):
    """D = (sum_t R^tT R^t)^{-1} and D^s = R^s D R^sT (Definition of D^s, Section 2.2).

    Returns the list of diagonals of the D^s.
    """
    d = 1.0 / multiplicity(n, subs)
    return [d[idx] for idx in subs]


def conflict_coloring(subs, M_pattern: sp.csr_matrix) -> np.ndarray:
    """Colors of the subdomains for the coloring constant N(M) (Definition of
    the coloring constant, Section 2.2).

    s and t conflict when R^s M R^tT != 0, i.e. when M has a nonzero (i, j)
    with i in Omega^s and j in Omega^t.  Greedy coloring of that conflict
    graph in subdomain order: each subdomain takes the smallest color that
    none of its conflicting predecessors holds.
    """
    N = len(subs)
    n = M_pattern.shape[0]
    P = sp.csr_matrix((np.ones(sum(len(s) for s in subs)),
                       (np.concatenate([np.full(len(s), k) for k, s in enumerate(subs)]),
                        np.concatenate(subs))), shape=(N, n))
    Mb = (abs(M_pattern) > 0).astype(np.float64)
    C = (P @ Mb @ P.T).toarray() > 0
    color = -np.ones(N, dtype=np.int64)
    for s in range(N):
        used = set(color[np.flatnonzero(C[s])].tolist())
        c = 0
        while c in used:
            c += 1
        color[s] = c
    return color


def coloring_constant(subs, M_pattern: sp.csr_matrix) -> int:
    """A valid coloring constant N(M): the number of colors of
    conflict_coloring (any valid coloring gives a valid bound)."""
    return int(conflict_coloring(subs, M_pattern).max() + 1)


# ---------------------------------------------------------------------------
# Section 3.1: algebraic splitting A = sum_s R^sT B^s R^s
# ---------------------------------------------------------------------------
def pair_multiplicity(A: sp.csr_matrix, subs) -> np.ndarray:
    """M_mu on the pattern of A: for each stored nonzero (i, j) of A (CSR order),
    the number of subdomains containing both i and j (Definition of B^s and the
    theorem that follows it, Section 3.1).  Counted directly."""
    n = A.shape[0]
    A = A.tocsr()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    cnt = np.zeros(A.nnz, dtype=np.int64)
    mask = np.zeros(n, dtype=bool)
    for idx in subs:
        mask[:] = False
        mask[idx] = True
        cnt += (mask[rows] & mask[cols])
    return cnt


def algebraic_B(A: sp.csr_matrix, cnt: np.ndarray) -> sp.csr_matrix:
    """B = A (Hadamard-divided by) M_mu on the pattern of A (Definition of B^s, Section 3.1)."""
    B = A.tocsr().copy()
    B.data = A.data / cnt
    return B


def local_block(M: sp.csr_matrix, idx) -> np.ndarray:
    """Dense R^s M R^sT."""
    return M[idx][:, idx].toarray()


# ---------------------------------------------------------------------------
# Section 3.2: B^s = A^s_+ - A^s_-, A_+ = sum R^sT A^s_+ R^s
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class LocalSplit:
    lam: np.ndarray        # all eigenvalues of B^s, ascending
    V: np.ndarray          # orthonormal eigenvectors (columns)
    nneg: int              # n^s_-: number of non-positive eigenvalues (incl. numerical zeros)
    nstrict: int           # number of strictly negative eigenvalues (second coarse space)
    thr: float             # eps0 * max|lambda|

    @property
    def V_minus(self):
        return self.V[:, :self.nneg]

    @property
    def L_minus(self):
        return self.lam[:self.nneg]

    @property
    def V_plus(self):
        return self.V[:, self.nneg:]

    @property
    def L_plus(self):
        return self.lam[self.nneg:]

    def A_plus(self):
        """A^s_+ = V_+ L_+ V_+^T (Definition of the splitting of B^s, Section 3.2)."""
        return (self.V_plus * self.L_plus) @ self.V_plus.T

    def A_minus(self):
        """A^s_- = - V_- L_- V_-^T."""
        return -(self.V_minus * self.L_minus) @ self.V_minus.T

    def A_plus_pinv(self):
        """(A^s_+)^dagger = V_+ L_+^{-1} V_+^T (Definition of H^NN, Section 3.3)."""
        return (self.V_plus / self.L_plus) @ self.V_plus.T


def split_local(Bs: np.ndarray, eps0: float = 1e-12) -> LocalSplit:
    """Diagonalise B^s (eigenvalues ascending) and split off the non-positive part.

    Zero eigenvalues go into L_- as the paper chooses (remark after the
    A_+ theorem); "zero" means |lambda| <= eps0 * max|lambda|.
    """
    lam, V = np.linalg.eigh(Bs)
    scale = np.max(np.abs(lam)) if lam.size else 0.0
    thr = eps0 * scale
    nneg = int(np.count_nonzero(lam <= thr))
    nstrict = int(np.count_nonzero(lam < -thr))
    return LocalSplit(lam, V, nneg, nstrict, thr)


# ---------------------------------------------------------------------------
# the whole setup
# ---------------------------------------------------------------------------
def gram_keep(E: np.ndarray, tol: float = 1e-10, return_pivots: bool = False):
    """Columns of a (possibly dependent) basis kept for a Gram matrix E.

    Reading of the basis assumption of Section 2 (a basis of V0 is assumed,
    none is constructed) and of Remark 1, Section 4.4 (dependent columns of
    the second coarse space may have to be removed): a left-to-right Cholesky
    factorisation deletes column k when its pivot (the squared norm, in the
    inner product of E, of the part of basis vector k outside the span of the
    kept earlier ones) is <= tol * E_kk.  The projection onto the span is then
    X_keep E_keep^{-1} X_keep^T.

    With return_pivots, also the relative pivots d_k / E_kk (0 where E_kk is
    not positive), which say how far each decision lies from the threshold.
    """
    n = E.shape[0]
    L = np.zeros((n, n))
    keep = []
    piv = np.zeros(n)
    for k in range(n):
        d = E[k, k] - L[k, keep] @ L[k, keep]
        piv[k] = d / E[k, k] if E[k, k] > 0 else 0.0
        if not d > tol * E[k, k]:
            continue
        L[k, k] = np.sqrt(d)
        L[k + 1:, k] = (E[k + 1:, k] - L[k + 1:, keep] @ L[k, keep]) / L[k, k]
        keep.append(k)
    keep = np.array(keep, dtype=np.int64)
    return (keep, piv) if return_pivots else keep


def deletion_margin(piv: np.ndarray, keep: np.ndarray, tol: float = 1e-10) -> float:
    """Factor by which the threshold of gram_keep would have to move before one
    keep / delete decision changes: min over kept columns of piv / tol and
    over deleted ones of tol / piv (inf for a non-positive deleted pivot, and
    inf when there is no column).  Below 100 the decision is left to rounding."""
    m = np.inf
    kept = np.zeros(piv.size, dtype=bool)
    kept[keep] = True
    if kept.any():
        m = min(m, float(np.min(piv[kept])) / tol)
    dp = piv[~kept]
    dp = dp[dp > 0]
    if dp.size:
        m = min(m, tol / float(np.max(dp)))
    return m


@dataclasses.dataclass
class AWGSetup:
    A: sp.csr_matrix
    subs: list
    tau: float
    Ds: list                      # partition of unity diagonals D^s
    cnt: np.ndarray               # M_mu on the pattern of A
    B: sp.csr_matrix
    split: list                   # LocalSplit per subdomain
    Y: list                       # GenEO vectors Y^s (n_s x m_s), M_B-normalised
    geneo_lam: list               # all GenEO eigenvalues per subdomain (ascending)
    R0T: sp.csr_matrix            # n x n0 coarse basis [R^1T Y^1 | ... ]
    E0: np.ndarray
    E0_cho: tuple
    W: np.ndarray                 # n x n_-
    EW: np.ndarray
    EW_cho: tuple
    Vg: np.ndarray                # prolongated strictly negative eigenvectors
    w_info: dict
    E0_keep: np.ndarray = None    # kept coarse vectors (gram_keep); all unless dependent
    EW_keep: np.ndarray = None
    E0_piv: np.ndarray = None     # relative pivots of the deletion (gram_keep)
    EW_piv: np.ndarray = None
    Lg: np.ndarray = None         # |strictly negative eigenvalues|, the columns of V_- (Vg)
    C: np.ndarray = None          # capacitance L_-^{-1} - V_-^T W (H3,inex)
    C_keep: np.ndarray = None
    C_cho: tuple = None
    MB: list = None               # M_B^s = R^s A_+ R^sT per subdomain (GenEO pencil, H^AS_+ local blocks)
    MB_cho: list = None           # their Cholesky factors, formed on first use by H^AS_+
    ash: dict = None              # coarse space and local factors of H^AS_hyb, formed on first use

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def n0(self):
        return self.R0T.shape[1]

    @property
    def n_minus(self):
        return self.W.shape[1]

    @property
    def n0_rank(self):
        return int(self.E0_keep.size)

    @property
    def n_minus_rank(self):
        return int(self.EW_keep.size)

    # -- A_- and A_+ actions (Definition of A_+ and A_-, Section 3.2) -----
    def A_minus_mv(self, X):
        """A_- X = sum_s R^sT A^s_- R^s X (A^s_- applied through its eigenvectors)."""
        X = np.asarray(X)
        out = np.zeros_like(X, dtype=np.float64)
        for idx, sp_ in zip(self.subs, self.split):
            if sp_.nneg == 0:
                continue
            Vm = sp_.V_minus
            out[idx] += -(Vm * sp_.L_minus) @ (Vm.T @ X[idx])
        return out

    def A_plus_mv(self, X):
        """A_+ X = A X + A_- X (item (i) of the A_+ theorem, Section 3.2)."""
        return self.A @ X + self.A_minus_mv(X)

    # -- one-level H^NN (Section 3.3) -----------------------------------
    def H_NN(self, X):
        out = np.zeros_like(X, dtype=np.float64)
        for idx, Ds, sp_ in zip(self.subs, self.Ds, self.split):
            Xs = X[idx]
            Xs = Ds[:, None] * Xs if Xs.ndim == 2 else Ds * Xs
            Ys = sp_.V_plus @ ((sp_.V_plus.T @ Xs) / (sp_.L_plus[:, None] if Xs.ndim == 2 else sp_.L_plus))
            out[idx] += Ds[:, None] * Ys if Xs.ndim == 2 else Ds * Ys
        return out

    # -- coarse solve with E0 -------------------------------------------
    def E0_solve(self, g):
        """E0^+ g on the kept coarse vectors (zero on the deleted ones)."""
        out = np.zeros_like(g, dtype=np.float64)
        out[self.E0_keep] = sla.cho_solve(self.E0_cho, g[self.E0_keep])
        return out

    def EW_solve(self, g):
        out = np.zeros_like(g, dtype=np.float64)
        out[self.EW_keep] = sla.cho_solve(self.EW_cho, g[self.EW_keep])
        return out

    def H2(self, r):
        """H2 = Pi H^NN Pi^T + R0^T E0^{-1} R0 (Theorem for H^NN_hyb, Section 3.4)."""
        u0 = self.E0_solve(self.R0T.T @ r)                    # E0^{-1} R0 r
        t = r - self.A_plus_mv(self.R0T @ u0)                 # Pi^T r
        y = self.H_NN(t)                                      # H^NN Pi^T r
        v = self.E0_solve(self.R0T.T @ self.A_plus_mv(y))     # E0^{-1} R0 A_+ y
        return y - self.R0T @ v + self.R0T @ u0               # Pi y + R0^T E0^{-1} R0 r

    # -- one-level H^AS_+ and its two-level forms (Section 3.4) -----------
    def H_AS_plus(self, X):
        """H^AS_+ X = sum_s R^sT (R^s A_+ R^sT)^{-1} R^s X: exact local solves
        with A_+, no partition of unity (one-level preconditioners for A_+,
        Section 3.3)."""
        if self.MB_cho is None:
            self.MB_cho = [sla.cho_factor(0.5 * (M + M.T), lower=True) for M in self.MB]
        out = np.zeros_like(X, dtype=np.float64)
        for idx, F in zip(self.subs, self.MB_cho):
            out[idx] += sla.cho_solve(F, X[idx])
        return out

    def H2_as_plus_hyb(self, r):
        """H^AS_{+,hyb}(tau_flat) = Pi H^AS_+ Pi^T + R0^T E0^{-1} R0 (Theorem on
        H^AS_{+,hyb/ad}, Section 3.4).  Its coarse space V0_{AS,+}(tau_flat) is
        spanned by the R^sT Y_L(1/tau_flat) of the pencil (D^-1 A^s_+ D^-1,
        R^s A_+ R^sT): with tau_flat = 1/tau it is the coarse space already
        built here, so R0 and E0 are shared."""
        u0 = self.E0_solve(self.R0T.T @ r)
        t = r - self.A_plus_mv(self.R0T @ u0)
        y = self.H_AS_plus(t)
        v = self.E0_solve(self.R0T.T @ self.A_plus_mv(y))
        return y - self.R0T @ v + self.R0T @ u0

    def H2_as_plus_ad(self, r):
        """H^AS_{+,ad}(tau_flat) = H^AS_+ + R0^T E0^{-1} R0 (same theorem and coarse space)."""
        return self.H_AS_plus(r) + self.R0T @ self.E0_solve(self.R0T.T @ r)

    # -- H^AS_hyb(tau_sharp, tau_flat) (Theorem on H^AS_hyb, Section 3.4) --
    def _as_hyb_space(self):
        """Coarse space V0_AS(tau_sharp, tau_flat), tau_sharp = tau and
        tau_flat = 1/tau: per subdomain the columns of
        Y_L(1/tau_flat, D^-1 A^s_+ D^-1, R^s A R^sT) followed by those of
        Y_L(tau_sharp, R^s A R^sT, R^s A_+ R^sT); E0 = R0 A_+ R0^T on it (its
        kept columns as for H^NN_hyb: the union may be dependent)."""
        if self.ash is not None:
            return self.ash
        rows, cols, vals, Ys, chol, m1s = [], [], [], [], [], []
        off = 0
        for s, idx in enumerate(self.subs):
            As = local_block(self.A, idx)
            As = 0.5 * (As + As.T)
            Dinv = 1.0 / self.Ds[s]
            MA = Dinv[:, None] * self.split[s].A_plus() * Dinv[None, :]
            lam1, Y1 = sla.eigh(0.5 * (MA + MA.T), As)
            lam2, Y2 = sla.eigh(As, 0.5 * (self.MB[s] + self.MB[s].T))
            Y = np.concatenate([Y1[:, lam1 < self.tau], Y2[:, lam2 < self.tau]], axis=1)
            Ys.append(Y)
            m1s.append(int(np.count_nonzero(lam1 < self.tau)))
            m = Y.shape[1]
            rows.append(np.repeat(idx, m))
            cols.append(np.tile(np.arange(off, off + m), idx.size))
            vals.append(Y.ravel())
            off += m
            chol.append(sla.cho_factor(As, lower=True))
        R0T = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                            shape=(self.n, off))
        E0 = np.asarray(R0T.T @ self.A_plus_mv(R0T.toarray()))
        E0 = 0.5 * (E0 + E0.T)
        # the union of the two pencils' vectors can be numerically dependent
        # across subdomains with every pivot of E0 well above GRAM_DROP_TOL:
        # its pseudo-inverse deflates the eigenvectors Z of the Jacobi-scaled
        # Es = S^-1 E0 S^-1 below 1e-10 instead,
        #   E0^+ = S^-1 ((Es + Z Z^T)^-1 - Z Z^T) S^-1
        sc = np.sqrt(np.diag(E0))
        Es = E0 / sc[:, None] / sc[None, :]
        lam, V = np.linalg.eigh(Es)
        Z = V[:, lam < 1e-10]
        Ms = Es + Z @ Z.T
        keep = gram_keep(Ms)
        self.ash = dict(Y=Ys, m1=m1s, R0T=R0T, E0=E0, keep=keep, scale=sc, Z=Z,
                        cho=sla.cho_factor(Ms[np.ix_(keep, keep)], lower=True), local=chol)
        return self.ash

    def E0_as_solve(self, g):
        """E0^+ g on the coarse space of H^AS_hyb (deflated pseudo-inverse)."""
        c = self._as_hyb_space()
        h = g / c["scale"] if g.ndim == 1 else g / c["scale"][:, None]
        out = np.zeros_like(h, dtype=np.float64)
        out[c["keep"]] = sla.cho_solve(c["cho"], h[c["keep"]])
        out -= c["Z"] @ (c["Z"].T @ h)
        return out / c["scale"] if g.ndim == 1 else out / c["scale"][:, None]

    def H_AS(self, X):
        """H^AS X = sum_s R^sT (R^s A R^sT)^{-1} R^s X (one-level, Section 3.3)."""
        c = self._as_hyb_space()
        out = np.zeros_like(X, dtype=np.float64)
        for idx, F in zip(self.subs, c["local"]):
            out[idx] += sla.cho_solve(F, X[idx])
        return out

    def H2_as_hyb(self, r):
        """H^AS_hyb(tau_sharp, tau_flat) = Pi_AS H^AS Pi_AS^T + R0^T E0^{-1} R0 on
        V0_AS(tau_sharp, tau_flat), Pi_AS = I - R0^T E0^{-1} R0 A_+."""
        c = self._as_hyb_space()
        R0T = c["R0T"]
        e0 = self.E0_as_solve
        u0 = e0(R0T.T @ r)
        t = r - self.A_plus_mv(R0T @ u0)
        y = self.H_AS(t)
        v = e0(R0T.T @ self.A_plus_mv(y))
        return y - R0T @ v + R0T @ u0

    def h2(self, kind: str):
        """The preconditioner for A_+ named by kind: "nn_hyb" (H^NN_hyb(tau)),
        "asp_hyb" or "asp_ad" (H^AS_{+,hyb/ad}(1/tau)), "as_hyb"
        (H^AS_hyb(tau, 1/tau))."""
        return {"nn_hyb": self.H2, "asp_hyb": self.H2_as_plus_hyb, "asp_ad": self.H2_as_plus_ad,
                "as_hyb": self.H2_as_hyb}[kind]

    def apply(self, r, h2=None):
        """H r with H = H3,ad = H2 + W (W^T A W)^{-1} W^T (Definition, Section 4.3).
        h2: a replacement for H2."""
        z = (h2 or self.H2)(r)
        if self.n_minus:
            z = z + self.W @ self.EW_solve(self.W.T @ r)
        return z

    # -- the other two second-coarse-space preconditioners (Section 4) ----
    def C_solve(self, g):
        """C^+ g for the capacitance C = L_-^{-1} - V_-^T A_+^{-1} V_- (kept columns)."""
        out = np.zeros_like(g, dtype=np.float64)
        out[self.C_keep] = sla.cho_solve(self.C_cho, g[self.C_keep])
        return out

    def apply_inex(self, r, h2=None):
        """H3,inex r = H2 r + A_+^{-1} V_- C^{-1} V_-^T A_+^{-1} r with W = A_+^{-1} V_-
        (Theorem on the AWG preconditioner with inexact coarse space, Section 4.2).
        h2: a replacement for H2 (the pins use the exact A_+^{-1})."""
        z = (h2 or self.H2)(r)
        if self.n_minus:
            z = z + self.W @ self.C_solve(self.W.T @ r)
        return z

    def apply_hyb(self, r, h2=None):
        """H3,hyb r = Pi3 H2 Pi3^T r + W (W^T A W)^{-1} W^T r with
        Pi3 = I - W (W^T A W)^{-1} W^T A (Definition of Pi_3 and H3, Section 4.3):
        t = E_W^{-1} W^T r, y = H2 (r - A W t), z = y - W E_W^{-1} W^T A y + W t."""
        if not self.n_minus:
            return (h2 or self.H2)(r)
        t = self.EW_solve(self.W.T @ r)
        y = (h2 or self.H2)(r - self.A @ (self.W @ t))
        s = self.EW_solve(self.W.T @ (self.A @ y))
        return y + self.W @ (t - s)


def geneo_local(sp_: LocalSplit, Ds: np.ndarray, MB: np.ndarray, tau: float):
    """GenEO modes of subdomain s for H^NN_hyb (Theorem, Section 3.4).

    Pencil M_A = (D^s)^{-1} A^s_+ (D^s)^{-1}, M_B = R^s A_+ R^sT.  All
    M_B-normalised eigenvectors with eigenvalue < tau (strict), ascending
    (Definition of Y_L).
    """
    Dinv = 1.0 / Ds
    MA = Dinv[:, None] * sp_.A_plus() * Dinv[None, :]
    MA = 0.5 * (MA + MA.T)
    MB = 0.5 * (MB + MB.T)
    lam, Y = sla.eigh(MA, MB)          # M_B-orthonormal, ascending
    m = int(np.count_nonzero(lam < tau))
    return Y[:, :m], lam


def local_MB(A: sp.csr_matrix, subs, split, s: int) -> np.ndarray:
    """M_B^s = R^s A_+ R^sT = R^s A R^sT + sum_t (R^s R^tT) A^t_- (R^t R^sT)
    (Definition of A_+, Section 3.2; written as in Remark 4, Section 4.4)."""
    idx = subs[s]
    MB = local_block(A, idx)
    for t, idt in enumerate(subs):
        if split[t].nneg == 0:
            continue
        common, ps, pt = np.intersect1d(idx, idt, assume_unique=True, return_indices=True)
        if common.size == 0:
            continue
        Vt = split[t].V_minus[pt]                       # rows of V^t_- on the common dofs
        MB[np.ix_(ps, ps)] += -(Vt * split[t].L_minus) @ Vt.T
    return MB


W_DIRECT_MAX_N = 100_000     # largest n for which w_solver="auto" factorises A


def setup(A: sp.csr_matrix, subs, tau: float, eps0: float = 1e-12, w_solver: str = "auto",
          w_rtol: float = 1e-13, w_maxit: int = 500, check: bool = True, stop_after: str = None,
          timings: dict = None) -> AWGSetup:
    """Build every ingredient of H3,ad with H2 = H^NN_hyb(tau).

    stop_after="coarse0" returns after E0 and its deletion (no second coarse
    space: W, E_W and C stay empty), for workloads whose W does not fit in
    memory.  timings, when given, receives the wall time of each phase (s)."""
    import time
    tm = timings if timings is not None else {}
    t0 = time.perf_counter()
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    n = A.shape[0]
    subs = [np.asarray(s, dtype=np.int64) for s in subs]
    if not (0.0 < tau < 1.0):
        raise OracleError("tau must lie in (0, 1) for H^NN_hyb")
    if check:
        check_inputs(A, subs)
    Ds = partition_of_unity(n, subs)
    cnt = pair_multiplicity(A, subs)
    B = algebraic_B(A, cnt)
    tm["maps"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    split = [split_local(local_block(B, idx), eps0) for idx in subs]
    tm["split"] = time.perf_counter() - t0
    t0 = time.perf_counter()

    # GenEO coarse space (Theorem for H^NN_hyb, Section 3.4)
    Ys, glam, MBs = [], [], []
    for s in range(len(subs)):
        MB = local_MB(A, subs, split, s)
        Y, lam = geneo_local(split[s], Ds[s], MB, tau)
        Ys.append(Y)
        glam.append(lam)
        MBs.append(MB)
    rows, cols, vals = [], [], []
    off = 0
    for idx, Y in zip(subs, Ys):
        m = Y.shape[1]
        rows.append(np.repeat(idx, m))
        cols.append(np.tile(np.arange(off, off + m), idx.size))
        vals.append(Y.ravel())
        off += m
    R0T = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(n, off))
    tm["geneo"] = time.perf_counter() - t0
    t0 = time.perf_counter()

    st = AWGSetup(A=A, subs=subs, tau=tau, Ds=Ds, cnt=cnt, B=B, split=split, Y=Ys,
                  geneo_lam=glam, R0T=R0T, E0=None, E0_cho=None, W=np.zeros((n, 0)),
                  EW=np.zeros((0, 0)), EW_cho=None, Vg=np.zeros((n, 0)), w_info={}, MB=MBs)
    # E0 = R0 A_+ R0^T (by column blocks of R0^T, which bounds the memory of
    # the dense products) and its Cholesky factor
    E0 = np.empty((off, off))
    R0 = R0T.T.tocsr()
    for c0 in range(0, off, 512):
        E0[:, c0:c0 + 512] = R0 @ st.A_plus_mv(R0T[:, c0:c0 + 512].toarray())
    st.E0 = 0.5 * (E0 + E0.T)
    st.E0_keep, st.E0_piv = gram_keep(st.E0, return_pivots=True)
    st.EW_keep = np.zeros(0, dtype=np.int64)
    st.EW_piv = np.zeros(0)
    try:
        st.E0_cho = sla.cho_factor(st.E0[np.ix_(st.E0_keep, st.E0_keep)], lower=True)
    except np.linalg.LinAlgError as e:
        raise OracleError("E0 is not positive semi-definite") from e
    tm["coarse0"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    if stop_after == "coarse0":
        return st

    # second coarse space W = A_+^{-1} [R^1T V^1_- | ... ] with strictly
    # negative eigenvalues only (Remark 1, Section 4.4)
    cols = []
    for idx, sp_ in zip(subs, split):
        if sp_.nstrict == 0:
            continue
        V = np.zeros((n, sp_.nstrict))
        V[idx] = sp_.V[:, :sp_.nstrict]
        cols.append(V)
    Vg = np.concatenate(cols, axis=1) if cols else np.zeros((n, 0))
    st.Vg = Vg
    if Vg.shape[1]:
        if w_solver == "auto":
            # a sparse LU of A is cheap for the 2D workloads; for the 3D ones its
            # fill makes it impractical, and the oracle takes the paper's own
            # route (Remark 2, Section 4.4): PCG with H2 on every column
            w_solver = "direct" if n <= W_DIRECT_MAX_N else "pcg"
        if w_solver == "direct":
            st.W = solve_A_plus_direct(st, Vg)
            st.w_info = dict(solver="direct")
        else:
            st.W, st.w_info = solve_A_plus_pcg(st, Vg, w_rtol, w_maxit)
        EW = st.W.T @ (A @ st.W)
        st.EW = 0.5 * (EW + EW.T)
        st.EW_keep, st.EW_piv = gram_keep(st.EW, return_pivots=True)
        try:
            st.EW_cho = sla.cho_factor(st.EW[np.ix_(st.EW_keep, st.EW_keep)], lower=True)
        except np.linalg.LinAlgError as e:
            raise OracleError("W^T A W is not positive semi-definite") from e
        # capacitance of the Woodbury form of A^{-1} = (A_+ - V_- L_- V_-^T)^{-1}
        # (Theorem on the AWG preconditioner with inexact coarse space, Section
        # 4.2): C = L_-^{-1} - V_-^T W, with L_- = |strictly negative eigenvalues|
        Lg = np.concatenate([np.abs(sp_.lam[:sp_.nstrict]) for sp_ in split if sp_.nstrict])
        st.Lg = Lg
        C = np.diag(1.0 / Lg) - Vg.T @ st.W
        st.C = 0.5 * (C + C.T)
        st.C_keep = gram_keep(st.C)
        try:
            st.C_cho = sla.cho_factor(st.C[np.ix_(st.C_keep, st.C_keep)], lower=True)
        except np.linalg.LinAlgError as e:
            raise OracleError("the capacitance matrix is not positive semi-definite") from e
    tm["W"] = time.perf_counter() - t0
    return st


def assemble_A_plus(st: AWGSetup) -> sp.csr_matrix:
    """A_+ = sum_s R^sT A^s_+ R^s assembled as a sparse matrix (Definition, Section 3.2)."""
    rows, cols, vals = [], [], []
    for idx, sp_ in zip(st.subs, st.split):
        Ap = sp_.A_plus()
        rows.append(np.repeat(idx, idx.size))
        cols.append(np.tile(idx, idx.size))
        vals.append(Ap.ravel())
    n = st.n
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    M.sum_duplicates()
    return M


def solve_A_plus_direct(st: AWGSetup, RHS: np.ndarray) -> np.ndarray:
    """A_+^{-1} RHS by direct factorisation.

    Small n: dense Cholesky of the assembled A_+.  Otherwise A_+ = A + U C U^T
    with U = [R^sT V^s_-] (strictly negative pairs; zero eigenvalues add
    nothing) and C = |L_-| (Definition of A_-, Section 3.2), and the
    Woodbury identity (Section 4.1) gives
    A_+^{-1} = A^{-1} - A^{-1} U (C^{-1} + U^T A^{-1} U)^{-1} U^T A^{-1}
    on top of a sparse LU factorisation of A.
    """
    if st.n <= 4000:
        Ap = assemble_A_plus(st)
        return sla.cho_solve(sla.cho_factor(Ap.toarray(), lower=True), RHS)
    lu = spla.splu(st.A.tocsc())
    cols, cdiag = [], []
    for idx, sp_ in zip(st.subs, st.split):
        if sp_.nstrict == 0:
            continue
        U = np.zeros((st.n, sp_.nstrict))
        U[idx] = sp_.V[:, :sp_.nstrict]
        cols.append(U)
        cdiag.append(-sp_.lam[:sp_.nstrict])
    X = lu.solve(RHS)
    if not cols:
        return X
    U = np.concatenate(cols, axis=1)
    c = np.concatenate(cdiag)
    AU = lu.solve(U)
    cap = np.diag(1.0 / c) + U.T @ AU
    return X - AU @ np.linalg.solve(cap, U.T @ X)


def solve_A_plus_pcg(st: AWGSetup, RHS: np.ndarray, rtol: float, maxit: int, block: int = 256):
    """A_+^{-1} RHS column by column with PCG preconditioned by H2 (Remark 2,
    Section 4.4); the columns of a block run side by side, each with its own
    recurrence and stopping test."""
    X = np.zeros_like(RHS)
    its = []
    for c0 in range(0, RHS.shape[1], block):
        Bk = RHS[:, c0:c0 + block]
        Xk, it = pcg_multi(st.A_plus_mv, st.H2, Bk, rtol, maxit)
        X[:, c0:c0 + block] = Xk
        its.append(it)
    its = np.concatenate(its)
    return X, dict(solver="pcg", rtol=rtol, iters_max=int(its.max()), iters_mean=float(its.mean()))


def pcg_multi(Amv, Mmv, Bk, rtol, maxit):
    """Independent PCG recurrences for every column of Bk (x0 = 0)."""
    X = np.zeros_like(Bk)
    R = Bk.copy()
    bn = np.linalg.norm(Bk, axis=0)
    bn[bn == 0] = 1.0
    Z = Mmv(R)
    P = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    active = np.ones(Bk.shape[1], dtype=bool)
    its = np.zeros(Bk.shape[1], dtype=np.int64)
    for _ in range(maxit):
        if not active.any():
            break
        a = np.flatnonzero(active)
        Q = Amv(P[:, a])
        pq = np.einsum("ij,ij->j", P[:, a], Q)
        alpha = rz[a] / pq
        X[:, a] += alpha * P[:, a]
        R[:, a] -= alpha * Q
        its[a] += 1
        rn = np.linalg.norm(R[:, a], axis=0) / bn[a]
        done = rn <= rtol
        active[a[done]] = False
        a = np.flatnonzero(active)
        if a.size == 0:
            break
        Za = Mmv(R[:, a])
        rz_new = np.einsum("ij,ij->j", R[:, a], Za)
        beta = rz_new / rz[a]
        rz[a] = rz_new
        P[:, a] = Za + beta * P[:, a]
    return X, its


# ---------------------------------------------------------------------------
# PCG (Saad, Section 9.2, as cited by the paper's introduction)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    res_hist: list            # ||r_k|| / ||b|| for k = 0..iters (recursive residual)
    alphas: list
    betas: list
    rel_res_true: float
    restarts: int = 0         # restarts from the true residual

    def lanczos_extremes(self):
        """Extreme Ritz values of HA from the PCG coefficients (Lanczos tridiagonal)."""
        k = len(self.alphas)
        if k == 0:
            return np.nan, np.nan
        T = np.zeros((k, k))
        for j in range(k):
            T[j, j] = 1.0 / self.alphas[j] + (self.betas[j - 1] / self.alphas[j - 1] if j > 0 else 0.0)
            if j + 1 < k:
                T[j, j + 1] = T[j + 1, j] = np.sqrt(self.betas[j]) / self.alphas[j]
        ev = np.linalg.eigvalsh(T)
        return float(ev[0]), float(ev[-1])


def pcg(A, b, M, tol: float = 1e-8, maxit: int = 1000, norm: str = "unpreconditioned",
        max_restarts: int = 5) -> PCGResult:
    """PCG from x0 = 0; stops at the first k with ||r_k||/||b|| <= tol.

    The textbook recurrence (Saad, Iterative Methods for Sparse Linear
    Systems, Algorithm 9.1).  Reading of the stopping rule (the paper states a
    relative residual tolerance only): when the recursive residual meets tol
    but the true residual b - A x_k does not (rounding drift on
    ill-conditioned A), the recurrence restarts from the true residual
    (at most max_restarts times; iterations keep counting).

    norm="preconditioned" instead tests ||H r_k|| / ||H b|| (the default
    of PETSc's CG, used only to compare iteration counts with the paper's
    tables).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn]
    alphas, betas = [], []
    if hist[0] <= tol:
        return PCGResult(x, 0, True, hist, alphas, betas, hist[0])
    z = M(r)
    zn0 = np.linalg.norm(z)
    p = z.copy()
    rz = r @ z
    k = 0
    converged = False
    restarts = 0
    while k < maxit:
        q = A @ p
        pq = p @ q
        if not pq > 0:
            raise OracleError("p^T A p <= 0: A or H is not SPD")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        k += 1
        if restarts == 0:
            alphas.append(alpha)
        hist.append(np.linalg.norm(r) / bn)
        if norm != "preconditioned" and hist[-1] <= tol:
            rt = b - A @ x
            if np.linalg.norm(rt) / bn <= tol or restarts >= max_restarts or k >= maxit:
                converged = np.linalg.norm(rt) / bn <= tol
                break
            restarts += 1
            r = rt
            z = M(r)
            p = z.copy()
            rz = r @ z
            continue
        z = M(r)
        if norm == "preconditioned" and np.linalg.norm(z) / zn0 <= tol:
            converged = True
            break
        rz_new = r @ z
        beta = rz_new / rz
        if restarts == 0:
            betas.append(beta)
        rz = rz_new
        p = z + beta * p
    true = np.linalg.norm(b - A @ x) / bn
    return PCGResult(x, k, converged, hist, alphas, betas, float(true), restarts)


# ---------------------------------------------------------------------------
# dense helpers for small problems (tests)
# ---------------------------------------------------------------------------
def dense_operator(apply, n: int, block: int = 512) -> np.ndarray:
    """Dense matrix of a linear operator from its action on unit vectors."""
    M = np.zeros((n, n))
    for c0 in range(0, n, block):
        E = np.zeros((n, min(block, n - c0)))
        E[np.arange(c0, c0 + E.shape[1]), np.arange(E.shape[1])] = 1.0
        M[:, c0:c0 + E.shape[1]] = apply(E)
    return M


def spectrum_HA(H: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Eigenvalues of HA for SPD H and A (via the symmetric L^T H L, A = L L^T)."""
    L = np.linalg.cholesky(A)
    S = L.T @ H @ L
    return np.linalg.eigvalsh(0.5 * (S + S.T))


def stats(st: AWGSetup) -> dict:
    return dict(
        n=st.n, N=len(st.subs), sum_ns=int(sum(len(s) for s in st.subs)),
        n_minus=st.n_minus, n0=st.n0,
        k_s=[sp_.nneg for sp_ in st.split], kstrict_s=[sp_.nstrict for sp_ in st.split],
        m_s=[Y.shape[1] for Y in st.Y],
        n0_rank=st.n0_rank, n_minus_rank=st.n_minus_rank,
        e0_margin=deletion_margin(st.E0_piv, st.E0_keep),
        ew_margin=deletion_margin(st.EW_piv, st.EW_keep),
    )
