"""Seeded synthetic sparse SPD systems shaped like the paper's workloads.

Input generation only: this module assembles matrices and right-hand sides
(finite differences and Q1 finite elements) and holds none of the AWG
method's arithmetic.  Both the FP64 oracle tests and the GPU path consume
what it produces.

Conventions
-----------
* Matrices are returned as ``scipy.sparse.csr_matrix`` (float64), full
  symmetric storage, sorted column indices, Dirichlet dofs eliminated.
* ``node_of_dof`` maps every kept dof to its grid node id; ``dof_per_node``
  is 1 (diffusion) or 2/3 (elasticity, dofs of a node are consecutive).
* Node ids are ``ix + nx1 * iy (+ nx1 * ny1 * iz)`` over the full grid of
  ``nx1 = nx + 1`` nodes per row, before Dirichlet elimination.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Problem:
    A: sp.csr_matrix
    b: np.ndarray
    node_of_dof: np.ndarray      # (n,) int64 node id of each kept dof
    dof_per_node: int
    node_adj: sp.csr_matrix      # node graph over ALL grid nodes (incl. Dirichlet)
    node_xyz: np.ndarray         # (nnodes, dim) coordinates of every grid node
    kept_node: np.ndarray        # (nnodes,) bool, False on Dirichlet nodes
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]


# ---------------------------------------------------------------------------
# reference-element quadrature (tensor Gauss-Legendre, 2 points per axis)
# ---------------------------------------------------------------------------
_G = np.array([-1.0, 1.0]) / np.sqrt(3.0)


def _q1_shape_grads(dim: int):
    """Gauss points and gradients of the Q1 shape functions on [-1,1]^dim.

    Local node order is lexicographic with x fastest:
    2D: (0,0),(1,0),(0,1),(1,1); 3D: same plus z as slowest index.
    Returns (weights (ng,), N (ng, nloc), dN (ng, nloc, dim)).
    """
    corners = np.array(np.meshgrid(*([[-1.0, 1.0]] * dim), indexing="ij"))
    corners = corners.reshape(dim, -1).T[:, ::-1]  # x fastest
    pts = np.array(np.meshgrid(*([_G] * dim), indexing="ij")).reshape(dim, -1).T
    ng, nloc = pts.shape[0], corners.shape[0]
    N = np.ones((ng, nloc))
    dN = np.ones((ng, nloc, dim))
    for a in range(nloc):
        fac = 0.5 * (1.0 + corners[a][None, :] * pts)          # (ng, dim)
        N[:, a] = np.prod(fac, axis=1)
        for d in range(dim):
            g = np.prod(np.delete(fac, d, axis=1), axis=1) * 0.5 * corners[a][d]
            dN[:, a, d] = g
    w = np.ones(ng)
    return w, N, dN


def q1_laplace_element(h: float, dim: int) -> np.ndarray:
    """Element matrix of int grad(phi_a).grad(phi_b) on a cube of side h."""
    w, _, dN = _q1_shape_grads(dim)
    jac = h / 2.0
    G = dN / jac                                   # physical gradients
    K = np.einsum("g,gad,gbd->ab", w, G, G) * jac ** dim
    return K


def q1_mass_lumped(h: float, dim: int) -> np.ndarray:
    """int phi_a over the element (all equal to h^dim / 2^dim)."""
    w, N, _ = _q1_shape_grads(dim)
    return np.einsum("g,ga->a", w, N) * (h / 2.0) ** dim


def q1_elasticity_element(h: float, dim: int, E: float, nu: float) -> np.ndarray:
    """Element matrix of int 2 mu eps(u):eps(v) + lam div u div v (isotropic).

    Dofs are node-major: (node a, component c) -> a * dim + c.
    Lame coefficients: mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu)(1 - 2 nu)).
    """
    w, _, dN = _q1_shape_grads(dim)
    jac = h / 2.0
    G = dN / jac
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    nloc = G.shape[1]
    K = np.zeros((nloc * dim, nloc * dim))
    for g in range(G.shape[0]):
        # strain of the basis function (a, c): eps_ij = 0.5 (d_j u_i + d_i u_j)
        # with u = e_c phi_a.  Bilinear form evaluated directly.
        for a in range(nloc):
            for c in range(dim):
                for bb in range(nloc):
                    for e in range(dim):
                        ga, gb = G[g, a], G[g, bb]
                        # 2 mu eps(phi_a e_c) : eps(phi_b e_e)
                        val = mu * (ga @ gb if c == e else 0.0) + mu * ga[e] * gb[c]
                        val += lam * ga[c] * gb[e]
                        K[a * dim + c, bb * dim + e] += w[g] * val
    return K * jac ** dim


# ---------------------------------------------------------------------------
# structured grids
# ---------------------------------------------------------------------------
def _grid_elements(shape_cells):
    """Connectivity (ne, 2^dim) of a structured cell grid, local order x fastest."""
    dim = len(shape_cells)
    ncell = np.array(shape_cells)
    nn = ncell + 1
    idx = np.indices(shape_cells).reshape(dim, -1)        # cell lower corners
    strides = np.cumprod(np.concatenate([[1], nn[:-1]]))
    base = (idx * strides[:, None]).sum(0)
    offs = []
    for corner in np.ndindex(*([2] * dim)):
        corner = corner[::-1]                              # x fastest
        offs.append(int(np.dot(corner, strides)))
    return base[:, None] + np.array(offs)[None, :]


def _node_coords(shape_cells, h):
    nn = [c + 1 for c in shape_cells]
    grids = np.meshgrid(*[np.arange(m) * h for m in nn], indexing="ij")
    # flatten with x fastest
    return np.stack([g.transpose(*range(len(nn) - 1, -1, -1)).ravel() for g in grids], axis=1)


def _node_graph_from_elements(conn, nnodes):
    ne, nloc = conn.shape
    rows = np.repeat(conn, nloc, axis=1).ravel()
    cols = np.tile(conn, (1, nloc)).ravel()
    G = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(nnodes, nnodes))
    G.data[:] = 1.0
    return G


def _assemble(conn, Ke_stack, dpn, nnodes, kept_node):
    """Assemble element matrices (ne, nd, nd) and eliminate Dirichlet dofs."""
    ne, nloc = conn.shape
    nd = nloc * dpn
    gdof = (conn[:, :, None] * dpn + np.arange(dpn)[None, None, :]).reshape(ne, nd)
    rows = np.repeat(gdof, nd, axis=1).ravel()
    cols = np.tile(gdof, (1, nd)).ravel()
    ntot = nnodes * dpn
    A = sp.csr_matrix((Ke_stack.ravel(), (rows, cols)), shape=(ntot, ntot))
    keep_dof = np.repeat(kept_node, dpn)
    kept = np.flatnonzero(keep_dof)
    A = A[kept][:, kept].tocsr()
    A.sum_duplicates()
    A = ((A + A.T) * 0.5).tocsr()      # bitwise symmetric (fp addition commutes)
    A.sort_indices()
    A.eliminate_zeros()
    return A, kept


def q1_diffusion(shape_cells, h, kcell, dirichlet, rhs="ones", name=""):
    """Q1 FEM for -div(k grad u) = f on a structured grid of cells.

    kcell: (ncells,) coefficient per cell in the connectivity order.
    dirichlet: function (node_xyz) -> bool mask of Dirichlet nodes.
    rhs: "ones" (b_i = 1) or "load" (b = int phi_i, f = 1).
    """
    dim = len(shape_cells)
    conn = _grid_elements(shape_cells)
    xyz = _node_coords(shape_cells, h)
    nnodes = xyz.shape[0]
    Kref = q1_laplace_element(h, dim)
    Ke = kcell[:, None, None] * Kref[None]
    kept_node = ~dirichlet(xyz)
    A, kept = _assemble(conn, Ke, 1, nnodes, kept_node)
    if rhs == "ones":
        b = np.ones(A.shape[0])
    else:
        m = q1_mass_lumped(h, dim)
        full = np.zeros(nnodes)
        np.add.at(full, conn.ravel(), np.tile(m, conn.shape[0]))
        b = full[kept]
    return Problem(A=A, b=b, node_of_dof=kept.astype(np.int64), dof_per_node=1,
                   node_adj=_node_graph_from_elements(conn, nnodes), node_xyz=xyz,
                   kept_node=kept_node, name=name)


def q1_elasticity(shape_cells, h, Ecell, nu, body_force, dirichlet, name=""):
    """Q1 FEM for isotropic linear elasticity (plane strain in 2D)."""
    dim = len(shape_cells)
    conn = _grid_elements(shape_cells)
    xyz = _node_coords(shape_cells, h)
    nnodes = xyz.shape[0]
    Kref = q1_elasticity_element(h, dim, 1.0, nu)   # linear in E
    Ke = Ecell[:, None, None] * Kref[None]
    kept_node = ~dirichlet(xyz)
    A, kept = _assemble(conn, Ke, dim, nnodes, kept_node)
    m = q1_mass_lumped(h, dim)
    full = np.zeros((nnodes, dim))
    for c in range(dim):
        np.add.at(full[:, c], conn.ravel(), np.tile(m * body_force[c], conn.shape[0]))
    b = full.ravel()[kept]
    return Problem(A=A, b=b, node_of_dof=(kept // dim).astype(np.int64), dof_per_node=dim,
                   node_adj=_node_graph_from_elements(conn, nnodes), node_xyz=xyz,
                   kept_node=kept_node, name=name)


def fd5_diffusion(nint, kcell, name=""):
    """5-point finite differences for -div(k grad u) = 1 on (0,1)^2.

    nint x nint interior nodes, h = 1/(nint+1), homogeneous Dirichlet on the
    whole boundary.  kcell is ((nint+1), (nint+1)) indexed [cx, cy] by the
    lower-left corner of each cell.  The coefficient on the edge between two
    neighbouring nodes is the arithmetic mean of the two cells sharing that
    edge.  The equation is scaled by h^2, so b_i = h^2.
    """
    m = nint
    h = 1.0 / (m + 1)
    N = m + 2                                     # nodes per row incl. boundary
    nid = lambda ix, iy: ix + N * iy              # noqa: E731
    rows, cols, vals = [], [], []
    diag = np.zeros(N * N)
    for iy in range(1, m + 1):
        for ix in range(0, m + 1):                # horizontal edge (ix,iy)-(ix+1,iy)
            kf = 0.5 * (kcell[ix, iy - 1] + kcell[ix, iy])
            a, bnode = nid(ix, iy), nid(ix + 1, iy)
            diag[a] += kf
            diag[bnode] += kf
            rows += [a, bnode]
            cols += [bnode, a]
            vals += [-kf, -kf]
    for ix in range(1, m + 1):
        for iy in range(0, m + 1):                # vertical edge (ix,iy)-(ix,iy+1)
            kf = 0.5 * (kcell[ix - 1, iy] + kcell[ix, iy])
            a, bnode = nid(ix, iy), nid(ix, iy + 1)
            diag[a] += kf
            diag[bnode] += kf
            rows += [a, bnode]
            cols += [bnode, a]
            vals += [-kf, -kf]
    nn = N * N
    rows = np.array(rows + list(range(nn)))
    cols = np.array(cols + list(range(nn)))
    vals = np.array(vals + list(diag))
    Af = sp.csr_matrix((vals, (rows, cols)), shape=(nn, nn))
    ixs, iys = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    kept_node = ((ixs >= 1) & (ixs <= m) & (iys >= 1) & (iys <= m)).ravel()
    kept = np.flatnonzero(kept_node)
    A = Af[kept][:, kept].tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.eliminate_zeros()
    b = np.full(A.shape[0], h * h)
    adj = (abs(Af) > 0).astype(np.float64).tocsr()
    xyz = np.stack([ixs.ravel() * h, iys.ravel() * h], axis=1)
    return Problem(A=A, b=b, node_of_dof=kept.astype(np.int64), dof_per_node=1,
                   node_adj=adj, node_xyz=xyz, kept_node=kept_node, name=name)
