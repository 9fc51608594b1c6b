"""Overlapping subdomain index sets for the synthetic problems.

Input generation only.  A subdomain is built as a set of grid nodes (a box,
or a recursive-coordinate-bisection part) extended by ``delta`` layers of
graph neighbours in the node graph of A; all dofs of a node go together.
With delta >= 1 every nonzero A_ij has both i and j in some subdomain, which
is the minimal-overlap assumption of the paper (Section 2.1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import Problem


def node_graph_of_A(prob: Problem):
    """Node-level adjacency of A's pattern over the kept nodes.

    Returns (G, kept_nodes): G is indexed by compressed node ids, kept_nodes
    maps a compressed id back to the grid node id.
    """
    A = prob.A.tocoo()
    kept_nodes = np.unique(prob.node_of_dof)
    comp = np.full(prob.node_xyz.shape[0], -1, dtype=np.int64)
    comp[kept_nodes] = np.arange(kept_nodes.size)
    r = comp[prob.node_of_dof[A.row]]
    c = comp[prob.node_of_dof[A.col]]
    m = kept_nodes.size
    G = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(m, m))
    G.data[:] = 1.0
    return G, kept_nodes


def extend_by_layers(G: sp.csr_matrix, parts: np.ndarray, nparts: int, delta: int):
    """Node sets: each part grown by ``delta`` hops in graph G.  Returns list of sorted node arrays."""
    out = []
    for p in range(nparts):
        x = (parts == p).astype(np.float64)
        for _ in range(delta):
            x = np.minimum(1.0, x + G @ x)
        out.append(np.flatnonzero(x > 0))
    return out


def nodes_to_dofs(prob: Problem, kept_nodes: np.ndarray, node_sets):
    """Map compressed node sets to sorted dof index arrays (int64)."""
    dpn = prob.dof_per_node
    # dofs are ordered node-major with dpn consecutive dofs per kept node
    first = np.zeros(prob.node_xyz.shape[0], dtype=np.int64) - 1
    uniq, start = np.unique(prob.node_of_dof, return_index=True)
    first[uniq] = start
    subs = []
    for ns in node_sets:
        gnodes = kept_nodes[ns]
        d = (first[gnodes][:, None] + np.arange(dpn)[None, :]).ravel()
        subs.append(np.sort(d).astype(np.int64))
    return subs


def box_parts(coords: np.ndarray, counts) -> np.ndarray:
    """Assign points to a grid of boxes: equal-count slabs along each axis.

    coords: (m, dim) node coordinates; counts: boxes per axis.  Along each
    axis the distinct coordinate values are split into ``counts[d]``
    contiguous groups of (nearly) equal size (numpy.array_split).
    """
    m, dim = coords.shape
    part = np.zeros(m, dtype=np.int64)
    mult = 1
    for d in range(dim):
        vals = np.unique(np.round(coords[:, d], 12))
        groups = np.array_split(vals, counts[d])
        lab = np.zeros(m, dtype=np.int64)
        cd = np.round(coords[:, d], 12)
        for gi, g in enumerate(groups):
            lab[(cd >= g[0]) & (cd <= g[-1])] = gi
        part += lab * mult
        mult *= counts[d]
    return part


def rcb_parts(coords: np.ndarray, nparts: int, rng: np.random.Generator,
              weight_range=(1.0, 3.0)) -> np.ndarray:
    """Seeded recursive coordinate bisection into ``nparts`` uneven parts.

    Each leaf gets a random target weight U(weight_range); a set is split on
    its longer axis at the quantile matching the weight of its two halves of
    the leaf list, so part sizes vary by up to the weight ratio.
    """
    w = rng.uniform(weight_range[0], weight_range[1], size=nparts)
    part = np.zeros(coords.shape[0], dtype=np.int64)

    def rec(idx, leaves):
        if len(leaves) == 1:
            part[idx] = leaves[0]
            return
        half = len(leaves) // 2
        la, lb = leaves[:half], leaves[half:]
        frac = w[la].sum() / w[leaves].sum()
        c = coords[idx]
        ext = c.max(0) - c.min(0)
        ax = int(np.argmax(ext))
        order = np.argsort(c[:, ax], kind="stable")
        k = int(round(frac * idx.size))
        k = min(max(k, 1), idx.size - 1)
        rec(idx[order[:k]], la)
        rec(idx[order[k:]], lb)

    rec(np.arange(coords.shape[0]), list(range(nparts)))
    return part


def make_subdomains(prob: Problem, parts_of_kept_nodes: np.ndarray, nparts: int, delta: int):
    G, kept_nodes = node_graph_of_A(prob)
    node_sets = extend_by_layers(G, parts_of_kept_nodes, nparts, delta)
    return nodes_to_dofs(prob, kept_nodes, node_sets)


def box_subdomains(prob: Problem, counts, delta: int):
    G, kept_nodes = node_graph_of_A(prob)
    parts = box_parts(prob.node_xyz[kept_nodes], counts)
    node_sets = extend_by_layers(G, parts, int(np.prod(counts)), delta)
    return nodes_to_dofs(prob, kept_nodes, node_sets)


def closed_box_subdomains(prob: Problem, lo_list, hi_list, tol=1e-9):
    """Subdomains = dofs of kept nodes inside closed boxes [lo, hi] (no extension).

    Neighbouring boxes then share exactly the nodes on their common face,
    which is the interface-only overlap of the paper's experiments
    (Section 5).
    """
    kept_nodes = np.unique(prob.node_of_dof)
    xyz = prob.node_xyz[kept_nodes]
    sets = []
    for lo, hi in zip(lo_list, hi_list):
        inside = np.all((xyz >= np.asarray(lo) - tol) & (xyz <= np.asarray(hi) + tol), axis=1)
        sets.append(np.flatnonzero(inside))
    return nodes_to_dofs(prob, kept_nodes, sets)
