"""Named synthetic workloads (matrix, right-hand side, subdomains, tau).

Input generation only.  Every random draw uses
``numpy.random.default_rng(seed)``.  The recipes are the ones stated in the
design notes of this repository:

* ``fd5_32``      2D -div(k grad u) = 1, 5-point FD, 32x32 interior nodes,
                  k = 1e4 on a cell with probability 0.2 else 1 (seed 0),
                  4x4 node boxes, overlap 1, tau = 0.1, b = h^2.
* ``q1_2d``       2D Q1 diffusion on an m x m cell grid of [0,1]^2, Dirichlet
                  on x = 0, log10 k ~ N(0, 1.5^2) per cell plus 8 horizontal
                  channels k = 1e5 centred at y = (c + 1/2)/8, b = 1,
                  8x8 node boxes with overlap 2 (256x256 is the bench
                  workload) or seeded uneven RCB parts (512x512).
* ``elast3d``     3D Q1 linear elasticity, nu = 0.3, E = 1 with seeded
                  spherical inclusions E = 1e5 filling >= 10 % of cells.
* ``diff3d_grf``  3D Q1 diffusion, log10 k = 1.5 * Gaussian random field.
* ``paper_x0``    the paper's 2D plane-strain elasticity test (Section 5):
                  [0,3]^2, h = 1/21, 9 unit-square subdomains overlapping
                  only on interfaces, layered E.
* ``paper_long``  the paper's long domain [0,N]x[0,1], h = 1/14 (Section 5).
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import fem
from . import partition as part


@dataclasses.dataclass
class Workload:
    prob: fem.Problem
    subs: list            # list of sorted int64 dof index arrays
    tau: float
    tol: float
    name: str
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def A(self):
        return self.prob.A

    @property
    def b(self):
        return self.prob.b

    @property
    def coords(self):
        """(n, dim) coordinates of the node of every dof."""
        return self.prob.node_xyz[self.prob.node_of_dof]


def cell_centroids(shape_cells, h):
    """Centroids of the cells in the element order used by the assemblers."""
    idx = np.indices(shape_cells).reshape(len(shape_cells), -1).T
    return (idx + 0.5) * h


# ---------------------------------------------------------------------------
def fd5_32(seed: int = 0, nint: int = 32, boxes=(4, 4), delta: int = 1, tau: float = 0.1):
    rng = np.random.default_rng(seed)
    u = rng.random((nint + 1, nint + 1))
    kcell = np.where(u < 0.2, 1e4, 1.0)
    prob = fem.fd5_diffusion(nint, kcell, name=f"fd5_{nint}")
    subs = part.box_subdomains(prob, boxes, delta)
    return Workload(prob, subs, tau, 1e-8, f"fd5_{nint}x{nint}_box{boxes[0]}x{boxes[1]}_d{delta}",
                    dict(seed=seed))


def _channels_2d(m, thick):
    rows = []
    for c in range(8):
        centre = (c + 0.5) / 8.0 * m                  # in cells
        lo = int(round(centre - thick / 2.0))
        rows += list(range(lo, lo + thick))
    return np.array(rows)


def q1_2d(m: int = 256, seed: int = 1, partition: str = "box", boxes=(8, 8), nparts: int = 256,
          part_seed: int = 3, delta: int = 2, tau: float = 0.1, thick=None):
    """2D Q1 diffusion; coefficient law and channels as in the module docstring."""
    h = 1.0 / m
    rng = np.random.default_rng(seed)
    logk = rng.normal(0.0, 1.5, size=(m, m))          # indexed [cx, cy]
    thick = thick if thick is not None else max(2, m // 128)
    logk[:, _channels_2d(m, thick)] = 5.0
    kcell = (10.0 ** logk).ravel()
    prob = fem.q1_diffusion((m, m), h, kcell, lambda xyz: xyz[:, 0] < 0.5 * h,
                            rhs="ones", name=f"q1_2d_{m}")
    if partition == "box":
        subs = part.box_subdomains(prob, boxes, delta)
        pname = f"box{boxes[0]}x{boxes[1]}"
    else:
        G, kept_nodes = part.node_graph_of_A(prob)
        parts = part.rcb_parts(prob.node_xyz[kept_nodes], nparts, np.random.default_rng(part_seed))
        subs = part.nodes_to_dofs(prob, kept_nodes, part.extend_by_layers(G, parts, nparts, delta))
        pname = f"rcb{nparts}"
    return Workload(prob, subs, tau, 1e-8, f"q1_2d_{m}x{m}_{pname}_d{delta}",
                    dict(seed=seed, part_seed=part_seed))


def spheres_3d(m: int, rng: np.random.Generator, fill: float = 0.10, rmin=2.0, rmax=4.0):
    """Boolean mask over cells (C order [cx,cy,cz]) covered by random balls."""
    cen = cell_centroids((m, m, m), 1.0)                # in cell units
    inside = np.zeros(cen.shape[0], dtype=bool)
    while inside.mean() < fill:
        c = rng.uniform(0.0, m, size=3)
        r = rng.uniform(rmin, rmax)
        inside |= ((cen - c) ** 2).sum(1) <= r * r
    return inside


def elast3d(m: int = 40, seed: int = 4, boxes=(8, 8, 8), delta: int = 1, tau: float = 0.05,
            nu: float = 0.3):
    h = 1.0 / m
    rng = np.random.default_rng(seed)
    hard = spheres_3d(m, rng)
    Ecell = np.where(hard, 1e5, 1.0)
    prob = fem.q1_elasticity((m, m, m), h, Ecell, nu, (0.0, 0.0, -1.0),
                             lambda xyz: xyz[:, 0] < 0.5 * h, name=f"elast3d_{m}")
    subs = part.box_subdomains(prob, boxes, delta)
    return Workload(prob, subs, tau, 1e-8, f"elast3d_{m}^3_box{boxes[0]}^3_d{delta}", dict(seed=seed))


def grf_3d(m: int, rng: np.random.Generator, ell_range=(4.0, 16.0)):
    """Unit-variance Gaussian random field on m^3 cells, Gaussian covariance.

    White noise is filtered in Fourier space by exp(-(k ell)^2 / 4) (the
    square root of a Gaussian spectral density with correlation length ell
    cells) and normalised to unit sample variance.
    """
    ell = rng.uniform(*ell_range)
    w = rng.standard_normal((m, m, m))
    f = np.fft.fftfreq(m) * 2.0 * np.pi
    kx, ky, kz = np.meshgrid(f, f, f, indexing="ij")
    filt = np.exp(-(kx ** 2 + ky ** 2 + kz ** 2) * ell * ell / 4.0)
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g = (g - g.mean()) / g.std()
    return g, ell


def diff3d_grf(m_cells: int = 65, seed: int = 1000, boxes=(8, 8, 8), delta: int = 1,
               tau: float = 0.1):
    h = 1.0 / m_cells
    rng = np.random.default_rng(seed)
    g, ell = grf_3d(m_cells, rng)
    kcell = (10.0 ** (1.5 * g)).ravel()
    def dirichlet(xyz):
        return np.any((xyz < 0.5 * h) | (xyz > 1.0 - 0.5 * h), axis=1)
    prob = fem.q1_diffusion((m_cells,) * 3, h, kcell, dirichlet, rhs="ones",
                            name=f"diff3d_{m_cells}")
    subs = part.box_subdomains(prob, boxes, delta)
    return Workload(prob, subs, tau, 1e-8, f"diff3d_grf_{m_cells}^3_box{boxes[0]}^3_d{delta}",
                    dict(seed=seed, ell=ell))


# ---------------------------------------------------------------------------
# the paper's own test problems (Section 5)
# ---------------------------------------------------------------------------
def _layer_E(ycent, intervals, E1, E2, periodic=True):
    frac = ycent - np.floor(ycent) if periodic else ycent
    hard = np.zeros(ycent.shape, dtype=bool)
    for lo, hi in intervals:
        hard |= (frac >= lo) & (frac <= hi)
    return np.where(hard, E1, E2)


SIX_LAYERS = [(1 / 7, 2 / 7), (3 / 7, 4 / 7)]
NINE_LAYERS = [(1 / 7, 2 / 7), (3 / 7, 4 / 7), (5 / 7, 6 / 7)]
THREE_LAYERS = [(1 / 7, 2 / 7)]


def paper_x0(E1: float = 1e11, E2: float = 1e7, nu: float = 0.3, layers=SIX_LAYERS,
             tau: float = 0.1, hinv: int = 21, L: int = 3):
    """Plane-strain Q1 elasticity on [0,L]^2, Dirichlet on x = 0, g = (0,-9.81).

    E is E1 on a cell whose centroid y satisfies y - floor(y) in one of the
    ``layers`` intervals, else E2; N = L^2 unit-square subdomains sharing
    only their interface nodes.
    """
    h = 1.0 / hinv
    m = L * hinv
    cen = cell_centroids((m, m), h)
    Ecell = _layer_E(cen[:, 1], layers, E1, E2)
    prob = fem.q1_elasticity((m, m), h, Ecell, nu, (0.0, -9.81),
                             lambda xyz: xyz[:, 0] < 0.5 * h, name="paper_x0")
    lo, hi = [], []
    for by in range(L):
        for bx in range(L):
            lo.append((bx, by))
            hi.append((bx + 1, by + 1))
    subs = part.closed_box_subdomains(prob, lo, hi)
    return Workload(prob, subs, tau, 1e-10, "paper_x0", dict(E1=E1, E2=E2, nu=nu))


def paper_x0_refined(hinv: int, per_unit: int, E1: float = 1e11, E2: float = 1e7, nu: float = 0.3,
                     layers=SIX_LAYERS, tau: float = 0.1, L: int = 3):
    """The problem of paper_x0 on a finer mesh (h = 1/hinv) with every unit
    square cut into per_unit x per_unit box subdomains (N = (L per_unit)^2)
    sharing only their interface nodes, so the subdomain size stays that of
    the paper's mesh when hinv = 21 per_unit."""
    h = 1.0 / hinv
    m = L * hinv
    cen = cell_centroids((m, m), h)
    Ecell = _layer_E(cen[:, 1], layers, E1, E2)
    prob = fem.q1_elasticity((m, m), h, Ecell, nu, (0.0, -9.81),
                             lambda xyz: xyz[:, 0] < 0.5 * h, name=f"paper_x0_h{hinv}_b{per_unit}")
    lo, hi = [], []
    d = 1.0 / per_unit
    for by in range(L * per_unit):
        for bx in range(L * per_unit):
            lo.append((bx * d, by * d))
            hi.append(((bx + 1) * d, (by + 1) * d))
    subs = part.closed_box_subdomains(prob, lo, hi)
    return Workload(prob, subs, tau, 1e-10, f"paper_x0_h{hinv}_b{per_unit}", dict(E1=E1, E2=E2, nu=nu))


def paper_long(N: int, tau: float = 0.1, hinv: int = 14, E1: float = 1e11, E2: float = 1e7,
               nu: float = 0.3):
    """Long domain [0,N]x[0,1] with two hard layers, h = 1/14 (Section 5)."""
    h = 1.0 / hinv
    shape = (N * hinv, hinv)
    cen = cell_centroids(shape, h)
    Ecell = _layer_E(cen[:, 1], SIX_LAYERS, E1, E2, periodic=False)
    prob = fem.q1_elasticity(shape, h, Ecell, nu, (0.0, -9.81),
                             lambda xyz: xyz[:, 0] < 0.5 * h, name=f"paper_long_{N}")
    lo = [(s, 0) for s in range(N)]
    hi = [(s + 1, 1) for s in range(N)]
    subs = part.closed_box_subdomains(prob, lo, hi)
    return Workload(prob, subs, tau, 1e-10, f"paper_long_{N}", dict(N=N))


def by_name(name: str, **kw) -> Workload:
    table = {
        "fd5_32": fd5_32,
        "q1_2d": q1_2d,
        "elast3d": elast3d,
        "diff3d_grf": diff3d_grf,
        "paper_x0": paper_x0,
        "paper_long": paper_long,
    }
    return table[name](**kw)
