"""Seeded problem instances: matrix, hierarchy and right-hand sides.

Random numbers come from NumPy's PCG64 (``numpy.random.default_rng(seed)``) in
a fixed draw order: element coefficients first, then right-hand sides, then
any further targets.

Instances
---------
* ``config_problem("poisson12")`` -- Poisson on 12^3 Q1 hexahedra, 2x2x2 box
  sub-domains (octree of height 1), f ~ U[-1,1] per free dof.
* ``config_problem("diffusion64")`` -- -div(k grad u) = f on 64^3 Q1 hexahedra,
  k_e = exp(z_e), z_e ~ N(0,1) per element, 4x4x4 box sub-domains (octree of
  height 2: two interface levels below three RSD recursion levels), f ~ U[-1,1].
* ``config_problem("adjoint32")`` -- 32^3, k_e = exp(theta_e), theta_e ~ N(0, 0.5^2),
  octree of height 2; b ~ U[-1,1] and a target x_t ~ U[-1,1].
* ``diffusion_problem(ne, height, ...)`` -- any size, for parity cases.
* ``skew_diffusion_problem(ne, height, ...)`` -- a non-symmetric K on the same
  pattern (Poisson plus a random antisymmetric part), for pins of the general path.
* ``strip_problem(N, P, ...)`` -- the paper's 2-D strip workloads (Section 4):
  P sub-domains of N x N nodes in a binary tree, manufactured right-hand side
  b = K x_true with x_true ~ U[-1,1].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .fem import (assemble_diffusion_3d, assemble_elasticity_3d, assemble_strip_2d, fe_map_grid,
                  laplace_element)
from .hierarchy import build_box_tree, dof_node_map


@dataclass
class Problem:
    name: str
    K: sp.csr_matrix
    parent: np.ndarray        # int32[T]
    dof_node: np.ndarray      # int32[n]
    b: np.ndarray             # float64[n, nrhs]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.K.shape[0]

    def csr_arrays(self):
        """(row_ptr int64[n+1], col_idx int32[nnz], values float64[nnz])."""
        K = self.K
        return (K.indptr.astype(np.int64), K.indices.astype(np.int32),
                K.data.astype(np.float64))


def diffusion_problem(ne: int, height: int, sigma: float = 0.0, seed: int = 0,
                      nrhs: int = 1, name: str | None = None, cut_fn=None,
                      tree: str = "octree") -> Problem:
    """-div(k grad u) = f on ne^3 Q1 hexahedra with a cut-plane tree of the given height:
    tree = "octree" cuts every box along all three axes, tree = "binary" along one axis
    per depth (x, y, z, x, ...), which gives deeper trees on small meshes.

    sigma = 0 gives Poisson (k = 1, no coefficient draw); otherwise
    k_e = exp(sigma * z_e) with z_e ~ N(0, 1) drawn first.  f ~ U[-1,1] per free
    dof, nrhs columns, drawn after the coefficients.
    """
    rng = np.random.default_rng(seed)
    k = None
    theta = np.zeros(ne ** 3)
    if sigma > 0.0:
        theta = sigma * rng.standard_normal(ne ** 3)
        k = np.exp(theta)
    sysm = assemble_diffusion_3d(ne, k)
    if tree not in ("octree", "binary"):
        raise ValueError(tree)
    axes = None if tree == "octree" else (lambda d: (d % 3,))
    box = build_box_tree(sysm.shape_nodes, height, axes_per_level=axes, cut_fn=cut_fn)
    dof_node = dof_node_map(box, sysm.free_ijk, 1)
    b = rng.uniform(-1.0, 1.0, size=(sysm.K.shape[0], nrhs))
    return Problem(name or f"diffusion{ne}_h{height}", sysm.K, box.parent, dof_node, b,
                   meta=dict(ne=ne, height=height, sigma=sigma, seed=seed, k_elem=k,
                             theta=theta, free_ijk=sysm.free_ijk, tree=box))


def diffusion_fe_map(p: Problem) -> dict:
    """Coefficient map of a diffusion problem: K = sum_e exp(theta_e) h K_ref."""
    ne = p.meta["ne"]
    return fe_map_grid((ne, ne, ne), (1.0 / ne) * laplace_element(3), p.K)


def config_problem(name: str, seed: int = 0, nrhs: int = 1) -> Problem:
    if name == "poisson12":
        return diffusion_problem(12, 1, 0.0, seed, nrhs, name)
    if name == "diffusion64":
        return diffusion_problem(64, 2, 1.0, seed, nrhs, name)
    if name == "elasticity48":
        return elasticity_problem(48, 3, seed, 8 if nrhs == 1 else nrhs, name)
    if name == "poisson256":
        # 256^3 Poisson, octree of height 5: 32,768 sub-domains of 8^3 elements (343
        # interior dofs), 16 right-hand sides ~ U[-1, 1]
        return diffusion_problem(256, 5, 0.0, seed, 16 if nrhs == 1 else nrhs, name)
    if name == "adjoint32":
        p = diffusion_problem(32, 2, 0.5, seed, nrhs, name)
        # draw order continues after b: the adjoint target
        rng = np.random.default_rng(seed)
        rng.standard_normal(32 ** 3)
        rng.uniform(-1.0, 1.0, size=(p.n, nrhs))
        p.meta["x_target"] = rng.uniform(-1.0, 1.0, size=p.n)
        return p
    raise KeyError(name)


def skew_diffusion_problem(ne: int, height: int, skew: float = 0.3, seed: int = 0,
                           nrhs: int = 1, tree: str = "octree") -> Problem:
    """A non-symmetric K on the 3-D diffusion pattern: K_d + skew (N - N^T), where K_d is
    Poisson on ne^3 Q1 hexahedra and N holds, on the entries of K_d above the diagonal,
    |K_d,ij| times U[-1, 1] drawn from `seed` (then f ~ U[-1, 1], nrhs columns).  The
    symmetric part is K_d, so every principal block and Schur complement is
    non-singular; the pattern stays symmetric."""
    base = diffusion_problem(ne, height, 0.0, seed, 1, tree=tree)
    rng = np.random.default_rng(seed)
    Kd = base.K.tocsr()
    U = sp.triu(Kd, k=1).tocoo()
    N = sp.coo_matrix((np.abs(U.data) * rng.uniform(-1.0, 1.0, U.nnz), (U.row, U.col)),
                      shape=Kd.shape)
    K = (Kd + skew * (N - N.T)).tocsr()
    K.sort_indices()
    b = rng.uniform(-1.0, 1.0, size=(K.shape[0], nrhs))
    return Problem(f"skew_diffusion{ne}_h{height}", K, base.parent, base.dof_node, b,
                   meta=dict(ne=ne, height=height, skew=skew, seed=seed))


def uneven_cuts(seed: int, lo_frac: float = 0.45, hi_frac: float = 0.55):
    """Random axis-aligned cut planes: each box is cut at a fraction drawn from
    U[lo_frac, hi_frac] of its extent; over an octree of height 3 the fractions
    compound (48^3 elasticity: leaf interiors of 192 to 882 dofs).  Drawn in the
    tree's breadth-first order from their own generator."""
    rng = np.random.default_rng(seed)

    def cut(depth, axis, lo, hi):
        m = lo + int(round(rng.uniform(lo_frac, hi_frac) * (hi - lo)))
        return min(max(m, lo + 1), hi - 1)
    return cut


def elasticity_problem(ne: int, height: int, seed: int = 0, nrhs: int = 8,
                       name: str | None = None) -> Problem:
    """3-D linear elasticity (E = 1, nu = 0.3) on ne^3 Q1 hexahedra, the face x = 0
    clamped, an octree of the given height over random uneven cut planes.

    Right-hand sides: the nodal body load (0, 0, -1) h^3 plus N(0, 0.1^2) h^3 per dof,
    nrhs columns.  Draw order: the cut planes (their own stream, seed + 1), then the
    load perturbations (seed).
    """
    sysm = assemble_elasticity_3d(ne)
    tree = build_box_tree(sysm.shape_nodes, height, cut_fn=uneven_cuts(seed + 1))
    dof_node = dof_node_map(tree, sysm.free_ijk, 3)
    n = sysm.K.shape[0]
    h3 = (1.0 / ne) ** 3
    body = np.tile(np.array([0.0, 0.0, -1.0]), n // 3)
    rng = np.random.default_rng(seed)
    b = (body[:, None] + 0.1 * rng.standard_normal((n, nrhs))) * h3
    return Problem(name or f"elasticity{ne}_h{height}", sysm.K, tree.parent, dof_node, b,
                   meta=dict(ne=ne, height=height, seed=seed, free_ijk=sysm.free_ijk,
                             tree=tree))


def strip_problem(N: int, P: int, problem: str = "poisson", seed: int = 0) -> Problem:
    """The paper's 2-D long strip with P = 2^H sub-domains of N x N nodes."""
    H = int(round(np.log2(P)))
    if 2 ** H != P:
        raise ValueError("P must be a power of two")
    sysm = assemble_strip_2d(N, P, problem)
    tree = build_box_tree(sysm.shape_nodes, H, axes_per_level=lambda d: (0,))
    dof_node = dof_node_map(tree, sysm.free_ijk, sysm.ndof)
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(-1.0, 1.0, size=sysm.K.shape[0])
    b = (sysm.K @ x_true)[:, None]
    return Problem(f"strip_{problem}_N{N}_P{P}", sysm.K, tree.parent, dof_node, b,
                   meta=dict(N=N, P=P, x_true=x_true, tree=tree, free_ijk=sysm.free_ijk))
