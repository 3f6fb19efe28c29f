"""Q1 finite-element assembly on uniform grids (input generation only).

The paper discretises its model problems with bilinear (2-D) finite elements on
regular grids with homogeneous Dirichlet conditions on every side (Section 4,
results set-up).  This module builds such systems, and their 3-D trilinear
analogue, as CSR matrices over the free (non-Dirichlet) nodes.  It holds no
part of the RSD method: it produces the sparse matrix ``K`` and load vectors
that the method and the oracle both take as input.

Element matrices are integrated with tensor Gauss rules that are exact for the
polynomial degree of the integrands (2 points per axis for stiffness, 3 for
mass / consistent loads).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_G2 = (np.array([-1.0, 1.0]) / np.sqrt(3.0) + 1.0) / 2.0  # 2-pt Gauss on [0,1]
_W2 = np.array([0.5, 0.5])
_G3 = (np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) + 1.0) / 2.0  # 3-pt Gauss on [0,1]
_W3 = np.array([5.0, 8.0, 5.0]) / 18.0


def _corners(dim: int) -> np.ndarray:
    """Reference-element corner bits, x varying fastest: corner a = sum_d bit_d 2^d."""
    return np.array([[(a >> d) & 1 for d in range(dim)] for a in range(2 ** dim)])


def _shape(dim: int, xi: np.ndarray):
    """Values and gradients of the 2^dim multilinear shape functions at point xi."""
    c = _corners(dim)
    n = 2 ** dim
    val = np.ones(n)
    grad = np.ones((n, dim))
    for a in range(n):
        for d in range(dim):
            f = xi[d] if c[a, d] else 1.0 - xi[d]
            df = 1.0 if c[a, d] else -1.0
            val[a] *= f
            for e in range(dim):
                grad[a, e] *= df if e == d else f
    return val, grad


def elasticity_element_3d(E: float, nu: float) -> np.ndarray:
    """Unit-cell linear-elasticity stiffness  int eps(v) : C : eps(u)  (24 x 24).

    Isotropic C with Lame constants lambda = E nu / ((1 + nu)(1 - 2 nu)) and
    mu = E / (2 (1 + nu)): sigma = 2 mu eps + lambda tr(eps) I.  Dofs are node-major:
    (u_x, u_y, u_z) per corner.  For an element of size h the matrix scales by h.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    K = np.zeros((24, 24))
    for q in itertools.product(range(2), repeat=3):
        xi = np.array([_G2[i] for i in q])
        w = np.prod([_W2[i] for i in q])
        _, g = _shape(3, xi)
        for a in range(8):
            for b in range(8):
                # 2 mu eps:eps = mu (grad u : grad v + grad u : grad v^T), plus lambda div div
                blk = mu * (g[a] @ g[b]) * np.eye(3) + mu * np.outer(g[b], g[a]) \
                    + lam * np.outer(g[a], g[b])
                K[3 * a:3 * a + 3, 3 * b:3 * b + 3] += w * blk
    return K


def laplace_element(dim: int) -> np.ndarray:
    """Unit-cell stiffness  int grad(phi_a) . grad(phi_b)  (2^dim x 2^dim)."""
    n = 2 ** dim
    K = np.zeros((n, n))
    for q in itertools.product(range(2), repeat=dim):
        xi = np.array([_G2[i] for i in q])
        w = np.prod([_W2[i] for i in q])
        _, g = _shape(dim, xi)
        K += w * g @ g.T
    return K


def mass_element(dim: int) -> np.ndarray:
    """Unit-cell mass matrix  int phi_a phi_b."""
    n = 2 ** dim
    M = np.zeros((n, n))
    for q in itertools.product(range(3), repeat=dim):
        xi = np.array([_G3[i] for i in q])
        w = np.prod([_W3[i] for i in q])
        v, _ = _shape(dim, xi)
        M += w * np.outer(v, v)
    return M


def navier_lame_element_2d(lam: float, mu: float) -> np.ndarray:
    """Unit-cell bilinear form  int mu grad u : grad v + (lam+mu) div u div v.

    This is the weak form of the elliptic Navier-Lame operator
    -mu Lap u - (lam+mu) grad div u (Problem 4 of the paper, with the sign that
    makes the operator elliptic).  Dofs are node-major: (u_x, u_y) per corner.
    """
    K = np.zeros((8, 8))
    for q in itertools.product(range(2), repeat=2):
        xi = np.array([_G2[i] for i in q])
        w = _W2[q[0]] * _W2[q[1]]
        _, g = _shape(2, xi)
        for a in range(4):
            for b in range(4):
                for i in range(2):
                    for j in range(2):
                        v = (lam + mu) * g[a, i] * g[b, j]
                        if i == j:
                            v += mu * (g[a] @ g[b])
                        K[2 * a + i, 2 * b + j] += w * v
    return K


@dataclass
class GridSystem:
    """A Q1 system on a uniform grid, restricted to free (non-Dirichlet) nodes.

    Attributes
    ----------
    K : scipy.sparse.csr_matrix  (n x n), sorted indices, no duplicates
    shape_nodes : number of grid nodes per axis (including boundary nodes)
    free_ijk : (n_free_nodes, dim) integer grid coordinates of the free nodes
    ndof : dofs per node (node-major numbering)
    h : element size per axis
    """

    K: sp.csr_matrix
    shape_nodes: tuple
    free_ijk: np.ndarray
    ndof: int
    h: tuple


def _element_connectivity(ne: tuple) -> np.ndarray:
    """(n_elem, 2^dim) global node ids (lexicographic, x fastest) of each element."""
    dim = len(ne)
    nn = tuple(e + 1 for e in ne)
    strides = np.cumprod((1,) + nn[:-1])
    grids = np.meshgrid(*[np.arange(e) for e in ne], indexing="ij")
    base = sum(g.ravel(order="F") * s for g, s in zip(grids, strides))
    c = _corners(dim)
    off = c @ strides
    return base[:, None] + off[None, :]


def assemble_grid(ne: tuple, elem: np.ndarray, coef: np.ndarray | None = None,
                  ndof: int = 1, dirichlet: str = "all", h: tuple | None = None,
                  symmetric: bool = True) -> GridSystem:
    """Assemble  sum_e coef_e * elem  over a uniform grid of ne elements per axis.

    ``elem`` is the element matrix already scaled for the element size.
    ``dirichlet`` is "all" (every boundary node constrained) or "x0" (only the
    face x = 0).  Constrained dofs are eliminated (rows and columns removed).
    ``symmetric``: make K bitwise symmetric (for a symmetric element matrix);
    False keeps a non-symmetric operator as assembled.
    """
    dim = len(ne)
    nn = tuple(e + 1 for e in ne)
    conn = _element_connectivity(ne)
    nel = conn.shape[0]
    if coef is None:
        coef = np.ones(nel)
    ijk = np.stack(np.unravel_index(np.arange(int(np.prod(nn))), nn, order="F"), axis=1)
    if dirichlet == "all":
        free = np.all((ijk > 0) & (ijk < np.array(nn) - 1), axis=1)
    elif dirichlet == "x0":
        free = ijk[:, 0] > 0
    else:
        raise ValueError(dirichlet)
    node_id = -np.ones(ijk.shape[0], dtype=np.int64)
    node_id[free] = np.arange(int(free.sum()))
    # element dof lists, node-major; -1 marks an eliminated (Dirichlet) dof
    gdof = np.where(np.repeat(free[conn], ndof, axis=1),
                    node_id[np.repeat(conn, ndof, axis=1)] * ndof
                    + np.tile(np.arange(ndof), conn.shape[1])[None, :], -1)
    ne_loc = gdof.shape[1]
    rows = np.repeat(gdof, ne_loc, axis=1).ravel()
    cols = np.tile(gdof, (1, ne_loc)).ravel()
    vals = (coef[:, None] * elem.ravel()[None, :]).ravel()
    keep = (rows >= 0) & (cols >= 0)
    n = int(free.sum()) * ndof
    K = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    K.sum_duplicates()
    if symmetric:
        # duplicates are summed in a data-dependent order, so K_ij and K_ji can differ
        # in the last bit; the average is symmetric bit for bit (a + b == b + a)
        K = ((K + K.T) * 0.5).tocsr()
        K.sum_duplicates()
    K.sort_indices()
    if h is None:
        h = tuple(1.0 / e for e in ne)
    return GridSystem(K=K, shape_nodes=nn, free_ijk=ijk[free], ndof=ndof, h=h)


def assemble_diffusion_3d(ne: int, k_elem: np.ndarray | None = None) -> GridSystem:
    """-div(k grad u) on the unit cube, ne^3 trilinear elements, Dirichlet on all faces.

    Element matrix = k_e * h * K_ref (the 3-D gradient integral scales with h^{3-2}).
    """
    h = 1.0 / ne
    return assemble_grid((ne, ne, ne), h * laplace_element(3), k_elem, 1, "all", (h, h, h))


def assemble_elasticity_3d(ne: int, E: float = 1.0, nu: float = 0.3) -> GridSystem:
    """Linear elasticity on the unit cube, ne^3 trilinear elements, the face x = 0
    clamped (its nodes eliminated), 3 dofs per node."""
    h = 1.0 / ne
    return assemble_grid((ne, ne, ne), h * elasticity_element_3d(E, nu), None, 3, "x0",
                         (h, h, h))


def anisotropic_laplace_element_2d(ax: float, ay: float) -> np.ndarray:
    """Unit-cell  int ax phi_a,x phi_b,x + ay phi_a,y phi_b,y  (4 x 4)."""
    K = np.zeros((4, 4))
    for q in itertools.product(range(2), repeat=2):
        xi = np.array([_G2[i] for i in q])
        w = np.prod([_W2[i] for i in q])
        _, g = _shape(2, xi)
        K += w * (ax * np.outer(g[:, 0], g[:, 0]) + ay * np.outer(g[:, 1], g[:, 1]))
    return K


def coupled_element_2d(c: float, h: float) -> np.ndarray:
    """Element of the paper's two-field systems (Problems 2 and 3), dofs (u, v) per node:
      -u_xx/100 - u_yy + c v = f,   -c u - v_xx - v_yy/100 = g
    as  [[A_u, c h^2 M], [-c h^2 M, A_v]]  with the unit-cell anisotropic stiffness
    matrices (scale-invariant in 2-D) and the consistent mass matrix of an h x h element.
    The coupling is antisymmetric, so the operator is not symmetric."""
    Au = anisotropic_laplace_element_2d(0.01, 1.0)
    Av = anisotropic_laplace_element_2d(1.0, 0.01)
    M = mass_element(2) * h * h
    E = np.zeros((8, 8))
    for a in range(4):
        for b in range(4):
            E[2 * a, 2 * b] = Au[a, b]
            E[2 * a + 1, 2 * b + 1] = Av[a, b]
            E[2 * a, 2 * b + 1] = c * M[a, b]
            E[2 * a + 1, 2 * b] = -c * M[a, b]
    return E


def assemble_strip_2d(N: int, P: int, problem: str) -> GridSystem:
    """The paper's 2-D strip: P true sub-domains of N x N nodes placed along x.

    Neighbouring sub-domains share one node line, so the domain has
    P(N-1) x (N-1) elements; Dirichlet on every side.  The stiffness forms used
    here are scale-invariant in 2-D; for the two-field systems each sub-domain is a
    unit square (element size h = 1/(N-1)), which sets the weight of the coupling.
    problem: "poisson" (Problem 1), "coupled_weak" (Problem 2, c = 1/100),
    "coupled_strong" (Problem 3, c = 100) or "navier_lame" (Problem 4, lambda=10,
    mu=1).
    """
    ne = (P * (N - 1), N - 1)
    if problem == "poisson":
        return assemble_grid(ne, laplace_element(2), None, 1, "all", (1.0, 1.0))
    if problem in ("coupled_weak", "coupled_strong"):
        c = 0.01 if problem == "coupled_weak" else 100.0
        return assemble_grid(ne, coupled_element_2d(c, 1.0 / (N - 1)), None, 2, "all",
                             (1.0, 1.0), symmetric=False)
    if problem == "navier_lame":
        return assemble_grid(ne, navier_lame_element_2d(10.0, 1.0), None, 2, "all", (1.0, 1.0))
    raise ValueError(problem)


def consistent_load_3d(ne: int, f) -> np.ndarray:
    """b_i = int f phi_i over the unit cube (3-pt Gauss per axis per element), free dofs only."""
    h = 1.0 / ne
    nn = ne + 1
    conn = _element_connectivity((ne, ne, ne))
    ex = np.stack(np.unravel_index(np.arange(ne ** 3), (ne, ne, ne), order="F"), axis=1) * h
    b_full = np.zeros(nn ** 3)
    for q in itertools.product(range(3), repeat=3):
        xi = np.array([_G3[i] for i in q])
        w = np.prod([_W3[i] for i in q]) * h ** 3
        v, _ = _shape(3, xi)
        pts = ex + xi * h
        fv = f(pts[:, 0], pts[:, 1], pts[:, 2])
        np.add.at(b_full, conn, w * fv[:, None] * v[None, :])
    ijk = np.stack(np.unravel_index(np.arange(nn ** 3), (nn, nn, nn), order="F"), axis=1)
    free = np.all((ijk > 0) & (ijk < nn - 1), axis=1)
    return b_full[free]


def fe_map_grid(ne: tuple, elem: np.ndarray, K: sp.csr_matrix, ndof: int = 1,
                dirichlet: str = "all") -> dict:
    """Coefficient map of ``assemble_grid(ne, elem, coef, ndof, dirichlet)``.

    Returns the element dof lists (E x d, -1 on eliminated dofs), the symmetrised
    element matrix ``ke`` (d x d) and, for every nonzero of ``K`` (CSR order), the list
    of element entries (e, a, b) that add to it, packed as e*d*d + a*d + b and sorted.
    Entries with ke[a, b] == 0 are omitted (they add nothing for any coefficient).
    """
    dim = len(ne)
    nn = tuple(e + 1 for e in ne)
    conn = _element_connectivity(ne)
    ijk = np.stack(np.unravel_index(np.arange(int(np.prod(nn))), nn, order="F"), axis=1)
    if dirichlet == "all":
        free = np.all((ijk > 0) & (ijk < np.array(nn) - 1), axis=1)
    elif dirichlet == "x0":
        free = ijk[:, 0] > 0
    else:
        raise ValueError(dirichlet)
    node_id = -np.ones(ijk.shape[0], dtype=np.int64)
    node_id[free] = np.arange(int(free.sum()))
    gdof = np.where(np.repeat(free[conn], ndof, axis=1),
                    node_id[np.repeat(conn, ndof, axis=1)] * ndof
                    + np.tile(np.arange(ndof), conn.shape[1])[None, :], -1)
    E, d = gdof.shape
    ke = 0.5 * (elem + elem.T)
    a_idx, b_idx = np.meshgrid(np.arange(d), np.arange(d), indexing="ij")
    a_idx, b_idx = a_idx.ravel(), b_idx.ravel()
    rows = gdof[:, a_idx]
    cols = gdof[:, b_idx]
    code = np.arange(E, dtype=np.int64)[:, None] * d * d + (a_idx * d + b_idx)[None, :]
    keep = (rows >= 0) & (cols >= 0) & (ke[a_idx, b_idx] != 0.0)[None, :]
    rows, cols, code = rows[keep], cols[keep], code[keep]
    n = K.shape[0]
    Kc = K.tocsr()
    row_of_nz = np.repeat(np.arange(n, dtype=np.int64), np.diff(Kc.indptr))
    kkeys = row_of_nz * n + Kc.indices.astype(np.int64)
    keys = rows * n + cols
    pos = np.searchsorted(kkeys, keys)
    if np.any(pos >= kkeys.size) or np.any(kkeys[np.minimum(pos, kkeys.size - 1)] != keys):
        raise ValueError("element entry outside the sparsity pattern of K")
    order = np.lexsort((code, pos))
    counts = np.bincount(pos, minlength=Kc.nnz)
    ptr = np.zeros(Kc.nnz + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    if E * d * d >= 2 ** 31:
        raise ValueError("too many element entries for 32-bit packed codes")
    return dict(elem_dofs=gdof.astype(np.int32), ke=np.ascontiguousarray(ke),
                contrib_ptr=ptr, contrib=code[order].astype(np.int32), nnz=int(Kc.nnz),
                num_elements=E, dofs_per_element=d)
