"""Pins for the seeded input generator (Q1 assembly and box hierarchies).

These check the generated systems against closed forms that do not depend on
the generator's own code path: the Q1 element integrals, the 27-point stencil,
the tensor-product eigenpairs of the Poisson matrix, the O(h^2) nodal error of
a manufactured solution, and the dof counts of every hierarchy level.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workloads.fem import (assemble_diffusion_3d, assemble_grid, consistent_load_3d,
                           laplace_element, navier_lame_element_2d)
from workloads.hierarchy import build_box_tree, dof_node_map


def test_element_closed_forms():
    K3 = laplace_element(3)
    # unit-cube trilinear stiffness: diagonal 1/3, edge neighbour 0,
    # face diagonal -1/12, body diagonal -1/12
    for a in range(8):
        for b in range(8):
            dist = bin(a ^ b).count("1")
            want = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[dist]
            assert abs(K3[a, b] - want) < 1e-15
    K2 = laplace_element(2)
    for a in range(4):
        for b in range(4):
            dist = bin(a ^ b).count("1")
            want = {0: 2 / 3, 1: -1 / 6, 2: -1 / 3}[dist]
            assert abs(K2[a, b] - want) < 1e-15


def test_interior_stencil_p1():
    ne = 8
    s = assemble_diffusion_3d(ne)
    h = 1.0 / ne
    K = s.K.tocsr()
    ijk = s.free_ijk
    idx = {tuple(v): i for i, v in enumerate(ijk)}
    centre = idx[(4, 4, 4)]
    row = K[centre].toarray().ravel()
    for j in np.nonzero(row)[0]:
        d = np.abs(ijk[j] - ijk[centre]).sum()
        want = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[d] * h
        assert abs(row[j] - want) < 1e-15
    # 27-point row of an interior node sums to zero
    assert abs(row.sum()) < 1e-15
    assert K[centre].nnz == 27


def test_sine_modes_are_eigenvectors_p2():
    ne = 10
    h = 1.0 / ne
    K = assemble_diffusion_3d(ne).K
    ijk = assemble_diffusion_3d(ne).free_ijk
    kap = lambda j: (2 / h) * (1 - np.cos(j * np.pi * h))    # noqa: E731
    mu = lambda j: (h / 3) * (2 + np.cos(j * np.pi * h))     # noqa: E731
    for (a, b, c) in [(1, 1, 1), (2, 5, 3), (9, 1, 4)]:
        u = (np.sin(a * np.pi * ijk[:, 0] * h) * np.sin(b * np.pi * ijk[:, 1] * h)
             * np.sin(c * np.pi * ijk[:, 2] * h))
        lam = kap(a) * mu(b) * mu(c) + mu(a) * kap(b) * mu(c) + mu(a) * mu(b) * kap(c)
        r = K @ u - lam * u
        assert np.abs(r).max() <= 1e-13 * np.abs(lam * u).max()


def test_manufactured_solution_second_order_p9():
    f = lambda x, y, z: 3 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)  # noqa: E731
    errs = []
    for ne in (8, 16):
        s = assemble_diffusion_3d(ne)
        b = consistent_load_3d(ne, f)
        u = spla.spsolve(s.K.tocsc(), b)
        x = s.free_ijk / ne
        exact = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2])
        errs.append(np.abs(u - exact).max())
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, ratio


def test_navier_lame_operator_is_elastic_form():
    """With Dirichlet data on every side, mu grad:grad + (lam+mu) div div and the
    elasticity form 2 mu eps:eps + lam div div assemble to the same matrix, and
    constant displacements lie in the element kernel."""
    lam, mu = 10.0, 1.0
    Ke = navier_lame_element_2d(lam, mu)
    for comp in range(2):
        t = np.zeros(8)
        t[comp::2] = 1.0
        assert np.abs(Ke @ t).max() < 1e-14
    # symmetric-gradient element, assembled independently
    from workloads.fem import _G2, _W2, _shape
    Ks = np.zeros((8, 8))
    for qx in range(2):
        for qy in range(2):
            _, g = _shape(2, np.array([_G2[qx], _G2[qy]]))
            B = np.zeros((3, 8))
            for a in range(4):
                B[0, 2 * a] = g[a, 0]
                B[1, 2 * a + 1] = g[a, 1]
                B[2, 2 * a] = g[a, 1]
                B[2, 2 * a + 1] = g[a, 0]
            D = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
            Ks += _W2[qx] * _W2[qy] * B.T @ D @ B
    A1 = assemble_grid((12, 6), Ke, None, 2, "all", (1.0, 1.0)).K
    A2 = assemble_grid((12, 6), Ks, None, 2, "all", (1.0, 1.0)).K
    assert abs(A1 - A2).max() < 1e-12


@pytest.mark.parametrize("name,n,nnz,counts", [
    ("poisson12", 1331, 29791, {0: [331], 1: [125] * 8}),
    ("diffusion64", 250047, 6539203, {0: [11719], 1: [2791] * 8, 2: [3375] * 64}),
])
def test_config_sizes(problem_cache, name, n, nnz, counts):
    p = problem_cache("config", name)
    assert p.n == n and p.K.nnz == nnz
    T = len(p.parent)
    assert p.parent[0] == -1 and all(p.parent[t] < t for t in range(1, T))
    depth = np.zeros(T, dtype=int)
    for t in range(1, T):
        depth[t] = depth[p.parent[t]] + 1
    per_node = np.bincount(p.dof_node, minlength=T)
    for lev, want in counts.items():
        assert sorted(per_node[depth == lev].tolist()) == sorted(want)


def test_hierarchy_ownership_rule():
    """Nodes on several cut planes go to the shallowest node; others to a leaf."""
    tree = build_box_tree((9, 9, 9), 2)
    ijk = np.array([[4, 4, 4], [4, 2, 6], [2, 2, 2], [1, 1, 1], [2, 6, 5], [3, 3, 3]])
    owner = dof_node_map(tree, ijk, 1)
    assert owner[0] == 0 and owner[1] == 0          # on root planes
    assert tree.depth[owner[2]] == 1                 # on level-1 planes of octant (0,0,0)
    assert tree.depth[owner[3]] == 2 and tree.depth[owner[5]] == 2
    assert tree.depth[owner[4]] == 1


def test_elasticity_element_rigid_body_modes():
    """The unconstrained element annihilates the 6 rigid-body modes and has rank 18;
    a single-node stretch has the closed-form energy of the isotropic law."""
    from workloads.fem import _corners, elasticity_element_3d
    K = elasticity_element_3d(1.0, 0.3)
    c = _corners(3).astype(float)
    modes = []
    for t in range(3):
        v = np.zeros(24)
        v[t::3] = 1.0
        modes.append(v)
    for i, j in [(0, 1), (1, 2), (0, 2)]:
        v = np.zeros(24)
        v[i::3] = -c[:, j]
        v[j::3] = c[:, i]
        modes.append(v)
    R = np.array(modes).T
    assert np.abs(K - K.T).max() == 0.0
    assert np.abs(K @ R).max() < 1e-14
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-10) == 18 and np.all(ev > -1e-12)
    # uniform strain u_x = x: energy = 1/2 (lambda + 2 mu) * volume
    lam, mu = 0.3 / (1.3 * 0.4), 1.0 / 2.6
    u = np.zeros(24)
    u[0::3] = c[:, 0]
    assert abs(0.5 * u @ K @ u - 0.5 * (lam + 2 * mu)) < 1e-14


def test_elasticity_workload_sizes():
    """48^3 clamped at x = 0: n = 3 * 49^2 * 48; octree of height 3 over uneven cuts
    (leaf interiors 192..882 dofs, root interface 20,880); 8 right-hand sides."""
    from workloads import config_problem
    p = config_problem("elasticity48")
    assert p.n == 3 * 49 * 49 * 48 == 345744
    assert p.b.shape == (p.n, 8)
    T = p.parent.size
    cnt = np.bincount(p.dof_node, minlength=T)
    isleaf = np.ones(T, bool)
    isleaf[p.parent[p.parent >= 0]] = False
    assert isleaf.sum() == 512 and cnt[isleaf].min() == 192 and cnt[isleaf].max() == 882
    assert cnt[0] == 20880
    assert abs(p.K - p.K.T).max() == 0.0
