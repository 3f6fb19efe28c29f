"""Pins of the oracle's interface modes against independent dense constructions.

The oracle follows the recursion of Alg. 2 (Section 3.2); tests/explicit_forms.py
builds the same preconditioner from the block algebra (static condensation, a block
forward sweep over the skeleton Schur complement, harmonic extension), written
without the oracle's code.  Pinned here:

* the leaf-only right-hand side of the interface systems (the strip formula of Alg. 2
  taken literally) in 3-D, at heights 2, 3 and 4, for a symmetric and a non-symmetric
  K: the explicit form with the direct interface-to-interface blocks of K dropped from
  the sweep; likewise the full right-hand side on the non-symmetric K;
* the per-level (hybrid) mode: the levels whose largest interface exceeds dense_max
  take gamma inner GMRES steps (Section 3.1's inexact interface solve), the others the
  exact solve.  The construction computes each inexact solve as GMRES's defining
  minimiser over the Krylov space, not by an Arnoldi process;
* planted mistakes: K_lI used in place of K_Il (a transposition that a symmetric K
  hides), and a level solved in the wrong mode, each break a pin.
"""
import numpy as np
import pytest

from explicit_forms import SkeletonForm, minimal_residual
from oracle import RSDOracle


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _vectors(n, k=3, seed=0):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, k))


# ----------------------------------------------------- the constructions themselves
def test_explicit_form_is_the_inverse_at_one_level(problem_cache):
    """One interface level: T is the whole skeleton Schur complement, so the explicit
    form is block Gaussian elimination, i.e. K^{-1} -- symmetric and not."""
    for key in (("config", "poisson12"), ("skew", 12, 1, 0.3, 2)):
        p = problem_cache(*key)
        F = SkeletonForm(p.K, p.parent, p.dof_node)
        Kinv = np.linalg.inv(p.K.toarray())
        assert rel(F.dense_form(), Kinv) < 1e-12
        assert rel(F.dense_form("leaf_only"), Kinv) < 1e-12


def test_minimal_residual_is_gmres_by_definition():
    rng = np.random.default_rng(3)
    S = 5.0 * np.eye(8) + 0.5 * rng.standard_normal((8, 8))   # non-symmetric, well conditioned
    g = rng.standard_normal(8)
    assert rel(minimal_residual(S, g, 8), np.linalg.solve(S, g)) < 1e-8   # finite termination
    u = minimal_residual(S, g, 3)
    Kr = np.column_stack([g, S @ g, S @ S @ g])
    best = np.linalg.norm(g - S @ u)
    for _ in range(200):                 # no vector of the Krylov space does better
        v = Kr @ rng.standard_normal(3) * 0.1 + u
        assert np.linalg.norm(g - S @ v) >= best * (1 - 1e-12)


# --------------------------------------------------------- coupling forms in 3-D
COUPLING_CASES = [
    ("diffusion", 13, 2, 1.0, 2),            # octree, height 2 (leaves of 27 dofs)
    ("diffusion_binary", 12, 3, 1.0, 3),     # height 3 (leaves of 125)
    ("diffusion_binary", 12, 4, 0.5, 1),     # height 4 (leaves of 50)
    ("skew", 13, 2, 0.3, 1),                 # non-symmetric K (LU sub-domain solves)
    ("skew_binary", 12, 3, 0.3, 5),
]


@pytest.mark.parametrize("key", COUPLING_CASES)
@pytest.mark.parametrize("coupling", ["full", "leaf_only"])
def test_coupling_forms_match_explicit_form(problem_cache, key, coupling):
    p = problem_cache(*key)
    o = RSDOracle(p.K, p.parent, p.dof_node, coupling=coupling)
    F = SkeletonForm(p.K, p.parent, p.dof_node)
    R = _vectors(p.n)
    assert rel(o.apply(R), F.dense_form(coupling) @ R) < 1e-11


def test_couplings_differ_in_3d(problem_cache):
    """The pin above tells the two forms apart: they differ by far more than rounding
    wherever interfaces couple directly to deeper interfaces."""
    for key in (("diffusion", 13, 2, 1.0, 2), ("diffusion_binary", 12, 3, 1.0, 3)):
        p = problem_cache(*key)
        F = SkeletonForm(p.K, p.parent, p.dof_node)
        assert rel(F.dense_form("leaf_only"), F.dense_form("full")) > 1e-3


@pytest.mark.parametrize("coupling", ["full", "leaf_only"])
def test_planted_transposition_is_caught(problem_cache, coupling):
    """K_lI^T in place of K_Il (the interface-to-leaf block) in S~ and in g: invisible
    for a symmetric K, caught on a non-symmetric one."""
    p = problem_cache("skew_binary", 12, 3, 0.3, 5)
    F = SkeletonForm(p.K, p.parent, p.dof_node)
    R = _vectors(p.n)
    ref = F.dense_form(coupling) @ R
    o = RSDOracle(p.K, p.parent, p.dof_node, coupling=coupling)
    assert rel(o.apply(R), ref) < 1e-11
    for (t, l) in list(o.K_Il):
        o.K_Il[(t, l)] = o.K_lI[(l, t)].T.tocsr()
    for t in o.S_chol:
        o.S_chol[t] = o._factor(o.schur_dense(t))
    assert rel(o.apply(R), ref) > 1e-3


# ------------------------------------------------------------- per-level (hybrid) mode
HYBRID_CASES = [  # (problem, gamma, dense_max)
    (("diffusion", 13, 2, 1.0, 2), 3, 200),          # root (397) inexact, level 1 exact
    (("diffusion_binary", 12, 3, 1.0, 3), 4, 30),    # levels 0-1 inexact, level 2 exact
    (("diffusion_binary", 12, 4, 0.5, 1), 3, 60),    # root inexact, levels 1-3 exact
    (("skew_binary", 12, 3, 0.3, 5), 3, 60),         # non-symmetric K
]


@pytest.mark.parametrize("key,gamma,dense_max", HYBRID_CASES)
@pytest.mark.parametrize("coupling", ["full", "leaf_only"])
def test_hybrid_matches_sweep(problem_cache, key, gamma, dense_max, coupling):
    p = problem_cache(*key)
    o = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=gamma,
                  dense_max=dense_max, coupling=coupling)
    F = SkeletonForm(p.K, p.parent, p.dof_node)
    inexact = F.level_choice(dense_max)
    assert inexact == o.inexact
    assert any(inexact.values()) and not all(inexact.values())
    for j, r in enumerate(_vectors(p.n, 2, seed=7).T):
        assert rel(o.apply(r), F.sweep_apply(r, inexact, gamma, coupling)) < 1e-9, j


def test_hybrid_extremes_are_the_pure_modes(problem_cache):
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    r = _vectors(p.n, 1)[:, 0]
    dense = RSDOracle(p.K, p.parent, p.dof_node).apply(r)
    gam = RSDOracle(p.K, p.parent, p.dof_node, interface="gamma", gamma=3).apply(r)
    hd = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=3, dense_max=10 ** 6)
    hg = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=3, dense_max=0)
    assert np.array_equal(hd.apply(r), dense) and np.array_equal(hg.apply(r), gam)
    # and the sweep with every node inexact agrees with the pure gamma mode
    F = SkeletonForm(p.K, p.parent, p.dof_node)
    assert rel(gam, F.sweep_apply(r, {t: True for t in F.internal}, 3)) < 1e-9


def test_planted_level_flip_is_caught(problem_cache):
    """The root solved exactly although its level is above dense_max: breaks the pin."""
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    o = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=3, dense_max=200)
    F = SkeletonForm(p.K, p.parent, p.dof_node)
    r = _vectors(p.n, 1)[:, 0]
    ref = F.sweep_apply(r, F.level_choice(200), 3)
    assert rel(o.apply(r), ref) < 1e-9
    o.inexact[0] = False
    o.S_chol[0] = o._factor(o.schur_dense(0))
    assert rel(o.apply(r), ref) > 1e-4
