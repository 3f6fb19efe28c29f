"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

* brute force: the preconditioned solve equals a dense direct solve;
* one interface level with exact interface solves reproduces K^{-1}
  (eqs. (schur) and (backSub) are exact block elimination);
* exact nested dissection on the same tree equals K^{-1} (tree plumbing);
* the preconditioner equals an explicit dense form derived independently:
  static condensation onto the skeleton, one bottom-up block Gauss-Seidel sweep
  with the skeleton Schur complement, and harmonic extension;
* gamma >= dim(S~) inner GMRES steps reproduce the exact interface solve;
* the outer iteration counts printed in Tables 1 and 10 (2-D strips, paper mode);
* symmetry / definiteness of K, S~_t;
* planted mistakes in the oracle (sign, dropped coupling, missing leaf) are caught.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import Hierarchy, RSDOracle, exact_block_solve, fgmres, pcg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def explicit_dense_form(K, parent, dof_node):
    """M^{-1} = [[I, -A^{-1}C],[0, I]] diag(A^{-1}, T^{-1}) [[I, 0],[-C^T A^{-1}, I]]
    with A = blockdiag(K_ll), C = K_{leaves, skeleton}, S^ = E - C^T A^{-1} C and T
    the block lower-triangular part of S^ over tree nodes ordered deepest first
    (block (s, t) kept when t = s or t lies in the sub-tree of s)."""
    Kd = K.toarray()
    H = Hierarchy(parent, dof_node, K.shape[0])
    leaves = [t for t in range(H.T) if H.is_leaf[t]]
    internal = sorted([t for t in range(H.T) if not H.is_leaf[t]], key=lambda t: -H.level[t])
    lam = np.concatenate([H.dofs[t] for t in leaves])
    skel_blocks = [H.dofs[t] for t in internal]
    skel = np.concatenate(skel_blocks)
    A = Kd[np.ix_(lam, lam)]
    C = Kd[np.ix_(lam, skel)]
    E = Kd[np.ix_(skel, skel)]
    Ainv = np.linalg.inv(A)
    S = E - C.T @ Ainv @ C
    T = np.zeros_like(S)
    off = np.cumsum([0] + [len(b) for b in skel_blocks])
    for a, s in enumerate(internal):
        for b, t in enumerate(internal):
            if t == s or H.in_subtree(t, s):
                T[off[a]:off[a + 1], off[b]:off[b + 1]] = S[off[a]:off[a + 1], off[b]:off[b + 1]]
    nl, ns = len(lam), len(skel)
    L = np.block([[np.eye(nl), np.zeros((nl, ns))], [-C.T @ Ainv, np.eye(ns)]])
    U = np.block([[np.eye(nl), -Ainv @ C], [np.zeros((ns, nl)), np.eye(ns)]])
    D = np.block([[Ainv, np.zeros((nl, ns))], [np.zeros((ns, nl)), np.linalg.inv(T)]])
    Mp = U @ D @ L                      # in the [leaves; skeleton] ordering
    perm = np.concatenate([lam, skel])
    M = np.zeros_like(Mp)
    M[np.ix_(perm, perm)] = Mp
    return M


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


# ---------------------------------------------------------------- brute force
def test_preconditioned_solution_equals_direct_solve_p3(problem_cache):
    p = problem_cache("diffusion", 10, 2, 1.0, 5)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    x, info = fgmres(p.K, p.b[:, 0], o.apply, rtol=1e-12)
    xd = np.linalg.solve(p.K.toarray(), p.b[:, 0])
    assert info["converged"] and rel(x, xd) < 1e-10


def test_one_level_exact_interface_is_inverse_p4(problem_cache):
    p = problem_cache("config", "poisson12")
    o = RSDOracle(p.K, p.parent, p.dof_node)
    assert rel(o.dense(), np.linalg.inv(p.K.toarray())) < 1e-13
    x, info = pcg(p.K, p.b[:, 0], o.apply, rtol=1e-10)
    assert info["iterations"] == 1 and info["relres"] < 1e-13


@pytest.mark.parametrize("ne,height,sigma", [(8, 2, 1.0), (11, 2, 0.5), (9, 3, 0.0)])
def test_exact_nested_dissection_is_inverse_p7(problem_cache, ne, height, sigma):
    p = problem_cache("diffusion", ne, height, sigma, 1)
    x = exact_block_solve(p.K, p.parent, p.dof_node, p.b[:, 0])
    assert rel(x, spla.spsolve(p.K.tocsc(), p.b[:, 0])) < 1e-12


@pytest.mark.parametrize("ne,height,sigma", [(8, 2, 1.0), (10, 2, 0.0), (13, 2, 1.0), (9, 3, 0.5)])
def test_matches_explicit_dense_form_p5(problem_cache, ne, height, sigma):
    p = problem_cache("diffusion", ne, height, sigma, 2)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    assert rel(o.dense(), explicit_dense_form(p.K, p.parent, p.dof_node)) < 1e-12


def test_gamma_to_dimension_equals_dense_p6(problem_cache):
    p = problem_cache("diffusion", 8, 2, 1.0, 4)
    dense = RSDOracle(p.K, p.parent, p.dof_node)
    big = max(len(d) for d in dense.I.values())
    gam = RSDOracle(p.K, p.parent, p.dof_node, interface="gamma", gamma=big)
    r = p.b[:, 0]
    assert rel(gam.apply(r), dense.apply(r)) < 1e-10


# ------------------------------------------------------------- paper tables
def _golden_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_outer_iterations.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                prob, N, P, g, beta = line.split()
                rows.append((prob, int(N), int(P), int(g), int(beta)))
    return rows


@pytest.mark.parametrize("prob,N,P,gamma,beta", _golden_rows())
def test_paper_outer_iteration_counts_p8(problem_cache, prob, N, P, gamma, beta):
    """Tables 1 and 10: the paper's beta within +-2 (PETSc's GMRES details are
    not stated, so the count is a soft pin)."""
    s = problem_cache("strip", N, P, prob, 0)
    o = RSDOracle(s.K, s.parent, s.dof_node, interface="gamma", gamma=gamma)
    x, info = fgmres(s.K, s.b[:, 0], o.apply, rtol=1e-12, restart=30, maxit=500)
    assert info["converged"]
    assert abs(info["iterations"] - beta) <= 2, (info["iterations"], beta)
    assert rel(x, s.meta["x_true"]) < 1e-8


def test_paper_trends_t2(problem_cache):
    """Section 4 discussion: beta does not grow with P, and falls as gamma grows."""
    its = {}
    for P in (8, 64):
        s = problem_cache("strip", 17, P, "poisson", 0)
        for g in (2, 8):
            o = RSDOracle(s.K, s.parent, s.dof_node, interface="gamma", gamma=g)
            its[(P, g)] = fgmres(s.K, s.b[:, 0], o.apply, rtol=1e-12)[1]["iterations"]
    assert its[(64, 2)] <= its[(8, 2)] + 2 and its[(64, 8)] <= its[(8, 8)] + 2
    assert its[(8, 8)] < its[(8, 2)] and its[(64, 8)] < its[(64, 2)]


# --------------------------------------------------------- structure / symmetry
def test_symmetry_and_definiteness_p10(problem_cache):
    p = problem_cache("diffusion", 10, 2, 1.0, 0)
    assert abs(p.K - p.K.T).max() == 0.0
    o = RSDOracle(p.K, p.parent, p.dof_node)
    for t in o.I:
        S = o.schur_dense(t)
        assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
        assert np.linalg.eigvalsh(S).min() > 0.0
    # one interface level: M^{-1} = K^{-1} is symmetric; two levels: not in general
    M = o.dense()
    assert np.abs(M - M.T).max() / np.abs(M).max() > 1e-3


def test_strip_couplings_coincide(problem_cache):
    """In a 2-D strip an interface couples only to L-hat and R-hat, so the full
    and leaf-only right-hand sides of the interface system coincide."""
    s = problem_cache("strip", 9, 8, "poisson", 0)
    a = RSDOracle(s.K, s.parent, s.dof_node, coupling="full")
    b = RSDOracle(s.K, s.parent, s.dof_node, coupling="leaf_only")
    assert all(len(a.C[t]) == 2 for t in a.C)
    r = s.b[:, 0]
    assert rel(a.apply(r), b.apply(r)) < 1e-14


def test_krylov_solvers_against_direct(problem_cache):
    p = problem_cache("diffusion", 9, 1, 1.0, 7)
    xd = spla.spsolve(p.K.tocsc(), p.b[:, 0])
    for solver in (lambda: fgmres(p.K, p.b[:, 0], lambda v: v.copy(), rtol=1e-12, restart=10),
                   lambda: pcg(p.K, p.b[:, 0], lambda v: v.copy(), rtol=1e-12)):
        x, info = solver()
        assert info["converged"] and rel(x, xd) < 1e-9


# ------------------------------------------------------------ planted mistakes
def test_planted_mistakes_are_caught(problem_cache, monkeypatch):
    """Each plausible oracle bug breaks at least one of the pins above."""
    p1 = problem_cache("config", "poisson12")
    Kinv = np.linalg.inv(p1.K.toarray())
    p2 = problem_cache("diffusion", 8, 2, 1.0, 2)
    E1 = explicit_dense_form(p2.K, p2.parent, p2.dof_node)

    # (a) dropped deeper-interface coupling in g: breaks the explicit form at h = 2
    o = RSDOracle(p2.K, p2.parent, p2.dof_node, coupling="leaf_only")
    assert rel(o.dense(), E1) > 1e-3

    # (b) wrong sign of the interface solution: breaks P4
    o = RSDOracle(p1.K, p1.parent, p1.dof_node)
    monkeypatch.setattr(o, "interface_solve", lambda t, g: -o._solve(o.S_chol[t], g))
    assert rel(o.dense(), Kinv) > 1e-3

    # (c) one leaf missing from C_t: breaks P4
    o = RSDOracle(p1.K, p1.parent, p1.dof_node)
    o.C[0] = o.C[0][1:]
    assert rel(o.dense(), Kinv) > 1e-3


# ------------------------------------------- the paper's two-field (non-symmetric) systems
def _golden_coupled_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_outer_iterations_coupled.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                prob, N, P, g, beta = line.split()
                rows.append((prob, int(N), int(P), int(g), int(beta)))
    return rows


@pytest.mark.parametrize("prob,N,P,gamma,beta", _golden_coupled_rows())
def test_paper_coupled_iteration_counts_p8(problem_cache, prob, N, P, gamma, beta):
    """Tables 4 and 7 with LU sub-domain solves.  Problem 3 within +-2.  Problem 2
    (weak coupling) drifts below the printed counts as they grow (80 vs 87 at N = 33,
    gamma = 2): within max(2, 12%).  The paper states neither the discretisation of the
    coupling terms nor the domain size; here each sub-domain is a unit square with the
    consistent mass matrix for the coupling, which sets the coupling's weight against
    the scale-invariant stiffness and hence how far Problem 2's counts can match."""
    s = problem_cache("strip", N, P, prob, 0)
    assert abs(s.K - s.K.T).max() > 0                   # really non-symmetric
    o = RSDOracle(s.K, s.parent, s.dof_node, interface="gamma", gamma=gamma)
    assert not o.symmetric
    x, info = fgmres(s.K, s.b[:, 0], o.apply, rtol=1e-12, restart=30, maxit=500)
    assert info["converged"]
    tol = 2 if prob == "coupled_strong" else max(2, int(0.12 * beta))
    assert abs(info["iterations"] - beta) <= tol, (info["iterations"], beta)
    assert rel(x, s.meta["x_true"]) < 1e-8


@pytest.mark.parametrize("prob", ["coupled_weak", "coupled_strong"])
def test_lu_path_one_level_is_exact(problem_cache, prob):
    """Two sub-domains, exact interface solve: M^{-1} = K^{-1} for a non-symmetric K
    (the LU sub-domain and interface solves of the oracle)."""
    s = problem_cache("strip", 9, 2, prob, 0)
    o = RSDOracle(s.K, s.parent, s.dof_node)
    Kinv = np.linalg.inv(s.K.toarray())
    assert np.abs(o.dense() - Kinv).max() <= 1e-11 * np.abs(Kinv).max()
    g = RSDOracle(s.K, s.parent, s.dof_node, interface="gamma", gamma=14)   # dim(S~) = 14
    r = np.random.default_rng(2).uniform(-1, 1, s.n)
    assert rel(g.apply(r), o.apply(r)) < 1e-10
