"""Plain FP64 CPU oracle for the Recursive Schur Decomposition preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It
shares no code with the HIP library; both read the same seeded inputs.

What it computes (Sampath et al., "Recursive Schur Decomposition"):

* Two sub-domains (Section 3.1): with dofs split into the two sub-domain
  interiors and their interface I, the interface unknowns solve the Schur
  complement system S u_I = g of eq. (schur), and the interiors follow by the
  back-substitution of eq. (backSub).  Sub-domain matrices are inverted
  exactly with a direct method (here: dense Cholesky; LU with partial pivoting
  when K is not symmetric, as for the paper's two-field Problems 2 and 3).
* Many sub-domains (Section 3.2): the pseudo sub-domain solves that produce
  K^{-1} f inside g are replaced by the same algorithm applied recursively to
  the sub-tree (Alg. 2, RSD); the two other uses of a pseudo sub-domain inverse
  (inside the S-MatVec and in the back-substitution) are approximated by the
  inverse of the true sub-domain that touches the interface (restrict, solve,
  prolong by zeros) -- the V-hat approximation.
* Alg. 1 (S-MatVec) therefore applies
      S~_t = K_II - sum_{l in C_t} K_Il K_ll^{-1} K_lI,
  and the interface system is solved either exactly (dense Cholesky of the
  assembled S~_t: the limit of infinitely many inner iterations) or, as in the
  paper's experiments, by a fixed number gamma of unpreconditioned GMRES
  iterations started from zero.  A third mode mixes the two per level of the tree
  (the internal nodes of one depth): the levels whose largest interface exceeds a
  size limit take the inexact solve, the others the exact one.

Readings taken where the paper describes only 2-D strips (binary trees):

* Generic trees: any number of children per node; every dof belongs either to
  a leaf interior or to the interface of one internal node (the ``dof_node`` map).
* C_t (the generalised V-hat): all leaves of subtree(t) whose interior is
  coupled to I_t by K.  In a 2-D strip that is exactly {L-hat, R-hat}.
* The right-hand side of the interface system: the paper's
  g = f_I - K_{I,L-hat} v_{L-hat} - K_{I,R-hat} v_{R-hat} equals
  f_I - K_{I,V} v in a strip, because I couples only to those two interiors.
  In 3-D an interface also couples directly to deeper interface dofs.  The
  default ("full") takes g = f_I - K_{I,V} v over all of V = D(t) minus I
  (eq. (schur) with the recursive solution in place of K_VV^{-1} f_V);
  "leaf_only" keeps only the C_t leaf terms (the literal 2-D formula).

Parity: this module is pinned by the CPU tests (closed forms, brute-force
dense inverses, the explicit dense form of the preconditioner -- with either
right-hand side, for symmetric and non-symmetric K --, a block sweep with
minimal-residual Krylov steps for the inexact and per-level modes, and the
paper's printed iteration counts).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class Hierarchy:
    """The tree (Section 2): children lists, levels, the dofs of every node and
    D(t), the dofs of the whole sub-tree rooted at t."""

    def __init__(self, parent, dof_node, n: int):
        parent = np.asarray(parent, dtype=np.int64)
        dof_node = np.asarray(dof_node, dtype=np.int64)
        T = len(parent)
        self.T = T
        self.parent = parent
        self.children = [[] for _ in range(T)]
        for t in range(1, T):
            self.children[parent[t]].append(t)
        self.level = np.zeros(T, dtype=np.int64)
        for t in range(1, T):
            self.level[t] = self.level[parent[t]] + 1
        order = np.argsort(dof_node, kind="stable")
        bounds = np.searchsorted(dof_node[order], np.arange(T + 1))
        self.dofs = [np.sort(order[bounds[t]:bounds[t + 1]]) for t in range(T)]
        self.is_leaf = np.array([len(c) == 0 for c in self.children])
        # D(t): every dof owned by a node in the sub-tree of t
        self.subtree_dofs = [None] * T
        for t in range(T - 1, -1, -1):
            parts = [self.dofs[t]] + [self.subtree_dofs[c] for c in self.children[t]]
            self.subtree_dofs[t] = np.sort(np.concatenate(parts))
        self.leaves = [t for t in range(T) if self.is_leaf[t]]
        self.subtree_leaves = [None] * T
        for t in range(T - 1, -1, -1):
            if self.is_leaf[t]:
                self.subtree_leaves[t] = [t]
            else:
                self.subtree_leaves[t] = sorted(
                    sum((self.subtree_leaves[c] for c in self.children[t]), []))

    def in_subtree(self, s: int, t: int) -> bool:
        """True if s lies in the sub-tree rooted at t."""
        while s != -1:
            if s == t:
                return True
            s = self.parent[s]
        return False


class RSDOracle:
    """RSD preconditioner z = M^{-1} r (Alg. 2) with Alg. 1's interface operator.

    interface: "dense"  -- solve S~_t u = g exactly (Cholesky of the assembled S~_t)
               "gamma"  -- gamma steps of unpreconditioned GMRES from zero (paper mode)
               "hybrid" -- per level of the tree (the internal nodes of one depth):
                           gamma steps where the level's largest interface has more
                           than dense_max dofs, exact solves elsewhere
    coupling:  "full" | "leaf_only"  (see the module docstring)
    """

    def __init__(self, K, parent, dof_node, interface: str = "dense", gamma: int | None = None,
                 coupling: str = "full", dense_max: int | None = None):
        if interface not in ("dense", "gamma", "hybrid"):
            raise ValueError(interface)
        if coupling not in ("full", "leaf_only"):
            raise ValueError(coupling)
        if interface in ("gamma", "hybrid") and (gamma is None or gamma < 1):
            raise ValueError("gamma and hybrid modes need gamma >= 1")
        if interface == "hybrid" and (dense_max is None or dense_max < 0):
            raise ValueError("hybrid mode needs dense_max >= 0")
        self.dense_max = dense_max
        self.K = sp.csr_matrix(K, dtype=np.float64)
        self.n = self.K.shape[0]
        self.interface = interface
        self.gamma = gamma
        self.coupling = coupling
        self.H = Hierarchy(parent, dof_node, self.n)
        H = self.H
        K = self.K
        # Direct solver on each true sub-domain (Section 3.1: exact inversion):
        # Cholesky for a symmetric K, LU with partial pivoting otherwise
        self.symmetric = abs(K - K.T).max() == 0.0
        self.leaf_chol = {}
        for l in H.leaves:
            d = H.dofs[l]
            if d.size:
                self.leaf_chol[l] = self._factor(K[d][:, d].toarray())
        # Per internal node: I, V = D(t) \ I, C_t and the coupling blocks
        self.I = {}
        self.V = {}
        self.C = {}
        self.K_IV = {}
        self.K_II = {}
        self.K_Il = {}
        self.K_lI = {}
        self.S_chol = {}
        for t in range(H.T):
            if H.is_leaf[t]:
                continue
            I = H.dofs[t]
            V = np.setdiff1d(H.subtree_dofs[t], I, assume_unique=True)
            self.I[t], self.V[t] = I, V
            self.K_II[t] = K[I][:, I]
            self.K_IV[t] = K[I][:, V]
            Ct = []
            for l in H.subtree_leaves[t]:
                d = H.dofs[l]
                if d.size == 0 or I.size == 0:
                    continue
                blk = K[I][:, d]
                if blk.nnz:
                    Ct.append(l)
                    self.K_Il[(t, l)] = blk
                    self.K_lI[(l, t)] = K[d][:, I]
            self.C[t] = Ct
        # interface solve of every internal node: exact or gamma inner GMRES steps
        internal = [t for t in range(H.T) if not H.is_leaf[t]]
        largest = {}
        for t in internal:
            d = int(H.level[t])
            largest[d] = max(largest.get(d, 0), self.I[t].size)
        self.inexact = {}
        for t in internal:
            if interface == "hybrid":
                self.inexact[t] = largest[int(H.level[t])] > dense_max
            else:
                self.inexact[t] = interface == "gamma"
            if not self.inexact[t] and self.I[t].size:
                self.S_chol[t] = self._factor(self.schur_dense(t))

    # -- building blocks -------------------------------------------------------------
    def _factor(self, A: np.ndarray):
        if self.symmetric:
            return ("chol", sla.cho_factor(A, lower=True))
        return ("lu", sla.lu_factor(A))

    @staticmethod
    def _solve(f, rhs: np.ndarray) -> np.ndarray:
        kind, fac = f
        return sla.cho_solve(fac, rhs) if kind == "chol" else sla.lu_solve(fac, rhs)

    def leaf_solve(self, l: int, rhs: np.ndarray) -> np.ndarray:
        """K_ll^{-1} rhs by the sub-domain's direct factorisation."""
        if rhs.size == 0:
            return rhs.copy()
        return self._solve(self.leaf_chol[l], rhs)

    def schur_dense(self, t: int) -> np.ndarray:
        """S~_t = K_II - sum_{l in C_t} K_Il K_ll^{-1} K_lI (the operator of Alg. 1).

        Only the columns of K_lI that are non-zero take part in each leaf's
        product; the omitted columns contribute exactly zero.
        """
        S = self.K_II[t].toarray()
        for l in self.C[t]:
            KlI = self.K_lI[(l, t)].tocsc()
            cols = np.unique(KlI.tocoo().col)
            W = self.leaf_solve(l, KlI[:, cols].toarray())       # K_ll^{-1} K_lI (non-zero cols)
            KIl = self.K_Il[(t, l)]
            rows = np.unique(KIl.tocoo().row)
            S[np.ix_(rows, cols)] -= KIl[rows].toarray() @ W
        return S

    def s_matvec(self, t: int, x: np.ndarray) -> np.ndarray:
        """Alg. 1: y = K_II x - sum over C_t of K_Il (K_ll^{-1} (K_lI x))."""
        y = self.K_II[t] @ x
        for l in self.C[t]:
            w = self.leaf_solve(l, self.K_lI[(l, t)] @ x)
            y -= self.K_Il[(t, l)] @ w
        return y

    def inner_gmres(self, t: int, g: np.ndarray, steps: int) -> np.ndarray:
        """`steps` iterations of unpreconditioned GMRES on S~_t u = g from u0 = 0
        (Section 3.1: the interface system is solved only approximately).  Stops
        early only at an exact (happy) breakdown."""
        beta = np.linalg.norm(g)
        if beta == 0.0:
            return np.zeros_like(g)
        m = g.size
        Vb = np.zeros((m, steps + 1))
        Hh = np.zeros((steps + 1, steps))
        Vb[:, 0] = g / beta
        k = 0
        for j in range(steps):
            w = self.s_matvec(t, Vb[:, j])
            for i in range(j + 1):                      # modified Gram-Schmidt
                Hh[i, j] = Vb[:, i] @ w
                w = w - Hh[i, j] * Vb[:, i]
            Hh[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            if Hh[j + 1, j] <= 1e-14 * beta:
                break
            Vb[:, j + 1] = w / Hh[j + 1, j]
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(Hh[:k + 1, :k], e1, rcond=None)
        return Vb[:, :k] @ y

    def interface_solve(self, t: int, g: np.ndarray) -> np.ndarray:
        if g.size == 0:
            return g.copy()
        if not self.inexact[t]:
            return self._solve(self.S_chol[t], g)
        return self.inner_gmres(t, g, self.gamma)

    # -- Alg. 2 ----------------------------------------------------------------------
    def _rsd(self, t: int, f: np.ndarray, v: np.ndarray) -> None:
        """RSD(K_D(t), f_D(t)): writes the approximate solution into v on D(t)."""
        H = self.H
        if H.is_leaf[t]:                                  # h = 0: direct solve
            d = H.dofs[t]
            v[d] = self.leaf_solve(t, f[d])
            return
        for c in H.children[t]:                           # recursion on every child
            self._rsd(c, f, v)
        I, V = self.I[t], self.V[t]
        if self.coupling == "full":                       # g of eq. (schur)
            g = f[I] - self.K_IV[t] @ v[V]
        else:
            g = f[I].copy()
            for l in self.C[t]:
                g -= self.K_Il[(t, l)] @ v[H.dofs[l]]
        u = self.interface_solve(t, g)                    # S u_I = g, approximately
        for l in self.C[t]:                               # eq. (backSub) on C_t only
            d = H.dofs[l]
            v[d] -= self.leaf_solve(l, self.K_lI[(l, t)] @ u)
        v[I] = u

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = M^{-1} r for one vector or for each column of a 2-D array."""
        r = np.asarray(r, dtype=np.float64)
        if r.ndim == 2:
            return np.stack([self.apply(r[:, j]) for j in range(r.shape[1])], axis=1)
        v = np.zeros(self.n)
        self._rsd(0, r, v)
        return v

    def dense(self) -> np.ndarray:
        """M^{-1} as a dense matrix (apply to the unit vectors; tiny systems only)."""
        return self.apply(np.eye(self.n))


def exact_block_solve(K, parent, dof_node, f: np.ndarray) -> np.ndarray:
    """Nested dissection without approximation: the same tree walk as RSD, but
    with the exact pseudo sub-domain inverses in all three places where the
    paper needs them (Section 3.2).  Equals K^{-1} f; used to pin the tree
    plumbing (D(t), children, interface sets).  f may hold several columns."""
    K = sp.csr_matrix(K, dtype=np.float64)
    H = Hierarchy(parent, dof_node, K.shape[0])

    def solve(t, rhs):
        # solve K[D(t), D(t)] X = rhs (rows of rhs follow the sorted D(t))
        dofs = H.subtree_dofs[t]
        if H.is_leaf[t]:
            return np.linalg.solve(K[dofs][:, dofs].toarray(), rhs) if dofs.size else rhs.copy()
        I = H.dofs[t]
        V = np.setdiff1d(dofs, I, assume_unique=True)
        iI = np.searchsorted(dofs, I)
        iV = np.searchsorted(dofs, V)

        def solve_V(B):
            # K_VV is block diagonal over the children: sub-trees are not coupled
            out = np.zeros_like(B)
            for c in H.children[t]:
                ic = np.searchsorted(V, H.subtree_dofs[c])
                out[ic] = solve(c, B[ic])
            return out

        y = solve_V(rhs[iV])
        if I.size:
            Z = solve_V(K[V][:, I].toarray())               # K_VV^{-1} K_VI
            K_IV = K[I][:, V].toarray()
            S = K[I][:, I].toarray() - K_IV @ Z              # exact Schur complement
            uI = np.linalg.solve(S, rhs[iI] - K_IV @ y)
            y = y - Z @ uI
        else:
            uI = np.zeros((0,) + rhs.shape[1:])
        x = np.zeros_like(rhs)
        x[iV] = y
        x[iI] = uI
        return x

    f = np.asarray(f, dtype=np.float64)
    return solve(0, f)
