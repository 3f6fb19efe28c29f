"""Independent dense constructions of the RSD preconditioner, for the oracle's pins.

Test infrastructure: written from the block algebra, not from the oracle's recursion,
and sharing no code with it or with the HIP library.

Order the dofs as [Lambda (leaf interiors); B (skeleton: every interface, deepest tree
level first)] and write K = [[A, C], [R, E]], A = blockdiag(K_ll).  With
Shat = E - R A^{-1} C (the skeleton Schur complement), the recursion of Alg. 2 is:

  1. y = A^{-1} r_Lambda and q = r_B - R y (static condensation);
  2. for every interface s, deepest first, u_s = solve_s(g_s) with
       g_s = q_s - sum over t below s of X_st u_t,
     where X_st = Shat_st for the full right-hand side of the interface systems and
     X_st = Shat_st - E_st = -(R A^{-1} C)_st for the leaf-only one (the couplings of
     I_s to the interiors of the leaves only, the strip formula of Alg. 2 taken
     literally), and solve_s is either the exact solve with Shat_ss (= S~_s, the
     operator of Alg. 1) or gamma steps of GMRES from zero on it (Section 3.1);
  3. z_Lambda = A^{-1} (r_Lambda - C u_B) (harmonic extension).

With exact interface solves step 2 is a block forward substitution with the block
lower-triangular matrix T (T_ss = Shat_ss, T_st = X_st), so

  M^{-1} = [[I, -A^{-1} C], [0, I]] diag(A^{-1}, T^{-1}) [[I, 0], [-R A^{-1}, I]].

GMRES with gamma steps from zero returns, by its definition, the vector of the Krylov
space span{g, S g, ..., S^{gamma-1} g} with the smallest residual ||g - S u||; here it is
computed from an orthonormal basis of that space (Householder QR of the normalised
power basis) and a least-squares solve, not by the Arnoldi process.
"""
from __future__ import annotations

import numpy as np


class SkeletonForm:
    """The dense blocks above for one (K, tree) pair (small systems only)."""

    def __init__(self, K, parent, dof_node):
        Kd = K.toarray() if hasattr(K, "toarray") else np.asarray(K, dtype=np.float64)
        parent = np.asarray(parent, dtype=np.int64)
        dof_node = np.asarray(dof_node, dtype=np.int64)
        T = len(parent)
        children = [[] for _ in range(T)]
        for t in range(1, T):
            children[parent[t]].append(t)
        depth = np.zeros(T, dtype=np.int64)
        for t in range(1, T):
            depth[t] = depth[parent[t]] + 1
        self.parent = parent
        leaves = [t for t in range(T) if not children[t]]
        internal = sorted([t for t in range(T) if children[t]], key=lambda t: (-depth[t], t))
        self.internal = internal
        self.depth = depth
        own = [np.nonzero(dof_node == t)[0] for t in range(T)]
        lam = np.concatenate([own[t] for t in leaves]) if leaves else np.zeros(0, np.int64)
        blocks = [own[t] for t in internal]
        skel = np.concatenate(blocks) if blocks else np.zeros(0, np.int64)
        self.lam, self.skel = lam, skel
        self.n, self.nl, self.ns = Kd.shape[0], len(lam), len(skel)
        off = np.cumsum([0] + [len(b) for b in blocks])
        self.blk = {t: slice(off[a], off[a + 1]) for a, t in enumerate(internal)}
        self.A = Kd[np.ix_(lam, lam)]
        self.C = Kd[np.ix_(lam, skel)]
        self.R = Kd[np.ix_(skel, lam)]
        self.E = Kd[np.ix_(skel, skel)]
        self.Ainv = np.linalg.inv(self.A) if self.nl else np.zeros((0, 0))
        self.RAC = self.R @ self.Ainv @ self.C
        self.Shat = self.E - self.RAC

    def below(self, s: int, t: int) -> bool:
        """True if t lies strictly inside the sub-tree of s."""
        if t == s:
            return False
        while t != -1:
            if t == s:
                return True
            t = int(self.parent[t])
        return False

    def coupling_block(self, s: int, t: int, coupling: str) -> np.ndarray:
        bs, bt = self.blk[s], self.blk[t]
        if coupling == "full":
            return self.Shat[bs, bt]
        if coupling == "leaf_only":
            return -self.RAC[bs, bt]
        raise ValueError(coupling)

    # -- exact interface solves: the explicit dense form -----------------------------
    def dense_form(self, coupling: str = "full") -> np.ndarray:
        """M^{-1} in the caller's dof order."""
        Tm = np.zeros_like(self.Shat)
        for s in self.internal:
            for t in self.internal:
                if t == s:
                    Tm[self.blk[s], self.blk[s]] = self.Shat[self.blk[s], self.blk[s]]
                elif self.below(s, t):
                    Tm[self.blk[s], self.blk[t]] = self.coupling_block(s, t, coupling)
        nl, ns = self.nl, self.ns
        Ai = self.Ainv
        L = np.block([[np.eye(nl), np.zeros((nl, ns))], [-self.R @ Ai, np.eye(ns)]])
        U = np.block([[np.eye(nl), -Ai @ self.C], [np.zeros((ns, nl)), np.eye(ns)]])
        D = np.block([[Ai, np.zeros((nl, ns))], [np.zeros((ns, nl)), np.linalg.inv(Tm)]])
        Mp = U @ D @ L
        perm = np.concatenate([self.lam, self.skel])
        M = np.zeros_like(Mp)
        M[np.ix_(perm, perm)] = Mp
        return M

    # -- any mix of exact and inexact interface solves: the sweep itself -------------
    def sweep_apply(self, r: np.ndarray, inexact: dict, gamma: int | None = None,
                    coupling: str = "full") -> np.ndarray:
        """z = M^{-1} r with node s solved by gamma GMRES steps where inexact[s]."""
        r = np.asarray(r, dtype=np.float64)
        rl, rb = r[self.lam], r[self.skel]
        q = rb - self.R @ (self.Ainv @ rl)
        u = np.zeros(self.ns)
        for s in self.internal:                        # deepest level first
            bs = self.blk[s]
            g = q[bs].copy()
            for t in self.internal:
                if self.below(s, t):
                    g -= self.coupling_block(s, t, coupling) @ u[self.blk[t]]
            S = self.Shat[bs, bs]
            if g.size == 0:
                continue
            u[bs] = minimal_residual(S, g, gamma) if inexact[s] else np.linalg.solve(S, g)
        z = np.zeros(self.n)
        z[self.lam] = self.Ainv @ (rl - self.C @ u)
        z[self.skel] = u
        return z

    def level_choice(self, dense_max: int) -> dict:
        """The hybrid rule: a level (internal nodes of one depth) is solved inexactly
        when its largest interface has more than dense_max dofs."""
        big = {}
        for t in self.internal:
            d = int(self.depth[t])
            big[d] = max(big.get(d, 0), self.blk[t].stop - self.blk[t].start)
        return {t: big[int(self.depth[t])] > dense_max for t in self.internal}


def minimal_residual(S: np.ndarray, g: np.ndarray, steps: int) -> np.ndarray:
    """argmin ||g - S u|| over u in span{g, S g, ..., S^{steps-1} g} (steps < dim)."""
    beta = np.linalg.norm(g)
    if beta == 0.0:
        return np.zeros_like(g)
    cols, v = [], g / beta
    for _ in range(steps):
        cols.append(v)
        v = S @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(np.column_stack(cols))
    y, *_ = np.linalg.lstsq(S @ Q, g, rcond=None)
    return Q @ y
