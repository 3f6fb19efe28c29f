"""Plain FP64 Krylov solvers for the oracle (TEST INFRASTRUCTURE ONLY).

The paper solves K u = f with GMRES preconditioned by RSD, from a zero initial
guess, to a relative 2-norm residual tolerance (Section 3 and Section 4).
Because the paper-mode preconditioner (gamma inner GMRES steps) is a
non-linear map, and the exact-interface preconditioner is non-symmetric once
the tree has two or more interface levels, the outer method here is the
right-preconditioned flexible GMRES(m) (Saad, Iterative Methods for Sparse
Linear Systems, 2nd ed., Alg. 9.6), with modified Gram-Schmidt and Givens
rotations.  Preconditioned CG (Saad, Alg. 9.1) is provided for the
symmetric positive definite case (one interface level with exact interface
solves, where M^{-1} = K^{-1}).

Convergence is decided on the true residual ||b - K x||_2 <= rtol ||b||_2:
the recurrence estimate only triggers a check, which is then confirmed with
an explicit residual (restarting when the check fails).
"""
from __future__ import annotations

import numpy as np


def fgmres(K, b: np.ndarray, apply_M, rtol: float = 1e-10, restart: int = 30,
           maxit: int = 1000, x0: np.ndarray | None = None):
    """Right-preconditioned flexible GMRES(restart).  Returns (x, info) with
    info = {iterations, relres, converged, history} (history: estimated
    relative residual after every Arnoldi step)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), dict(iterations=0, relres=0.0, converged=True, history=[])
    tol = rtol * bnorm
    its = 0
    history = []
    r = b - K @ x
    beta = np.linalg.norm(r)
    while True:
        if beta <= tol:
            return x, dict(iterations=its, relres=beta / bnorm, converged=True, history=history)
        if its >= maxit:
            return x, dict(iterations=its, relres=beta / bnorm, converged=False, history=history)
        V = np.zeros((n, restart + 1))
        Z = np.zeros((n, restart))
        Hh = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        s = np.zeros(restart + 1)
        V[:, 0] = r / beta
        s[0] = beta
        k = 0
        for j in range(restart):
            Z[:, j] = apply_M(V[:, j])
            w = K @ Z[:, j]
            for i in range(j + 1):
                Hh[i, j] = V[:, i] @ w
                w = w - Hh[i, j] * V[:, i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] > 0.0:
                V[:, j + 1] = w / Hh[j + 1, j]
            for i in range(j):                                  # previous rotations
                tmp = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = tmp
            den = np.hypot(Hh[j, j], Hh[j + 1, j])
            cs[j] = Hh[j, j] / den
            sn[j] = Hh[j + 1, j] / den
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            s[j + 1] = -sn[j] * s[j]
            s[j] = cs[j] * s[j]
            its += 1
            k = j + 1
            history.append(abs(s[j + 1]) / bnorm)
            if abs(s[j + 1]) <= tol or its >= maxit:
                break
        y = np.linalg.solve(np.triu(Hh[:k, :k]), s[:k])
        x = x + Z[:, :k] @ y
        r = b - K @ x
        beta = np.linalg.norm(r)


def pcg(K, b: np.ndarray, apply_M, rtol: float = 1e-10, maxit: int = 1000):
    """Preconditioned conjugate gradients from x0 = 0.  Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, dict(iterations=0, relres=0.0, converged=True, history=[])
    tol = rtol * bnorm
    r = b.copy()
    z = apply_M(r)
    p = z.copy()
    rz = r @ z
    history = []
    its = 0
    while its < maxit:
        q = K @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        its += 1
        rn = np.linalg.norm(r)
        history.append(rn / bnorm)
        if rn <= tol:
            rt = np.linalg.norm(b - K @ x)
            if rt <= tol:
                return x, dict(iterations=its, relres=rt / bnorm, converged=True, history=history)
            r = b - K @ x                                       # replace the drifted residual
        z = apply_M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    rt = np.linalg.norm(b - K @ x)
    return x, dict(iterations=its, relres=rt / bnorm, converged=rt <= tol, history=history)
