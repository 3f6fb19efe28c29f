"""TEST INFRASTRUCTURE ONLY -- the FP64 reference for differentiable RSD solves.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use this module;
it shares no code with the HIP library.

Definitions (the adjoint method for x = K(theta)^{-1} b with K = sum_e k(theta_e) K_e,
the per-element coefficient of the Q1 model problems of Section 4):
  * assemble(fe, theta): K(theta) written out from the element map;
  * loss L = 1/2 ||x - x_target||^2;
  * lambda = K^{-T} (x - x_target);  dL/db = lambda;
    dL/dtheta_e = -k'(theta_e) lambda_e^T K_e x_e   (differentiating K x = b).
Solves are direct (scipy's sparse LU), i.e. the exact x and lambda.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

LINEAR, EXP = 0, 1


def coef(theta: np.ndarray, kind: int = EXP) -> np.ndarray:
    return np.exp(theta) if kind == EXP else np.asarray(theta, dtype=np.float64)


def dcoef(theta: np.ndarray, kind: int = EXP) -> np.ndarray:
    return np.exp(theta) if kind == EXP else np.ones_like(theta, dtype=np.float64)


def assemble(fe: dict, theta: np.ndarray, n: int, kind: int = EXP) -> sp.csr_matrix:
    """K(theta) = sum_e k(theta_e) ke scattered by the element dof lists."""
    dofs = fe["elem_dofs"].astype(np.int64)
    ke = fe["ke"]
    E, d = dofs.shape
    rows = np.repeat(dofs, d, axis=1)              # (E, d*d): row a for entry (a, b)
    cols = np.tile(dofs, (1, d))                   # column b
    vals = coef(theta, kind)[:, None] * ke.ravel()[None, :]
    keep = (rows >= 0) & (cols >= 0)
    K = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def element_gradient(fe: dict, theta: np.ndarray, lam: np.ndarray, x: np.ndarray,
                     kind: int = EXP) -> np.ndarray:
    """dL/dtheta_e = -k'(theta_e) lambda_e^T ke x_e (zero on eliminated dofs)."""
    dofs = fe["elem_dofs"].astype(np.int64)
    lam_e = np.where(dofs >= 0, lam[np.maximum(dofs, 0)], 0.0)
    x_e = np.where(dofs >= 0, x[np.maximum(dofs, 0)], 0.0)
    return -dcoef(theta, kind) * np.einsum("ea,ab,eb->e", lam_e, fe["ke"], x_e)


def solve_loss_grad(fe: dict, theta: np.ndarray, b: np.ndarray, x_target: np.ndarray,
                    kind: int = EXP):
    """(L, x, dL/dtheta, dL/db) with exact solves."""
    n = b.shape[0]
    K = assemble(fe, theta, n, kind).tocsc()
    x = spla.spsolve(K, b)
    r = x - x_target
    lam = spla.spsolve(K.T.tocsc(), r)
    return 0.5 * float(r @ r), x, element_gradient(fe, theta, lam, x, kind), lam
