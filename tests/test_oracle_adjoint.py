"""Pins of the oracle's adjoint gradient (no GPU).

The gradient formula (dL/dtheta_e = -k'(theta_e) lambda_e^T K_e x_e, dL/db = lambda) is
checked against central finite differences of the loss, each loss value computed by
an independent direct solve -- a dropped coefficient derivative, a sign error or a
transposed element product fails these.  The oracle's assembly is checked against
the generator's own Q1 assembly (a separate construction from the same mesh).
"""
import numpy as np

from oracle import adjoint as A
from workloads import diffusion_fe_map, diffusion_problem


def _setup(ne=4, seed=3, sigma=0.5):
    p = diffusion_problem(ne, 1, sigma, seed)
    fe = diffusion_fe_map(p)
    rng = np.random.default_rng(seed + 100)
    xt = rng.uniform(-1, 1, p.n)
    return p, fe, xt


def test_assembly_matches_generator():
    p, fe, _ = _setup(ne=6)
    K = A.assemble(fe, p.meta["theta"], p.n)
    D = (K - p.K).tocoo()
    assert np.abs(D.data).max() <= 1e-14 * np.abs(p.K.data).max()


def test_theta_gradient_matches_central_differences():
    p, fe, xt = _setup()
    th = p.meta["theta"]
    b = p.b[:, 0]
    L, x, g, lam = A.solve_loss_grad(fe, th, b, xt)
    eps = 1e-6
    for e in range(th.size):                    # every element of the 4^3 mesh
        d = np.zeros_like(th)
        d[e] = eps
        Lp = A.solve_loss_grad(fe, th + d, b, xt)[0]
        Lm = A.solve_loss_grad(fe, th - d, b, xt)[0]
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g[e]) <= 1e-6 * np.abs(g).max() + 1e-12, (e, fd, g[e])


def test_b_gradient_matches_central_differences():
    p, fe, xt = _setup(ne=4, seed=5)
    th = p.meta["theta"]
    b = p.b[:, 0]
    _, _, _, lam = A.solve_loss_grad(fe, th, b, xt)
    rng = np.random.default_rng(1)
    eps = 1e-6
    for _ in range(5):
        d = rng.standard_normal(b.size)
        fd = (A.solve_loss_grad(fe, th, b + eps * d, xt)[0]
              - A.solve_loss_grad(fe, th, b - eps * d, xt)[0]) / (2 * eps)
        assert abs(fd - lam @ d) <= 1e-7 * abs(lam @ d) + 1e-10


def test_linear_coefficient_kind():
    """k = theta: the gradient is -lambda_e^T K_e x_e (no exp factor)."""
    p, fe, xt = _setup(ne=3, seed=2)
    th = 1.0 + 0.3 * np.random.default_rng(0).random(p.meta["theta"].size)
    b = p.b[:, 0]
    L, x, g, lam = A.solve_loss_grad(fe, th, b, xt, kind=A.LINEAR)
    eps = 1e-6
    for e in range(0, th.size, 3):
        d = np.zeros_like(th)
        d[e] = eps
        fd = (A.solve_loss_grad(fe, th + d, b, xt, kind=A.LINEAR)[0]
              - A.solve_loss_grad(fe, th - d, b, xt, kind=A.LINEAR)[0]) / (2 * eps)
        assert abs(fd - g[e]) <= 1e-6 * np.abs(g).max() + 1e-12


def test_planted_sign_error_is_caught():
    """A gradient with the wrong sign disagrees with the differences."""
    p, fe, xt = _setup(ne=3, seed=4)
    th = p.meta["theta"]
    b = p.b[:, 0]
    L, x, g, lam = A.solve_loss_grad(fe, th, b, xt)
    e = int(np.argmax(np.abs(g)))
    d = np.zeros_like(th)
    d[e] = 1e-6
    fd = (A.solve_loss_grad(fe, th + d, b, xt)[0] - A.solve_loss_grad(fe, th - d, b, xt)[0]) / 2e-6
    assert abs(fd - g[e]) < 1e-6 * abs(g[e])
    assert abs(fd + g[e]) > 0.5 * abs(g[e])
