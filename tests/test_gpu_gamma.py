"""GPU parity of the inexact interface solves (the paper's mode, Section 3.1 and
Section 4): gamma steps of unpreconditioned GMRES from zero on every interface system.

The HIP path runs the inner GMRES on the assembled S~_t, which is the operator of
Alg. 1; the oracle applies Alg. 1 matrix-free.  The two differ by rounding only, and
the inner GMRES result is a smooth function of g away from breakdown, so the apply bar
is 1e-8 relative (max norm).  Pins on the GPU path itself:
  * gamma >= dim(S~_t) gives back the exact interface solves (dense mode) to 1e-10;
  * the hybrid mode equals the pure modes bitwise when dense_max puts every level on
    one side, and the oracle's per-level mode (same level rule) to 1e-8 otherwise;
  * the outer FGMRES iteration counts of the paper's Table 1 (Poisson) and Table 10
    (Navier-Lame) strips -- the fixtures the oracle is pinned to -- within +-2, and
    within +-1 of the oracle's own count, with the solution to 1e-8 of the
    manufactured one;
  * several right-hand sides: each column bitwise equal to its solo apply.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import RSDOracle, fgmres  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _log(msg):
    print(msg, flush=True)


def _handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    return RSD(rp, ci, v, p.parent, p.dof_node, **kw)


def _vec(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _cm(a):
    return torch.as_tensor(np.ascontiguousarray(a.T)).cuda().t()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


APPLY_CASES = [  # (cache key, gamma)
    (("strip", 17, 8, "poisson", 0), 2),
    (("strip", 17, 8, "poisson", 0), 8),
    (("strip", 33, 8, "poisson", 0), 4),
    (("strip", 17, 8, "navier_lame", 0), 4),
    (("strip", 17, 128, "poisson", 0), 4),
    (("diffusion", 13, 2, 1.0, 2), 3),
    (("diffusion", 9, 3, 0.0, 4), 5),
]


@pytest.mark.parametrize("key,gamma", APPLY_CASES)
def test_gamma_apply_matches_oracle(problem_cache, key, gamma):
    _log(f"gamma apply {key} gamma={gamma}")
    p = problem_cache(*key)
    o = RSDOracle(p.K, p.parent, p.dof_node, interface="gamma", gamma=gamma)
    r = np.random.default_rng(31).uniform(-1, 1, p.n)
    zo = o.apply(r)
    h = _handle(p, interface="gamma", gamma=gamma)
    z = h.apply(_vec(r)).cpu().numpy()
    assert _rel(z, zo) <= 1e-8, _rel(z, zo)
    h.close()


def test_gamma_at_dimension_is_exact(problem_cache):
    """Strip of 9 x 9 node sub-domains: interfaces of 7 dofs, gamma = 8 >= dim(S~)."""
    p = problem_cache("strip", 9, 8, "poisson", 0)
    r = np.random.default_rng(5).uniform(-1, 1, p.n)
    hd = _handle(p)
    hg = _handle(p, interface="gamma", gamma=8)
    zd = hd.apply(_vec(r)).cpu().numpy()
    zg = hg.apply(_vec(r)).cpu().numpy()
    assert _rel(zg, zd) <= 1e-10, _rel(zg, zd)
    hd.close()
    hg.close()


def test_hybrid_mode_selects_levels(problem_cache):
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    rh = np.random.default_rng(8).uniform(-1, 1, p.n)
    r = _vec(rh)
    z = {}
    for name, kw in (("dense", {}), ("gamma", dict(interface="gamma", gamma=3)),
                     ("hyb_all_dense", dict(interface="hybrid", gamma=3, dense_max=10 ** 6)),
                     ("hyb_all_gamma", dict(interface="hybrid", gamma=3, dense_max=0)),
                     ("hyb_root_gamma", dict(interface="hybrid", gamma=3, dense_max=200))):
        h = _handle(p, **kw)
        z[name] = h.apply(r).cpu().numpy()
        h.close()
    assert np.array_equal(z["hyb_all_dense"], z["dense"])
    assert np.array_equal(z["hyb_all_gamma"], z["gamma"])
    o = RSDOracle(p.K, p.parent, p.dof_node)
    assert _rel(z["dense"], o.apply(rh)) <= 1e-10
    # root interface (397 dofs) inexact, level-1 interfaces (61-91 dofs) exact: the
    # oracle's per-level mode with the same rule
    oh = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=3, dense_max=200)
    assert oh.inexact[0] and not any(oh.inexact[t] for t in oh.inexact if t != 0)
    assert _rel(z["hyb_root_gamma"], oh.apply(rh)) <= 1e-8, _rel(z["hyb_root_gamma"], oh.apply(rh))


HYBRID_CASES = [  # (problem, gamma, dense_max, coupling): a mix of exact and inexact levels
    (("diffusion_binary", 12, 3, 1.0, 3), 4, 30, "full"),       # levels 0-1 gamma, 2 exact
    (("diffusion_binary", 12, 3, 1.0, 3), 4, 30, "leaf_only"),
    (("diffusion_binary", 12, 4, 0.5, 1), 3, 60, "full"),       # root gamma, levels 1-3 exact
    (("diffusion", 17, 2, 1.0, 4), 5, 500, "full"),             # root of 721 dofs inexact
]


@pytest.mark.parametrize("key,gamma,dense_max,coupling", HYBRID_CASES)
def test_hybrid_apply_matches_oracle(problem_cache, key, gamma, dense_max, coupling):
    _log(f"hybrid apply {key} gamma={gamma} dense_max={dense_max} {coupling}")
    p = problem_cache(*key)
    o = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=gamma,
                  dense_max=dense_max, coupling=coupling)
    assert any(o.inexact.values()) and not all(o.inexact.values())
    R = np.random.default_rng(19).uniform(-1, 1, size=(p.n, 3))
    h = _handle(p, interface="hybrid", gamma=gamma, dense_max=dense_max, coupling=coupling)
    Z = h.apply(_cm(R)).cpu().numpy()
    for j in range(3):
        zo = o.apply(R[:, j])
        assert _rel(Z[:, j], zo) <= 1e-8, (j, _rel(Z[:, j], zo))
    h.close()


@pytest.mark.parametrize("key,gamma", [(("skew", 13, 2, 0.3, 1), 4),
                                       (("skew_binary", 12, 3, 0.3, 5), 3)])
def test_nonsymmetric_3d_gamma_matches_oracle(problem_cache, key, gamma):
    """A non-symmetric K in 3-D (Poisson plus a random antisymmetric part on its
    pattern): general sub-domain inverses and gamma inner steps at every level, against
    the oracle's LU path."""
    _log(f"non-symmetric 3-D gamma {key}")
    p = problem_cache(*key)
    o = RSDOracle(p.K, p.parent, p.dof_node, interface="gamma", gamma=gamma)
    assert not o.symmetric
    r = np.random.default_rng(23).uniform(-1, 1, p.n)
    h = _handle(p, interface="gamma", gamma=gamma, symmetric=False)
    z = h.apply(_vec(r)).cpu().numpy()
    assert _rel(z, o.apply(r)) <= 1e-8, _rel(z, o.apply(r))
    x, st, info = h.solve(_vec(p.b[:, 0]), rtol=1e-10)
    x = x.cpu().numpy()
    assert st == 0
    assert np.linalg.norm(p.b[:, 0] - p.K @ x) <= 1e-10 * np.linalg.norm(p.b[:, 0])
    h.close()


def _golden_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_outer_iterations.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                prob, N, P, g, beta = line.split()
                rows.append((prob, int(N), int(P), int(g), int(beta)))
    return rows


@pytest.mark.parametrize("prob,N,P,gamma,beta", _golden_rows())
def test_paper_outer_iteration_counts_on_gpu(problem_cache, prob, N, P, gamma, beta):
    _log(f"paper table {prob} N={N} P={P} gamma={gamma}")
    s = problem_cache("strip", N, P, prob, 0)
    b = s.b[:, 0]
    o = RSDOracle(s.K, s.parent, s.dof_node, interface="gamma", gamma=gamma)
    _, io = fgmres(s.K, b, o.apply, rtol=1e-12, restart=30, maxit=500)
    h = _handle(s, interface="gamma", gamma=gamma)
    x, st, info = h.solve(_vec(b), rtol=1e-12, restart=30, maxit=500)
    x = x.cpu().numpy()
    its = info[0]["iterations"]
    assert st == 0
    assert abs(its - beta) <= 2, (its, beta)
    assert abs(its - io["iterations"]) <= 1, (its, io["iterations"])
    assert np.linalg.norm(b - s.K @ x) <= 1e-12 * np.linalg.norm(b)
    assert _rel(x, s.meta["x_true"]) < 1e-8
    h.close()


def test_gamma_multi_rhs_columns_bitwise(problem_cache):
    p = problem_cache("strip", 17, 8, "navier_lame", 0)
    h = _handle(p, interface="gamma", gamma=4)
    R = np.random.default_rng(12).uniform(-1, 1, size=(p.n, 6))
    R[:, 2] = 0.0                               # g = 0 on every interface: u = 0
    Z = h.apply(_cm(R)).cpu().numpy()
    for j in range(6):
        assert np.array_equal(Z[:, j], h.apply(_vec(R[:, j])).cpu().numpy()), j
    assert np.all(Z[:, 2] == 0.0)
    X, st, info = h.solve(_cm(R[:, :3]), rtol=1e-10)
    for j in range(3):
        xj, _, ij = h.solve(_vec(R[:, j]), rtol=1e-10)
        assert ij[0] == info[j] and np.array_equal(X.cpu().numpy()[:, j], xj.cpu().numpy())
    h.close()


def test_gamma_chunked_large_interface():
    """Root interface of 5,256 dofs (elasticity 24^3, octree of height 1, uneven cuts):
    above one work chunk (4,096 rows), so the inner GMRES runs on the chunked kernels
    (classical Gram-Schmidt twice, two-pass sums).  Apply vs the oracle's gamma mode to
    1e-8, several right-hand sides bitwise, and a hybrid solve to 1e-10."""
    from workloads import elasticity_problem
    _log("gamma chunked elasticity 24^3 h=1")
    p = elasticity_problem(24, 1, 2, nrhs=3)
    o = RSDOracle(p.K, p.parent, p.dof_node, interface="gamma", gamma=6)
    R = np.random.default_rng(17).uniform(-1, 1, size=(p.n, 3))
    h = _handle(p, interface="gamma", gamma=6)
    Z = h.apply(_cm(R)).cpu().numpy()
    zo = o.apply(R[:, 0])
    assert _rel(Z[:, 0], zo) <= 1e-8, _rel(Z[:, 0], zo)
    for j in range(3):
        assert np.array_equal(Z[:, j], h.apply(_vec(R[:, j])).cpu().numpy()), j
    h.close()
    h = _handle(p, interface="hybrid", gamma=6, dense_max=4000,
                leaf_prec="fp32", sigma_prec="fp32", iface_prec="fp32")
    X, st, info = h.solve(_cm(p.b), rtol=1e-10)
    assert st == 0
    X = X.cpu().numpy()
    for j in range(3):
        assert np.linalg.norm(p.b[:, j] - p.K @ X[:, j]) <= 1e-10 * np.linalg.norm(p.b[:, j])
    h.close()
