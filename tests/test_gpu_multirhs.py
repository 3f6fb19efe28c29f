"""Several right-hand sides at once, through the C ABI.

The apply and the SpMV read the factors and K once per group of vectors, and FGMRES
advances up to eight right-hand sides in lockstep (one host wait per iteration for the
group).  Each column's arithmetic is the one it has alone, so the bar is bitwise
equality with one-column calls, for every column position, group size (1 .. 11, two
groups past eight) and precision; columns that stop early (b = 0, NaN in b, different
convergence speed) leave the others untouched.  The first column of each block is also
checked against the FP64 oracle (1e-10 for FP64 factors, 2e-4 for FP32 factors, as in
the single-vector parity tests).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import RSDOracle  # noqa: E402
from workloads import elasticity_problem  # noqa: E402

pytestmark = pytest.mark.gpu

FP32 = dict(leaf_prec="fp32", sigma_prec="fp32", iface_prec="fp32")
CASES = [  # (name, problem key, handle options, oracle bar)
    ("diffusion13-fp64", ("diffusion", 13, 2, 1.0, 2), {}, 1e-10),
    ("diffusion20-fp32", ("diffusion", 20, 2, 1.0, 5), FP32, 2e-4),
    ("elasticity8-fp32", ("elasticity", 8, 2, 1), FP32, 2e-4),
    ("diffusion20-bf16", ("diffusion", 20, 2, 1.0, 5), dict(leaf_prec="bf16"), 1e-1),
]


def _log(msg):
    print(msg, flush=True)


def _problem(problem_cache, key):
    if key[0] == "elasticity":
        return elasticity_problem(key[1], key[2], key[3], nrhs=2)
    return problem_cache(*key)


def _handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    return RSD(rp, ci, v, p.parent, p.dof_node, **kw)


def _cm(a):
    """column-major device copy of an (n, k) array"""
    return torch.as_tensor(np.ascontiguousarray(a.T)).cuda().t()


def _vec(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,key,opts,bar", CASES)
def test_apply_and_spmv_columns_bitwise(problem_cache, name, key, opts, bar):
    _log(f"multi apply {name}")
    p = _problem(problem_cache, key)
    h = _handle(p, **opts)
    R = np.random.default_rng(21).uniform(-1, 1, size=(p.n, 11))
    for k in (11, 3, 2):
        Z = h.apply(_cm(R[:, :k])).cpu().numpy()
        Y = h.spmv(_cm(R[:, :k])).cpu().numpy()
        for j in range(k):
            assert np.array_equal(Z[:, j], h.apply(_vec(R[:, j])).cpu().numpy()), (k, j)
            assert np.array_equal(Y[:, j], h.spmv(_vec(R[:, j])).cpu().numpy()), (k, j)
    zo = RSDOracle(p.K, p.parent, p.dof_node).apply(R[:, 0])
    assert np.abs(Z[:, 0] - zo).max() <= bar * np.abs(zo).max()
    h.close()


@pytest.mark.parametrize("name,key,opts,bar", CASES)
def test_lockstep_fgmres_columns_bitwise(problem_cache, name, key, opts, bar):
    _log(f"lockstep fgmres {name}")
    p = _problem(problem_cache, key)
    h = _handle(p, **opts)
    rng = np.random.default_rng(4)
    B = rng.uniform(-1, 1, size=(p.n, 10))
    B[:, 1] *= 1e3                 # other scale
    B[:, 3] = 0.0                  # stops at once, inside the active range
    B[:, 5] = p.K @ np.ones(p.n)   # smooth: converges at another iteration
    X, st, info = h.solve(_cm(B), rtol=1e-10, restart=30)
    X = X.cpu().numpy()
    assert st == 0
    assert info[3]["iterations"] == 0 and np.all(X[:, 3] == 0.0)
    for j in range(10):
        xj, stj, ij = h.solve(_vec(B[:, j]), rtol=1e-10, restart=30)
        assert stj == 0 and ij[0] == info[j], (j, ij[0], info[j])
        assert np.array_equal(X[:, j], xj.cpu().numpy()), j
        nb = np.linalg.norm(B[:, j])
        if nb > 0:
            assert np.linalg.norm(B[:, j] - p.K @ X[:, j]) <= 1e-10 * nb
    h.close()


def test_lockstep_breakdown_and_maxit_columns(problem_cache):
    _log("lockstep breakdown / maxit")
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    h = _handle(p)
    B = np.random.default_rng(6).uniform(-1, 1, size=(p.n, 4))
    B[7, 1] = np.nan
    X, st, info = h.solve(_cm(B), rtol=1e-10, restart=30)
    X = X.cpu().numpy()
    assert st == 5 and info[1]["status"] == 5
    for j in (0, 2, 3):
        xj, stj, ij = h.solve(_vec(B[:, j]), rtol=1e-10, restart=30)
        assert info[j]["status"] == 0 and ij[0] == info[j]
        assert np.array_equal(X[:, j], xj.cpu().numpy())
    # maxit inside the first restart cycle and across a restart
    for maxit, restart in ((3, 30), (7, 4)):
        B2 = np.delete(B, 1, axis=1)
        X2, st2, info2 = h.solve(_cm(B2), rtol=1e-14, restart=restart, maxit=maxit)
        assert st2 == 4
        for j in range(3):
            assert info2[j]["status"] == 4 and info2[j]["iterations"] == maxit
            xj, _, ij = h.solve(_vec(B2[:, j]), rtol=1e-14, restart=restart, maxit=maxit)
            assert ij[0] == info2[j] and np.array_equal(X2.cpu().numpy()[:, j], xj.cpu().numpy())
    h.close()
