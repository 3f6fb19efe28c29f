"""GPU parity at the tree shape of the 256^3 Poisson workload, at the largest size the
FP64 oracle follows in about a minute: Poisson on 64^3 Q1 hexahedra with an octree of
height 3, i.e. the same sub-domains of 8^3 elements (512 x 343 interior dofs), level-2
interfaces of 631 dofs (64), level-1 interfaces of 2,791 (8) and a root of 11,719 --
the four deepest levels of the 256^3 tree (Alg. 2 recursion, Section 3.2).

* FP64, exact interface solves: the whole apply vector against the oracle to 1e-10.
* FP64, per-level mode with the 256^3 workload's rule (gamma = 8 inner GMRES steps on
  the levels whose interfaces exceed dense_max = 5,000 dofs: here the root): against
  the oracle's per-level mode (same rule) to 1e-8.
* The 256^3 workload's option set (BF16 sub-domain inverses formed in FP32, FP32 Sigma
  and interface inverses, FP64 root steps, the same per-level rule) with 16 right-hand
  sides in two lockstep groups of 8: every column to a true relative residual of 1e-10
  (scipy), and the apply error against the FP64 oracle printed and bounded by 4 kappa u.
  The bound: a BF16-stored inverse X~ of a sub-domain matrix has entries within u = 2^-9
  (round to nearest) of X = K_ll^{-1}; K_ll is an M-matrix (every off-diagonal entry of
  the Q1 Laplacian is <= 0), so X >= 0 and ||(X~ - X) r|| <= u ||X |r| || <=
  u kappa(K_ll) ||X r||.  Each apply runs two sub-domain sweeps, whose errors reach z
  directly and through the interface right-hand sides: 4 kappa u covers both with a
  factor of two for the FP32 blocks and the propagation.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import RSDOracle  # noqa: E402

pytestmark = pytest.mark.gpu
DENSE_MAX = 5000
GAMMA = 8


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def c5():
    from workloads import diffusion_problem
    _log("c5 shape: generating Poisson 64^3, octree height 3, 16 right-hand sides")
    return diffusion_problem(64, 3, 0.0, seed=0, nrhs=16, name="poisson64_h3")


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


def test_c5_tree_shape(c5):
    from paper_1210_6266_amd.rsd import rsd_analyze
    rp, ci, _ = c5.csr_arrays()
    a = rsd_analyze(rp, ci, c5.parent, c5.dof_node)
    assert (a["num_leaves"], a["num_levels"], a["max_leaf_dofs"], a["max_iface_dofs"]) == \
        (512, 3, 343, 11719)
    assert a["leaf_dofs"] == 512 * 343
    assert a["skeleton_dofs"] == 64 * 631 + 8 * 2791 + 11719


@pytest.mark.timeout(400)
def test_c5_shape_fp64_dense_apply(c5):
    r = np.random.default_rng(41).uniform(-1.0, 1.0, c5.n)
    h = _handle(c5)
    z = h.apply(_vec(r)).cpu().numpy()
    h.close()
    _log("c5 shape: FP64 dense oracle set-up (about a minute on the host)")
    zo = RSDOracle(c5.K, c5.parent, c5.dof_node).apply(r)
    err = _rel(z, zo)
    _log(f"c5 shape: FP64 dense apply vs oracle {err:.2e}")
    assert err <= 1e-10, err


@pytest.fixture(scope="module")
def c5_hybrid_oracle(c5):
    _log("c5 shape: per-level oracle set-up (root by gamma steps)")
    o = RSDOracle(c5.K, c5.parent, c5.dof_node, interface="hybrid", gamma=GAMMA,
                  dense_max=DENSE_MAX)
    assert [t for t in o.inexact if o.inexact[t]] == [0]
    return o


@pytest.mark.timeout(400)
def test_c5_shape_fp64_hybrid_apply(c5, c5_hybrid_oracle):
    r = np.random.default_rng(43).uniform(-1.0, 1.0, c5.n)
    h = _handle(c5, interface="hybrid", gamma=GAMMA, dense_max=DENSE_MAX)
    z = h.apply(_vec(r)).cpu().numpy()
    h.close()
    err = _rel(z, c5_hybrid_oracle.apply(r))
    _log(f"c5 shape: FP64 hybrid apply vs oracle {err:.2e}")
    assert err <= 1e-8, err


@pytest.mark.timeout(400)
def test_c5_shape_bf16_hybrid_16rhs(c5, c5_hybrid_oracle):
    opts = dict(leaf_prec="bf16", sigma_prec="fp32", iface_prec="fp32", root_prec="fp64",
                interface="hybrid", gamma=GAMMA, dense_max=DENSE_MAX)
    h = _handle(c5, **opts)
    # apply error against the FP64 oracle, with the bound of the module docstring
    r = c5.b[:, 0]
    z = h.apply(_vec(r)).cpu().numpy()
    zo = c5_hybrid_oracle.apply(r)
    err = float(np.linalg.norm(z - zo) / np.linalg.norm(zo))
    leaf = np.nonzero(c5.dof_node == c5_hybrid_oracle.H.leaves[0])[0]
    kappa = float(np.linalg.cond(c5.K[leaf][:, leaf].toarray()))
    bar = 4.0 * kappa * 2.0 ** -9
    _log(f"c5 shape: BF16/FP32 hybrid apply vs FP64 oracle {err:.3e} "
         f"(kappa(K_ll) = {kappa:.2f}, bar 4 kappa u = {bar:.3e})")
    assert 1e-6 < err <= bar, (err, bar)
    # 16 right-hand sides: two lockstep groups of 8 through FGMRES(30)
    X, st, info = h.solve(_cm(c5.b), rtol=1e-10, restart=30, maxit=1000)
    X = X.cpu().numpy()
    h.close()
    assert st == 0, st
    its = [i["iterations"] for i in info]
    rel = [float(np.linalg.norm(c5.b[:, j] - c5.K @ X[:, j]) / np.linalg.norm(c5.b[:, j]))
           for j in range(16)]
    _log(f"c5 shape: 16 columns, iterations {its}, max true relres {max(rel):.2e}")
    assert max(rel) <= 1e-10, rel
