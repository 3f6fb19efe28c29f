"""Parity at the benchmarked sizes, with the handle options and device-resident inputs
the benchmark uses.

64^3 variable-coefficient diffusion (250,047 dofs, 64 sub-domains of 3,375 dofs, a
root interface of 11,719 dofs over 8 level-1 interfaces):
  * FP64 factors: the whole apply vector against the FP64 oracle apply, 1e-10
    relative (max norm), as in the small parity cases;
  * mixed factors (FP32 sub-domains, Sigma and level-1 interfaces, FP64 root): apply
    within 2e-4 of the oracle; FGMRES(30) to 1e-10 with a true relative residual
    (scipy SpMV) <= 1e-10, the FP64 handle's iteration count within 1 and the two
    solutions within 1e-8 of each other.
48^3 elasticity on 512 uneven sub-domains, 8 right-hand sides in lockstep:
  * FP64 factors: one apply column against the oracle, 1e-10;
  * mixed factors: every column converged with a true relative residual <= 1e-10, and
    column 0 bitwise equal to its solve alone on the same handle.
The oracle set-ups take tens of seconds on the host; each is built once per module.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import RSDOracle  # noqa: E402
from workloads import config_problem  # noqa: E402

pytestmark = pytest.mark.gpu

MIXED = dict(leaf_prec="fp32", sigma_prec="fp32", iface_prec="fp32", root_prec="fp64")


def _log(msg):
    print(msg, flush=True)


def _device_handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    d = [torch.as_tensor(a, device="cuda") for a in
         (rp, ci, v, p.parent.astype(np.int32), p.dof_node.astype(np.int32))]
    return RSD(*d, **kw)


def _cm(a):
    return torch.as_tensor(np.ascontiguousarray(a.T), device="cuda").t()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def d64():
    _log("64^3 diffusion: problem and FP64 oracle set-up")
    p = config_problem("diffusion64")
    return p, RSDOracle(p.K, p.parent, p.dof_node)


@pytest.fixture(scope="module")
def e48():
    _log("48^3 elasticity: problem and FP64 oracle set-up")
    p = config_problem("elasticity48")
    return p, RSDOracle(p.K, p.parent, p.dof_node)


def test_diffusion64_apply(d64):
    p, o = d64
    r = np.random.default_rng(11).uniform(-1, 1, p.n)
    zo = o.apply(r)
    for name, kw, bar in (("fp64", {}, 1e-10), ("mixed", MIXED, 2e-4)):
        _log(f"64^3 apply {name}")
        h = _device_handle(p, **kw)
        z = h.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
        h.close()
        assert _rel(z, zo) <= bar, (name, _rel(z, zo))


def test_diffusion64_solve(d64):
    p, _ = d64
    b = np.ascontiguousarray(p.b[:, 0])
    x = {}
    its = {}
    for name, kw in (("fp64", {}), ("mixed", MIXED)):
        _log(f"64^3 solve {name}")
        h = _device_handle(p, **kw)
        xd, st, info = h.solve(torch.as_tensor(b, device="cuda"), rtol=1e-10, restart=30)
        h.close()
        assert st == 0
        x[name] = xd.cpu().numpy()
        its[name] = info[0]["iterations"]
        assert np.linalg.norm(b - p.K @ x[name]) <= 1e-10 * np.linalg.norm(b)
    assert abs(its["mixed"] - its["fp64"]) <= 1, its
    assert _rel(x["mixed"], x["fp64"]) <= 1e-8


def test_elasticity48_apply_fp64(e48):
    p, o = e48
    _log("48^3 elasticity apply fp64")
    r = np.random.default_rng(12).uniform(-1, 1, p.n)
    zo = o.apply(r)
    h = _device_handle(p)
    z = h.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    h.close()
    assert _rel(z, zo) <= 1e-10, _rel(z, zo)


def test_elasticity48_eight_rhs_mixed(e48):
    p, _ = e48
    _log("48^3 elasticity 8 rhs mixed")
    assert p.b.shape[1] == 8
    h = _device_handle(p, **MIXED)
    B = _cm(p.b)
    X, st, info = h.solve(B, rtol=1e-10, restart=30, maxit=2000)
    assert st == 0 and all(i["status"] == 0 for i in info)
    Xh = X.cpu().numpy()
    for j in range(8):
        bj = p.b[:, j]
        assert np.linalg.norm(bj - p.K @ Xh[:, j]) <= 1e-10 * np.linalg.norm(bj), j
    x0, st0, info0 = h.solve(B[:, :1], rtol=1e-10, restart=30, maxit=2000)
    h.close()
    assert st0 == 0 and info0[0] == info[0]
    assert np.array_equal(x0.cpu().numpy()[:, 0], Xh[:, 0])
