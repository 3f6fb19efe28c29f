"""GPU parity of the differentiable RSD solve (adjoint method) against the FP64 oracle.

Cases: the adjoint configuration (diffusion 32^3, k = exp(theta), theta ~ N(0, 0.5^2),
octree of height 2, L = 1/2 ||x - x_target||^2) and a small mesh for the kernels.
Bars:
  * rsd_fe_assemble: every CSR value within 1e-14 (relative to max |K|) of the
    oracle's assembly -- sums of at most 8 terms in a different order;
  * rsd_fe_grad on given vectors: within 1e-13 relative (64-term sums);
  * dL/dtheta and dL/db from the GPU solves (rtol 1e-12) within 1e-7 relative of the
    oracle's exact-solve gradient, for FP64 and for FP32 factors (the outer Krylov
    iteration is FP64, so the factor precision changes iterations, not the result);
  * 20 random directions d: (L(theta + eps d) - L(theta - eps d)) / (2 eps), eps =
    1e-6, with GPU solves at rtol 1e-13, within 1e-5 relative of <dL/dtheta, d>.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as A  # noqa: E402
from workloads import config_problem, diffusion_fe_map, diffusion_problem  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def _system(p, fe, **kw):
    from paper_1210_6266_amd.adjoint import DifferentiableSolve
    rp, ci, _ = p.csr_arrays()
    return DifferentiableSolve(rp, ci, p.parent, p.dof_node, fe, **kw)


@pytest.fixture(scope="module")
def adj32():
    p = config_problem("adjoint32")
    return p, diffusion_fe_map(p)


def test_fe_assemble_matches_oracle():
    _log("fe assemble 6^3")
    from paper_1210_6266_amd.rsd import FEMap, rsd_fe_assemble
    p = diffusion_problem(6, 1, 0.5, 7)
    fe = diffusion_fe_map(p)
    th = p.meta["theta"]
    fm = FEMap(fe)
    vals = torch.empty(fe["nnz"], dtype=torch.float64, device="cuda")
    for kind, k in (("exp", A.EXP), ("linear", A.LINEAR)):
        t = th if kind == "exp" else np.exp(th)
        rsd_fe_assemble(fm, _dev(t), kind, vals)
        K = A.assemble(fe, t, p.n, k)
        assert np.array_equal(K.indptr, p.K.indptr) and np.array_equal(K.indices, p.K.indices)
        v = vals.cpu().numpy()
        assert np.abs(v - K.data).max() <= 1e-14 * np.abs(K.data).max()


def test_fe_grad_kernel_matches_oracle():
    _log("fe grad kernel 6^3")
    from paper_1210_6266_amd.rsd import FEMap, rsd_fe_grad
    p = diffusion_problem(6, 1, 0.5, 8)
    fe = diffusion_fe_map(p)
    th = p.meta["theta"]
    rng = np.random.default_rng(4)
    lam, x = rng.standard_normal(p.n), rng.standard_normal(p.n)
    g = torch.empty(th.size, dtype=torch.float64, device="cuda")
    rsd_fe_grad(FEMap(fe), _dev(th), "exp", _dev(lam), _dev(x), g)
    go = A.element_gradient(fe, th, lam, x)
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-13 * np.abs(go).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_gradient_matches_oracle(adj32, prec):
    _log(f"adjoint32 gradient {prec}")
    p, fe = adj32
    th, b, xt = p.meta["theta"], p.b[:, 0], p.meta["x_target"]
    Lo, xo, go, lo = A.solve_loss_grad(fe, th, b, xt)
    kw = {} if prec == "fp64" else dict(leaf_prec="fp32", root_prec="fp64")
    s = _system(p, fe, rtol=1e-12, **kw)
    theta = _dev(th).requires_grad_(True)
    bb = _dev(b).requires_grad_(True)
    x = s(theta, bb)
    L = 0.5 * ((x - _dev(xt)) ** 2).sum()
    L.backward()
    assert abs(L.item() - Lo) <= 1e-9 * Lo
    gt, gb = theta.grad.cpu().numpy(), bb.grad.cpu().numpy()
    assert np.linalg.norm(gt - go) <= 1e-7 * np.linalg.norm(go)
    assert np.linalg.norm(gb - lo) <= 1e-7 * np.linalg.norm(lo)
    assert all(i["status"] == 0 for i in s.last_info)
    s.close()


def test_adjoint_central_differences(adj32):
    _log("adjoint32 central differences (20 directions)")
    p, fe = adj32
    th, b, xt = p.meta["theta"], p.b[:, 0], p.meta["x_target"]
    s = _system(p, fe, rtol=1e-13)
    xt_d, b_d = _dev(xt), _dev(b)

    def loss(t):
        with torch.no_grad():
            x = s(t, b_d)
        return 0.5 * float(((x - xt_d) ** 2).sum())

    theta = _dev(th).requires_grad_(True)
    x = s(theta, b_d)
    (0.5 * ((x - xt_d) ** 2).sum()).backward()
    g = theta.grad.detach()
    rng = np.random.default_rng(20)
    eps = 1e-6
    for k in range(20):
        d = _dev(rng.standard_normal(th.size))
        fd = (loss(theta.detach() + eps * d) - loss(theta.detach() - eps * d)) / (2 * eps)
        gd = float((g * d).sum())
        assert abs(fd - gd) <= 1e-5 * abs(gd), (k, fd, gd)
    s.close()
