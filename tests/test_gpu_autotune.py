"""The vectors-per-pass autotuner (rsd_options.autotune).

Before the first application to 2..8 columns the handle times passes of 1, 2 and 4
vectors for each dense batch's symmetric product and keeps the fastest.  Every grouping
gives the same bits, so a tuned handle must agree bitwise with an untuned one; the
choices are reported by rsd_get_stats.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import elasticity_problem  # noqa: E402

pytestmark = pytest.mark.gpu


def _handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    return RSD(rp, ci, v, p.parent, p.dof_node, **kw)


def _cm(a):
    return torch.as_tensor(np.ascontiguousarray(a.T)).cuda().t()


@pytest.mark.parametrize("opts", [dict(), dict(leaf_prec="fp32", sigma_prec="fp32",
                                                iface_prec="fp32"),
                                  dict(leaf_prec="bf16")])
def test_autotuned_applies_match_untuned(opts):
    p = elasticity_problem(10, 2, 0, nrhs=2)
    ht = _handle(p, autotune=True, **opts)
    hu = _handle(p, autotune=False, **opts)
    R = np.random.default_rng(5).uniform(-1, 1, size=(p.n, 8))
    for k in (8, 5, 3, 2):
        zt = ht.apply(_cm(R[:, :k])).cpu().numpy()
        zu = hu.apply(_cm(R[:, :k])).cpu().numpy()
        assert np.array_equal(zt, zu), k
    vp = ht.stats()["vec_pass"]
    nlev = 2                                  # octree of height 2: two dense levels
    assert all(v in (1, 2, 4) for v in vp[:1 + nlev]), vp
    assert all(v == 0 for v in vp[1 + nlev:]), vp
    assert all(v == 0 for v in hu.stats()["vec_pass"])
    B = _cm(R[:, :4])
    Xt, st, it = ht.solve(B, rtol=1e-10)
    Xu, su, iu = hu.solve(B, rtol=1e-10)
    assert st == su == 0 and it == iu and np.array_equal(Xt.cpu().numpy(), Xu.cpu().numpy())
    ht.close()
    hu.close()
