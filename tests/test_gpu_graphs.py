"""Graph-captured preconditioner applications (rsd_options.graphs) against eager ones.

A handle with graphs replays each application from a HIP graph captured on first use
(one per number of columns); a handle without runs the same kernels eagerly.  The bar
is bitwise equality, replay after replay, with eager work of other kinds in between
(SpMVs, applies with other column counts, torch reductions, solves), after a change of
the matrix values, and for every interface mode and leaf precision.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import elasticity_problem  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [  # (name, problem key, handle options)
    ("diffusion13-fp64", ("diffusion", 13, 2, 1.0, 2), {}),
    ("elasticity8-fp32", ("elasticity", 8, 2, 1),
     dict(leaf_prec="fp32", sigma_prec="fp32", iface_prec="fp32")),
    ("diffusion20-bf16", ("diffusion", 20, 2, 1.0, 5), dict(leaf_prec="bf16")),
    ("strip-gamma", ("strip", 17, 8, "navier_lame", 0), dict(interface="gamma", gamma=4)),
    ("diffusion13-hybrid", ("diffusion", 13, 2, 1.0, 2),
     dict(interface="hybrid", gamma=3, dense_max=200)),
]


def _log(msg):
    print(msg, flush=True)


def _problem(problem_cache, key):
    if key[0] == "elasticity":
        return elasticity_problem(key[1], key[2], key[3], nrhs=3)
    return problem_cache(*key)


def _handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    return RSD(rp, ci, v, p.parent, p.dof_node, **kw)


def _cm(a):
    return torch.as_tensor(np.ascontiguousarray(a.T)).cuda().t()


def _vec(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,key,opts", CASES)
def test_graph_replays_match_eager(problem_cache, name, key, opts):
    _log(f"graphs {name}")
    p = _problem(problem_cache, key)
    hg = _handle(p, graphs=True, **opts)
    he = _handle(p, graphs=False, **opts)
    rng = np.random.default_rng(3)
    R = _cm(rng.uniform(-1, 1, size=(p.n, 5)))
    r1 = _vec(rng.uniform(-1, 1, p.n))
    for rep in range(3):
        zg = hg.apply(R).cpu().numpy()
        ze = he.apply(R).cpu().numpy()
        assert np.array_equal(zg, ze), rep
        # other eager work between the replays
        _ = hg.spmv(R)
        s = float(torch.sum(R * R))
        assert np.array_equal(hg.apply(r1).cpu().numpy(), he.apply(r1).cpu().numpy())
        assert s > 0
    B = _cm(rng.uniform(-1, 1, size=(p.n, 3)))
    Xg, stg, ig = hg.solve(B, rtol=1e-10)
    Xe, ste, ie = he.solve(B, rtol=1e-10)
    assert stg == ste == 0 and ig == ie
    assert np.array_equal(Xg.cpu().numpy(), Xe.cpu().numpy())
    hg.close()
    he.close()


def test_graph_after_value_update(problem_cache):
    """rsd_update_values keeps every buffer the captured graphs use; the replays then
    apply the new factors (the same bits as a fresh eager handle on the new values)."""
    p1 = problem_cache("diffusion", 13, 2, 1.0, 2)
    p2 = problem_cache("diffusion", 13, 2, 1.0, 3)
    hg = _handle(p1, graphs=True)
    r = _vec(np.random.default_rng(4).uniform(-1, 1, p1.n))
    z1 = hg.apply(r).cpu().numpy()                 # captured here
    hg.update_values(p2.csr_arrays()[2])
    z2 = hg.apply(r).cpu().numpy()                 # replayed with the new factors
    he = _handle(p2, graphs=False)
    assert np.array_equal(z2, he.apply(r).cpu().numpy())
    assert not np.array_equal(z1, z2)
    hg.close()
    he.close()
