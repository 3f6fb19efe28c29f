"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Every case is a seeded synthetic Q1 problem.  Sizes span several 64 x 64 tiles
with ragged tails (leaf interiors of 125, 343, 729 and 3,375 dofs; interfaces of
331 to 11,719 dofs).  Bars:
  * SpMV: |y - y_ref| <= 1e-14 * (|K| |x|) per row (rounding of a 27-term sum);
  * preconditioner apply, FP64: max |z - z_oracle| <= 1e-10 * max |z_oracle|
    (the oracle uses Cholesky solves, the device explicit inverses: both exact to
    kappa * eps ~ 1e-13 here);
  * solves: true relative residual <= 1e-10, computed on the CPU by scipy;
  * FP32 factors: apply error <= 2e-4 (kappa(K_ll) * eps_32 with kappa <~ 1e3),
    solve still to 1e-10 through the FP64 outer iteration;
  * determinism: two applies are bitwise identical.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from oracle import RSDOracle, fgmres  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def _handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    return RSD(rp, ci, v, p.parent, p.dof_node, **kw)


def _log(msg):
    print(msg, flush=True)


CASES = [  # (ne, height, sigma, seed)
    (12, 1, 0.0, 0),     # the 12^3 Poisson configuration: exact at one level
    (8, 2, 1.0, 1),
    (13, 2, 1.0, 2),     # uneven cuts, ragged tiles
    (24, 2, 0.5, 3),     # root interface 1,519 dofs (24 tiles)
    (9, 3, 0.0, 4),      # three interface levels
    (20, 2, 1.0, 5),     # leaves of 729 dofs (12 tiles, ragged)
]


@pytest.mark.parametrize("ne,height,sigma,seed", CASES)
def test_spmv_parity(problem_cache, ne, height, sigma, seed):
    _log(f"spmv ne={ne} h={height}")
    p = problem_cache("diffusion", ne, height, sigma, seed)
    h = _handle(p)
    x = np.random.default_rng(seed).uniform(-1, 1, size=(p.n, 2))
    y = h.spmv(_dev(x, torch.float64)).cpu().numpy()
    ref = p.K @ x
    bound = abs(p.K) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-14 * bound + 1e-300)
    h.close()


@pytest.mark.parametrize("group", [1, 2, 4])
@pytest.mark.parametrize("ne,height,sigma,seed", CASES)
def test_apply_parity_fp64(problem_cache, monkeypatch, ne, height, sigma, seed, group):
    monkeypatch.setenv("RSD_SWEEP_GROUP", str(group))
    _log(f"apply ne={ne} h={height} group={group}")
    p = problem_cache("diffusion", ne, height, sigma, seed)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    r = np.random.default_rng(100 + seed).uniform(-1, 1, size=(p.n, 2))
    zo = o.apply(r)
    h = _handle(p)
    z = h.apply(_dev(r, torch.float64)).cpu().numpy()
    err = np.abs(z - zo).max() / np.abs(zo).max()
    assert err <= 1e-10, err
    h.close()


def test_apply_is_deterministic(problem_cache):
    p = problem_cache("diffusion", 24, 2, 0.5, 3)
    h = _handle(p)
    r = _dev(np.random.default_rng(7).uniform(-1, 1, p.n), torch.float64)
    z1 = h.apply(r).cpu().numpy()
    z2 = h.apply(r).cpu().numpy()
    assert np.array_equal(z1, z2)
    h.close()


def test_pcg_one_level_converges_in_one_iteration(problem_cache):
    """Poisson 12^3, 2x2x2 sub-domains: one interface level with exact interface
    solves makes M^{-1} = K^{-1}, so PCG stops after one iteration."""
    p = problem_cache("config", "poisson12")
    h = _handle(p)
    b = p.b[:, 0]
    x, st, info = h.solve(_dev(b, torch.float64), method="pcg", rtol=1e-10)
    x = x.cpu().numpy()
    assert st == 0 and info[0]["iterations"] == 1
    assert np.linalg.norm(b - p.K @ x) / np.linalg.norm(b) <= 1e-10
    h.close()


@pytest.mark.parametrize("ne,height,sigma,seed", [(24, 2, 0.5, 3), (20, 2, 1.0, 5), (9, 3, 0.0, 4)])
def test_fgmres_matches_oracle(problem_cache, ne, height, sigma, seed):
    _log(f"fgmres ne={ne} h={height}")
    p = problem_cache("diffusion", ne, height, sigma, seed)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    b = p.b[:, 0]
    xo, io = fgmres(p.K, b, o.apply, rtol=1e-10, restart=30)
    h = _handle(p)
    x, st, info = h.solve(_dev(b, torch.float64), method="fgmres", restart=30, rtol=1e-10)
    x = x.cpu().numpy()
    assert st == 0
    assert np.linalg.norm(b - p.K @ x) / np.linalg.norm(b) <= 1e-10
    assert abs(info[0]["iterations"] - io["iterations"]) <= 1
    xd = spla.spsolve(p.K.tocsc(), b)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    h.close()


def test_multiple_rhs_and_leading_dimension(problem_cache):
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    rng = np.random.default_rng(11)
    ld = p.n + 5
    R = np.zeros((3, ld))
    R[:, :p.n] = rng.uniform(-1, 1, size=(3, p.n))
    r_dev = _dev(R, torch.float64)            # rows of R are the columns (ld = n + 5)
    z_dev = torch.zeros_like(r_dev)
    from paper_1210_6266_amd import rsd as Rb
    h = _handle(p)
    lib = Rb.load()
    st = lib.rsd_apply(h.handle, 3, r_dev.data_ptr(), ld, z_dev.data_ptr(), ld,
                       torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    Z = z_dev.cpu().numpy()
    for j in range(3):
        zo = o.apply(R[j, :p.n])
        assert np.abs(Z[j, :p.n] - zo).max() <= 1e-10 * np.abs(zo).max()
        assert np.all(Z[j, p.n:] == 0.0)
    # nrhs = 0 is a no-op
    assert lib.rsd_apply(h.handle, 0, r_dev.data_ptr(), ld, z_dev.data_ptr(), ld, 0) == 0
    h.close()


def test_single_leaf_tree_is_direct_solve(problem_cache):
    """Height 0: the root is the only (true) sub-domain; RSD is the direct solve."""
    p = problem_cache("diffusion", 7, 1, 1.0, 8)
    parent = np.array([-1], dtype=np.int32)
    dof_node = np.zeros(p.n, dtype=np.int32)
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    h = RSD(rp, ci, v, parent, dof_node)
    r = np.random.default_rng(3).uniform(-1, 1, p.n)
    z = h.apply(_dev(r, torch.float64)).cpu().numpy()
    zd = spla.spsolve(p.K.tocsc(), r)
    assert np.abs(z - zd).max() <= 1e-11 * np.abs(zd).max()
    h.close()


def test_mixed_precision_factors(problem_cache):
    p = problem_cache("diffusion", 20, 2, 1.0, 5)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    r = np.random.default_rng(9).uniform(-1, 1, p.n)
    zo = o.apply(r)
    h = _handle(p, leaf_prec="fp32", root_prec="fp64")
    z = h.apply(_dev(r, torch.float64)).cpu().numpy()
    err = np.abs(z - zo).max() / np.abs(zo).max()
    assert 1e-9 < err <= 2e-4, err
    b = p.b[:, 0]
    x, st, info = h.solve(_dev(b, torch.float64), rtol=1e-10)
    x = x.cpu().numpy()
    assert st == 0 and np.linalg.norm(b - p.K @ x) / np.linalg.norm(b) <= 1e-10
    h.close()


@pytest.mark.parametrize("ne", [32, 48])
def test_bf16_split_updates(problem_cache, ne):
    """FP32 sub-domain and level-1 interface blocks inverted with their trailing updates on
    the BF16 matrix cores (operands split exactly into three BF16 parts: the default,
    rsd_options.bf16_split = 1) or on the FP32 ones: both within the FP32 bar of the FP64
    oracle, different bits (the BF16 path ran), iteration counts within 1 of each other.
    32^3: leaves of 343 dofs (two-tile pivot groups); 48^3: 1,331 (four-tile groups)."""
    _log(f"bf16 split updates {ne}^3")
    p = problem_cache("diffusion", ne, 2, 1.0, 6)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    r = np.random.default_rng(21).uniform(-1, 1, p.n)
    zo = o.apply(r)
    b = p.b[:, 0]
    res = {}
    for split in (True, False):
        h = _handle(p, leaf_prec="fp32", iface_prec="fp32", root_prec="fp64", bf16_split=split)
        z = h.apply(_dev(r, torch.float64)).cpu().numpy()
        err = np.abs(z - zo).max() / np.abs(zo).max()
        _log(f"  bf16_split={split}: apply error vs oracle {err:.2e}")
        assert 1e-9 < err <= 2e-4, (split, err)
        x, st, info = h.solve(_dev(b, torch.float64), rtol=1e-10)
        x = x.cpu().numpy()
        assert st == 0 and np.linalg.norm(b - p.K @ x) / np.linalg.norm(b) <= 1e-10
        res[split] = (z, info[0]["iterations"])
        h.close()
    assert not np.array_equal(res[True][0], res[False][0])
    assert abs(res[True][1] - res[False][1]) <= 1


def test_update_values(problem_cache):
    p1 = problem_cache("diffusion", 13, 2, 1.0, 2)
    p2 = problem_cache("diffusion", 13, 2, 1.0, 3)   # same pattern, new coefficients
    h = _handle(p1)
    rp, ci, v2 = p2.csr_arrays()
    assert np.array_equal(rp, p1.csr_arrays()[0]) and np.array_equal(ci, p1.csr_arrays()[1])
    h.update_values(v2)
    o = RSDOracle(p2.K, p2.parent, p2.dof_node)
    r = np.random.default_rng(5).uniform(-1, 1, p2.n)
    zo = o.apply(r)
    z = h.apply(_dev(r, torch.float64)).cpu().numpy()
    assert np.abs(z - zo).max() <= 1e-10 * np.abs(zo).max()
    h.close()


def test_not_spd_leaf_is_reported(problem_cache):
    from paper_1210_6266_amd import RSD, RSDError
    p = problem_cache("diffusion", 8, 2, 0.0, 0)
    rp, ci, v = p.csr_arrays()
    v = v.copy()
    leaf = p.parent.size - 1                    # the last leaf
    d = int(np.nonzero(p.dof_node == leaf)[0][0])
    k = rp[d] + int(np.nonzero(ci[rp[d]:rp[d + 1]] == d)[0][0])
    v[k] = -v[k]                                # negative diagonal entry
    with pytest.raises(RSDError) as ei:
        RSD(rp, ci, v, p.parent, p.dof_node)
    assert ei.value.status == 3 and f"leaf node {leaf}" in str(ei.value)


def test_invalid_structure_on_the_device_is_reported(problem_cache):
    """rsd_setup with the structure in device memory copies it to the host for the
    analysis; a malformed CSR or map (23^3 dofs: the analysis checks the rows in several
    parallel chunks) is rejected before any kernel with the message the host analysis
    (rsd_analyze) gives, and a valid set-up in the same process still solves."""
    from paper_1210_6266_amd import RSD, RSDError
    from paper_1210_6266_amd import rsd as R
    p = problem_cache("diffusion", 24, 2, 0.0, 0)
    rp, ci, v = p.csr_arrays()
    par, dn = p.parent.astype(np.int32), p.dof_node.astype(np.int32)
    n, hi_row = p.n, p.n - 100
    cases = {}
    a = rp.copy()
    a[hi_row + 1] = a[hi_row] - 1
    cases["row_ptr"] = (a, ci, dn, 1)
    c = ci.copy()
    c[rp[hi_row + 1] - 1] = n
    cases["col_range"] = (rp, c, dn, 1)
    d = dn.copy()
    T = len(par)
    leaves = [t for t in range(T) if t not in set(par[1:].tolist())]
    d[np.nonzero(dn == leaves[0])[0][0]] = leaves[-1]
    cases["not_separable"] = (rp, ci, d, 2)
    for name, (rpx, cix, dnx, status) in cases.items():
        with pytest.raises(R.RSDError) as eh:
            R.rsd_analyze(rpx, cix, par, dnx)
        with pytest.raises(RSDError) as ed:
            RSD(rpx, cix, v, par, dnx)
        assert ed.value.status == eh.value.status == status, name
        assert str(eh.value).split(": ", 1)[-1] in str(ed.value), (name, str(ed.value))
    h = _handle(p)
    x, st, info = h.solve(_dev(p.b[:, 0], torch.float64), rtol=1e-10)
    assert st == 0
    h.close()


def test_nan_rhs_reports_breakdown(problem_cache):
    p = problem_cache("config", "poisson12")
    h = _handle(p)
    b = p.b[:, 0].copy()
    b[3] = np.nan
    x, st, info = h.solve(_dev(b, torch.float64), rtol=1e-10)
    assert st == 5 and info[0]["status"] == 5
    h.close()


def test_maxit_reports_not_converged(problem_cache):
    p = problem_cache("diffusion", 20, 2, 1.0, 5)
    h = _handle(p)
    b = p.b[:, 0]
    x, st, info = h.solve(_dev(b, torch.float64), rtol=1e-14, maxit=2)
    assert st == 4 and info[0]["iterations"] == 2
    assert info[0]["relres"] > 1e-14
    h.close()


@pytest.mark.parametrize("prec,bar", [("fp16", 2e-2), ("bf16", 1e-1)])
def test_half_precision_leaves(problem_cache, prec, bar):
    """16-bit sub-domain inverses (formed in FP32, stored in 16 bits, FP32 products):
    the apply error is of order kappa(K_ll) * eps_16 (eps = 2^-11 FP16, 2^-8 BF16) and
    clearly above the FP32 one; the FP64 FGMRES still reaches 1e-10."""
    _log(f"16-bit leaves {prec}")
    p = problem_cache("diffusion", 20, 2, 1.0, 5)
    o = RSDOracle(p.K, p.parent, p.dof_node)
    r = np.random.default_rng(9).uniform(-1, 1, p.n)
    zo = o.apply(r)
    h = _handle(p, leaf_prec=prec, root_prec="fp64")
    z = h.apply(_dev(r, torch.float64)).cpu().numpy()
    err = np.abs(z - zo).max() / np.abs(zo).max()
    assert 1e-6 < err <= bar, err
    b = p.b[:, 0]
    x, st, info = h.solve(_dev(b, torch.float64), rtol=1e-10)
    x = x.cpu().numpy()
    assert st == 0 and np.linalg.norm(b - p.K @ x) / np.linalg.norm(b) <= 1e-10
    h.close()
