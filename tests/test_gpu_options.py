"""The right-hand side form of the interface systems (rsd_options.g_coupling) and a
caller-supplied device allocator (rsd_options.alloc / free), through the C ABI.

* LEAF_ONLY keeps only the couplings of an interface to sub-domain interiors (the strip
  formula of Alg. 2 taken literally): against the oracle's "leaf_only" form to 1e-10
  on 3-D octrees of height 2 and 3, where it differs from FULL; in a strip and with one
  level no deeper-interface coupling exists and it gives FULL's bits.
* allocator="torch": every device block of the handle comes from PyTorch's caching
  allocator (closing the handle returns exactly its device bytes there; the default
  handle's blocks are not PyTorch's), and applies and solves give the default handle's
  bits.
* a handle on a caller's stream gives the default-stream handle's bits.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import RSDOracle  # noqa: E402

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("key", [("diffusion", 13, 2, 1.0, 2), ("diffusion", 9, 3, 0.0, 4)])
def test_leaf_only_matches_oracle(problem_cache, key):
    _log(f"leaf_only {key}")
    p = problem_cache(*key)
    r = np.random.default_rng(41).uniform(-1, 1, p.n)
    zo = RSDOracle(p.K, p.parent, p.dof_node, coupling="leaf_only").apply(r)
    h = _handle(p, coupling="leaf_only")
    z = h.apply(_vec(r)).cpu().numpy()
    h.close()
    assert _rel(z, zo) <= 1e-10, _rel(z, zo)
    hf = _handle(p)
    zf = hf.apply(_vec(r)).cpu().numpy()
    hf.close()
    assert _rel(zf, zo) > 1e-6          # the forms differ in 3-D


@pytest.mark.parametrize("key", [("strip", 17, 8, "poisson", 0), ("diffusion", 12, 1, 0.0, 0)])
def test_leaf_only_equals_full_without_deeper_couplings(problem_cache, key):
    _log(f"leaf_only = full {key}")
    p = problem_cache(*key)
    r = _vec(np.random.default_rng(42).uniform(-1, 1, p.n))
    hl = _handle(p, coupling="leaf_only")
    hf = _handle(p)
    assert np.array_equal(hl.apply(r).cpu().numpy(), hf.apply(r).cpu().numpy())
    hl.close()
    hf.close()


def test_torch_allocator(problem_cache):
    _log("torch allocator")
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    rng = np.random.default_rng(43)
    R = rng.uniform(-1, 1, size=(p.n, 3))
    out = {}
    for name, kw in (("default", {}), ("torch", dict(allocator="torch"))):
        h = _handle(p, leaf_prec="fp32", **kw)
        z = h.apply(_cm(R)).cpu().numpy()
        X, st, info = h.solve(_cm(R), rtol=1e-10)      # solve workspace for 3 columns
        assert st == 0
        torch.cuda.synchronize()
        db = h.stats()["device_bytes"]
        m1 = torch.cuda.memory_allocated()
        h.close()
        m2 = torch.cuda.memory_allocated()
        out[name] = (z, X.cpu().numpy(), db, m1 - m2)
    assert out["torch"][2] > 0 and out["torch"][3] == out["torch"][2]
    assert out["default"][3] == 0
    assert np.array_equal(out["torch"][0], out["default"][0])
    assert np.array_equal(out["torch"][1], out["default"][1])


def test_user_stream(problem_cache):
    """A handle on a caller's stream (rsd_setup / apply / solve all on it, the applies
    eager and then replayed from the captured graph): the default-stream handle's bits."""
    _log("user stream")
    p = problem_cache("diffusion", 13, 2, 1.0, 2)
    R = np.random.default_rng(44).uniform(-1, 1, size=(p.n, 3))
    hd = _handle(p)
    zd = hd.apply(_cm(R)).cpu().numpy()
    Xd, std, infod = hd.solve(_cm(R), rtol=1e-10)
    Xd = Xd.cpu().numpy()
    hd.close()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = _handle(p, stream=s)
        Rs = _cm(R)
        for rep in range(3):
            z = h.apply(Rs).cpu().numpy()
            X, st, info = h.solve(Rs, rtol=1e-10)
            X = X.cpu().numpy()
            assert np.array_equal(z, zd), rep
            assert st == std == 0 and info == infod and np.array_equal(X, Xd), rep
        h.close()
    torch.cuda.synchronize()


def test_calls_on_two_streams_are_ordered(problem_cache):
    """Two applies on one handle from different streams with no synchronisation between
    them share the handle's work buffers: the library makes the second stream wait for
    the first call, so both give the single-stream results bitwise.  Then an update of
    the values on a third stream waits for the applies still reading the old blocks."""
    _log("calls on two streams")
    p = problem_cache("diffusion", 20, 2, 1.0, 3)
    h = _handle(p)
    rng = np.random.default_rng(4)
    R = [torch.as_tensor(rng.uniform(-1, 1, p.n)).cuda() for _ in range(2)]
    ref = [h.apply(r).clone() for r in R]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out = [torch.empty_like(R[0]) for _ in range(2)]
    for _ in range(3):
        with torch.cuda.stream(s1):
            h.apply(R[0], out=out[0])
        with torch.cuda.stream(s2):
            h.apply(R[1], out=out[1])
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    # values scaled by 2 on a third stream right behind an apply on s1: z halves exactly
    rp, ci, v = p.csr_arrays()
    v2 = torch.as_tensor(2.0 * v).cuda()
    s3 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        h.apply(R[0], out=out[0])
    with torch.cuda.stream(s3):
        h.update_values(v2)
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0])
    assert torch.equal(h.apply(R[0]), 0.5 * ref[0])
    h.close()


def test_timing_events_pooled_and_cache_release(problem_cache):
    """timing = 1: per-class kernel times and launch counts in rsd_get_stats; the timing
    events of a destroyed handle serve the next handle (process-wide pool), and after
    rsd_release_cache (idle streams, events and blocks returned to the runtime) a new
    handle refills the pools and gives the same bits."""
    from paper_1210_6266_amd.rsd import rsd_release_cache
    _log("timing events and cache release")
    p = problem_cache("diffusion", 20, 2, 1.0, 3)
    r = torch.as_tensor(np.random.default_rng(9).uniform(-1, 1, p.n)).cuda()
    ref = None
    for k in range(3):
        h = _handle(p, timing=True)
        z = h.apply(r)
        st = h.stats()
        h.close()
        assert st["launches"]["leaf_update"] > 0 and st["time_ms"]["leaf_update"] > 0.0, st
        assert st["time_ms"]["leaf_apply"] > 0.0, st
        if ref is None:
            ref = z.clone()
        assert torch.equal(z, ref)
        if k == 1:
            rsd_release_cache()
    h = _handle(p)
    assert torch.equal(h.apply(r), ref)
    h.close()


def test_timing_classes_selects_the_timed_classes(problem_cache):
    """rsd_options.timing_classes: with timing = 1, only the selected kernel classes are
    timed (the others report 0 ms), every class still counts its launches, the
    applications replay from graphs when none of their classes is timed, and the results
    are those of an untimed handle."""
    _log("timing classes")
    p = problem_cache("diffusion", 20, 2, 1.0, 3)
    r = torch.as_tensor(np.random.default_rng(10).uniform(-1, 1, p.n)).cuda()
    hu = _handle(p)
    zu = hu.apply(r)
    Xu, su, iu = hu.solve(r, rtol=1e-10)
    hu.close()
    for classes in (["leaf_update"], ["leaf_update", "leaf_apply"]):
        h = _handle(p, timing=True, timed_classes=classes)
        assert torch.equal(h.apply(r), zu)
        X, s, info = h.solve(r, rtol=1e-10)
        assert s == su == 0 and info[0]["iterations"] == iu[0]["iterations"]
        assert torch.equal(X, Xu)
        st = h.stats()
        h.close()
        for name, ms in st["time_ms"].items():
            if name in classes:
                assert ms > 0.0, (name, st["time_ms"])
            else:
                assert ms == 0.0, (name, st["time_ms"])
        assert st["launches"]["leaf_apply"] > 0 and st["launches"]["krylov"] > 0, st["launches"]
    with pytest.raises(ValueError):
        _handle(p, timing=True, timed_classes=[])
