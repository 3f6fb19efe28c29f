"""rsd_apply_noalloc (the application on the library's static work area) against
rsd_apply, through the C ABI: two calls in a row, the second with a smaller input, on
every interface mode and leaf precision; each column bitwise what rsd_apply gives it
(the same kernels in the same order on other memory).  Also: calls from two streams
with no synchronisation between them are ordered by the library, and invalid arguments
are rejected."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _handle(p, **kw):
    from paper_1210_6266_amd import RSD
    rp, ci, v = p.csr_arrays()
    return RSD(rp, ci, v, p.parent, p.dof_node, **kw)


def _cm(a):
    return torch.as_tensor(np.ascontiguousarray(a.T)).cuda().t()


def _noalloc(h, r, z, stream=None):
    """Direct ctypes call of the C entry point (the binding's column rule for nrhs and ld;
    a single column may carry any stride, so ld = n describes it)."""
    from paper_1210_6266_amd.rsd import _cols, _stream, load, rsd_last_error
    nrhs, ldr = _cols(r, r.shape[0])
    _, ldz = _cols(z, z.shape[0])
    st = load().rsd_apply_noalloc(C.c_void_p(h.handle), nrhs, C.c_void_p(r.data_ptr()), ldr,
                                  C.c_void_p(z.data_ptr()), ldz, C.c_void_p(_stream(stream)))
    if st != 0:
        print("rsd_apply_noalloc:", st, rsd_last_error(h.handle), flush=True)
    return st


CASES = [  # (problem, handle options, right-hand sides of the first and second call)
    (("diffusion", 13, 2, 1.0, 2), {}, 5, 2),
    (("diffusion", 13, 2, 1.0, 2), dict(leaf_prec="fp32", root_prec="fp64"), 8, 3),
    (("diffusion", 13, 2, 1.0, 2), dict(leaf_prec="bf16"), 11, 1),
    (("diffusion", 13, 2, 1.0, 2), dict(interface="hybrid", gamma=3, dense_max=200), 4, 1),
    (("diffusion_binary", 12, 3, 1.0, 3), dict(interface="gamma", gamma=4), 3, 2),
    (("strip", 17, 8, "navier_lame", 0), dict(interface="gamma", gamma=4), 2, 1),
]


@pytest.mark.parametrize("key,opts,n1,n2", CASES)
def test_noalloc_matches_apply(problem_cache, key, opts, n1, n2):
    _log(f"noalloc {key} {opts} nrhs {n1} then {n2}")
    p = problem_cache(*key)
    h = _handle(p, **opts)
    rng = np.random.default_rng(61)
    for nrhs in (n1, n2):
        R = _cm(rng.uniform(-1, 1, size=(p.n, nrhs)))
        Z = _cm(np.zeros((p.n, nrhs)))
        assert _noalloc(h, R, Z) == 0
        ref = h.apply(R)                      # the allocating entry point
        torch.cuda.synchronize()
        assert torch.equal(Z, ref), float((Z - ref).abs().max())
    h.close()


def test_noalloc_second_handle_smaller(problem_cache):
    """A larger handle, then a smaller one on the same area: the area keeps the first
    call's contents, which the second must not depend on."""
    big = problem_cache("diffusion", 20, 2, 1.0, 3)
    small = problem_cache("diffusion", 9, 2, 0.5, 1)
    rng = np.random.default_rng(62)
    for p, nrhs in ((big, 6), (small, 2)):
        h = _handle(p)
        R = _cm(rng.uniform(-1, 1, size=(p.n, nrhs)))
        Z = _cm(np.zeros((p.n, nrhs)))
        assert _noalloc(h, R, Z) == 0
        ref = h.apply(R)
        torch.cuda.synchronize()
        assert torch.equal(Z, ref)
        h.close()


def test_noalloc_two_streams_ordered(problem_cache):
    """Two handles, two streams, no synchronisation between the calls: the library orders
    them on the shared area, so both give their rsd_apply results."""
    pa = problem_cache("diffusion", 20, 2, 1.0, 3)
    pb = problem_cache("diffusion", 13, 2, 1.0, 2)
    ha, hb = _handle(pa), _handle(pb)
    rng = np.random.default_rng(63)
    Ra = torch.as_tensor(rng.uniform(-1, 1, pa.n)).cuda()
    Rb = torch.as_tensor(rng.uniform(-1, 1, pb.n)).cuda()
    refa, refb = ha.apply(Ra), hb.apply(Rb)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    Za, Zb = torch.empty_like(Ra), torch.empty_like(Rb)
    for _ in range(3):
        with torch.cuda.stream(s1):
            assert _noalloc(ha, Ra, Za, s1) == 0
        with torch.cuda.stream(s2):
            assert _noalloc(hb, Rb, Zb, s2) == 0
        torch.cuda.synchronize()
        assert torch.equal(Za, refa) and torch.equal(Zb, refb)
    ha.close()
    hb.close()


def test_noalloc_rejects_invalid(problem_cache):
    from paper_1210_6266_amd.rsd import load
    p = problem_cache("diffusion", 9, 2, 0.5, 1)
    h = _handle(p)
    R = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    Z = torch.zeros_like(R)
    lib = load()
    assert lib.rsd_apply_noalloc(C.c_void_p(h.handle), -1, C.c_void_p(R.data_ptr()), p.n,
                                 C.c_void_p(Z.data_ptr()), p.n, None) == 1
    assert lib.rsd_apply_noalloc(C.c_void_p(h.handle), 1, C.c_void_p(R.data_ptr()), p.n - 1,
                                 C.c_void_p(Z.data_ptr()), p.n, None) == 1
    assert lib.rsd_apply_noalloc(C.c_void_p(h.handle), 1, C.c_void_p(R.data_ptr()), p.n,
                                 C.c_void_p(R.data_ptr()), p.n, None) == 1
    assert lib.rsd_apply_noalloc(None, 1, C.c_void_p(R.data_ptr()), p.n,
                                 C.c_void_p(Z.data_ptr()), p.n, None) == 1
    assert lib.rsd_apply_noalloc(C.c_void_p(h.handle), 0, None, 0, None, 0, None) == 0
    h.close()
