"""The host analysis (hierarchy validation, separability check, ordering) built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only) and driven by the
host tests' malformed inputs, a non-separable map and valid trees: every case returns
its status and the sanitizers report nothing.  The analysis parses caller-supplied CSR
and tree arrays, so its error paths are exercised under the sanitizers here."""
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from test_capi_host import INVALID_CASES, _arrays, invalid_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1210_6266_amd", "csrc")

RUNNER = r"""
import ctypes, sys
import numpy as np
lib = ctypes.CDLL(sys.argv[1])
cases = np.load(sys.argv[2])
names = sorted({k.split("/")[0] for k in cases.files})
buf = ctypes.create_string_buffer(512)
for name in names:
    rp, ci, par, dn = (np.ascontiguousarray(cases[name + "/" + f]) for f in ("rp", "ci", "par", "dn"))
    st = lib.plan_check(ctypes.c_int32(len(rp) - 1), ctypes.c_int64(len(ci)),
                        rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                        ctypes.c_int32(len(par)), par.ctypes.data_as(ctypes.c_void_p),
                        dn.ctypes.data_as(ctypes.c_void_p), buf, 512)
    print(name, st, buf.value.decode(), flush=True)
"""


def _build(tmp):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    so = os.path.join(tmp, "libplan_sanitized.so")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-shared",
           "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", CSRC, os.path.join(CSRC, "plan.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "plan_entry.cpp"), "-o", so]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return gxx, so


def test_host_analysis_under_sanitizers(problem_cache):
    p = problem_cache("diffusion", 6, 1, 0.0, 0)
    cases = {name: invalid_case(p, name) for name in INVALID_CASES}
    # a map that is not separable: one interior dof of a leaf moved to a far leaf
    q = problem_cache("diffusion", 8, 2, 0.0, 0)
    rp, ci, par, dn = [x.copy() for x in _arrays(q)]
    T = len(par)
    leaves = [t for t in range(T) if t not in set(par[1:].tolist())]
    dn[np.nonzero(dn == leaves[0])[0][0]] = leaves[-1]
    cases["not_separable"] = (rp, ci, par, dn)
    cases["valid_h1"] = _arrays(p)
    cases["valid_h2"] = _arrays(problem_cache("diffusion", 13, 2, 1.0, 2))
    cases["valid_strip"] = _arrays(problem_cache("strip", 9, 8, "poisson", 0))
    # 23^3 dofs: the passes over the rows run in several chunks
    big = problem_cache("diffusion", 24, 2, 0.0, 0)
    cases["valid_chunks"] = _arrays(big)
    rp, ci, par, dn = [x.copy() for x in _arrays(big)]
    for r in (100, big.n - 100):
        rp[r + 1] = rp[r] - 1
    cases["row_ptr_chunks"] = (rp, ci, par, dn)
    rp, ci, par, dn = [x.copy() for x in _arrays(big)]
    for r in (100, big.n - 100):
        ci[rp[r + 1] - 1] = big.n
        dn[r] = len(par)
    cases["col_range_chunks"] = (rp, ci, par, dn)
    expect = {name: 1 for name in INVALID_CASES}
    expect.update(not_separable=2, valid_h1=0, valid_h2=0, valid_strip=0, valid_chunks=0,
                  row_ptr_chunks=1, col_range_chunks=1)
    tmp = tempfile.mkdtemp(prefix="rsd_san_")
    try:
        gxx, so = _build(tmp)
        npz = os.path.join(tmp, "cases.npz")
        np.savez(npz, **{f"{name}/{f}": a for name, arrs in cases.items()
                         for f, a in zip(("rp", "ci", "par", "dn"), arrs)})
        libasan = subprocess.run([gxx, "-print-file-name=libasan.so"], capture_output=True,
                                 text=True).stdout.strip()
        env = dict(os.environ, LD_PRELOAD=libasan,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", RUNNER, so, npz], capture_output=True,
                           text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
        got = {}
        for line in r.stdout.splitlines():
            name, st = line.split(" ", 2)[:2]
            got[name] = int(st)
        assert got == expect, (got, r.stdout)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
