"""Host-side tests of the C ABI (no GPU): the library loads, exports every entry
point declared in include/rsd.h, and its host analysis validates input and
reproduces the hierarchy counts computed independently from the matrix."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_1210_6266_amd import rsd as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = "".join(open(p).read() for p in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(R.library_path()):
        pytest.fail("librsd.so is not built (run __graft_entry__.build())")
    return R.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert set(names) == set(R.EXPORTS), names
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(lib):
    o = R.rsd_options_default()
    # 17 int32 fields (4 bytes of padding), then the allocator's two function pointers
    # and its context
    assert o.struct_size == 18 * 4 + 3 * 8 == ctypes.sizeof(R.rsd_options)
    assert R.rsd_options.dev_alloc.offset == 18 * 4
    assert R.rsd_options.timing_classes.offset == 16 * 4 and o.timing_classes == 0
    assert R.rsd_options.bf16_split.offset == 14 * 4 and o.bf16_split == 1
    assert R.rsd_options.sym_form.offset == 15 * 4 and o.sym_form == 0
    assert o.leaf_prec == 0 and o.timing == 0 and o.graphs == 1
    assert o.symmetric == 1 and o.autotune == 1 and o.g_coupling == 0
    assert o.iface_mode == 0 and o.gamma == 8 and o.dense_max == 32768
    assert not o.dev_alloc and not o.dev_free and o.alloc_ctx is None


def _arrays(p):
    rp, ci, _ = p.csr_arrays()
    return rp, ci, p.parent.astype(np.int32), p.dof_node.astype(np.int32)


def test_analysis_counts(problem_cache, lib):
    """Counts from the library's planner against counts computed here from K."""
    p = problem_cache("diffusion", 13, 2, 1.0, 0)
    rp, ci, par, dn = _arrays(p)
    a = R.rsd_analyze(rp, ci, par, dn)
    T = len(par)
    children = [[] for _ in range(T)]
    for t in range(1, T):
        children[par[t]].append(t)
    leaves = [t for t in range(T) if not children[t]]
    sizes = np.bincount(dn, minlength=T)
    K = p.K.tocsr()
    is_leaf = np.array([not children[t] for t in range(T)])
    m = []
    for l in leaves:
        rows = np.nonzero(dn == l)[0]
        cols = np.unique(K[rows].indices)
        m.append(int(np.sum(~is_leaf[dn[cols]])))
    depth = np.zeros(T, dtype=int)
    for t in range(1, T):
        depth[t] = depth[par[t]] + 1
    inner = [t for t in range(T) if children[t] and sizes[t] > 0]
    assert a["num_leaves"] == len(leaves)
    assert a["num_levels"] == len({depth[t] for t in inner})
    assert a["leaf_dofs"] == int(sizes[leaves].sum())
    assert a["skeleton_dofs"] == p.n - int(sizes[leaves].sum())
    assert a["max_leaf_dofs"] == int(sizes[leaves].max())
    assert a["max_iface_dofs"] == int(sizes[inner].max())
    assert a["max_boundary_dofs"] == max(m)
    assert a["sum_sigma_sq"] == sum(x * x for x in m)
    assert a["sum_leaf_sq"] == int((sizes[leaves].astype(np.int64) ** 2).sum())


def test_config_analysis_c2(problem_cache, lib):
    p = problem_cache("config", "diffusion64")
    a = R.rsd_analyze(*_arrays(p))
    assert (a["num_leaves"], a["num_levels"], a["max_leaf_dofs"], a["max_iface_dofs"]) == \
        (64, 2, 3375, 11719)
    assert a["leaf_dofs"] == 216000 and a["skeleton_dofs"] == 34047
    assert a["max_boundary_dofs"] == 1538


def _expect(status, fn):
    with pytest.raises(R.RSDError) as ei:
        fn()
    assert ei.value.status == status, (ei.value.status, str(ei.value))
    return str(ei.value)


def test_rejects_non_separable_map(problem_cache, lib):
    p = problem_cache("diffusion", 8, 2, 0.0, 0)
    rp, ci, par, dn = _arrays(p)
    dn = dn.copy()
    T = len(par)
    children = [[] for _ in range(T)]
    for t in range(1, T):
        children[par[t]].append(t)
    leaves = [t for t in range(T) if not children[t]]
    # move one interior dof of leaf A into leaf B, far away: K then couples A and B
    a_dof = np.nonzero(dn == leaves[0])[0][0]
    dn[a_dof] = leaves[-1]
    msg = _expect(2, lambda: R.rsd_analyze(rp, ci, par, dn))
    assert "root-to-leaf" in msg


INVALID_CASES = ["unsorted", "col_range", "row_ptr", "parent", "dof_node", "asymmetric",
                 "asymmetric_lower"]


def invalid_case(p, case):
    """(row_ptr, col_idx, parent, dof_node) of the 6^3 one-level problem with one defect."""
    rp, ci, par, dn = [x.copy() for x in _arrays(p)]
    if case == "unsorted":
        ci[rp[3]], ci[rp[3] + 1] = ci[rp[3] + 1], ci[rp[3]]
    elif case == "col_range":
        ci[5] = p.n
    elif case == "row_ptr":
        rp[-1] += 1
    elif case == "parent":
        par[3] = 5
    elif case == "dof_node":
        dn[0] = len(par)
    elif case == "asymmetric":
        # drop one off-diagonal entry of row 0 (keep row 1's mirror): an entry below
        # the diagonal is left without its transpose
        k = rp[0] + 1
        ci = np.delete(ci, k)
        rp = rp.copy()
        rp[1:] -= 1
    elif case == "asymmetric_lower":
        # drop the first entry below the diagonal of row 5: an entry above the diagonal
        # (in the row of its column) is left without its transpose
        k = rp[5]
        assert ci[k] < 5
        ci = np.delete(ci, k)
        rp = rp.copy()
        rp[6:] -= 1
    return rp, ci, par, dn


@pytest.mark.parametrize("case", INVALID_CASES)
def test_rejects_invalid_input(problem_cache, lib, case):
    p = problem_cache("diffusion", 6, 1, 0.0, 0)
    rp, ci, par, dn = invalid_case(p, case)
    msg = _expect(1, lambda: R.rsd_analyze(rp, ci, par, dn))
    if case.startswith("asymmetric"):
        assert "structurally symmetric" in msg


def test_reports_the_lowest_failing_row(problem_cache, lib):
    """The analysis checks the rows in parallel chunks (23^3 dofs: several chunks); with
    the same defect planted in two rows of different chunks, the message names the lower
    row, and a defect of the CSR is reported before one of the tree."""
    p = problem_cache("diffusion", 24, 1, 0.0, 0)
    base = _arrays(p)
    n, T = p.n, len(base[2])
    lo_row, hi_row = 100, n - 100

    def planted(kind, rows):
        rp, ci, par, dn = [x.copy() for x in base]
        for r in rows:
            if kind == "row_ptr":
                rp[r + 1] = rp[r] - 1
            elif kind == "col_range":
                ci[rp[r + 1] - 1] = n
            elif kind == "unsorted":
                ci[rp[r]], ci[rp[r] + 1] = ci[rp[r] + 1], ci[rp[r]]
            elif kind == "dof_node":
                dn[r] = T
        return rp, ci, par, dn

    expect = {"row_ptr": f"row_ptr decreases at row {lo_row}",
              "col_range": f"column index {n} out of range in row {lo_row}",
              "unsorted": f"columns of row {lo_row} not strictly increasing",
              "dof_node": f"dof_node[{lo_row}] = {T} out of range"}
    for kind, want in expect.items():
        for rows in ((lo_row, hi_row), (hi_row, lo_row)):
            msg = _expect(1, lambda: R.rsd_analyze(*planted(kind, rows)))
            assert want in msg, (kind, msg)
    # a column defect in a late row and a tree defect in an early one: the CSR's first
    rp, ci, par, dn = planted("col_range", (hi_row,))
    dn[lo_row] = T
    msg = _expect(1, lambda: R.rsd_analyze(rp, ci, par, dn))
    assert f"out of range in row {hi_row}" in msg, msg


def test_setup_validates_before_device_work(problem_cache, lib):
    """With host pointers and an invalid map, rsd_setup fails in the host analysis
    (no device call is reached) and reports the error thread-locally."""
    p = problem_cache("diffusion", 6, 1, 0.0, 0)
    rp, ci, v = p.csr_arrays()
    par = p.parent.astype(np.int32).copy()
    par[0] = 0
    o = R.rsd_options_default()
    o.host_pointers = 1
    msg = _expect(1, lambda: R.rsd_setup(rp, ci, v, par, p.dof_node.astype(np.int32), o, stream=0))
    assert "parent[0]" in msg
    o.leaf_prec = 7
    _expect(1, lambda: R.rsd_setup(rp, ci, v, p.parent.astype(np.int32),
                                   p.dof_node.astype(np.int32), o, stream=0))
    # interface-solve options: unknown mode, gamma out of 1..64, negative dense_max
    for mode, gamma, dmax, what in ((5, 8, 0, "interface mode"), (1, 0, 0, "gamma"),
                                    (2, 65, 0, "gamma"), (2, 4, -1, "dense_max")):
        o = R.rsd_options_default()
        o.host_pointers = 1
        o.iface_mode, o.gamma, o.dense_max = mode, gamma, dmax
        msg = _expect(1, lambda: R.rsd_setup(rp, ci, v, p.parent.astype(np.int32),
                                             p.dof_node.astype(np.int32), o, stream=0))
        assert what in msg, msg
    # coupling form; an allocator needs both functions
    o = R.rsd_options_default()
    o.host_pointers = 1
    o.g_coupling = 2
    msg = _expect(1, lambda: R.rsd_setup(rp, ci, v, p.parent.astype(np.int32),
                                         p.dof_node.astype(np.int32), o, stream=0))
    assert "g_coupling" in msg, msg
    o = R.rsd_options_default()
    o.host_pointers = 1
    only_alloc = R.ALLOC_FN(lambda nbytes, ctx: None)
    o.dev_alloc = only_alloc
    msg = _expect(1, lambda: R.rsd_setup(rp, ci, v, p.parent.astype(np.int32),
                                         p.dof_node.astype(np.int32), o, stream=0))
    assert "dev_alloc and dev_free" in msg, msg
    # a non-symmetric K needs the gamma interface mode and FP64 / FP32 sub-domains
    for mode, prec, code in ((0, 0, 8), (2, 0, 8), (1, 2, 8), (1, 0, None)):
        o = R.rsd_options_default()
        o.host_pointers = 1
        o.symmetric, o.iface_mode, o.leaf_prec = 0, mode, prec
        if code is not None:
            msg = _expect(code, lambda: R.rsd_setup(rp, ci, v, p.parent.astype(np.int32),
                                                    p.dof_node.astype(np.int32), o, stream=0))
            assert "symmetric = 0" in msg, msg


def test_column_block_layout_checks():
    """The binding's (nrhs, ld) of vector blocks: 1-D, column-major 2-D, and a single
    column whose stride torch normalised (any ld >= n describes one column)."""
    import torch
    from paper_1210_6266_amd.rsd import _cols, colmajor
    n = 7
    assert _cols(torch.zeros(n, dtype=torch.float64), n) == (1, n)
    b = colmajor(torch.zeros(n, 3, dtype=torch.float64))
    assert _cols(b, n) == (3, n)
    one = colmajor(torch.zeros(n, 1, dtype=torch.float64))
    assert _cols(one, n) == (1, n)
    assert _cols(torch.zeros(3, n, dtype=torch.float64).t()[:, :1], n) == (1, n)
    with pytest.raises(ValueError):
        _cols(torch.zeros(n, 3, dtype=torch.float64), n)     # row-major block
