#!/usr/bin/env python3
"""Benchmark of the RSD-preconditioned Krylov solve on one MI355X.

Workload: -div(k grad u) = f on 64^3 trilinear hexahedra of the unit cube,
k_e = exp(z_e), z_e ~ N(0, 1) per element, f ~ U[-1, 1] per free dof (n = 250,047),
4 x 4 x 4 box sub-domains (octree of height 2: 64 true sub-domains of 3,375 dofs,
8 level-1 interfaces of 2,791 dofs, a root interface of 11,719 dofs).

One step = one pass of the whole hot path on inputs already resident in HBM:
rsd_setup (host analysis of the hierarchy, extraction and exact inversion of the
sub-domain matrices, Sigma blocks, interface Schur assembly and inversion), then
rsd_solve (FGMRES(30) preconditioned by RSD to a true relative residual of 1e-10),
then rsd_destroy.  The headline variant keeps sub-domain, Sigma and non-root
interface blocks in FP32 and the root interface, the Krylov vectors, dot products,
orthogonalisation and residuals in FP64; the plain FP64 variant is timed beside it.

value = solves per second of the mixed variant (1 / time-to-1e-10 including set-up).

Secondary blocks on the same line: the differentiable solve on diffusion 32^3
(forward + adjoint + gradient per pass), 3-D elasticity 48^3 on 512 uneven
sub-domains with 8 right-hand sides solved in lockstep, and Poisson 256^3 on 32,768
sub-domains with 16 right-hand sides (16-bit sub-domain inverses, matrix-free gamma
steps on the two largest interface levels).  `--blocks elasticity48` (without
`main`) runs only the chosen blocks, for profiling.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 residual & solves/s, mixed-batched vs FP64 RSD; GB/s, MFMA %"
PEAK = {"hbm_GBps": 8000.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3}
MIXED = dict(leaf_prec="fp32", sigma_prec="fp32", iface_prec="fp32", root_prec="fp64")
FP64 = dict(leaf_prec="fp64", sigma_prec="fp64", iface_prec="fp64", root_prec="fp64")
TILE = 64


def leaf_apply_bytes(p, es):
    """Algorithmic bytes of one leaf pass of an apply, averaged over its two passes.  The
    first reads the lower triangle of every sub-domain inverse (es bytes per entry) and
    16 bytes of vectors per leaf dof; the second (the back-substitution's correction
    K_ll^{-1} w, w zero outside the leaf's shell, which the library orders last) only the
    tile rows from the first one that holds shell rows, and 24 bytes per leaf dof (w, the
    first pass's result and the sum).  The shell: leaf dofs coupled to a dof of another
    tree node."""
    K = p.K.tocsr()
    node = np.asarray(p.dof_node)
    rows = np.repeat(np.arange(p.n), np.diff(K.indptr))
    outer = np.bincount(rows[node[K.indices] != node[rows]], minlength=p.n) > 0
    T = len(p.parent)
    has_child = np.zeros(T, bool)
    has_child[np.asarray(p.parent)[1:]] = True
    n_of = np.bincount(node, minlength=T)
    s_of = np.bincount(node[outer], minlength=T)
    full = corr = 0
    for t in np.nonzero(~has_child)[0]:
        n, r0 = int(n_of[t]), (int(n_of[t] - s_of[t]) // TILE) * TILE
        full += n * (n + 1) // 2
        corr += n * (n + 1) // 2 - r0 * (r0 + 1) // 2
    nleaf = int(n_of[~has_child].sum())
    return ((full + corr) * es + (16 + 24) * nleaf) / 2


def group_tiles(n):
    """Pivot tiles per sweep step that the library picks for matrices of order n."""
    return 4 if (n + TILE - 1) // TILE >= 16 else 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    # (the library's set-up autotuner times up to four inversion schedules per batch shape,
    # the first of them twice, on the first five set-ups of a process: the warm-up steps
    # cover them)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--reuse-solves", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="time one variant only (for profiling runs)")
    ap.add_argument("--adjoint-steps", type=int, default=5,
                    help="forward+backward passes timed on the 32^3 adjoint workload (0: skip)")
    ap.add_argument("--elasticity-steps", type=int, default=2,
                    help="set-up + 8-RHS solves timed on the 48^3 elasticity workload (0: skip)")
    ap.add_argument("--profile-setups", type=int, default=0,
                    help="counter-run mode: K set-up + solve passes of the 64^3 headline "
                         "workload (mixed) with the inversion schedule fixed to the one the "
                         "autotuner keeps there (look-ahead, 128 x 128 super-tiles), one line "
                         "of text, no benchmark line")
    ap.add_argument("--blocks", default="main,adjoint32,elasticity48,poisson256",
                    help="comma list of what to run: main (the 64^3 diffusion line), adjoint32, "
                         "elasticity48, poisson256; without main only the chosen blocks are run "
                         "and printed (a profiling aid, not the benchmark line)")
    return ap.parse_args()


def update_flops(sizes):
    """Algorithmic flops of the MFMA trailing updates of one blocked sweep inversion
    per matrix of order n: per step with w real pivot columns, the n - w other rows
    and columns receive a rank-w update of their lower triangle: w (n-w)(n-w+1)."""
    tot = 0.0
    for n in sizes:
        steps_group = group_tiles(max(sizes))
        nt = (n + TILE - 1) // TILE
        for c0 in range(0, nt, steps_group):
            lo = c0 * TILE
            w = min(n, (c0 + steps_group) * TILE) - lo
            if w <= 0:
                continue
            r = n - w
            tot += float(w) * r * (r + 1)
    return tot


def potrf_flops(sizes):
    """The set-up rows' unit of work: one Cholesky factorisation, n^3 / 3 flops per
    matrix of order n (the sweep inversion executes about three times as many)."""
    return sum(float(n) ** 3 / 3.0 for n in sizes)


def measured_traffic(key):
    """HBM bytes per launch of kernel `key` (FETCH_SIZE + WRITE_SIZE, each scaled by
    what the counter reads for a plain copy of known size), as recorded by the
    counter runs under profiles/; None unless the kernel source is unchanged since."""
    rec_path = os.path.join(ROOT, "profiles", "traffic_diffusion64_mixed.json")
    src_path = os.path.join(ROOT, "paper_1210_6266_amd", "csrc", "kernels.hip")
    try:
        with open(rec_path) as f:
            rec = json.load(f)
        with open(src_path, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    k = rec.get("kernels", {}).get(key)
    if rec.get("source_sha256") != sha or k is None:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def bench_adjoint(a, dev):
    """Differentiable solve on the 32^3 adjoint workload (None when skipped)."""
    import torch

    from workloads import config_problem
    # ---- differentiable solve (adjoint method) on the 32^3 adjoint workload: one pass
    # = assembly of K(theta) + set-up refresh + forward solve + adjoint solve + gradient
    adjoint = None
    if a.adjoint_steps > 0:
        from paper_1210_6266_amd.adjoint import DifferentiableSolve
        from workloads import diffusion_fe_map
        pa = config_problem("adjoint32", seed=a.seed)
        fe = diffusion_fe_map(pa)
        rpa, cia, _ = pa.csr_arrays()
        th0 = torch.as_tensor(pa.meta["theta"], device=dev)
        ba = torch.as_tensor(np.ascontiguousarray(pa.b[:, 0]), device=dev)
        xt = torch.as_tensor(pa.meta["x_target"], device=dev)
        adjoint = {}
        for name, prec in (("mixed", dict(leaf_prec="fp32", sigma_prec="fp32",
                                          iface_prec="fp32", root_prec="fp64")), ("fp64", {})):
            sysd = DifferentiableSolve(rpa, cia, pa.parent, pa.dof_node, fe, rtol=1e-10, **prec)

            def one(k):
                theta = (th0 + 1e-3 * k).requires_grad_(True)   # a new K every pass
                x = sysd(theta, ba)
                loss = 0.5 * ((x - xt) ** 2).sum()
                loss.backward()
                return theta.grad

            one(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(a.adjoint_steps):
                one(k + 1)
            torch.cuda.synchronize()
            its = [i["iterations"] for i in sysd.last_info[-2 * a.adjoint_steps:]]
            adjoint[name] = dict(ms_per_fwd_bwd=1e3 * (time.perf_counter() - t0) / a.adjoint_steps,
                                 krylov_iterations=its[:2])
            sysd.close()
        adjoint["workload"] = ("diffusion 32^3 Q1, k = exp(theta), theta ~ N(0, 0.5^2), octree h=2; "
                               "L = 1/2 ||x - x_t||^2; FGMRES(30) to 1e-10 forward and adjoint")

    return adjoint


def bench_elasticity(a, dev):
    """Set-up + lockstep 8-RHS solves on the 48^3 elasticity workload (None when skipped)."""
    import torch

    from paper_1210_6266_amd import RSD
    from workloads import config_problem
    # ---- 3-D elasticity 48^3 on 512 uneven sub-domains with 8 right-hand sides: one pass
    # = set-up + lockstep FGMRES(30) of the 8 columns to 1e-10 + destroy
    elastic = None
    if a.elasticity_steps > 0:
        pe = config_problem("elasticity48", seed=a.seed)
        rpe, cie, ve = pe.csr_arrays()
        de = [torch.as_tensor(t, device=dev) for t in
              (rpe, cie, ve, pe.parent.astype(np.int32), pe.dof_node.astype(np.int32))]
        Be = torch.as_tensor(np.ascontiguousarray(pe.b.T), device=dev).t()   # n x 8, column-major
        elastic = {}
        for name, prec in (("mixed", dict(leaf_prec="fp32", sigma_prec="fp32",
                                          iface_prec="fp32", root_prec="fp64")), ("fp64", {})):
            if a.only is not None and name != a.only:
                continue

            def one():
                h = RSD(*de, **prec)
                X, st, info = h.solve(Be, rtol=1e-10, restart=30, maxit=2000)
                torch.cuda.synchronize()
                return h, X, st, info

            h, X, st, info = one()
            # one column alone on the same handle: what the group saves per column
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st1, info1 = h.solve(Be[:, :1], rtol=1e-10, restart=30, maxit=2000)
            torch.cuda.synchronize()
            single = time.perf_counter() - t0
            h.close()
            t0 = time.perf_counter()
            for _ in range(a.elasticity_steps):
                h, X, st, info = one()
                h.close()
            sec = (time.perf_counter() - t0) / a.elasticity_steps
            Xh = X.cpu().numpy()
            rel = max(float(np.linalg.norm(pe.b[:, j] - pe.K @ Xh[:, j]) / np.linalg.norm(pe.b[:, j]))
                      for j in range(pe.b.shape[1]))
            elastic[name] = dict(ms_setup_plus_8rhs_solve=1e3 * sec,
                                 solves_per_s=pe.b.shape[1] / sec,
                                 status=int(st), iterations=[i["iterations"] for i in info],
                                 max_true_relres=rel,
                                 ms_one_column_solve_alone=1e3 * single,
                                 iterations_one_column=info1[0]["iterations"])
        elastic["workload"] = ("3-D linear elasticity Q1 48^3 (E = 1, nu = 0.3, clamped x = 0), "
                               f"n = {pe.n}, nnz = {pe.K.nnz}; octree h = 3 over uneven cut planes "
                               "(512 leaves of 192-882 dofs); 8 right-hand sides (body load + "
                               "N(0, 0.1^2) per dof); lockstep FGMRES(30) to 1e-10")

    return elastic


def bench_poisson256(a, dev):
    """256^3 Poisson on 32,768 sub-domains with 16 right-hand sides: one cold pass of
    set-up + two lockstep groups of FGMRES(30) to 1e-10 (None when skipped; the error
    text when it fails, so that the benchmark line still prints)."""
    import torch

    from paper_1210_6266_amd import RSD
    from workloads import config_problem
    try:
        t0 = time.perf_counter()
        p = config_problem("poisson256", seed=a.seed)
        gen_s = time.perf_counter() - t0
        rp, ci, v = p.csr_arrays()
        d = [torch.as_tensor(t, device=dev) for t in
             (rp, ci, v, p.parent.astype(np.int32), p.dof_node.astype(np.int32))]
        B = torch.as_tensor(np.ascontiguousarray(p.b.T), device=dev).t()      # n x 16
        opts = dict(leaf_prec="bf16", sigma_prec="fp32", iface_prec="fp32", root_prec="fp64",
                    interface="hybrid", gamma=8, dense_max=5000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = RSD(*d, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X, st, info = h.solve(B, rtol=1e-10, restart=30, maxit=1000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # true residuals: every column with the library's FP64 SpMV, column 0 also by scipy
        R = B - h.spmv(X)
        rel = (torch.linalg.vector_norm(R, dim=0) / torch.linalg.vector_norm(B, dim=0)).cpu()
        x0 = X[:, 0].cpu().numpy()
        rel0 = float(np.linalg.norm(p.b[:, 0] - p.K @ x0) / np.linalg.norm(p.b[:, 0]))
        dev_bytes = h.stats()["device_bytes"]
        h.close()
        return dict(ms_setup=1e3 * (t1 - t0), ms_solve_16rhs=1e3 * (t2 - t1),
                    solves_per_s=p.b.shape[1] / (t2 - t0), status=int(st),
                    iterations=[i["iterations"] for i in info],
                    max_true_relres=float(rel.max()), relres_col0_scipy=rel0,
                    device_bytes=int(dev_bytes), host_generation_s=gen_s,
                    options="BF16 sub-domain inverses (formed in FP32), FP32 Sigma and level "
                            "3-4 interface inverses, levels 0-2 (interfaces > 5,000 dofs) by "
                            "8 matrix-free GMRES steps, FP64 Krylov; one cold pass",
                    workload=(f"Poisson Q1 256^3, n = {p.n}, nnz = {p.K.nnz}; octree h = 5: "
                              "32,768 sub-domains of 343 dofs; 16 right-hand sides U[-1, 1]; "
                              "two lockstep groups of 8, FGMRES(30) to 1e-10"))
    except Exception as e:  # a secondary block: report, do not fail the line
        return dict(error=repr(e))


def bf16_shape_error(a, dev):
    """The 256^3 block's option set (BF16 sub-domain inverses formed in FP32, FP32 Sigma
    and interface inverses, 8 matrix-free GMRES steps on interfaces above 5,000 dofs) on
    the same tree shape at 64^3 -- octree of height 3, sub-domains of 8^3 elements (343
    dofs), interfaces of 631 / 2,791 / 11,719 dofs -- applied to one right-hand side and
    compared with the FP64 oracle's per-level mode: the error of the 16-bit path at the
    largest size the oracle follows (the 256^3 tree itself is beyond it)."""
    import torch

    from oracle import RSDOracle
    from paper_1210_6266_amd import RSD
    from workloads import diffusion_problem
    try:
        p = diffusion_problem(64, 3, 0.0, a.seed)
        rp, ci, v = p.csr_arrays()
        opts = dict(leaf_prec="bf16", sigma_prec="fp32", iface_prec="fp32", root_prec="fp64",
                    interface="hybrid", gamma=8, dense_max=5000)
        h = RSD(rp, ci, v, p.parent, p.dof_node, **opts)
        r = p.b[:, 0]
        zg = h.apply(torch.as_tensor(r, device=dev)).cpu().numpy()
        h.close()
        zo = RSDOracle(p.K, p.parent, p.dof_node, interface="hybrid", gamma=8,
                       dense_max=5000).apply(r)
        return dict(max_rel=float(np.abs(zg - zo).max() / np.abs(zo).max()),
                    l2_rel=float(np.linalg.norm(zg - zo) / np.linalg.norm(zo)),
                    workload="Poisson 64^3, octree height 3 (512 sub-domains of 343 dofs; "
                             "interfaces of 631, 2,791, 11,719 dofs), the poisson256 options")
    except Exception as e:  # a report, not the product
        return dict(error=repr(e))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {a.gpus}).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1210_6266_amd import RSD
    from paper_1210_6266_amd.rsd import rsd_analyze
    from workloads import config_problem

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if a.profile_setups > 0:
        p = config_problem("diffusion64", seed=a.seed)
        rp, ci, v = p.csr_arrays()
        d = [torch.as_tensor(t, device=dev) for t in
             (rp, ci, v, p.parent.astype(np.int32), p.dof_node.astype(np.int32))]
        b = torch.as_tensor(np.ascontiguousarray(p.b[:, 0]), device=dev)
        its = []
        t0 = time.perf_counter()
        for _ in range(a.profile_setups):
            h = RSD(*d, autotune=False, **MIXED)
            _, st, info = h.solve(b, rtol=1e-10, restart=30, maxit=1000)
            its.append(info[0]["iterations"])
            h.close()
        torch.cuda.synchronize()
        print(f"profile-setups: {a.profile_setups} set-up + solve passes, "
              f"{1e3 * (time.perf_counter() - t0) / a.profile_setups:.1f} ms each, "
              f"iterations {its}", flush=True)
        return
    if "main" not in a.blocks.split(","):
        blocks = set(a.blocks.split(","))
        out = {"adjoint32": bench_adjoint(a, dev) if "adjoint32" in blocks else None,
               "elasticity48": bench_elasticity(a, dev) if "elasticity48" in blocks else None,
               "poisson256": bench_poisson256(a, dev) if "poisson256" in blocks else None}
        print(json.dumps(out), flush=True)
        return
    p = config_problem("diffusion64", seed=a.seed)
    rp, ci, v = p.csr_arrays()
    ana = rsd_analyze(rp, ci, p.parent, p.dof_node)
    d_rp = torch.as_tensor(rp, device=dev)
    d_ci = torch.as_tensor(ci, device=dev)
    d_v = torch.as_tensor(v, device=dev)
    d_par = torch.as_tensor(p.parent.astype(np.int32), device=dev)
    d_dn = torch.as_tensor(p.dof_node.astype(np.int32), device=dev)
    b = torch.as_tensor(np.ascontiguousarray(p.b[:, 0]), device=dev)
    torch.cuda.synchronize()

    def step(prec, timing, classes=None):
        t0 = time.perf_counter()
        h = RSD(d_rp, d_ci, d_v, d_par, d_dn, timing=timing, timed_classes=classes, **prec)
        t1 = time.perf_counter()
        x, st, info = h.solve(b, rtol=1e-10, restart=30, maxit=1000)
        t2 = time.perf_counter()
        stats = h.stats() if timing else None
        h.close()
        t3 = time.perf_counter()
        stats["wall_ms"] = [1e3 * (t1 - t0), 1e3 * (t2 - t1), 1e3 * (t3 - t2)]
        return x, st, info[0], stats

    # The timed steps carry HIP events around the roofline's kernel class only (each event
    # between two launches costs a few microseconds of queue time); the phase breakdown
    # and the choice of that class come from the last warm-up step, timed in every class.
    def timed(prec, k, w):
        for _ in range(max(0, w - 1)):
            step(prec, True)
        _, _, _, full = step(prec, True)
        tm = full["time_ms"]
        dom_cls = max(("leaf_update", "root_update", "leaf_apply"), key=lambda c: tm.get(c, 0.0))
        torch.cuda.synchronize()
        acc_ms, acc_n = {}, {}
        its = []
        t0 = time.perf_counter()
        for _ in range(k):
            x, st, info, stats = step(prec, True, [dom_cls])
            its.append(info["iterations"])
            for kk, vv in stats["time_ms"].items():
                acc_ms[kk] = acc_ms.get(kk, 0.0) + vv
            for kk, vv in stats["launches"].items():
                acc_n[kk] = acc_n.get(kk, 0) + vv
            for i, kk in enumerate(["setup", "solve", "stats+destroy"]):
                acc_ms["wall_" + kk] = acc_ms.get("wall_" + kk, 0.0) + stats["wall_ms"][i]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if st != 0:
            raise RuntimeError(f"solve did not converge: status {st}, {info}")
        return (t1 - t0) / k, x, its, acc_ms, acc_n, stats, full

    def reuse(prec, r):
        h = RSD(d_rp, d_ci, d_v, d_par, d_dn, **prec)
        h.solve(b, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(r):
            x, st, info = h.solve(b, rtol=1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h.close()
        return r / (t1 - t0)

    variants = ["mixed", "fp64"] if a.only is None else [a.only]
    res = {}
    for name in variants:
        prec = MIXED if name == "mixed" else FP64
        k = a.steps if (name == "mixed" or a.only) else max(1, (a.steps + 1) // 2)
        sec, x, its, ms, nl, last, full = timed(prec, k, a.warmup)
        xh = x.cpu().numpy()
        bh = p.b[:, 0]
        relres = float(np.linalg.norm(bh - p.K @ xh) / np.linalg.norm(bh))
        res[name] = dict(sec=sec, x=xh, its=its, ms={kk: vv / k for kk, vv in ms.items()},
                         launches={kk: vv / k for kk, vv in nl.items()}, relres=relres,
                         device_bytes=last["device_bytes"], host_ms=last["host_analysis_ms"],
                         setup_wall_ms=last["setup_wall_ms"], steps=k,
                         phase_ms=dict(full["time_ms"], **{"wall_" + kk: full["wall_ms"][i] for i, kk
                                                            in enumerate(["setup", "solve",
                                                                          "stats+destroy"])}),
                         phase_launches=dict(full["launches"]))
    # the same steps without the per-kernel HIP events (the library's defaults, graphs on)
    plain_ms = {}
    for name in variants:
        prec = MIXED if name == "mixed" else FP64
        k = res[name]["steps"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            h = RSD(d_rp, d_ci, d_v, d_par, d_dn, **prec)
            _, st, _ = h.solve(b, rtol=1e-10, restart=30, maxit=1000)
            h.close()
        torch.cuda.synchronize()
        plain_ms[name] = 1e3 * (time.perf_counter() - t0) / k
    reuse_sps = {}
    if a.reuse_solves > 0:
        for name in variants:
            reuse_sps[name] = reuse(MIXED if name == "mixed" else FP64, a.reuse_solves)

    head = "mixed" if "mixed" in res else variants[0]
    R0 = res[head]
    value = 1.0 / R0["sec"]

    # ---- roofline of the dominant kernel class of the headline variant
    ms = R0["ms"]
    nlch = R0["launches"]
    leaf_sizes = [ana["max_leaf_dofs"]] * ana["num_leaves"]   # uniform leaves here
    fp32_leaf = head == "mixed"
    cand = {
        "leaf_update": ms.get("leaf_update", 0.0),
        "root_update": ms.get("root_update", 0.0),
        "leaf_apply": ms.get("leaf_apply", 0.0),
    }
    dom = max(cand, key=cand.get)
    if dom in ("leaf_update", "root_update"):
        # achieved: n^3/3 per matrix (a Cholesky factorisation, the set-up rows' unit)
        # spread over the inversion's MFMA update launches; executed: the flops those
        # launches perform (the sweep inverts in place: about n^3 per matrix)
        sizes = leaf_sizes if dom == "leaf_update" else [ana["max_iface_dofs"]]
        fp32 = fp32_leaf and dom == "leaf_update"
        nl = nlch[dom]
        dur = ms[dom] / nl * 1e-3
        per_launch = potrf_flops(sizes) / nl
        executed = update_flops(sizes) / nl
        peak = PEAK["fp32_TFLOPs"] if fp32 else PEAK["fp64_TFLOPs"]
        roof = dict(kernel=("k_sweep_update_bf3s / k_sweep_update2 (sub-domain batch)"
                            if dom == "leaf_update" else
                            "k_sweep_update2<double> + k_sweep_update_la<double> (root interface: "
                            "bulk and look-ahead launches of each step)"),
                    bound="mfma", achieved=per_launch / dur / 1e12, peak=peak, unit="TFLOP/s",
                    work_unit="n^3/3 flops per matrix (Cholesky-equivalent) over the "
                              "inversion's update launches",
                    executed_TFLOPs=executed / dur / 1e12,
                    executed_frac=executed / dur / 1e12 / peak,
                    profile_key=("k_sweep_update_bf3s<%d>" % group_tiles(max(sizes)) if fp32
                                 else "root_update"))
    else:
        per_launch = leaf_apply_bytes(p, 4 if fp32_leaf else 8)
        dur = ms["leaf_apply"] / nlch["leaf_apply"] * 1e-3
        roof = dict(kernel="k_symv1+k_symv2 (sub-domain batch)", bound="hbm",
                    achieved=per_launch / dur / 1e9, peak=PEAK["hbm_GBps"], unit="GB/s",
                    profile_key="k_symv1<%s, 1, false>" % ("float" if fp32_leaf else "double"))
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["avg_launch_ms"] = dur * 1e3
    roof["traffic"] = measured_traffic(roof.pop("profile_key"))
    # secondary figures (not the roofline object): leaf apply bandwidth, root update rate,
    # from the fully instrumented warm-up step
    extra = {}
    ms, nlch = R0["phase_ms"], R0["phase_launches"]
    if R0["launches"].get("leaf_apply"):
        lb = leaf_apply_bytes(p, 4 if fp32_leaf else 8)
        extra["leaf_apply_GBps"] = lb / (ms["leaf_apply"] / nlch["leaf_apply"] * 1e-3) / 1e9
    if R0["launches"].get("spmv"):
        # K in internal order: values 8 B + column 4 B per nonzero, row pointers 8 B per
        # row, x (gathered, read once from HBM at best) and y 8 B per row
        sb = 12 * p.K.nnz + 24 * p.n
        extra["spmv_GBps"] = sb / (ms["spmv"] / nlch["spmv"] * 1e-3) / 1e9
    for cls, sizes in (("root_update", [ana["max_iface_dofs"]]), ("leaf_update", leaf_sizes)):
        if R0["launches"].get(cls):
            sec_cls = ms[cls] * 1e-3
            extra[cls + "_TFLOPs_potrf_unit"] = potrf_flops(sizes) / sec_cls / 1e12
            extra[cls + "_TFLOPs_executed"] = update_flops(sizes) / sec_cls / 1e12

    blocks = set(a.blocks.split(","))
    adjoint = bench_adjoint(a, dev) if "adjoint32" in blocks and a.only is None else None
    elastic = bench_elasticity(a, dev) if "elasticity48" in blocks and a.only is None else None
    big = bench_poisson256(a, dev) if "poisson256" in blocks and a.only is None else None

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload, and the
    # error of every non-FP64 result against it
    cpu = None
    errors = None
    if not a.no_cpu_baseline and a.only is None:
        try:
            from threadpoolctl import threadpool_info

            from oracle import RSDOracle
            threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
            c0, t0 = time.process_time(), time.perf_counter()
            orc = RSDOracle(p.K, p.parent, p.dof_node)
            t1 = time.perf_counter()
            z = orc.apply(p.b[:, 0])
            t2 = time.perf_counter()
            _ = p.K @ z
            t3 = time.perf_counter()
            c1 = time.process_time()
            beta = float(np.mean(res["fp64"]["its"])) if "fp64" in res else float(np.mean(R0["its"]))
            sec_solve = (t1 - t0) + beta * ((t2 - t1) + (t3 - t2))
            cpu = dict(value=1.0 / sec_solve, unit="solves/s", cores=threads, kind="oracle",
                       estimate=True, effective_cores=(c1 - c0) / (t3 - t0),
                       sample=(f"measured: FP64 oracle set-up ({t1 - t0:.1f} s), one RSD apply "
                               f"({t2 - t1:.2f} s) and one SpMV on the full 64^3 problem; "
                               f"estimated time per solve = set-up + {beta:.0f} x (apply + SpMV), "
                               f"beta = the FP64 FGMRES iteration count on the GPU.  cores = "
                               f"the BLAS thread pool (dense factorisations and solves); the "
                               f"recursion itself is one Python thread (effective_cores = CPU "
                               f"time / wall time of the sample)"))
            # apply error of each variant against the FP64 oracle (same right-hand side)
            errors = {}
            for name in variants:
                h = RSD(d_rp, d_ci, d_v, d_par, d_dn, **(MIXED if name == "mixed" else FP64))
                zg = h.apply(b).cpu().numpy()
                h.close()
                errors[name] = dict(max_rel=float(np.abs(zg - z).max() / np.abs(z).max()),
                                    l2_rel=float(np.linalg.norm(zg - z) / np.linalg.norm(z)))
            errors["workload"] = "diffusion 64^3 (the headline problem): z = M^{-1} b"
        except Exception as e:  # the baseline is a report, not the product
            cpu = dict(value=None, unit="solves/s", cores=None, kind="oracle",
                       sample=f"failed: {e!r}")
        if "poisson256" in set(a.blocks.split(",")):
            errors = errors if errors is not None else {}
            errors["bf16_hybrid_256cube_tree_shape"] = bf16_shape_error(a, dev)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": R0["steps"],
        "warmup": a.warmup,
        "ms_per_step": R0["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "diffusion 64^3 Q1 hex, log-normal k (sigma 1), 4x4x4 box "
                               "sub-domains (octree, 2 interface levels), FGMRES(30) to 1e-10, "
                               + ("FP32 sub-domain/Sigma/level-1 blocks + FP64 root and Krylov"
                                  if head == "mixed" else "all FP64"),
                   "n": int(p.n), "nnz": int(p.K.nnz), "seed": a.seed, "nrhs": 1},
        "time_to_1e-10_s": {k: r["sec"] for k, r in res.items()},
        "iterations": {k: r["its"][-1] for k, r in res.items()},
        "relres": {k: r["relres"] for k, r in res.items()},
        "solves_per_s_handle_reuse": reuse_sps,
        "host_analysis_ms": {k: r["host_ms"] for k, r in res.items()},
        "setup_wall_ms": {k: r["setup_wall_ms"] for k, r in res.items()},
        "phase_ms_per_step": {k: r["phase_ms"] for k, r in res.items()},
        "device_bytes": {k: r["device_bytes"] for k, r in res.items()},
        "roofline": roof,
        "secondary": extra,
        "adjoint32": adjoint,
        "elasticity48": elastic,
        "poisson256": big,
        "cpu_baseline": cpu,
        "timing_instrumented": "the roofline's kernel class (HIP events around its launches); "
                               "phase_ms_per_step from one step timed in every class",
        "ms_per_step_uninstrumented": plain_ms,
        "apply_error_vs_fp64_oracle": errors,
    }
    if "mixed" in res and "fp64" in res:
        out["mixed_vs_fp64_speedup"] = res["fp64"]["sec"] / res["mixed"]["sec"]
        xm, xd = res["mixed"]["x"], res["fp64"]["x"]
        out["mixed_solution_rel_diff_vs_fp64"] = float(np.linalg.norm(xm - xd) / np.linalg.norm(xd))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
