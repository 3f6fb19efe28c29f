"""ctypes binding of the C ABI in include/rsd.h (argument marshalling only).

The functions keep the C names (rsd_setup, rsd_apply, rsd_solve, rsd_spmv,
rsd_update_values, rsd_get_stats, rsd_destroy, rsd_last_error, rsd_release_cache,
rsd_apply_noalloc, rsd_analyze).
Device arrays are PyTorch tensors on the current HIP device; PyTorch only
provides the device memory and the stream.  Every step of the method runs in
librsd.so; when the library is missing, loading raises instead of falling back.

``RSD`` wraps a handle for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "librsd.so")
_lib = None

RSD_OK = 0
STATUS = {0: "RSD_OK", 1: "RSD_ERR_INVALID_ARGUMENT", 2: "RSD_ERR_MAP_NOT_SEPARABLE",
          3: "RSD_ERR_NOT_SPD", 4: "RSD_ERR_NOT_CONVERGED", 5: "RSD_ERR_BREAKDOWN",
          6: "RSD_ERR_OUT_OF_MEMORY", 7: "RSD_ERR_DEVICE", 8: "RSD_ERR_UNSUPPORTED"}
PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
SOLVER = {"fgmres": 0, "pcg": 1}
COUPLING = {"full": 0, "leaf_only": 1}
IFACE = {"dense": 0, "gamma": 1, "hybrid": 2}
TIMER_NAMES = ["setup_extract", "leaf_inverse", "leaf_update", "sigma", "iface_assembly",
               "iface_inverse", "iface_update", "root_update", "leaf_apply", "iface_apply",
               "coupling", "spmv", "krylov", "permute"]


class rsd_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p)]


class rsd_hierarchy(C.Structure):
    _fields_ = [("num_nodes", C.c_int32), ("parent", C.c_void_p), ("dof_node", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class rsd_options(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("leaf_prec", C.c_int32), ("sigma_prec", C.c_int32),
                ("iface_prec", C.c_int32), ("root_prec", C.c_int32),
                ("host_pointers", C.c_int32), ("timing", C.c_int32),
                ("iface_mode", C.c_int32), ("gamma", C.c_int32), ("dense_max", C.c_int32),
                ("graphs", C.c_int32), ("autotune", C.c_int32), ("symmetric", C.c_int32),
                ("g_coupling", C.c_int32), ("bf16_split", C.c_int32), ("sym_form", C.c_int32),
                ("timing_classes", C.c_int32),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_ctx", C.c_void_p)]


class rsd_solve_options(C.Structure):
    _fields_ = [("method", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("rtol", C.c_double), ("use_x0", C.c_int32)]


class rsd_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("relres", C.c_double), ("status", C.c_int32)]


class rsd_analysis(C.Structure):
    _fields_ = [("num_leaves", C.c_int32), ("num_levels", C.c_int32),
                ("max_leaf_dofs", C.c_int32), ("max_iface_dofs", C.c_int32),
                ("max_boundary_dofs", C.c_int32), ("leaf_dofs", C.c_int64),
                ("skeleton_dofs", C.c_int64), ("sum_leaf_sq", C.c_int64),
                ("sum_iface_sq", C.c_int64), ("sum_sigma_apply", C.c_int64),
                ("sum_sigma_sq", C.c_int64), ("leaf_inverse_flops", C.c_double),
                ("iface_inverse_flops", C.c_double)]


class rsd_stats(C.Structure):
    _fields_ = [("analysis", rsd_analysis), ("time_ms", C.c_double * 14),
                ("launches", C.c_int64 * 14), ("host_analysis_ms", C.c_double),
                ("device_bytes", C.c_int64), ("setup_wall_ms", C.c_double * 4),
                ("vec_pass", C.c_int32 * 8), ("setup_variant", C.c_int32 * 8),
                ("sym_persist", C.c_int32 * 8)]


class rsd_fe_map(C.Structure):
    _fields_ = [("num_elements", C.c_int32), ("dofs_per_element", C.c_int32),
                ("nnz", C.c_int64), ("elem_dofs", C.c_void_p), ("ke", C.c_void_p),
                ("contrib_ptr", C.c_void_p), ("contrib", C.c_void_p)]


COEF = {"linear": 0, "exp": 1}

EXPORTS = ["rsd_options_default", "rsd_analyze", "rsd_setup", "rsd_apply", "rsd_spmv",
           "rsd_solve", "rsd_update_values", "rsd_get_stats", "rsd_destroy", "rsd_last_error",
           "rsd_release_cache", "rsd_apply_noalloc", "rsd_fe_assemble", "rsd_fe_grad"]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Loads librsd.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built: run `python -m paper_1210_6266_amd.build`")
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library links against)
    except ImportError:
        pass
    lib = C.CDLL(_LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.rsd_options_default.argtypes = [C.POINTER(rsd_options)]
    lib.rsd_options_default.restype = None
    lib.rsd_analyze.argtypes = [C.POINTER(rsd_csr), C.POINTER(rsd_hierarchy), C.POINTER(rsd_analysis)]
    lib.rsd_setup.argtypes = [C.POINTER(rsd_csr), C.POINTER(rsd_hierarchy), C.POINTER(rsd_options),
                              vp, C.POINTER(vp)]
    lib.rsd_apply.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    lib.rsd_apply_noalloc.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    lib.rsd_spmv.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    lib.rsd_solve.argtypes = [vp, i32, vp, i64, vp, i64, C.POINTER(rsd_solve_options),
                              C.POINTER(rsd_solve_info), vp]
    lib.rsd_update_values.argtypes = [vp, vp, vp]
    lib.rsd_get_stats.argtypes = [vp, C.POINTER(rsd_stats), i32, vp]
    lib.rsd_destroy.argtypes = [vp]
    lib.rsd_destroy.restype = None
    lib.rsd_last_error.argtypes = [vp]
    lib.rsd_last_error.restype = C.c_char_p
    lib.rsd_release_cache.argtypes = [i32]
    lib.rsd_release_cache.restype = None
    lib.rsd_fe_assemble.argtypes = [C.POINTER(rsd_fe_map), vp, i32, vp, vp]
    lib.rsd_fe_grad.argtypes = [C.POINTER(rsd_fe_map), vp, i32, vp, vp, vp, vp]
    for f in ["rsd_analyze", "rsd_setup", "rsd_apply", "rsd_apply_noalloc", "rsd_spmv",
              "rsd_solve", "rsd_update_values", "rsd_get_stats", "rsd_fe_assemble",
              "rsd_fe_grad"]:
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


class RSDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _check(st: int, handle=None):
    if st != RSD_OK:
        raise RSDError(st, rsd_last_error(handle))


# ------------------------------------------------------------------ C names
def rsd_last_error(handle=None) -> str:
    return load().rsd_last_error(handle).decode()


def rsd_options_default() -> rsd_options:
    o = rsd_options()
    load().rsd_options_default(C.byref(o))
    return o


def rsd_analyze(row_ptr: np.ndarray, col_idx: np.ndarray, parent: np.ndarray,
                dof_node: np.ndarray) -> dict:
    """Host-only analysis (numpy int64 row_ptr, int32 col_idx / parent / dof_node)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    dof_node = np.ascontiguousarray(dof_node, dtype=np.int32)
    csr = rsd_csr(len(row_ptr) - 1, int(row_ptr[-1]) if len(row_ptr) else 0, _ptr(row_ptr),
                  _ptr(col_idx), None)
    hier = rsd_hierarchy(len(parent), _ptr(parent), _ptr(dof_node))
    out = rsd_analysis()
    _check(load().rsd_analyze(C.byref(csr), C.byref(hier), C.byref(out)))
    return {k: getattr(out, k) for k, _ in rsd_analysis._fields_}


def rsd_setup(row_ptr, col_idx, values, parent, dof_node, options: rsd_options | None = None,
              stream=None) -> int:
    """Arrays: torch tensors on the device (or numpy arrays with options.host_pointers = 1)."""
    n = int(row_ptr.shape[0]) - 1
    nnz = int(col_idx.shape[0])
    csr = rsd_csr(n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(values))
    hier = rsd_hierarchy(int(parent.shape[0]), _ptr(parent), _ptr(dof_node))
    h = C.c_void_p()
    opt = C.byref(options) if options is not None else None
    _check(load().rsd_setup(C.byref(csr), C.byref(hier), opt, _stream(stream), C.byref(h)))
    return h.value


def _cols(t, n):
    """(nrhs, ld) of a device vector block: 1-D (n,) or 2-D (n, nrhs) column-major."""
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError("vectors must be contiguous")
        return 1, t.shape[0]
    if t.shape[1] <= 1 and (t.stride(0) == 1 or t.shape[0] <= 1):
        return t.shape[1], max(n, 1)       # one column: any ld >= n describes it
    if t.stride(0) != 1 or t.stride(1) < n:
        raise ValueError("2-D blocks must be column-major (stride (1, ld) with ld >= n)")
    return t.shape[1], t.stride(1)


def colmajor(t):
    """A column-major copy of a 1-D or 2-D tensor (the layout the C ABI takes)."""
    return t.contiguous() if t.dim() == 1 else t.t().contiguous().t()


def rsd_apply(handle, r, z, stream=None):
    nrhs, ldr = _cols(r, r.shape[0])
    _, ldz = _cols(z, z.shape[0])
    _check(load().rsd_apply(handle, nrhs, _ptr(r), ldr, _ptr(z), ldz, _stream(stream)), handle)


def rsd_apply_noalloc(handle, r, z, stream=None):
    """rsd_apply on the library's static work area (no device allocation)."""
    nrhs, ldr = _cols(r, r.shape[0])
    _, ldz = _cols(z, z.shape[0])
    _check(load().rsd_apply_noalloc(handle, nrhs, _ptr(r), ldr, _ptr(z), ldz, _stream(stream)),
           handle)


def rsd_spmv(handle, x, y, stream=None):
    nrhs, ldx = _cols(x, x.shape[0])
    _, ldy = _cols(y, y.shape[0])
    _check(load().rsd_spmv(handle, nrhs, _ptr(x), ldx, _ptr(y), ldy, _stream(stream)), handle)


def rsd_solve(handle, b, x, method="fgmres", restart=30, maxit=500, rtol=1e-10, use_x0=False,
              stream=None):
    """Returns (status, [info dicts]); x is overwritten.  Does not raise on NOT_CONVERGED
    or BREAKDOWN (the per-column status says which)."""
    nrhs, ldb = _cols(b, b.shape[0])
    _, ldx = _cols(x, x.shape[0])
    o = rsd_solve_options(SOLVER[method], restart, maxit, rtol, 1 if use_x0 else 0)
    info = (rsd_solve_info * max(1, nrhs))()
    st = load().rsd_solve(handle, nrhs, _ptr(b), ldb, _ptr(x), ldx, C.byref(o), info,
                          _stream(stream))
    if st not in (RSD_OK, 4, 5):
        _check(st, handle)
    return st, [dict(iterations=info[j].iterations, relres=info[j].relres, status=info[j].status)
                for j in range(nrhs)]


def rsd_update_values(handle, values, stream=None):
    _check(load().rsd_update_values(handle, _ptr(values), _stream(stream)), handle)


def rsd_get_stats(handle, reset=False, stream=None) -> dict:
    s = rsd_stats()
    _check(load().rsd_get_stats(handle, C.byref(s), 1 if reset else 0, _stream(stream)), handle)
    out = {k: getattr(s.analysis, k) for k, _ in rsd_analysis._fields_}
    out["time_ms"] = {TIMER_NAMES[i]: s.time_ms[i] for i in range(len(TIMER_NAMES))}
    out["launches"] = {TIMER_NAMES[i]: s.launches[i] for i in range(len(TIMER_NAMES))}
    out["host_analysis_ms"] = s.host_analysis_ms
    out["device_bytes"] = s.device_bytes
    out["setup_wall_ms"] = list(s.setup_wall_ms)
    out["vec_pass"] = list(s.vec_pass)
    out["setup_variant"] = list(s.setup_variant)
    out["sym_persist"] = list(s.sym_persist)
    return out


def rsd_destroy(handle):
    if handle:
        load().rsd_destroy(handle)


def rsd_release_cache(device: int = -1):
    """Returns the library's cached device blocks, pinned buffers and idle streams to the
    runtime (device < 0: every device)."""
    load().rsd_release_cache(int(device))


# ------------------------------------------------------------------ convenience
def torch_empty_like(t):
    return t.new_empty(t.shape)


class RSD:
    """One RSD preconditioner handle over a CSR matrix on the current HIP device."""

    def __init__(self, row_ptr, col_idx, values, parent, dof_node, leaf_prec="fp64",
                 sigma_prec=None, iface_prec=None, root_prec="fp64", timing=False, stream=None,
                 interface="dense", gamma=8, dense_max=32768, graphs=True, autotune=True,
                 symmetric=True, coupling="full", allocator=None, bf16_split=True,
                 persistent_symv=False, timed_classes=None):
        """interface: "dense" (exact interface solves), "gamma" (gamma steps of GMRES on
        every interface system, the paper's mode) or "hybrid" (gamma steps where an
        interface has more than dense_max dofs).  coupling: "full" or "leaf_only" (the
        right-hand side of the interface systems, rsd_options.g_coupling).  allocator:
        None (the library's own block cache) or "torch" (the handle's device memory
        comes from PyTorch's caching allocator, tied to the stream given here or, without
        one, to the stream current at construction: blocks the handle grows later come
        from that stream's pool too).  stream: None (torch's current stream at each
        call) or a fixed stream; calls on other streams are ordered by the library.
        bf16_split: FP32 blocks inverted with their trailing updates on the BF16 matrix
        cores (operands split exactly into three BF16 parts), rsd_options.bf16_split.
        persistent_symv: the applies' symmetric products always as persistent work-queue
        launches (rsd_options.sym_form = 1; otherwise the autotuner may pick them).
        timed_classes: with timing, the names (TIMER_NAMES) of the kernel classes timed
        (rsd_options.timing_classes); None: all."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())

        def dv(a, dt):
            t = torch.as_tensor(a)
            return t.to(device=dev, dtype=dt).contiguous()

        self.row_ptr = dv(row_ptr, torch.int64)
        self.col_idx = dv(col_idx, torch.int32)
        self.values = dv(values, torch.float64)
        self.parent = dv(parent, torch.int32)
        self.dof_node = dv(dof_node, torch.int32)
        self.n = self.row_ptr.numel() - 1
        o = rsd_options_default()
        o.leaf_prec = PREC[leaf_prec]
        low = "fp32" if leaf_prec in ("fp16", "bf16") else leaf_prec   # 16 bits: leaves only
        o.sigma_prec = PREC[sigma_prec or low]
        o.iface_prec = PREC[iface_prec or low]
        o.root_prec = PREC[root_prec]
        o.timing = 1 if timing else 0
        if timed_classes is not None:
            mask = 0
            for name in timed_classes:
                mask |= 1 << TIMER_NAMES.index(name)
            if mask == 0:
                raise ValueError("timed_classes: no class")
            o.timing_classes = mask
        o.iface_mode = IFACE[interface]
        o.gamma = int(gamma)
        o.dense_max = int(dense_max)
        o.graphs = 1 if graphs else 0
        o.symmetric = 1 if symmetric else 0
        o.autotune = 1 if autotune else 0
        o.g_coupling = COUPLING[coupling]
        o.bf16_split = 1 if bf16_split else 0
        o.sym_form = 1 if persistent_symv else 0
        self._alloc_cbs = None
        if allocator == "torch":
            if stream is None:
                stream_obj = torch.cuda.current_stream(dev)
            elif isinstance(stream, int):
                stream_obj = torch.cuda.ExternalStream(stream)
            else:
                stream_obj = stream

            def _alloc(nbytes, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream_obj)
                except Exception:   # out of memory: the library reports RSD_ERR_OUT_OF_MEMORY
                    return None

            def _free(p, ctx):
                torch.cuda.caching_allocator_delete(p)

            self._alloc_cbs = (ALLOC_FN(_alloc), FREE_FN(_free))   # kept alive with the handle
            o.dev_alloc, o.dev_free = self._alloc_cbs
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        self.stream = stream
        self.handle = rsd_setup(self.row_ptr, self.col_idx, self.values, self.parent,
                                self.dof_node, o, stream)

    def apply(self, r, out=None):
        r = colmajor(r)
        z = out if out is not None else colmajor(torch_empty_like(r))
        rsd_apply(self.handle, r, z, self.stream)
        return z

    def spmv(self, x, out=None):
        x = colmajor(x)
        y = out if out is not None else colmajor(torch_empty_like(x))
        rsd_spmv(self.handle, x, y, self.stream)
        return y

    def solve(self, b, x=None, **kw):
        b = colmajor(b)
        use_x0 = x is not None
        x = colmajor(x) if x is not None else colmajor(b.new_zeros(b.shape))
        st, info = rsd_solve(self.handle, b, x, use_x0=use_x0, stream=self.stream, **kw)
        return x, st, info

    def update_values(self, values):
        import torch
        self.values = torch.as_tensor(values).to(self.values.device, torch.float64).contiguous()
        rsd_update_values(self.handle, self.values, self.stream)

    def stats(self, reset=False):
        return rsd_get_stats(self.handle, reset, self.stream)

    def close(self):
        if self.handle:
            rsd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ coefficient maps
class FEMap:
    """Device copy of a coefficient map (include/rsd_fe.h) built from numpy arrays
    (elem_dofs int32 E x d, ke d x d, contrib_ptr int64 nnz+1, contrib int32)."""

    def __init__(self, fe: dict, device=None):
        import torch
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.elem_dofs = torch.as_tensor(np.ascontiguousarray(fe["elem_dofs"], dtype=np.int32), device=dev)
        self.ke = torch.as_tensor(np.asfortranarray(fe["ke"], dtype=np.float64).ravel(order="F"), device=dev)
        self.contrib_ptr = torch.as_tensor(np.ascontiguousarray(fe["contrib_ptr"], dtype=np.int64), device=dev)
        self.contrib = torch.as_tensor(np.ascontiguousarray(fe["contrib"], dtype=np.int32), device=dev)
        self.num_elements = int(fe["elem_dofs"].shape[0])
        self.dofs_per_element = int(fe["elem_dofs"].shape[1])
        self.nnz = int(fe["contrib_ptr"].shape[0]) - 1
        self.c = rsd_fe_map(self.num_elements, self.dofs_per_element, self.nnz,
                            _ptr(self.elem_dofs), _ptr(self.ke), _ptr(self.contrib_ptr),
                            _ptr(self.contrib))


def rsd_fe_assemble(fmap: FEMap, theta, kind: str, values, stream=None):
    _check(load().rsd_fe_assemble(C.byref(fmap.c), _ptr(theta), COEF[kind], _ptr(values),
                                  _stream(stream)))


def rsd_fe_grad(fmap: FEMap, theta, kind: str, lam, x, grad, stream=None):
    _check(load().rsd_fe_grad(C.byref(fmap.c), _ptr(theta), COEF[kind], _ptr(lam), _ptr(x),
                              _ptr(grad), _stream(stream)))
