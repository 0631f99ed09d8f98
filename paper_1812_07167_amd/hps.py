"""Thin ctypes binding of libhps.so (include/hps.h).

Argument marshalling only: every step of the build and the solve runs in the library's
HIP kernels.  Torch is used for device memory and streams: the device-pointer entry
points take torch tensors on the GPU and pass their data pointers through.  There is no
CPU fallback; calling a compute entry point without the built library raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhps.so")

HPS_OK, HPS_E_INVALID, HPS_E_NOMEM, HPS_E_SINGULAR, HPS_E_DEVICE, HPS_E_NOT_CONVERGED, HPS_E_BUSY = range(7)
OP_PSI, OP_Y, OP_R, OP_WINV, OP_PHI_A, OP_PHI_B, OP_R33A, OP_R33B, OP_R13A, OP_R23B = range(10)

EXPORTS = [
    "hps_last_error", "hps_version", "hps_default_opts", "hps_nodes", "hps_build",
    "hps_build_batch", "hps_solve", "hps_solve_batch", "hps_solve_jumps", "hps_residual",
    "hps_solve_noalloc",
    "hps_last_solve_info", "hps_factor_query",
    "hps_factor_get", "hps_factor_box", "hps_stage_times", "hps_free", "hps_estimate_bytes",
    "hps_release_cached", "hps_set_allocator", "hps_autotune_entries", "hps_autotune_clear",
    "hps_autotune_save", "hps_autotune_load",
    "hps_server_default_opts", "hps_server_create", "hps_server_submit_build",
    "hps_server_submit_solve", "hps_server_release", "hps_server_poll", "hps_server_stats",
    "hps_server_destroy",
]
HPS_REQ_BUILD, HPS_REQ_SOLVE = 0, 1
HPS_PREC_C128, HPS_PREC_MIXED = 0, 1


# hps_alloc_fn / hps_free_fn of include/hps.h
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class HPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"HPS error {code}: {msg}")
        self.code = code


class Domain(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("keep_all_R", C.c_int32), ("store_root_R", C.c_int32),
                ("profile", C.c_int32), ("stream", C.c_void_p), ("fp64_top_levels", C.c_int32),
                ("refine_max_iter", C.c_int32), ("refine_tol", C.c_double),
                ("autotune", C.c_int32), ("leaf_route", C.c_int32),
                ("interface_pivoting", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("correction", C.c_double)]


class StageTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int32), ("reserved", C.c_int32),
                ("ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


class FactorInfo(C.Structure):
    _fields_ = [("p", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("levels", C.c_int32),
                ("nleaf", C.c_int64), ("n_leaf_nodes", C.c_int64), ("n_interior", C.c_int64),
                ("n_root", C.c_int64), ("device_bytes", C.c_int64)]


class ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_batch_rhs", C.c_int32),
                ("max_pending_builds", C.c_int32), ("evict_idle", C.c_int32),
                ("solve_slots", C.c_int32), ("share_problems", C.c_int32)]


class Completion(C.Structure):
    _fields_ = [("req", C.c_uint64), ("problem", C.c_uint64), ("kind", C.c_int32),
                ("status", C.c_int32), ("nrhs", C.c_int32), ("batch_rhs", C.c_int32),
                ("iterations", C.c_int32), ("rebuilt", C.c_int32), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_end", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("builds", C.c_int64), ("rebuilds", C.c_int64), ("evictions", C.c_int64),
                ("solves", C.c_int64), ("rhs", C.c_int64), ("batches", C.c_int64),
                ("rejected", C.c_int64), ("failed", C.c_int64), ("resident", C.c_int32),
                ("pending", C.c_int32), ("max_concurrent", C.c_int32), ("slots", C.c_int32),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double),
                ("wall_s", C.c_double), ("rhs_per_s", C.c_double), ("solves_per_s", C.c_double),
                ("budget_bytes", C.c_int64), ("committed_bytes", C.c_int64),
                ("peak_committed_bytes", C.c_int64), ("shared_batches", C.c_int64),
                ("shared_problems", C.c_int64), ("retried", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_1812_07167_amd.build")
    # One HIP runtime per process: when torch is present its bundled runtime is loaded
    # first, and libhps.so's libamdhip64.so.7 dependency then resolves to it by soname.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P, D, I32, I64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
    lib.hps_last_error.restype = C.c_char_p
    lib.hps_version.restype = I32
    lib.hps_default_opts.argtypes = [C.POINTER(Opts)]
    lib.hps_default_opts.restype = None
    lib.hps_nodes.argtypes = [C.POINTER(Domain), I32, P, P, P, P]
    lib.hps_build.argtypes = [C.POINTER(Domain), I32, D, D, D, P, C.POINTER(Opts), C.POINTER(P)]
    lib.hps_solve.argtypes = [P, I32, P, P, P]
    lib.hps_solve_noalloc.argtypes = [P, I32, P, P, P]
    lib.hps_solve_jumps.argtypes = [P, I32, P, P, P, P]
    lib.hps_build_batch.argtypes = [I32, P, P, P, P, P, P, C.POINTER(Opts), P]
    lib.hps_solve_batch.argtypes = [I32, P, P, P, P, P]
    lib.hps_residual.argtypes = [P, I32, P, P, P, P, P]
    lib.hps_last_solve_info.argtypes = [P, C.POINTER(SolveInfo)]
    lib.hps_factor_query.argtypes = [P, C.POINTER(FactorInfo)]
    lib.hps_factor_get.argtypes = [P, I32, I32, I32, P, I64, C.POINTER(I32), C.POINTER(I32)]
    lib.hps_factor_box.argtypes = [P, I32, I32] + [C.POINTER(I32)] * 4
    lib.hps_stage_times.argtypes = [P, I32, C.POINTER(StageTime), I32, C.POINTER(I32)]
    lib.hps_free.argtypes = [P]
    lib.hps_free.restype = None
    lib.hps_release_cached.argtypes = []
    lib.hps_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
    lib.hps_autotune_entries.argtypes = [C.POINTER(I32)]
    lib.hps_autotune_clear.argtypes = []
    lib.hps_autotune_save.argtypes = [C.c_char_p]
    lib.hps_autotune_load.argtypes = [C.c_char_p]
    lib.hps_estimate_bytes.argtypes = [C.POINTER(Domain), I32, C.POINTER(Opts), C.POINTER(I64),
                                       C.POINTER(I64)]
    lib.hps_server_default_opts.argtypes = [C.POINTER(ServerOpts)]
    lib.hps_server_default_opts.restype = None
    lib.hps_server_create.argtypes = [C.c_size_t, C.POINTER(ServerOpts), C.POINTER(P)]
    U64 = C.c_uint64
    lib.hps_server_submit_build.argtypes = [P, C.POINTER(Domain), I32, D, D, D, P,
                                            C.POINTER(Opts), C.POINTER(U64), C.POINTER(U64)]
    lib.hps_server_submit_solve.argtypes = [P, U64, I32, P, P, P, C.POINTER(U64)]
    lib.hps_server_release.argtypes = [P, U64]
    lib.hps_server_poll.argtypes = [P, C.POINTER(Completion), I32, I32, C.POINTER(I32)]
    lib.hps_server_stats.argtypes = [P, C.POINTER(Stats)]
    lib.hps_server_destroy.argtypes = [P]
    lib.hps_server_destroy.restype = None
    for name in ["hps_nodes", "hps_build", "hps_build_batch", "hps_solve", "hps_solve_batch",
                 "hps_solve_noalloc",
                 "hps_solve_jumps", "hps_residual",
                 "hps_last_solve_info", "hps_factor_query", "hps_factor_get", "hps_factor_box",
                 "hps_stage_times", "hps_estimate_bytes", "hps_release_cached",
                 "hps_set_allocator", "hps_server_create",
                 "hps_autotune_entries", "hps_autotune_clear", "hps_autotune_save",
                 "hps_autotune_load",
                 "hps_server_submit_build", "hps_server_submit_solve", "hps_server_release",
                 "hps_server_poll", "hps_server_stats"]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(code):
    if code != HPS_OK:
        raise HPSError(code, load().hps_last_error().decode())


def domain(nx, ny, box=(0.0, 1.0, 0.0, 1.0)):
    return Domain(box[0], box[1], box[2], box[3], nx, ny)


def hps_nodes(dom: Domain, p: int):
    """Host arrays (xy_leaf, xy_interior, xy_root, nrm_root) in the ordering contract."""
    lib = load()
    nl, m = dom.nx * dom.ny, p - 2
    xy = np.zeros((nl * (p * p - 4), 2))
    xyi = np.zeros((nl * m * m, 2))
    nt = 2 * (dom.nx + dom.ny) * m
    xyb = np.zeros((nt, 2))
    nrm = np.zeros((nt, 2))
    _check(lib.hps_nodes(C.byref(dom), p, xy.ctypes.data, xyi.ctypes.data, xyb.ctypes.data,
                         nrm.ctypes.data))
    return xy, xyi, xyb, nrm


def _dev_ptr(t, dtype_name):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if str(t.dtype) != dtype_name:
        raise ValueError(f"expected dtype {dtype_name}, got {t.dtype}")
    return t.data_ptr()


class Factor:
    """Owning handle of a built factorization (hps_build / hps_free)."""

    def __init__(self, handle, stream_ptr):
        self.h = handle
        self.stream_ptr = stream_ptr
        info = FactorInfo()
        _check(load().hps_factor_query(self.h, C.byref(info)))
        self.info = info

    def free(self):
        if self.h:
            load().hps_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def get(self, what, level, box):
        """Copy one stored operator to a complex128 numpy array."""
        lib = load()
        rows, cols = C.c_int32(), C.c_int32()
        cap = 1
        while True:
            buf = np.zeros(cap, dtype=np.complex128)
            code = lib.hps_factor_get(self.h, what, level, box, buf.ctypes.data, cap,
                                      C.byref(rows), C.byref(cols))
            if code == HPS_OK:
                return buf[: rows.value * cols.value].reshape(cols.value, rows.value).T
            if rows.value * cols.value > cap:
                cap = rows.value * cols.value
                continue
            _check(code)

    def stage_times(self, which):
        """[(name, launches, ms, flops, bytes)] of the build (0) or the last solve (1)."""
        cap = 4096
        buf = (StageTime * cap)()
        n = C.c_int32()
        _check(load().hps_stage_times(self.h, which, buf, cap, C.byref(n)))
        return [(buf[i].name.decode(), buf[i].launches, buf[i].ms, buf[i].flops, buf[i].bytes)
                for i in range(n.value)]

    def last_solve_info(self):
        """(iterations, converged, last relative correction) of the most recent solve."""
        info = SolveInfo()
        _check(load().hps_last_solve_info(self.h, C.byref(info)))
        return info.iterations, bool(info.converged), info.correction

    def box(self, level, box):
        v = [C.c_int32() for _ in range(4)]
        _check(load().hps_factor_box(self.h, level, box, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)


def _opts(keep_all_R, store_root_R, stream, profile, precision, fp64_top_levels,
          refine_max_iter, refine_tol, autotune=False, leaf_route=0, interface_pivoting=0):
    import torch
    lib = load()
    opts = Opts()
    lib.hps_default_opts(C.byref(opts))
    opts.keep_all_R = int(keep_all_R)
    opts.store_root_R = int(store_root_R)
    opts.profile = int(profile)
    opts.precision = int(precision)
    if fp64_top_levels is not None:
        opts.fp64_top_levels = int(fp64_top_levels)
    if refine_max_iter is not None:
        opts.refine_max_iter = int(refine_max_iter)
    if refine_tol is not None:
        opts.refine_tol = float(refine_tol)
    opts.autotune = int(autotune)
    opts.leaf_route = int(leaf_route)
    opts.interface_pivoting = int(interface_pivoting)
    st = stream if stream is not None else torch.cuda.current_stream()
    opts.stream = C.c_void_p(st.cuda_stream)
    return opts, st


def hps_build_batch(doms, ps, kappas, etas, cs, keep_all_R=False, store_root_R=True,
                    stream=None, profile=False, precision=HPS_PREC_C128, fp64_top_levels=None,
                    refine_max_iter=None, refine_tol=None, autotune=False, leaf_route=0,
                    interface_pivoting=0):
    """Build several problems at once (problems of one shape share every launch).  doms:
    list of Domain; cs: list of float64 device tensors.  Returns a list of Factors."""
    lib = load()
    n = len(doms)
    opts, st = _opts(keep_all_R, store_root_R, stream, profile, precision, fp64_top_levels,
                     refine_max_iter, refine_tol, autotune, leaf_route, interface_pivoting)
    D = (Domain * n)(*doms)
    P = (C.c_int32 * n)(*[int(p) for p in ps])
    K = (C.c_double * n)(*[float(k) for k in kappas])
    ER = (C.c_double * n)(*[float(np.real(e)) for e in etas])
    EI = (C.c_double * n)(*[float(np.imag(e)) for e in etas])
    CP = (C.c_void_p * n)(*[_dev_ptr(c, "torch.float64") for c in cs])
    out = (C.c_void_p * n)()
    _check(lib.hps_build_batch(n, D, P, K, ER, EI, CP, C.byref(opts), out))
    return [Factor(C.c_void_p(out[i]), st.cuda_stream) for i in range(n)]


def hps_solve_batch(fs, ts, ss=None, us=None):
    """Solve several problems at once: ts[i] complex128 device tensor [nrhs_i, n_root];
    ss[i] [nrhs_i, n_interior] or None.  Returns the list of u tensors."""
    import torch
    lib = load()
    n = len(fs)
    if us is None:
        us = [torch.empty((t.shape[0], f.info.n_leaf_nodes), dtype=torch.complex128,
                          device=t.device) for f, t in zip(fs, ts)]
    H = (C.c_void_p * n)(*[f.h for f in fs])
    NR = (C.c_int32 * n)(*[int(t.shape[0]) for t in ts])
    S = None
    if ss is not None:
        S = (C.c_void_p * n)(*[(_dev_ptr(s, "torch.complex128") if s is not None else None)
                              for s in ss])
    T = (C.c_void_p * n)(*[_dev_ptr(t, "torch.complex128") for t in ts])
    U = (C.c_void_p * n)(*[_dev_ptr(u, "torch.complex128") for u in us])
    _check(lib.hps_solve_batch(n, H, NR, S, T, U))
    return us


def hps_build(dom: Domain, p: int, kappa: float, eta: complex, c_interior, keep_all_R=False,
              store_root_R=True, stream=None, profile=False, precision=HPS_PREC_C128,
              fp64_top_levels=None, refine_max_iter=None, refine_tol=None,
              autotune=False, leaf_route=0, interface_pivoting=0) -> Factor:
    """c_interior: float64 device tensor [nx*ny*(p-2)^2].  Returns a Factor.  Options left
    at None keep the library's defaults."""
    import torch
    lib = load()
    opts = Opts()
    lib.hps_default_opts(C.byref(opts))
    opts.keep_all_R = int(keep_all_R)
    opts.store_root_R = int(store_root_R)
    opts.profile = int(profile)
    opts.precision = int(precision)
    if fp64_top_levels is not None:
        opts.fp64_top_levels = int(fp64_top_levels)
    if refine_max_iter is not None:
        opts.refine_max_iter = int(refine_max_iter)
    if refine_tol is not None:
        opts.refine_tol = float(refine_tol)
    opts.autotune = int(autotune)
    opts.leaf_route = int(leaf_route)
    opts.interface_pivoting = int(interface_pivoting)
    st = stream if stream is not None else torch.cuda.current_stream()
    opts.stream = C.c_void_p(st.cuda_stream)
    out = C.c_void_p()
    ptr = _dev_ptr(c_interior, "torch.float64")
    _check(lib.hps_build(C.byref(dom), p, float(kappa), float(np.real(eta)), float(np.imag(eta)),
                         ptr, C.byref(opts), C.byref(out)))
    return Factor(out, st.cuda_stream)


def hps_solve(f: Factor, t, s=None, u=None):
    """t: complex128 device tensor [nrhs, n_root]; s: [nrhs, n_interior] or None.
    Returns u: complex128 device tensor [nrhs, n_leaf_nodes] (stream-ordered)."""
    import torch
    nrhs = t.shape[0]
    if u is None:
        u = torch.empty((nrhs, f.info.n_leaf_nodes), dtype=torch.complex128, device=t.device)
    sp = _dev_ptr(s, "torch.complex128") if s is not None else None
    _check(load().hps_solve(f.h, nrhs, sp, _dev_ptr(t, "torch.complex128"),
                            _dev_ptr(u, "torch.complex128")))
    return u


def hps_solve_noalloc(f: Factor, t, u, s=None):
    """As hps_solve, through the allocation-free entry point: the caller passes u
    (complex128 device tensor [nrhs, n_leaf_nodes]); the library allocates nothing."""
    nrhs = t.shape[0]
    sp = _dev_ptr(s, "torch.complex128") if s is not None else None
    _check(load().hps_solve_noalloc(f.h, nrhs, sp, _dev_ptr(t, "torch.complex128"),
                                    _dev_ptr(u, "torch.complex128")))
    return u


NOALLOC_SCRATCH_BYTES = 64 << 20


def hps_solve_jumps(f: Factor, t, s=None, jumps=None, u=None):
    """As hps_solve, with right-hand sides jumps [nrhs, nleaf, n_b] (complex128 device
    tensor or None) on the shared-edge rows of the global system."""
    import torch
    nrhs = t.shape[0]
    if u is None:
        u = torch.empty((nrhs, f.info.n_leaf_nodes), dtype=torch.complex128, device=t.device)
    sp = _dev_ptr(s, "torch.complex128") if s is not None else None
    jp = _dev_ptr(jumps, "torch.complex128") if jumps is not None else None
    _check(load().hps_solve_jumps(f.h, nrhs, sp, _dev_ptr(t, "torch.complex128"), jp,
                                  _dev_ptr(u, "torch.complex128")))
    return u


def hps_residual(f: Factor, u, t=None, s=None, jumps=None, r=None):
    """FP64 residual of the global collocation system at u [nrhs, n_leaf_nodes]; returns r
    of the same shape (per leaf: n_b boundary rows, then n_i interior rows)."""
    import torch
    nrhs = u.shape[0]
    if r is None:
        r = torch.empty_like(u)
    sp = _dev_ptr(s, "torch.complex128") if s is not None else None
    tp = _dev_ptr(t, "torch.complex128") if t is not None else None
    jp = _dev_ptr(jumps, "torch.complex128") if jumps is not None else None
    _check(load().hps_residual(f.h, nrhs, sp, tp, jp, _dev_ptr(u, "torch.complex128"),
                               _dev_ptr(r, "torch.complex128")))
    return r


def _plain_opts(precision=HPS_PREC_C128, fp64_top_levels=None, refine_max_iter=None,
                refine_tol=None, keep_all_R=False, store_root_R=True):
    """hps_opts without a stream (host-only calls and the request loop)."""
    opts = Opts()
    load().hps_default_opts(C.byref(opts))
    opts.precision = int(precision)
    opts.keep_all_R = int(keep_all_R)
    opts.store_root_R = int(store_root_R)
    if fp64_top_levels is not None:
        opts.fp64_top_levels = int(fp64_top_levels)
    if refine_max_iter is not None:
        opts.refine_max_iter = int(refine_max_iter)
    if refine_tol is not None:
        opts.refine_tol = float(refine_tol)
    return opts


def autotune_entries():
    n = C.c_int32()
    _check(load().hps_autotune_entries(C.byref(n)))
    return n.value


def autotune_clear():
    _check(load().hps_autotune_clear())


def autotune_save(path):
    _check(load().hps_autotune_save(str(path).encode()))


def autotune_load(path):
    _check(load().hps_autotune_load(str(path).encode()))


def hps_release_cached():
    """Return the library's cached workspace memory on the current device."""
    _check(load().hps_release_cached())


_hooks = []  # the installed callbacks (ctypes keeps no reference of its own)


def set_allocator(alloc=None, free=None):
    """Route the library's device memory through alloc(bytes, stream) -> int pointer and
    free(pointer, stream) (stream: the hipStream_t handle as an int, 0 for buffers that
    live across calls); with no arguments the library's own allocator returns.  Memory
    already handed out goes back to whoever provided it."""
    if (alloc is None) != (free is None):
        raise ValueError("set_allocator: give both alloc and free, or neither")
    if alloc is None:
        _check(load().hps_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    def a(nbytes, stream, ctx):
        try:
            return alloc(int(nbytes), int(stream or 0)) or None
        except Exception:  # an exception cannot cross into C: report no memory
            return None

    def f(ptr, stream, ctx):
        try:
            free(int(ptr), int(stream or 0))
        except Exception:
            pass

    cb = (ALLOC_FN(a), FREE_FN(f))
    _hooks.append(cb)  # kept for as long as memory they handed out may come back
    _check(load().hps_set_allocator(cb[0], cb[1], None))


def use_torch_allocator():
    """Serve the library's device memory from torch's caching allocator on the current
    device (stream-ordered on the stream the library names)."""
    import torch
    dev = torch.cuda.current_device()
    set_allocator(lambda n, st: torch.cuda.caching_allocator_alloc(n, dev, st),
                  lambda ptr, st: torch.cuda.caching_allocator_delete(ptr))


def hps_estimate_bytes(dom: Domain, p: int, **opts):
    """(build_peak, resident) device bytes of one problem's factorization (host only)."""
    peak, res = C.c_int64(), C.c_int64()
    o = _plain_opts(**opts)
    _check(load().hps_estimate_bytes(C.byref(dom), p, C.byref(o), C.byref(peak), C.byref(res)))
    return peak.value, res.value


class Server:
    """Request loop over resident factorizations (hps_server_*).  Tensors handed to
    solve() are kept referenced here until their completion has been polled."""

    def __init__(self, budget_bytes=0, slots=None, max_batch_rhs=None, max_pending_builds=None,
                 evict_idle=None, solve_slots=None, share_problems=None):
        lib = load()
        o = ServerOpts()
        lib.hps_server_default_opts(C.byref(o))
        if slots is not None:
            o.slots = int(slots)
        if max_batch_rhs is not None:
            o.max_batch_rhs = int(max_batch_rhs)
        if max_pending_builds is not None:
            o.max_pending_builds = int(max_pending_builds)
        if evict_idle is not None:
            o.evict_idle = int(evict_idle)
        if solve_slots is not None:
            o.solve_slots = int(solve_slots)
        if share_problems is not None:
            o.share_problems = int(share_problems)
        h = C.c_void_p()
        _check(lib.hps_server_create(int(budget_bytes), C.byref(o), C.byref(h)))
        self.h = h
        self._held = {}   # req -> tensors that must outlive the request
        self.shapes = {}  # problem -> (n_leaf_nodes, n_interior, n_root)

    def build(self, dom: Domain, p: int, kappa: float, eta: complex, c_interior, **opts):
        """Queue a build; c_interior (float64 device tensor) is copied before returning.
        Returns (problem_id, request_id)."""
        import torch
        o = _plain_opts(**opts)
        pid, req = C.c_uint64(), C.c_uint64()
        torch.cuda.synchronize()  # the server's streams do not wait on torch's
        _check(load().hps_server_submit_build(
            self.h, C.byref(dom), p, float(kappa), float(np.real(eta)), float(np.imag(eta)),
            _dev_ptr(c_interior, "torch.float64"), C.byref(o), C.byref(pid), C.byref(req)))
        nl, m = dom.nx * dom.ny, p - 2
        self.shapes[pid.value] = (nl * (p * p - 4), nl * m * m, 2 * (dom.nx + dom.ny) * m)
        return pid.value, req.value

    def solve(self, problem, t, s=None, u=None, sync=True):
        """Queue a solve: t [nrhs, n_root], s [nrhs, n_interior] or None (complex128 device
        tensors, complete on the device: sync=True synchronizes torch first).  Returns
        (request_id, u); u is valid once the request's completion is polled."""
        import torch
        nrhs = t.shape[0]
        if u is None:
            u = torch.empty((nrhs, self.shapes[problem][0]), dtype=torch.complex128,
                            device=t.device)
        if sync:
            torch.cuda.synchronize()
        req = C.c_uint64()
        sp = _dev_ptr(s, "torch.complex128") if s is not None else None
        _check(load().hps_server_submit_solve(self.h, problem, nrhs, sp,
                                              _dev_ptr(t, "torch.complex128"),
                                              _dev_ptr(u, "torch.complex128"), C.byref(req)))
        self._held[req.value] = (t, s, u)
        return req.value, u

    def release(self, problem):
        _check(load().hps_server_release(self.h, problem))

    def poll(self, max_n=256, timeout_ms=0):
        """List of completions (dicts); waits up to timeout_ms for the first."""
        buf = (Completion * max_n)()
        n = C.c_int32()
        _check(load().hps_server_poll(self.h, buf, max_n, int(timeout_ms), C.byref(n)))
        out = []
        for i in range(n.value):
            c = buf[i]
            out.append({k: getattr(c, k) for k, _ in Completion._fields_})
            self._held.pop(c.req, None)
        return out

    def wait(self, reqs, timeout_s=120.0):
        """Poll until every request id in reqs has completed; returns {req: completion}."""
        import time
        want, got = set(reqs), {}
        t_end = time.monotonic() + timeout_s
        while want - set(got):
            if time.monotonic() > t_end:
                raise TimeoutError(f"requests not completed: {sorted(want - set(got))[:8]}")
            for c in self.poll(256, 100):
                got[c["req"]] = c
        return got

    def stats(self):
        st = Stats()
        _check(load().hps_server_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def close(self):
        if self.h:
            load().hps_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
