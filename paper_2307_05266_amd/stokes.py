"""Thin ctypes binding of libstokes.so (include/stokes.h, include/stokes_server.h).

Argument marshalling only: every step of the solve runs in the HIP library.
The functions keep the C names; `Stokes` wraps one context.  torch is
imported before the library is loaded so that the process holds a single HIP
runtime (torch's), and torch provides the device memory of caller-side
tensors and the stream the library runs on.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede the library load: one HIP runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstokes.so")

STOKES_OK, STOKES_NOT_CONVERGED = 0, 1
STOKES_E_ARG, STOKES_E_NOMEM, STOKES_E_DEVICE, STOKES_E_BREAKDOWN, STOKES_E_STATE, STOKES_E_LIMIT = \
    -1, -2, -3, -4, -5, -6
STOKES_UZAWA, STOKES_SIMPLE = 0, 1
(STOKES_OP_A, STOKES_OP_B, STOKES_OP_BT, STOKES_OP_SHAT, STOKES_OP_DIAG_A, STOKES_OP_DIAG_SHAT,
 STOKES_OP_PROJECT, STOKES_OP_S, STOKES_OP_MG_SHAT, STOKES_OP_MG_A) = range(10)
STOKES_KEEP_ALL_COMPONENTS = 0x1
STOKES_FLAG_NO_FLOW, STOKES_FLAG_ZERO_RHS, STOKES_FLAG_INNER_MAXIT, STOKES_FLAG_MG_TWO_VISITS = 0x1, 0x2, 0x4, 0x8

EXPORTED = [
    "stokes_setup", "stokes_setup_ex", "stokes_set_stream", "stokes_set_option", "stokes_solve",
    "stokes_permeability", "stokes_get_report", "stokes_history", "stokes_get_fields",
    "stokes_apply", "stokes_apply_device", "stokes_info", "stokes_kernel_timing",
    "stokes_destroy", "stokes_status_str", "stokes_preprocess", "stokes_setup_on_stream",
    "stokes_estimate_bytes", "stokes_apply_device_noalloc", "stokes_setup_with_allocator",
    "stokes_setup_batch", "stokes_batch_result", "stokes_solve_rhs",
]
EXPORTED_SERVER = [
    "stokes_server_create", "stokes_server_submit", "stokes_server_wait", "stokes_server_stats",
    "stokes_server_clock", "stokes_server_destroy", "stokes_server_set_batching",
]


class StokesReport(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("flags", ctypes.c_uint),
        ("outer_iters", ctypes.c_int), ("inner_A_iters", ctypes.c_int), ("inner_S_iters", ctypes.c_int),
        ("n_components", ctypes.c_int), ("n_components_kept", ctypes.c_int),
        ("k_hat", ctypes.c_double), ("k_vox", ctypes.c_double), ("mean_u", ctypes.c_double * 3),
        ("rel_res", ctypes.c_double), ("rel_res_prec", ctypes.c_double), ("r0_norm", ctypes.c_double),
        ("div_norm", ctypes.c_double), ("cond_est", ctypes.c_double),
        ("ritz_min", ctypes.c_double), ("ritz_max", ctypes.c_double),
        ("porosity", ctypes.c_double), ("porosity_effective", ctypes.c_double),
        ("stv_ratio", ctypes.c_double), ("seconds", ctypes.c_double),
    ]

    def to_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "mean_u" else v
        return d


class StokesRequestResult(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64), ("status", ctypes.c_int), ("N", ctypes.c_int), ("k_hat", ctypes.c_double),
        ("outer_iters", ctypes.c_int), ("inner_A_iters", ctypes.c_int), ("inner_S_iters", ctypes.c_int),
        ("rel_res", ctypes.c_double), ("div_norm", ctypes.c_double), ("device_bytes", ctypes.c_int64),
        ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_end", ctypes.c_double),
        ("batch_members", ctypes.c_int),
    ]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class StokesAllocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class TorchDeviceMemory:
    """Device memory of a context from PyTorch's caching allocator, on the torch
    stream the context runs on.  Holds the ctypes callbacks (they must outlive
    the context) and the blocks it handed out."""

    def __init__(self, stream):
        self.stream = stream
        self.device = stream.device
        self.live = {}

        def alloc(nbytes, _stream, _user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:   # out of memory: the library reports STOKES_E_NOMEM
                return None
            self.live[ptr] = int(nbytes)
            return ptr

        def free(ptr, _nbytes, _stream, _user):
            if self.live.pop(ptr, None) is not None:
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:   # interpreter shutdown: torch is already gone
                    pass

        self._alloc = _ALLOC_FN(alloc)
        self._free = _FREE_FN(free)
        self.struct = StokesAllocator(self._alloc, self._free, None)

    @property
    def bytes_held(self):
        return sum(self.live.values())


class StokesError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


_lib = None


def load():
    """Load libstokes.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run paper_2307_05266_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "stokes_setup": ([ctypes.POINTER(vp), vp, ip, dp], ip),
        "stokes_setup_ex": ([ctypes.POINTER(vp), vp, ip, dp, ctypes.c_uint], ip),
        "stokes_set_stream": ([vp, vp], ip),
        "stokes_set_option": ([vp, ctypes.c_char_p, ctypes.c_double], ip),
        "stokes_solve": ([vp, ip, ctypes.c_double, ctypes.POINTER(StokesReport)], ip),
        "stokes_permeability": ([vp, dp], ip),
        "stokes_get_report": ([vp, ctypes.POINTER(StokesReport)], ip),
        "stokes_history": ([vp, vp, ip, ctypes.POINTER(ip)], ip),
        "stokes_get_fields": ([vp, vp, vp], ip),
        "stokes_apply": ([vp, ip, vp, vp], ip),
        "stokes_apply_device": ([vp, ip, vp, vp], ip),
        "stokes_apply_device_noalloc": ([vp, ip, vp, vp], ip),
        "stokes_info": ([vp, i64p], ip),
        "stokes_kernel_timing": ([vp, ip, dp, i64p, dp], ip),
        "stokes_destroy": ([vp], None),
        "stokes_status_str": ([ip], ctypes.c_char_p),
        "stokes_preprocess": ([vp, ip, dp, ctypes.c_uint, i64p, vp, vp], ip),
        "stokes_setup_on_stream": ([ctypes.POINTER(vp), vp, ip, dp, ctypes.c_uint, vp], ip),
        "stokes_setup_with_allocator": ([ctypes.POINTER(vp), vp, ip, dp, ctypes.c_uint, vp,
                                         ctypes.POINTER(StokesAllocator)], ip),
        "stokes_setup_batch": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ip, ip, dp, ctypes.c_uint, vp], ip),
        "stokes_batch_result": ([vp, ip, ctypes.POINTER(StokesReport), vp, vp], ip),
        "stokes_solve_rhs": ([vp, ip, ctypes.c_double, vp, ctypes.POINTER(StokesReport)], ip),
        "stokes_estimate_bytes": ([ip, ctypes.c_uint, ip, i64p], ip),
        "stokes_server_create": ([ctypes.POINTER(vp), ip, ctypes.c_int64], ip),
        "stokes_server_submit": ([vp, vp, ip, dp, ip, ctypes.c_double, ip, i64p], ip),
        "stokes_server_wait": ([vp, ctypes.c_int64, ctypes.POINTER(StokesRequestResult)], ip),
        "stokes_server_stats": ([vp, i64p], ip),
        "stokes_server_set_batching": ([vp, ip, ctypes.c_int64], ip),
        "stokes_server_clock": ([vp], ctypes.c_double),
        "stokes_server_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def status_str(s: int) -> str:
    return load().stokes_status_str(int(s)).decode()


def _check(st, what, ok=(STOKES_OK,)):
    if st not in ok:
        raise StokesError(st, what)
    return st


# ---- functions with the C names ---------------------------------------------------
def stokes_setup(mask, N, force, flags=0):
    lib = load()
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    if m.size != N ** 3:
        raise ValueError("mask must hold N^3 bytes")
    f = np.ascontiguousarray(force, dtype=np.float64)
    h = ctypes.c_void_p()
    st = lib.stokes_setup_ex(ctypes.byref(h), m.ctypes.data, int(N),
                             f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_uint(flags))
    _check(st, "stokes_setup")
    return h


def stokes_setup_with_allocator(mask, N, force, flags, stream, allocator):
    """stream: a hipStream_t as an int (0 = default); allocator: a StokesAllocator."""
    lib = load()
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    if m.size != N ** 3:
        raise ValueError("mask must hold N^3 bytes")
    f = np.ascontiguousarray(force, dtype=np.float64)
    h = ctypes.c_void_p()
    st = lib.stokes_setup_with_allocator(ctypes.byref(h), m.ctypes.data, int(N),
                                         f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_uint(flags),
                                         ctypes.c_void_p(stream), ctypes.byref(allocator))
    _check(st, "stokes_setup_with_allocator")
    return h


def stokes_preprocess(mask, N, force, flags=0, want_fields=True):
    """Host-only geometry preprocessing: counts, kept-fluid mask, component labels."""
    lib = load()
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    if m.size != N ** 3:
        raise ValueError("mask must hold N^3 bytes")
    f = np.ascontiguousarray(force, dtype=np.float64)
    counts = (ctypes.c_int64 * 6)()
    fluid = np.zeros(N ** 3, dtype=np.uint8) if want_fields else None
    label = np.zeros(N ** 3, dtype=np.int32) if want_fields else None
    st = lib.stokes_preprocess(m.ctypes.data, int(N), f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.c_uint(flags), counts,
                               fluid.ctypes.data if want_fields else None,
                               label.ctypes.data if want_fields else None)
    _check(st, "stokes_preprocess")
    keys = ["nfluid_in", "nfluid", "nsurf", "ncomp_all", "ncomp_kept"]
    out = {k: int(counts[i]) for i, k in enumerate(keys)}
    if want_fields:
        out["fluid"] = fluid.reshape(N, N, N)
        out["label"] = label.reshape(N, N, N)
    return out


def stokes_set_stream(ctx, stream):
    return _check(load().stokes_set_stream(ctx, ctypes.c_void_p(stream)), "stokes_set_stream")


def stokes_set_option(ctx, key, value):
    return _check(load().stokes_set_option(ctx, key.encode(), float(value)), f"stokes_set_option({key})")


def stokes_solve(ctx, precond, tol):
    rep = StokesReport()
    st = load().stokes_solve(ctx, int(precond), float(tol), ctypes.byref(rep))
    _check(st, "stokes_solve", ok=(STOKES_OK, STOKES_NOT_CONVERGED))
    return st, rep.to_dict()


def stokes_permeability(ctx):
    k = ctypes.c_double()
    _check(load().stokes_permeability(ctx, ctypes.byref(k)), "stokes_permeability")
    return k.value


def stokes_history(ctx, cap=100000):
    n = ctypes.c_int()
    out = np.zeros((cap, 8))
    _check(load().stokes_history(ctx, out.ctypes.data, cap, ctypes.byref(n)), "stokes_history")
    return out[:min(n.value, cap)].copy()


def stokes_get_fields(ctx, N):
    p = np.zeros(N ** 3)
    u = np.zeros(3 * N ** 3)
    _check(load().stokes_get_fields(ctx, p.ctypes.data, u.ctypes.data), "stokes_get_fields")
    return p.reshape(N, N, N), u.reshape(3, N, N, N)


def _op_shapes(op, N):
    face_in = op in (STOKES_OP_A, STOKES_OP_B, STOKES_OP_MG_A)
    face_out = op in (STOKES_OP_A, STOKES_OP_BT, STOKES_OP_DIAG_A, STOKES_OP_MG_A)
    return (3 * N ** 3 if face_in else N ** 3), (3 * N ** 3 if face_out else N ** 3), face_out


def stokes_apply(ctx, op, x, N):
    nin, nout, face_out = _op_shapes(op, N)
    if x is None:
        xin = np.zeros(nin)
    else:
        xin = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        if xin.size != nin:
            raise ValueError("input has the wrong size for this operator")
    out = np.zeros(nout)
    _check(load().stokes_apply(ctx, int(op), xin.ctypes.data, out.ctypes.data), "stokes_apply")
    return out.reshape((3, N, N, N) if face_out else (N, N, N))


def stokes_apply_device(ctx, op, x, out):
    """x, out: contiguous float64 torch tensors on the GPU (sizes as in stokes_apply)."""
    for t in (x, out):
        if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()):
            raise ValueError("stokes_apply_device needs contiguous float64 GPU tensors")
    xp = x.data_ptr() if x is not None else None
    return _check(load().stokes_apply_device(ctx, int(op), ctypes.c_void_p(xp), ctypes.c_void_p(out.data_ptr())),
                  "stokes_apply_device")


def stokes_apply_device_noalloc(ctx, op, x, out, ok=(STOKES_OK,)):
    """As stokes_apply_device, through the entry point that allocates nothing
    (its scratch is the library's fixed device array).  Returns the status;
    statuses outside `ok` raise StokesError."""
    for t in (x, out):
        if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()):
            raise ValueError("stokes_apply_device_noalloc needs contiguous float64 GPU tensors")
    xp = x.data_ptr() if x is not None else None
    return _check(load().stokes_apply_device_noalloc(ctx, int(op), ctypes.c_void_p(xp),
                                                     ctypes.c_void_p(out.data_ptr())),
                  "stokes_apply_device_noalloc", ok)


def stokes_info(ctx):
    info = (ctypes.c_int64 * 12)()
    _check(load().stokes_info(ctx, info), "stokes_info")
    keys = ["N", "nfluid_in", "nfluid", "nsurf", "ncomp_all", "ncomp_kept", "nface_x", "nface_y", "nface_z",
            "device_bytes", "mg_levels_S", "mg_levels_A"]
    return {k: int(info[i]) for i, k in enumerate(keys)}


KERNEL_NAMES = ["k_cgA_dir", "k_cgA_stencil_tiled", "k_cgA_update", "k_cgS_dir", "k_cgS_stencil_tiled", "k_cgS_update",
                "k_mgf_tiled<A,restrict>", "k_mgf_tiled<A,smooth>", "k_mgf_tiled<S,restrict>",
                "k_mgf_tiled<S,smooth>", "k_mgf_update_restrict<A>", "k_mgf_update_restrict<S>",
                "k_cgA_dirstencil_tiled", "k_cgS_dirstencil_tiled",
                "k_mgf_update_restrict_S_pipe", "k_mgf_smooth_S_pipe", "k_cgS_dirstencil_pipe"]


def stokes_kernel_timing(ctx, kernel):
    """(total ms, launches, algorithmic bytes per launch) of one inner-loop kernel."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    nbytes = ctypes.c_double()
    _check(load().stokes_kernel_timing(ctx, int(kernel), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(nbytes)),
           "stokes_kernel_timing")
    return ms.value, n.value, nbytes.value


def stokes_destroy(ctx):
    if ctx:
        load().stokes_destroy(ctx)


# ---- convenience wrapper ------------------------------------------------------------
class Stokes:
    """One geometry on the GPU.  mask: uint8 (N, N, N) indexed [k][j][i], 1 = fluid."""

    def __init__(self, mask, force=(1.0, 0.0, 0.0), keep_all=False, stream=None, torch_memory=True, **options):
        """stream: a torch.cuda.Stream or a raw hipStream_t (int); default the
        current torch stream.  torch_memory: the context's device memory comes
        from torch's caching allocator on that stream (default); False: the
        library allocates it with hipMalloc."""
        mask = np.asarray(mask)
        self.N = int(mask.shape[0])
        flags = STOKES_KEEP_ALL_COMPONENTS if keep_all else 0
        self._mem = None
        if torch.cuda.is_available():
            if stream is None:
                stream = torch.cuda.current_stream()
            elif isinstance(stream, int):
                stream = torch.cuda.ExternalStream(stream)
            if torch_memory:
                self._mem = TorchDeviceMemory(stream)
                self._ctx = stokes_setup_with_allocator(mask, self.N, force, flags, stream.cuda_stream,
                                                        self._mem.struct)
            else:
                self._ctx = stokes_setup(mask, self.N, force, flags)
                stokes_set_stream(self._ctx, stream.cuda_stream)
        else:
            self._ctx = stokes_setup(mask, self.N, force, flags)
            if stream is not None:
                stokes_set_stream(self._ctx, stream if isinstance(stream, int) else stream.cuda_stream)
        for k, v in options.items():
            stokes_set_option(self._ctx, k, v)

    def set_option(self, key, value):
        stokes_set_option(self._ctx, key, value)

    def solve(self, precond=STOKES_SIMPLE, tol=1e-8):
        if isinstance(precond, str):
            precond = {"uzawa": STOKES_UZAWA, "simple": STOKES_SIMPLE}[precond.lower()]
        st, rep = stokes_solve(self._ctx, precond, tol)
        return rep

    def solve_rhs(self, g, precond=STOKES_SIMPLE, tol=1e-8):
        """CG on S p = g for a given g (N^3 cells, in the range of B); FP64."""
        if isinstance(precond, str):
            precond = {"uzawa": STOKES_UZAWA, "simple": STOKES_SIMPLE}[precond.lower()]
        gd = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        if gd.size != self.N ** 3:
            raise ValueError("g must hold N^3 values")
        rep = StokesReport()
        st = load().stokes_solve_rhs(self._ctx, int(precond), float(tol), gd.ctypes.data, ctypes.byref(rep))
        _check(st, "stokes_solve_rhs", ok=(STOKES_OK, STOKES_NOT_CONVERGED))
        return rep.to_dict()

    def permeability(self):
        return stokes_permeability(self._ctx)

    def history(self):
        return stokes_history(self._ctx)

    def fields(self):
        return stokes_get_fields(self._ctx, self.N)

    def apply(self, op, x=None):
        return stokes_apply(self._ctx, op, x, self.N)

    def apply_device(self, op, x, out):
        return stokes_apply_device(self._ctx, op, x, out)

    def apply_device_noalloc(self, op, x, out, ok=(STOKES_OK,)):
        return stokes_apply_device_noalloc(self._ctx, op, x, out, ok)

    def info(self):
        return stokes_info(self._ctx)

    def kernel_timing(self, kernel):
        return stokes_kernel_timing(self._ctx, kernel)

    def close(self):
        if getattr(self, "_ctx", None):
            stokes_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stokes_estimate_bytes(N, precision=0, flags=0):
    """Upper bound of the device bytes of a context for an N^3 box (host-only)."""
    out = ctypes.c_int64()
    _check(load().stokes_estimate_bytes(int(N), ctypes.c_uint(flags), int(precision), ctypes.byref(out)),
           "stokes_estimate_bytes")
    return out.value


def stokes_setup_on_stream(mask, N, force, flags, stream):
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    f = (ctypes.c_double * 3)(*[float(x) for x in force])
    ctx = ctypes.c_void_p()
    _check(load().stokes_setup_on_stream(ctypes.byref(ctx), mask.ctypes.data, int(N), f, ctypes.c_uint(flags),
                                         ctypes.c_void_p(stream)), "stokes_setup_on_stream")
    return ctx


class StokesBatch:
    """Several geometries of one size solved together (stokes_setup_batch):
    every kernel launch advances all members; mixed precision.  masks: a list
    of uint8 (N, N, N) arrays indexed [k][j][i], 1 = fluid."""

    def __init__(self, masks, force=(1.0, 0.0, 0.0), keep_all=False, stream=None, **options):
        arrs = [np.ascontiguousarray(m, dtype=np.uint8) for m in masks]
        if not arrs:
            raise ValueError("a batch needs at least one mask")
        self.N = int(arrs[0].shape[0])
        if any(a.shape != (self.N,) * 3 for a in arrs):
            raise ValueError("all members need the same N^3 shape")
        self.size = len(arrs)
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        ptrs = (ctypes.c_void_p * self.size)(*[a.ctypes.data for a in arrs])
        f = np.ascontiguousarray(force, dtype=np.float64)
        self._ctx = ctypes.c_void_p()
        _check(load().stokes_setup_batch(ctypes.byref(self._ctx), ptrs, self.size, self.N,
                                         f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.c_uint(STOKES_KEEP_ALL_COMPONENTS if keep_all else 0),
                                         ctypes.c_void_p(stream)), "stokes_setup_batch")
        for k, v in options.items():
            stokes_set_option(self._ctx, k, v)

    def set_option(self, key, value):
        stokes_set_option(self._ctx, key, value)

    def solve(self, precond=STOKES_SIMPLE, tol=1e-8):
        """Solves every member; returns the list of their reports."""
        if isinstance(precond, str):
            precond = {"uzawa": STOKES_UZAWA, "simple": STOKES_SIMPLE}[precond.lower()]
        rep = StokesReport()
        load().stokes_solve(self._ctx, int(precond), float(tol), ctypes.byref(rep))
        return [self.result(m)[0] for m in range(self.size)]

    def result(self, member, fields=False):
        """(report, p, u) of one member; p and u only with fields=True."""
        rep = StokesReport()
        N = self.N
        p = np.zeros(N ** 3) if fields else None
        u = np.zeros(3 * N ** 3) if fields else None
        _check(load().stokes_batch_result(self._ctx, int(member), ctypes.byref(rep),
                                          p.ctypes.data if fields else None, u.ctypes.data if fields else None),
               "stokes_batch_result")
        if fields:
            return rep.to_dict(), p.reshape(N, N, N), u.reshape(3, N, N, N)
        return rep.to_dict(), None, None

    def info(self):
        return stokes_info(self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            stokes_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SERVER_STATS = ["submitted", "completed", "queued", "running", "bytes_in_use", "peak_bytes", "peak_running",
                "budget", "contexts", "requests_on_contexts"]


class Server:
    """Request server (include/stokes_server.h): `slots` workers, each with its
    own stream, admit queued solves as slots and HBM budget free up."""

    def __init__(self, slots, hbm_budget_bytes, max_members=None, max_cells=None):
        lib = load()
        self._srv = ctypes.c_void_p()
        _check(lib.stokes_server_create(ctypes.byref(self._srv), int(slots), ctypes.c_int64(int(hbm_budget_bytes))),
               "stokes_server_create")
        if max_members is not None or max_cells is not None:
            self.set_batching(32 if max_members is None else max_members, 1 << 21 if max_cells is None else max_cells)

    def set_batching(self, max_members, max_cells=1 << 21):
        _check(load().stokes_server_set_batching(self._srv, int(max_members), ctypes.c_int64(int(max_cells))),
               "stokes_server_set_batching")

    def submit(self, mask, force=(1.0, 0.0, 0.0), precond=STOKES_SIMPLE, tol=1e-8, precision=1):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        N = int(mask.shape[0])
        f = (ctypes.c_double * 3)(*[float(x) for x in force])
        rid = ctypes.c_int64()
        _check(load().stokes_server_submit(self._srv, mask.ctypes.data, N, f, int(precond), float(tol),
                                           int(precision), ctypes.byref(rid)), "stokes_server_submit")
        return rid.value

    def wait(self, rid):
        out = StokesRequestResult()
        _check(load().stokes_server_wait(self._srv, ctypes.c_int64(rid), ctypes.byref(out)), "stokes_server_wait")
        return out.to_dict()

    def stats(self):
        st = (ctypes.c_int64 * 10)()
        _check(load().stokes_server_stats(self._srv, st), "stokes_server_stats")
        return {k: int(st[i]) for i, k in enumerate(SERVER_STATS)}

    def clock(self):
        return load().stokes_server_clock(self._srv)

    def close(self):
        if getattr(self, "_srv", None):
            load().stokes_server_destroy(self._srv)
            self._srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
