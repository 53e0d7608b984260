"""Space-time parabolic solver for MI355X: Python binding of ``libstp.so``.

The library (HIP kernels for gfx950 behind the C-ABI declared in
``include/stp.h``) does all of the computation; this module only marshals
arguments.  Functions carry the C names.  Host arrays are NumPy float64
arrays; device arrays are contiguous float64 torch CUDA tensors (torch is
used for device memory and streams only).  The library must have been built
(``python -m paper_2009_08875_amd.build``); importing without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_HERE, "libstp.so")

STP_OK = 0
STP_NOT_CONVERGED = 1
STP_E_INVALID_ARG = -1
STP_E_OUT_OF_MEMORY = -2
STP_E_BREAKDOWN = -3
STP_E_DEVICE = -4
STP_E_UNSUPPORTED = -5
STP_E_BUSY = -6

STP_FP64 = 0
STP_MIXED = 1

STP_OP_W, STP_OP_WT, STP_OP_S, STP_OP_SHAT, STP_OP_KX, STP_OP_KSPACE, STP_OP_RHS, STP_OP_A, STP_OP_M = range(9)


class stp_options(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("vcycles", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("maxit", ctypes.c_int), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("graph", ctypes.c_int), ("nested", ctypes.c_int),
                ("diffusion", ctypes.c_double * 3), ("reaction", ctypes.c_double),
                ("dim", ctypes.c_int), ("lookahead", ctypes.c_int)]


class stp_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("status", ctypes.c_int), ("coarse_iterations", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class stp_request(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int), ("K", ctypes.c_int), ("precision", ctypes.c_int),
                ("rel_tol", ctypes.c_double), ("u0", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("on_device", ctypes.c_int)]


class stp_server_stats(ctypes.Structure):
    _fields_ = [("waiting", ctypes.c_int), ("running_groups", ctypes.c_int),
                ("unfinished", ctypes.c_int), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t), ("groups_started", ctypes.c_int64),
                ("requests_started", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class stp_kernel_stat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int), ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


(STP_KERNEL_MG_PRE, STP_KERNEL_MG_POST, STP_KERNEL_SYN_UPDATE, STP_KERNEL_ANA_DOT,
 STP_KERNEL_TIME_STENCIL, STP_KERNEL_COMBINE, STP_KERNEL_UPDATE_WR, STP_KERNEL_DOT) = range(8)
STP_KERNEL_NAMES = {STP_KERNEL_MG_PRE: "mg_pre", STP_KERNEL_MG_POST: "mg_post",
                    STP_KERNEL_SYN_UPDATE: "syn_update", STP_KERNEL_ANA_DOT: "ana_dot",
                    STP_KERNEL_TIME_STENCIL: "time_stencil", STP_KERNEL_COMBINE: "combine",
                    STP_KERNEL_UPDATE_WR: "update_wr", STP_KERNEL_DOT: "dot"}


class StpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _load():
    # torch carries its own HIP runtime (libamdhip64, soname libamdhip64.so.7)
    # and loads it by an unversioned name, so a process that loaded the system
    # runtime first would end up with two.  Importing torch first makes this
    # library bind to the runtime torch already loaded.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIBRARY_PATH):
        raise ImportError(
            f"{LIBRARY_PATH} is missing: build it with `python -m paper_2009_08875_amd.build` "
            "(the solver has no fallback path)")
    lib = ctypes.CDLL(LIBRARY_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sigs = {
        "stp_create": [i, i, i, i, ctypes.POINTER(stp_options), vp, ctypes.POINTER(vp)],
        "stp_set_u0": [vp, i, vp, i],
        "stp_set_g": [vp, i, vp, i],
        "stp_solve": [vp, d, ctypes.POINTER(stp_stats)],
        "stp_get_solution": [vp, i, vp, i],
        "stp_get_iterations": [vp, i, ctypes.POINTER(i)],
        "stp_footprint": [i, i, i, i, ctypes.POINTER(sz)],
        "stp_apply": [vp, i, i, i, vp, vp, i],
        "stp_profile": [vp, i],
        "stp_profile_read": [vp, i, ctypes.POINTER(stp_kernel_stat)],
        "stp_server_create": [sz, i, i, ctypes.POINTER(stp_options), ctypes.POINTER(vp)],
        "stp_server_submit": [vp, ctypes.POINTER(stp_request), ctypes.POINTER(ctypes.c_uint64)],
        "stp_server_poll": [vp, ctypes.c_uint64, ctypes.POINTER(stp_stats),
                            ctypes.POINTER(ctypes.c_double)],
        "stp_server_drain": [vp],
        "stp_server_info": [vp, ctypes.POINTER(stp_server_stats)],
        "stp_server_destroy": [vp],
        "stp_kspace_apply_static": [i, i, vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i
    lib.stp_destroy.argtypes = [vp]
    lib.stp_destroy.restype = None
    lib.stp_status_string.argtypes = [i]
    lib.stp_status_string.restype = ctypes.c_char_p
    lib.stp_last_error.argtypes = []
    lib.stp_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def _check(status, allow_warning=True):
    if status < 0 or (status > 0 and not allow_warning):
        msg = _lib.stp_last_error().decode() or _lib.stp_status_string(status).decode()
        raise StpError(status, msg)
    return status


def _ptr(a, count=None):
    """(address, on_device) of a float64 NumPy array or torch CUDA tensor."""
    if a is None:
        return None, 0
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
            raise TypeError("host arrays must be C-contiguous float64")
        if count is not None and a.size != count:
            raise ValueError(f"expected {count} values, got {a.size}")
        return a.ctypes.data, 0
    import torch  # device buffers only

    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise TypeError("expected a NumPy array or a CUDA tensor")
    if a.dtype != torch.float64 or not a.is_contiguous():
        raise TypeError("device tensors must be contiguous float64")
    if count is not None and a.numel() != count:
        raise ValueError(f"expected {count} values, got {a.numel()}")
    return a.data_ptr(), 1


def _options(options):
    if options is None:
        return None
    if isinstance(options, stp_options):
        return ctypes.byref(options)
    opts = dict(options)
    if "diffusion" in opts:
        opts["diffusion"] = (ctypes.c_double * 3)(*[float(v) for v in opts["diffusion"]])
    o = stp_options(**opts)
    return ctypes.byref(o)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def grid_n(K):
    return 2 ** K - 1


# ------------------------------------------------------------ solver C-ABI

def stp_create(J, K, nrhs=1, precision=STP_FP64, options=None, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.stp_create(J, K, nrhs, precision, _options(options), _stream(stream), ctypes.byref(h)))
    return h


def stp_destroy(ctx):
    _lib.stp_destroy(ctx)


def stp_set_u0(ctx, rhs, u0, K=None):
    p, dev = _ptr(u0, None if K is None else grid_n(K) ** 2)
    return _check(_lib.stp_set_u0(ctx, rhs, p, dev))


def stp_set_g(ctx, rhs, g):
    p, dev = _ptr(g)
    return _check(_lib.stp_set_g(ctx, rhs, p, dev))


def stp_solve(ctx, rel_tol, nrhs=1):
    stats = (stp_stats * nrhs)()
    status = _check(_lib.stp_solve(ctx, rel_tol, stats))
    return status, [s.as_dict() for s in stats]


def stp_get_solution(ctx, rhs, out):
    p, dev = _ptr(out)
    _check(_lib.stp_get_solution(ctx, rhs, p, dev))
    return out


def stp_get_iterations(ctx, rhs):
    v = ctypes.c_int()
    _check(_lib.stp_get_iterations(ctx, rhs, ctypes.byref(v)))
    return v.value


def stp_footprint(J, K, nrhs=1, precision=STP_FP64):
    v = ctypes.c_size_t()
    _check(_lib.stp_footprint(J, K, nrhs, precision, ctypes.byref(v)))
    return v.value


def stp_apply(ctx, op, precision, rhs, inp, out):
    pi, dev_i = _ptr(inp)
    po, dev_o = _ptr(out)
    if inp is not None and dev_i != dev_o:
        raise ValueError("input and output must both be host or both device arrays")
    return _check(_lib.stp_apply(ctx, op, precision, rhs, pi, po, dev_o))


def stp_profile(ctx, enable):
    return _check(_lib.stp_profile(ctx, 1 if enable else 0))


def stp_profile_read(ctx, kernel):
    st = stp_kernel_stat()
    _check(_lib.stp_profile_read(ctx, kernel, ctypes.byref(st)))
    return st.as_dict()


def stp_status_string(status):
    return _lib.stp_status_string(status).decode()


def stp_last_error():
    return _lib.stp_last_error().decode()


STP_STATIC_SCRATCH_BYTES = 256 << 20


def stp_kspace_apply_static(K, rows, inp, out, stream=None):
    """K_x on `rows` rows (device tensors of rows x N_x float64), every
    intermediate in the library's fixed device array: no allocation."""
    n = grid_n(K) ** 2
    pi, dev_i = _ptr(inp, rows * n)
    po, dev_o = _ptr(out, rows * n)
    if not (dev_i and dev_o):
        raise TypeError("stp_kspace_apply_static takes device tensors")
    return _check(_lib.stp_kspace_apply_static(K, rows, pi, po, _stream(stream)))


# ------------------------------------------------------------ serving C-ABI

# Buffers of submitted requests stay referenced here until the request is
# collected by stp_server_poll (the library reads and writes them meanwhile).
_server_refs = {}


def stp_server_create(hbm_budget_bytes, max_slots, max_batch=1, options=None):
    h = ctypes.c_void_p()
    _check(_lib.stp_server_create(int(hbm_budget_bytes), max_slots, max_batch, _options(options),
                                  ctypes.byref(h)))
    return h


def stp_server_submit(server, J, K, precision, rel_tol, u0=None, g=None, u=None):
    """Queue one solve.  u0 (N_x), g ((2^J+1) N_x) and u (output, same size as
    g) are float64 host arrays or CUDA tensors (all on the same side); None
    means zero data / no output."""
    n = grid_n(K) ** 2
    bufs = [(u0, n), (g, ((1 << J) + 1) * n), (u, ((1 << J) + 1) * n)]
    ptrs, sides = [], set()
    for a, count in bufs:
        p, dev = _ptr(a, count)
        ptrs.append(p)
        if a is not None:
            sides.add(dev)
    if len(sides) > 1:
        raise TypeError("u0, g and u must all be host arrays or all be device tensors")
    req = stp_request(J, K, precision, rel_tol, ptrs[0], ptrs[1], ptrs[2], sides.pop() if sides else 0)
    rid = ctypes.c_uint64()
    _check(_lib.stp_server_submit(server, ctypes.byref(req), ctypes.byref(rid)))
    _server_refs[(server.value, rid.value)] = (u0, g, u)
    return rid.value


def stp_server_poll(server, rid):
    """None while the request waits or runs; then (status, stats, latency_s).
    A failed request raises StpError."""
    st = stp_stats()
    lat = ctypes.c_double()
    status = _lib.stp_server_poll(server, rid, ctypes.byref(st), ctypes.byref(lat))
    if status == STP_E_BUSY:
        return None
    _server_refs.pop((server.value, rid), None)
    _check(status)
    return status, st.as_dict(), lat.value


def stp_server_drain(server):
    return _check(_lib.stp_server_drain(server))


def stp_server_info(server):
    out = stp_server_stats()
    _check(_lib.stp_server_info(server, ctypes.byref(out)))
    return out.as_dict()


def stp_server_destroy(server):
    status = _check(_lib.stp_server_destroy(server))
    for key in [k for k in _server_refs if k[0] == server.value]:
        del _server_refs[key]
    return status
