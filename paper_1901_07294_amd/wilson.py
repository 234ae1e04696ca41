"""Python binding of the C ABI in include/wilson.h (argument marshalling only).

Every function has the name of its C entry point and forwards to it through
ctypes; all arithmetic runs in the HIP library. Device buffers may be given as
torch tensors (their ``data_ptr()`` is passed) or as integer addresses.
``stream=None`` means torch's current stream on the current device.

The library must have been built (``python -m paper_1901_07294_amd.build``);
the first call raises ImportError if ``libwilson.so`` is missing. There is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwilson.so")

WD_OK = 0
WD_PENDING = 1
WD_ERR_INVALID_ARG = -1
WD_ERR_SHAPE = -2
WD_ERR_UNSUPPORTED = -3
WD_ERR_NOMEM = -4
WD_ERR_DEVICE = -5
WD_ERR_NOT_CONVERGED = -6
WD_ERR_NUMERIC = -7
WD_ERR_UNKNOWN_TICKET = -8
WD_ERR_CANCELLED = -9
WD_ERR_INTERNAL = -10

WD_FP64 = 0
WD_FP32 = 1
WD_FP16 = 2

WD_FLAG_GAMMA5 = 1

ABI_VERSION = 4  # the structures below match this version of include/wilson.h

STATUS_NAMES = {v: k for k, v in dict(globals()).items()
                if k.startswith("WD_ERR_") or k in ("WD_OK", "WD_PENDING")}


class wd_cg_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("delta", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("x0_given", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class wd_cg_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters,
                "reliable_updates": self.reliable_updates,
                "true_rel_residual": self.true_rel_residual, "seconds": self.seconds}

class wd_tune_result(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("eligible", ctypes.c_int32), ("tb", ctypes.c_int32),
                ("gw", ctypes.c_int32), ("group", ctypes.c_int32), ("rb", ctypes.c_int32),
                ("default_us", ctypes.c_double), ("best_us", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class wd_server_cfg(ctypes.Structure):
    _fields_ = [("arena_dev", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("inner", ctypes.c_int32), ("check_every", ctypes.c_int32), ("delta", ctypes.c_double),
                ("max_rhs_per_group", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("evict_idle_gauges", ctypes.c_int32)]


class wd_request(ctypes.Structure):
    _fields_ = [("gauge_id", ctypes.c_uint64), ("nrhs", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("masses", ctypes.c_double * 16),
                ("b_dev", ctypes.c_void_p), ("x_dev", ctypes.c_void_p)]


class wd_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("stats", wd_cg_stats * 16)]

    def as_dict(self):
        return {"status": self.status, "nrhs": self.nrhs, "t_submit": self.t_submit,
                "t_start": self.t_start, "t_done": self.t_done,
                "stats": [self.stats[k].as_dict() for k in range(self.nrhs)]}


class wd_server_state(ctypes.Structure):
    _fields_ = [("arena_in_use", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
                ("unfinished", ctypes.c_int32), ("gauges", ctypes.c_int32),
                ("evictions", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# Exported C symbols and their ctypes signatures.
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p
_dims_t = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = {
    "wd_abi_version": (ctypes.c_int, []),
    "wd_last_error": (ctypes.c_char_p, []),
    "wd_spinor_bytes": (ctypes.c_size_t, [_dims_t, _i32, _i32]),
    "wd_gauge_bytes": (ctypes.c_size_t, [_dims_t, _i32, _i32]),
    "wd_gauge_import": (ctypes.c_int, [_dims_t, _vp, _i32, _i32, _vp, ctypes.c_size_t, _vp,
                                       ctypes.POINTER(_vp)]),
    "wd_gauge_release": (ctypes.c_int, [_vp]),
    "wd_spinor_import": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp]),
    "wd_spinor_export": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp]),
    "dslash_apply": (ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp, _i32, _i32, _vp]),
    "dslash_apply_multi": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), _i32, _vp, _vp,
                                          _i32, _i32, _vp]),
    "cg_workspace_bytes": (ctypes.c_size_t, [_dims_t, _i32, _i32]),
    "wd_server_create": (ctypes.c_int, [ctypes.POINTER(wd_server_cfg), ctypes.POINTER(_vp)]),
    "wd_server_add_gauge": (ctypes.c_int, [_vp, _dims_t, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "wd_server_remove_gauge": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "cg_submit": (ctypes.c_int, [_vp, ctypes.POINTER(wd_request), ctypes.POINTER(ctypes.c_uint64)]),
    "cg_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(wd_result)]),
    "wd_server_info": (ctypes.c_int, [_vp, ctypes.POINTER(wd_server_state)]),
    "wd_server_destroy": (ctypes.c_int, [_vp]),
    "cg_solve_normal": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double), _i32, _vp, _vp,
                                       ctypes.POINTER(wd_cg_params), ctypes.POINTER(wd_cg_stats),
                                       _vp, ctypes.c_size_t, _vp]),
    "wd_gauge_eo_bytes": (ctypes.c_size_t, [_dims_t, _i32, _i32]),
    "wd_spinor_eo_bytes": (ctypes.c_size_t, [_dims_t, _i32, _i32]),
    "wd_gauge_import_eo": (ctypes.c_int, [_dims_t, _vp, _i32, _i32, _vp, ctypes.c_size_t, _vp,
                                          ctypes.POINTER(_vp)]),
    "wd_spinor_import_eo": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "wd_spinor_export_eo": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "dslash_apply_eo": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), _i32, _vp, _vp, _vp,
                                       _i32, _i32, _vp]),
    "wilson_workspace_bytes": (ctypes.c_size_t, [_dims_t, _i32, _i32, _i32]),
    "cg_solve_wilson": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double), _i32, _vp, _vp,
                                       ctypes.POINTER(wd_cg_params), ctypes.POINTER(wd_cg_stats),
                                       _vp, ctypes.c_size_t, _vp]),
    "cg_solve_normal_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double), _i32, _vp,
                                               _vp, ctypes.POINTER(wd_cg_params),
                                               ctypes.POINTER(wd_cg_stats), _vp]),
    "wd_tune_dslash": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _i32, _vp,
                                      ctypes.POINTER(wd_tune_result)]),
    "wd_tune_lookup": (ctypes.c_int, [_dims_t, _i32, _i32, _i32, ctypes.POINTER(ctypes.c_int32)]),
    "wd_tune_reset": (ctypes.c_int, []),
    "wd_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "wd_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
}


class WilsonError(RuntimeError):
    """A negative status returned by the library."""

    def __init__(self, func: str, code: int, message: str):
        self.code = code
        super().__init__(f"{func}: {STATUS_NAMES.get(code, code)}: {message}")


def _load(path=_LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is not built; run `python -m paper_1901_07294_amd.build` first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.wd_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} implements ABI version {lib.wd_abi_version()}, "
                          f"this binding expects {ABI_VERSION}; rebuild the library")
    return lib


_lib = None
LIB_PATH = _LIB_PATH


def _L():
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _dims(dims):
    d = [int(v) for v in dims]
    if len(d) != 4:
        raise ValueError("dims must have 4 entries (X, Y, Z, T)")
    return (ctypes.c_int32 * 4)(*d)


def _ptr(buf):
    if buf is None:
        return None
    if hasattr(buf, "data_ptr"):
        return buf.data_ptr()
    return int(buf)


def _nbytes(buf):
    if hasattr(buf, "untyped_storage"):
        return buf.numel() * buf.element_size()
    raise TypeError("pass dst_bytes explicitly for a raw address")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _check(func, rc):
    if rc < 0:
        raise WilsonError(func, rc, _L().wd_last_error().decode())
    return rc


def wd_abi_version() -> int:
    return _L().wd_abi_version()


def wd_last_error() -> str:
    return _L().wd_last_error().decode()


def wd_spinor_bytes(dims, prec, nrhs=1) -> int:
    return _L().wd_spinor_bytes(_dims(dims), prec, nrhs)


def wd_gauge_bytes(dims, prec, compress12=0) -> int:
    return _L().wd_gauge_bytes(_dims(dims), prec, int(bool(compress12)))


class Gauge:
    """Owns a wd_gauge* handle (released on close/GC) and keeps its buffer alive."""

    def __init__(self, handle, dims, prec, compress12, buf):
        self.handle = handle
        self.dims = tuple(int(v) for v in dims)
        self.prec = prec
        self.compress12 = bool(compress12)
        self._buf = buf

    @property
    def _as_parameter_(self):
        return self.handle

    def close(self):
        if self.handle:
            _check("wd_gauge_release", _L().wd_gauge_release(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wd_gauge_import(dims, U_canon, prec, compress12, dst, dst_bytes=None, stream=None) -> Gauge:
    out = ctypes.c_void_p()
    nb = _nbytes(dst) if dst_bytes is None else int(dst_bytes)
    _check("wd_gauge_import", _L().wd_gauge_import(
        _dims(dims), _ptr(U_canon), prec, int(bool(compress12)), _ptr(dst), nb,
        _stream(stream), ctypes.byref(out)))
    return Gauge(out.value, dims, prec, compress12, dst)


def wd_gauge_release(g) -> int:
    if isinstance(g, Gauge):
        g.close()
        return WD_OK
    return _check("wd_gauge_release", _L().wd_gauge_release(g))


def _h(g):
    return g.handle if isinstance(g, Gauge) else g


def wd_spinor_import(g, canon, prec, nrhs, dst, stream=None) -> int:
    return _check("wd_spinor_import", _L().wd_spinor_import(
        _h(g), _ptr(canon), prec, nrhs, _ptr(dst), _stream(stream)))


def wd_spinor_export(g, src, prec, nrhs, canon, stream=None) -> int:
    return _check("wd_spinor_export", _L().wd_spinor_export(
        _h(g), _ptr(src), prec, nrhs, _ptr(canon), _stream(stream)))


def dslash_apply(g, mass, inp, out, prec, flags=0, stream=None) -> int:
    return _check("dslash_apply", _L().dslash_apply(
        _h(g), float(mass), _ptr(inp), _ptr(out), prec, flags, _stream(stream)))


def dslash_apply_multi(g, masses, nrhs, inp, out, prec, flags=0, stream=None) -> int:
    m = (ctypes.c_double * max(1, nrhs))(*[float(v) for v in masses])
    return _check("dslash_apply_multi", _L().dslash_apply_multi(
        _h(g), m, nrhs, _ptr(inp), _ptr(out), prec, flags, _stream(stream)))


def cg_workspace_bytes(dims, nrhs, inner) -> int:
    return _L().cg_workspace_bytes(_dims(dims), nrhs, inner)


def cg_solve_normal(g_hi, g_lo, masses, nrhs, b, x, params, ws, ws_bytes=None, stream=None,
                    check=True):
    """Calls cg_solve_normal; returns (status, [per right-hand side stats dicts]).

    params: a wd_cg_params or a dict of its fields. With check=True a negative
    status other than WD_ERR_NOT_CONVERGED / WD_ERR_NUMERIC raises WilsonError.
    """
    if isinstance(params, dict):
        params = wd_cg_params(**params)
    m = (ctypes.c_double * nrhs)(*[float(v) for v in masses])
    stats = (wd_cg_stats * max(1, nrhs))()
    nb = _nbytes(ws) if ws_bytes is None else int(ws_bytes)
    rc = _L().cg_solve_normal(_h(g_hi), _h(g_lo) if g_lo is not None else None, m, nrhs, _ptr(b),
                              _ptr(x), ctypes.byref(params), stats, _ptr(ws), nb, _stream(stream))
    if check and rc < 0 and rc not in (WD_ERR_NOT_CONVERGED, WD_ERR_NUMERIC):
        raise WilsonError("cg_solve_normal", rc, _L().wd_last_error().decode())
    return rc, [stats[k].as_dict() for k in range(nrhs)]


def wd_gauge_eo_bytes(dims, prec, compress12=0) -> int:
    return _L().wd_gauge_eo_bytes(_dims(dims), prec, int(bool(compress12)))


def wd_spinor_eo_bytes(dims, prec, nrhs=1) -> int:
    return _L().wd_spinor_eo_bytes(_dims(dims), prec, nrhs)


def wd_gauge_import_eo(dims, U_canon, prec, compress12, dst, dst_bytes=None, stream=None) -> Gauge:
    out = ctypes.c_void_p()
    nb = _nbytes(dst) if dst_bytes is None else int(dst_bytes)
    _check("wd_gauge_import_eo", _L().wd_gauge_import_eo(
        _dims(dims), _ptr(U_canon), prec, int(bool(compress12)), _ptr(dst), nb,
        _stream(stream), ctypes.byref(out)))
    return Gauge(out.value, dims, prec, compress12, dst)


def wd_spinor_import_eo(g, canon, prec, nrhs, parity, dst, stream=None) -> int:
    return _check("wd_spinor_import_eo", _L().wd_spinor_import_eo(
        _h(g), _ptr(canon), prec, nrhs, parity, _ptr(dst), _stream(stream)))


def wd_spinor_export_eo(g, src, prec, nrhs, parity, canon, stream=None) -> int:
    return _check("wd_spinor_export_eo", _L().wd_spinor_export_eo(
        _h(g), _ptr(src), prec, nrhs, parity, _ptr(canon), _stream(stream)))


def dslash_apply_eo(g, masses, nrhs, inp, out, tmp, prec, flags=0, stream=None) -> int:
    m = (ctypes.c_double * max(1, nrhs))(*[float(v) for v in masses])
    return _check("dslash_apply_eo", _L().dslash_apply_eo(
        _h(g), m, nrhs, _ptr(inp), _ptr(out), _ptr(tmp), prec, flags, _stream(stream)))


def wilson_workspace_bytes(dims, nrhs, inner, eo) -> int:
    return _L().wilson_workspace_bytes(_dims(dims), nrhs, inner, int(bool(eo)))


def cg_solve_wilson(g_hi, g_lo, masses, nrhs, b, x, params, ws, ws_bytes=None, stream=None,
                    check=True):
    """Calls cg_solve_wilson; returns (status, [per right-hand side stats dicts])."""
    if isinstance(params, dict):
        params = wd_cg_params(**params)
    m = (ctypes.c_double * nrhs)(*[float(v) for v in masses])
    stats = (wd_cg_stats * max(1, nrhs))()
    nb = _nbytes(ws) if ws_bytes is None else int(ws_bytes)
    rc = _L().cg_solve_wilson(_h(g_hi), _h(g_lo) if g_lo is not None else None, m, nrhs, _ptr(b),
                              _ptr(x), ctypes.byref(params), stats, _ptr(ws), nb, _stream(stream))
    if check and rc < 0 and rc not in (WD_ERR_NOT_CONVERGED, WD_ERR_NUMERIC):
        raise WilsonError("cg_solve_wilson", rc, _L().wd_last_error().decode())
    return rc, [stats[k].as_dict() for k in range(nrhs)]


def cg_solve_normal_noalloc(g_hi, g_lo, masses, nrhs, b, x, params, stream=None, check=True):
    """Calls cg_solve_normal_noalloc (the library's static workspace); returns
    (status, [per right-hand side stats dicts]) as cg_solve_normal does."""
    if isinstance(params, dict):
        params = wd_cg_params(**params)
    m = (ctypes.c_double * nrhs)(*[float(v) for v in masses])
    stats = (wd_cg_stats * max(1, nrhs))()
    rc = _L().cg_solve_normal_noalloc(_h(g_hi), _h(g_lo) if g_lo is not None else None, m, nrhs,
                                      _ptr(b), _ptr(x), ctypes.byref(params), stats, _stream(stream))
    if check and rc < 0 and rc not in (WD_ERR_NOT_CONVERGED, WD_ERR_NUMERIC):
        raise WilsonError("cg_solve_normal_noalloc", rc, _L().wd_last_error().decode())
    return rc, [stats[k].as_dict() for k in range(nrhs)]


def wd_server_create(arena, inner, check_every=8, delta=0.1, max_rhs_per_group=16, n_streams=4,
                     arena_bytes=None, evict_idle_gauges=False) -> int:
    """Returns the server handle (an integer address)."""
    nb = _nbytes(arena) if arena_bytes is None else int(arena_bytes)
    cfg = wd_server_cfg(_ptr(arena), nb, inner, check_every, delta, max_rhs_per_group, n_streams,
                        int(bool(evict_idle_gauges)))
    out = ctypes.c_void_p()
    _check("wd_server_create", _L().wd_server_create(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def wd_server_add_gauge(server, dims, U_canon) -> int:
    gid = ctypes.c_uint64()
    _check("wd_server_add_gauge", _L().wd_server_add_gauge(server, _dims(dims), _ptr(U_canon),
                                                           ctypes.byref(gid)))
    return gid.value


def wd_server_remove_gauge(server, gauge_id) -> int:
    return _check("wd_server_remove_gauge", _L().wd_server_remove_gauge(server, gauge_id))


def cg_submit(server, gauge_id, masses, b, x, tol=1e-10, max_iter=20000) -> int:
    """Queues a solve of len(masses) right-hand sides; returns the ticket."""
    req = wd_request()
    req.gauge_id = gauge_id
    req.nrhs = len(masses)
    req.max_iter = max_iter
    req.tol = tol
    for k, m in enumerate(masses):
        req.masses[k] = float(m)
    req.b_dev = _ptr(b)
    req.x_dev = _ptr(x)
    t = ctypes.c_uint64()
    _check("cg_submit", _L().cg_submit(server, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def cg_poll(server, ticket):
    """(status, result dict). WD_PENDING while running; a final status once."""
    res = wd_result()
    rc = _L().cg_poll(server, ticket, ctypes.byref(res))
    if rc in (WD_ERR_UNKNOWN_TICKET, WD_ERR_INVALID_ARG, WD_ERR_DEVICE, WD_ERR_INTERNAL):
        raise WilsonError("cg_poll", rc, _L().wd_last_error().decode())
    return rc, res.as_dict()


def wd_server_info(server) -> dict:
    st = wd_server_state()
    _check("wd_server_info", _L().wd_server_info(server, ctypes.byref(st)))
    return {"arena_in_use": st.arena_in_use, "arena_peak": st.arena_peak,
            "unfinished": st.unfinished, "gauges": st.gauges, "evictions": st.evictions}


def wd_server_destroy(server) -> int:
    return _check("wd_server_destroy", _L().wd_server_destroy(server))


def wd_tune_dslash(g, nrhs, inp, out, ref, reps=10, stream=None) -> dict:
    """Tunes the dslash launch for g's lattice and nrhs; returns the result fields."""
    res = wd_tune_result()
    _check("wd_tune_dslash", _L().wd_tune_dslash(_h(g), nrhs, _ptr(inp), _ptr(out), _ptr(ref), reps,
                                                 _stream(stream), ctypes.byref(res)))
    return res.as_dict()


def wd_tune_lookup(dims, prec, compress12, nrhs):
    """(tb, gw, group, rb) registered for the key, or None."""
    choice = (ctypes.c_int32 * 4)()
    rc = _check("wd_tune_lookup", _L().wd_tune_lookup(_dims(dims), prec, int(bool(compress12)), nrhs,
                                                      choice))
    return tuple(choice) if rc == 1 else None


def wd_tune_reset() -> int:
    return _check("wd_tune_reset", _L().wd_tune_reset())


def wd_tune_save(path) -> int:
    return _check("wd_tune_save", _L().wd_tune_save(os.fsencode(path)))


def wd_tune_load(path) -> int:
    return _check("wd_tune_load", _L().wd_tune_load(os.fsencode(path)))
