"""Python binding of libmrs.so, the MI355X (gfx950) MRS filament library.

Argument marshalling only: every function forwards to the C entry point of
the same name declared in include/mrs.h, and every step of the computation
runs in the library's HIP kernels.  torch is imported first so that the
library shares torch's HIP runtime; torch tensors may be passed where the C
call takes device pointers (their data_ptr is used) and the current torch
stream may be passed as `stream`.

The library must be built (``python -m paper_2604_12083_amd.build`` or
``__graft_entry__.build()``); without it the package imports (so that the
build module can run) but every entry point raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

try:  # share torch's HIP runtime when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mrs.h")



class _MissingLibrary:
    """Stands in for libmrs.so until it is built: every call raises, so
    nothing runs without the HIP library (there is no other code path)."""

    def __getattr__(self, name):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_12083_amd.build` "
                          f"(needed for {name})")


_lib = _MissingLibrary()

MRS_OK, MRS_EINVAL, MRS_ENOMEM, MRS_EDEVICE, MRS_ENOTREADY, MRS_EBUSY, MRS_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
MRS_FP64, MRS_FP32C = 0, 1
MRS_EULER, MRS_RK2, MRS_RK4 = 1, 2, 4
STATUS_NAMES = {0: "MRS_OK", -1: "MRS_EINVAL", -2: "MRS_ENOMEM", -3: "MRS_EDEVICE", -4: "MRS_ENOTREADY",
                -5: "MRS_EBUSY", -6: "MRS_ENUMERIC"}


class mrs_rod_params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * 3), ("b", ctypes.c_double * 3), ("omega0", ctypes.c_double * 3),
                ("ds", ctypes.c_double)]


class mrs_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_fil", ctypes.c_int32), ("offsets", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("D", ctypes.c_void_p), ("f_ext", ctypes.c_void_p),
                ("n_ext", ctypes.c_void_p), ("eps", ctypes.c_double), ("mu", ctypes.c_double),
                ("dt", ctypes.c_double), ("nsteps", ctypes.c_int32), ("integ", ctypes.c_int32),
                ("include_elastic", ctypes.c_int32), ("rod", mrs_rod_params)]


class mrs_result_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("n", ctypes.c_int64),
                ("steps_done", ctypes.c_int32), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class mrs_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("ticks", ctypes.c_int64), ("failed_ticks", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("busy_s", ctypes.c_double), ("active", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("hbm_in_use", ctypes.c_int64), ("hbm_budget", ctypes.c_int64),
                ("wall_s", ctypes.c_double)]


MRS_REQ_EVAL, MRS_REQ_STEPS = 0, 1
MRS_ADMIT_ARRIVAL, MRS_ADMIT_LEAST_WORK = 0, 1


class mrs_pair_config(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("targets_per_lane", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("schedule", ctypes.c_int32)]


class MrsError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_vp = ctypes.c_void_p
_d = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double

_SIGS = {
    "mrs_context_create": (_int, [_int, ctypes.POINTER(_vp)]),
    "mrs_context_destroy": (None, [_vp]),
    "mrs_last_error": (ctypes.c_char_p, [_vp]),
    "mrs_context_set_stream": (_int, [_vp, _vp]),
    "mrs_context_synchronize": (_int, [_vp]),
    "mrs_eval_host": (_int, [_vp, _i64, _vp, _vp, _vp, _dbl, _dbl, _int, _vp, _vp]),
    "mrs_eval_device": (_int, [_vp, _i64, _vp, _vp, _vp, _dbl, _dbl, _int, _vp, _vp, _vp]),
    "mrs_eval_device_noalloc": (_int, [_vp, _i64, _vp, _vp, _vp, _dbl, _dbl, _int, _vp, _vp, _vp]),
    "mrs_rod_forces_device": (_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.POINTER(mrs_rod_params), _vp, _vp,
                                     _vp, _vp, _vp]),
    "mrs_rotsqrt_device": (_int, [_vp, _i64, _vp, _vp, _vp]),
    "mrs_ensemble_create": (_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl,
                                   ctypes.POINTER(mrs_rod_params), ctypes.POINTER(_vp)]),
    "mrs_ensemble_set_state": (_int, [_vp, _vp, _vp]),
    "mrs_ensemble_size": (_int, [_vp, ctypes.POINTER(_i64)]),
    "mrs_ensemble_set_swimming": (_int, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "mrs_ensemble_set_external": (_int, [_vp, _vp, _vp]),
    "mrs_ensemble_set_time": (_int, [_vp, _dbl]),
    "mrs_ensemble_get_time": (_int, [_vp, ctypes.POINTER(_dbl)]),
    "mrs_ensemble_eval": (_int, [_vp, _int, _int]),
    "mrs_ensemble_step": (_int, [_vp, _int, _dbl, ctypes.c_int32, _int, _int]),
    "mrs_ensemble_get": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "mrs_ensemble_destroy": (None, [_vp]),
    "mrs_batch_step": (_int, [_vp, ctypes.c_int32, _vp, _int, _dbl, ctypes.c_int32, _int, _int, _int]),
    "mrs_batch_eval": (_int, [_vp, ctypes.c_int32, _vp, _int, _int]),
    "mrs_server_start": (_int, [_vp, _int, _i64, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "mrs_server_submit": (_int, [_vp, ctypes.POINTER(mrs_request), ctypes.POINTER(ctypes.c_uint64)]),
    "mrs_server_poll": (_int, [_vp, ctypes.c_uint64, ctypes.POINTER(mrs_result_info), _vp, _vp, _vp, _vp]),
    "mrs_server_wait": (_int, [_vp, ctypes.c_uint64, _dbl, ctypes.POINTER(mrs_result_info), _vp, _vp, _vp, _vp]),
    "mrs_server_stats_get": (_int, [_vp, ctypes.POINTER(mrs_server_stats)]),
    "mrs_server_stop": (_int, [_vp]),
    "mrs_server_set_tick_pairs": (_int, [_vp, _i64]),
    "mrs_server_set_admission": (_int, [_vp, ctypes.c_int32, _dbl]),
    "mrs_autotune": (_int, [_vp, _i64, _int, ctypes.c_int32, ctypes.POINTER(mrs_pair_config),
                            ctypes.POINTER(_dbl)]),
    "mrs_tune_get": (_int, [_vp, _i64, _int, ctypes.POINTER(mrs_pair_config)]),
    "mrs_tune_set": (_int, [_vp, _i64, _int, ctypes.POINTER(mrs_pair_config)]),
    "mrs_tune_on_first_use": (_int, [_vp, ctypes.c_int32, ctypes.c_char_p]),
    "mrs_tune_save": (_int, [_vp, ctypes.c_char_p]),
    "mrs_tune_load": (_int, [_vp, ctypes.c_char_p]),
    "mrs_parareal": (_int, [_vp, ctypes.c_int32, _int, _dbl, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dbl,
                            _int, _int, _vp, ctypes.POINTER(ctypes.c_int32)]),
    "mrs_plan_items": (_int, [ctypes.c_int64, _int, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, _vp,
                              ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "mrs_parareal_pipelined": (_int, [_vp, ctypes.c_int32, _int, _dbl, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _dbl, _int, _int, ctypes.c_int32, _vp,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "mrs_profile_enable": (_int, [_vp, _int]),
    "mrs_profile_select": (_int, [_vp, ctypes.c_char_p]),
    "mrs_profile_reset": (_int, [_vp]),
    "mrs_profile_clock": (_int, [_vp, ctypes.POINTER(_dbl)]),
    "mrs_profile_query": (_int, [_vp, ctypes.c_char_p, ctypes.POINTER(_i64), ctypes.POINTER(_dbl)]),
}



def _load_library():
    """Load libmrs.so and declare the C signatures."""
    global _lib
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
    _lib = lib


def library_loaded() -> bool:
    return not isinstance(_lib, _MissingLibrary)


# The build step (paper_2604_12083_amd.build) imports this package before the
# library exists; every entry point raises ImportError until it is built and
# the package is reloaded.
if os.path.exists(LIB_PATH):
    _load_library()


def declared_functions(header: str = HEADER):
    """Names of the functions include/mrs.h declares."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrs_[a-z0-9_]+)\s*\(", text)))


def _ptr(x):
    """Address of a host numpy array, a torch tensor (device or host), an int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if torch is not None and isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    if isinstance(x, ctypes.c_void_p):
        return x.value
    raise TypeError(f"cannot pass {type(x)} as a pointer")


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    if torch is not None and isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    raise TypeError("stream must be None, an int handle or a torch.cuda.Stream")


def _check(status, ctx=None):
    if status != MRS_OK:
        msg = _lib.mrs_last_error(ctx).decode() if ctx else ""
        raise MrsError(status, msg)


def _f64(a, cols):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(-1, cols)


def rod_params(a=(1e-4, 1e-4, 1e-4), b=(1.0, 1.0, 1.0), omega0=(0.0, 0.0, 0.0), ds=1.0 / 64) -> mrs_rod_params:
    p = mrs_rod_params()
    p.a[:] = [float(v) for v in a]
    p.b[:] = [float(v) for v in b]
    p.omega0[:] = [float(v) for v in omega0]
    p.ds = float(ds)
    return p


# ---- thin wrappers with the C names ------------------------------------


def mrs_context_create(device: int = 0):
    h = _vp()
    _check(_lib.mrs_context_create(int(device), ctypes.byref(h)))
    return h


def mrs_context_destroy(ctx) -> None:
    _lib.mrs_context_destroy(ctx)


def mrs_last_error(ctx) -> str:
    return _lib.mrs_last_error(ctx).decode()


def mrs_context_set_stream(ctx, stream=None) -> None:
    _check(_lib.mrs_context_set_stream(ctx, _stream(stream)), ctx)


def mrs_context_synchronize(ctx) -> None:
    _check(_lib.mrs_context_synchronize(ctx), ctx)


def mrs_eval_host(ctx, X, f, n, eps, mu=1.0, prec=MRS_FP64):
    X, f, n = _f64(X, 3), _f64(f, 3), _f64(n, 3)
    U = np.empty_like(X)
    W = np.empty_like(X)
    _check(_lib.mrs_eval_host(ctx, X.shape[0], _ptr(X), _ptr(f), _ptr(n), float(eps), float(mu), int(prec),
                              _ptr(U), _ptr(W)), ctx)
    return U, W


def mrs_eval_device(ctx, n_points, dX, df, dn, eps, mu, prec, dU, dW, stream=None) -> None:
    _check(_lib.mrs_eval_device(ctx, int(n_points), _ptr(dX), _ptr(df), _ptr(dn), float(eps), float(mu), int(prec),
                                _ptr(dU), _ptr(dW), _stream(stream)), ctx)


def mrs_eval_device_noalloc(ctx, n_points, dX, df, dn, eps, mu, prec, dU, dW, stream=None) -> None:
    _check(_lib.mrs_eval_device_noalloc(ctx, int(n_points), _ptr(dX), _ptr(df), _ptr(dn), float(eps), float(mu),
                                        int(prec), _ptr(dU), _ptr(dW), _stream(stream)), ctx)


def mrs_rod_forces_device(ctx, offsets, dX, dD, rod, dfext, dnext, dg, dm, stream=None) -> None:
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    _check(_lib.mrs_rod_forces_device(ctx, len(off) - 1, _ptr(off), _ptr(dX), _ptr(dD), ctypes.byref(rod),
                                      _ptr(dfext), _ptr(dnext), _ptr(dg), _ptr(dm), _stream(stream)), ctx)


def mrs_rotsqrt_device(ctx, count, dR, dS, stream=None) -> None:
    _check(_lib.mrs_rotsqrt_device(ctx, int(count), _ptr(dR), _ptr(dS), _stream(stream)), ctx)


def mrs_ensemble_create(ctx, offsets, X, D, f_ext, n_ext, eps, mu, rod):
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X, D = _f64(X, 3), _f64(D, 9)
    fe = None if f_ext is None else _f64(f_ext, 3)
    ne = None if n_ext is None else _f64(n_ext, 3)
    h = _vp()
    _check(_lib.mrs_ensemble_create(ctx, len(off) - 1, _ptr(off), _ptr(X), _ptr(D), _ptr(fe), _ptr(ne), float(eps),
                                    float(mu), ctypes.byref(rod), ctypes.byref(h)), ctx)
    return h


def mrs_ensemble_set_state(ctx, ens, X=None, D=None) -> None:
    X = None if X is None else _f64(X, 3)
    D = None if D is None else _f64(D, 9)
    _check(_lib.mrs_ensemble_set_state(ens, _ptr(X), _ptr(D)), ctx)


def mrs_ensemble_set_external(ctx, ens, f_ext=None, n_ext=None) -> None:
    """Replace the external point loads (n x 3 host arrays; None = zero)."""
    fe = None if f_ext is None else _f64(f_ext, 3)
    ne = None if n_ext is None else _f64(n_ext, 3)
    _check(_lib.mrs_ensemble_set_external(ens, _ptr(fe), _ptr(ne)), ctx)


def mrs_ensemble_size(ens) -> int:
    n = _i64()
    _check(_lib.mrs_ensemble_size(ens, ctypes.byref(n)))
    return int(n.value)


def mrs_ensemble_set_swimming(ctx, ens, wave=None, lj=None) -> None:
    """Swimming waveform (A, k, f) and Lennard-Jones repulsion (sigma, energy); None switches either off."""
    w = None if wave is None else (_dbl * 3)(*[float(v) for v in wave])
    l = None if lj is None else (_dbl * 2)(*[float(v) for v in lj])
    _check(_lib.mrs_ensemble_set_swimming(ens, w, l), ctx)


def mrs_ensemble_set_time(ctx, ens, t) -> None:
    _check(_lib.mrs_ensemble_set_time(ens, float(t)), ctx)


def mrs_ensemble_get_time(ctx, ens) -> float:
    t = _dbl()
    _check(_lib.mrs_ensemble_get_time(ens, ctypes.byref(t)), ctx)
    return t.value


def mrs_ensemble_eval(ctx, ens, prec=MRS_FP64, include_elastic=True) -> None:
    _check(_lib.mrs_ensemble_eval(ens, int(prec), int(bool(include_elastic))), ctx)


def mrs_ensemble_step(ctx, ens, integ, dt, nsteps, prec=MRS_FP64, include_elastic=True) -> None:
    _check(_lib.mrs_ensemble_step(ens, int(integ), float(dt), int(nsteps), int(prec), int(bool(include_elastic))),
           ctx)


def mrs_ensemble_get(ctx, ens):
    n = mrs_ensemble_size(ens)
    X, D, U, W = np.empty((n, 3)), np.empty((n, 9)), np.empty((n, 3)), np.empty((n, 3))
    _check(_lib.mrs_ensemble_get(ens, _ptr(X), _ptr(D), _ptr(U), _ptr(W)), ctx)
    return X, D, U, W


def mrs_ensemble_destroy(ens) -> None:
    _lib.mrs_ensemble_destroy(ens)


def _ens_array(ens_list):
    arr = (_vp * len(ens_list))(*[e.value if isinstance(e, _vp) else e for e in ens_list])
    return arr


def mrs_batch_step(ctx, ens_list, integ, dt, nsteps, prec=MRS_FP32C, include_elastic=True, use_graph=True) -> None:
    arr = _ens_array(ens_list)
    _check(_lib.mrs_batch_step(ctx, len(ens_list), ctypes.cast(arr, _vp), int(integ), float(dt), int(nsteps),
                               int(prec), int(bool(include_elastic)), int(bool(use_graph))), ctx)


def mrs_batch_eval(ctx, ens_list, prec=MRS_FP32C, include_elastic=True) -> None:
    arr = _ens_array(ens_list)
    _check(_lib.mrs_batch_eval(ctx, len(ens_list), ctypes.cast(arr, _vp), int(prec), int(bool(include_elastic))), ctx)


def mrs_profile_enable(ctx, on=True) -> None:
    _check(_lib.mrs_profile_enable(ctx, int(bool(on))), ctx)


def mrs_profile_select(ctx, kernel="") -> None:
    _check(_lib.mrs_profile_select(ctx, kernel.encode() if kernel else None), ctx)


def mrs_profile_reset(ctx) -> None:
    _check(_lib.mrs_profile_reset(ctx), ctx)


def mrs_profile_clock(ctx) -> float:
    """Shader clock (MHz) measured by a short spin on the device."""
    v = _dbl()
    _check(_lib.mrs_profile_clock(ctx, ctypes.byref(v)), ctx)
    return float(v.value)


def mrs_profile_query(ctx, kernel=""):
    n = _i64()
    ms = _dbl()
    _check(_lib.mrs_profile_query(ctx, kernel.encode() if kernel else None, ctypes.byref(n), ctypes.byref(ms)), ctx)
    return int(n.value), float(ms.value)


# ---- serving ------------------------------------------------------------


def mrs_server_start(ctx, prec=MRS_FP32C, hbm_budget_bytes=8 << 30, max_slots=64):
    h = _vp()
    _check(_lib.mrs_server_start(ctx, int(prec), int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)), ctx)
    return h


def mrs_server_submit(srv, kind, offsets, X, D, f_ext, n_ext, eps, mu, rod, dt=0.0, nsteps=0, integ=MRS_RK4,
                      include_elastic=True):
    """Submit one request (inputs are copied); returns its ticket."""
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X, D = _f64(X, 3), _f64(D, 9)
    fe = None if f_ext is None else _f64(f_ext, 3)
    ne = None if n_ext is None else _f64(n_ext, 3)
    q = mrs_request(int(kind), len(off) - 1, _ptr(off), _ptr(X), _ptr(D), _ptr(fe), _ptr(ne), float(eps),
                    float(mu), float(dt), int(nsteps), int(integ), int(bool(include_elastic)), rod)
    t = ctypes.c_uint64()
    _check(_lib.mrs_server_submit(srv, ctypes.byref(q), ctypes.byref(t)))
    return int(t.value)


def _server_out(n):
    return np.empty((n, 3)), np.empty((n, 9)), np.empty((n, 3)), np.empty((n, 3))


def mrs_server_poll(srv, ticket, n):
    """(status, info, (X, D, U, Omega)); outputs are None unless done with
    MRS_OK or MRS_ENUMERIC (a result with non-finite values)."""
    info = mrs_result_info()
    X, D, U, W = _server_out(n)
    st = _lib.mrs_server_poll(srv, ctypes.c_uint64(ticket), ctypes.byref(info), _ptr(X), _ptr(D), _ptr(U), _ptr(W))
    return st, info, ((X, D, U, W) if st in (MRS_OK, MRS_ENUMERIC) else None)


def mrs_server_wait(srv, ticket, n, timeout_s=60.0):
    info = mrs_result_info()
    X, D, U, W = _server_out(n)
    st = _lib.mrs_server_wait(srv, ctypes.c_uint64(ticket), float(timeout_s), ctypes.byref(info), _ptr(X), _ptr(D),
                              _ptr(U), _ptr(W))
    return st, info, ((X, D, U, W) if st in (MRS_OK, MRS_ENUMERIC) else None)


def mrs_server_stats_get(srv):
    s = mrs_server_stats()
    _check(_lib.mrs_server_stats_get(srv, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in mrs_server_stats._fields_}


def mrs_server_set_tick_pairs(srv, max_pairs) -> None:
    _check(_lib.mrs_server_set_tick_pairs(srv, int(max_pairs)))


def mrs_server_set_admission(srv, order, max_wait_s=0.0) -> None:
    """order: MRS_ADMIT_ARRIVAL or MRS_ADMIT_LEAST_WORK (requests waiting
    longer than max_wait_s > 0 go first, in arrival order)."""
    _check(_lib.mrs_server_set_admission(srv, int(order), float(max_wait_s)))


def mrs_server_stop(srv) -> None:
    _check(_lib.mrs_server_stop(srv))


# ---- tuning -------------------------------------------------------------


def mrs_autotune(ctx, n, prec=MRS_FP32C, reps=3):
    """Returns ({mode, targets_per_lane, chunks, schedule}, median device ms
    of one evaluation with it)."""
    c = mrs_pair_config()
    ms = _dbl()
    _check(_lib.mrs_autotune(ctx, int(n), int(prec), int(reps), ctypes.byref(c), ctypes.byref(ms)), ctx)
    return {"mode": c.mode, "targets_per_lane": c.targets_per_lane, "chunks": c.chunks,
            "schedule": c.schedule}, float(ms.value)


def mrs_tune_get(ctx, n, prec=MRS_FP32C):
    c = mrs_pair_config()
    _check(_lib.mrs_tune_get(ctx, int(n), int(prec), ctypes.byref(c)), ctx)
    return {"mode": c.mode, "targets_per_lane": c.targets_per_lane, "chunks": c.chunks, "schedule": c.schedule}


def mrs_plan_items(n, prec, n_cu=256):
    """Host-only work list of the automatic pair-kernel configuration:
    (config dict, int32 array of blocks x (tgt0, ntgt, src0, nsrc, slot)) in
    dispatch order."""
    m, t, k, ts = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    cnt = ctypes.c_int64()
    _check(_lib.mrs_plan_items(int(n), int(prec), int(n_cu), ctypes.byref(m), ctypes.byref(t), ctypes.byref(k),
                               ctypes.byref(ts), None, 0, ctypes.byref(cnt)))
    items = np.zeros((cnt.value, 5), dtype=np.int32)
    _check(_lib.mrs_plan_items(int(n), int(prec), int(n_cu), None, None, None, None, items.ctypes.data, cnt.value,
                               ctypes.byref(cnt)))
    return {"mode": m.value, "targets_per_lane": t.value, "chunks": k.value, "tail_start": ts.value}, items


def mrs_tune_set(ctx, n, prec, mode, targets_per_lane=1, chunks=0, schedule=0) -> None:
    c = mrs_pair_config(int(mode), int(targets_per_lane), int(chunks), int(schedule))
    _check(_lib.mrs_tune_set(ctx, int(n), int(prec), ctypes.byref(c)), ctx)


def mrs_tune_on_first_use(ctx, reps=3, table_path=None) -> None:
    """Tune unseen size classes when an ensemble plan is first built (reps = 0
    turns it off); table_path: tuning table read now and rewritten after every
    tuning."""
    path = None if table_path is None else os.fsencode(table_path)
    _check(_lib.mrs_tune_on_first_use(ctx, int(reps), path), ctx)


def mrs_tune_save(ctx, path) -> None:
    _check(_lib.mrs_tune_save(ctx, os.fsencode(path)), ctx)


def mrs_tune_load(ctx, path) -> None:
    _check(_lib.mrs_tune_load(ctx, os.fsencode(path)), ctx)


# ---- Parareal -----------------------------------------------------------


def mrs_parareal(ctx, ens, n_slices, fine_integ, fine_dt, fine_steps, coarse_steps, max_iter, tol=0.0,
                 prec=MRS_FP64, include_elastic=True):
    """Returns (iterations done, relative increment per iteration)."""
    hist = np.zeros(max(int(max_iter), 1))
    it = ctypes.c_int32()
    _check(_lib.mrs_parareal(ens, int(n_slices), int(fine_integ), float(fine_dt), int(fine_steps), int(coarse_steps),
                             int(max_iter), float(tol), int(prec), int(bool(include_elastic)), _ptr(hist),
                             ctypes.byref(it)), ctx)
    return int(it.value), hist[: it.value].copy()


def mrs_parareal_pipelined(ctx, ens, n_slices, fine_integ, fine_dt, fine_steps, coarse_steps, max_iter, tol=0.0,
                           prec=MRS_FP64, include_elastic=True, group=0):
    """Pipelined schedule; returns (iterations done, relative increment per iteration)."""
    hist = np.zeros(max(int(max_iter), 1))
    it = ctypes.c_int32()
    _check(_lib.mrs_parareal_pipelined(ens, int(n_slices), int(fine_integ), float(fine_dt), int(fine_steps),
                                       int(coarse_steps), int(max_iter), float(tol), int(prec),
                                       int(bool(include_elastic)), int(group), _ptr(hist), ctypes.byref(it)), ctx)
    return int(it.value), hist[: it.value].copy()
