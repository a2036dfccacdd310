"""Python binding of the C library ``libbhx.so`` (include/bhx.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Functions keep the C names without the ``bhx_`` prefix.  Device arrays are
passed as torch tensors (float64, contiguous, on the handle's device) or as
raw integer device addresses; streams as torch streams or raw handles.

Importing this module raises ``ImportError`` if the library has not been
built (``python -m paper_1704_08897_amd.build`` or ``__graft_entry__.build()``);
there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import itertools
import os
import re
import sys
import weakref

_HERE = os.path.dirname(os.path.abspath(__file__))
# BHX_LIB selects a debugging build of the library (build.py VARIANTS).
LIB_PATH = os.environ.get("BHX_LIB") or os.path.join(_HERE, "libbhx.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "bhx.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_1704_08897_amd/build.py")
# torch ships its own HIP runtime.  Loaded after this library, it would be a
# second runtime in the process, and the one that reaches the GPU second finds
# no device.  Loaded first, it also satisfies this library's libamdhip64
# dependency, so the process holds one runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)

NEUMANN, PERIODIC, DIRICHLET = 0, 1, 2
OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_SINGULAR, ERR_NONFINITE, ERR_NOMEM, ERR_HIP, BUSY, ERR_BREAKDOWN = (
    -1, -2, -3, -4, -5, -6, -7)
PREC_FP64, PREC_FP32 = 0, 1


def BC(bx: int, by: int) -> int:
    return int(bx) | (int(by) << 4)


def BC3(bx: int, by: int, bz: int) -> int:
    return int(bx) | (int(by) << 4) | (int(bz) << 8)


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("maxit", ctypes.c_int),
                ("precond", ctypes.c_int), ("accurate", ctypes.c_int),
                ("tol_inner", ctypes.c_double), ("flexible", ctypes.c_int),
                ("chunk", ctypes.c_int), ("rows", ctypes.c_int), ("occupancy", ctypes.c_int),
                ("autotune", ctypes.c_int),
                ("profile", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("solver", ctypes.c_int), ("transform", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("restarts", ctypes.c_int), ("n_unknown", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("true_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("pass_ms", ctypes.c_double * 4),
                ("pass_launches", ctypes.c_int * 4)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["pass_ms"] = list(self.pass_ms)
        d["pass_launches"] = list(self.pass_launches)
        return d


_vp, _ci, _cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_sig = {
    "bhx_default_opts": (None, [ctypes.POINTER(Opts)]),
    "bhx_create": (_ci, [ctypes.POINTER(_vp), _ci]),
    "bhx_destroy": (None, [_vp]),
    "bhx_extend": (_ci, [_vp, _vp, _ci, _ci, _cd, _ci, _cd]),
    "bhx_extend_ex": (_ci, [_vp, _vp, _vp, _ci, _ci, _cd, _ci, _cd, ctypes.POINTER(Opts), _vp,
                            ctypes.POINTER(Stats)]),
    "bhx_extend_noalloc": (_ci, [_vp, _vp, _vp, _ci, _ci, _cd, _ci, _cd, ctypes.POINTER(Opts),
                                 _vp, ctypes.POINTER(Stats)]),
    "bhx_extend_batched": (_ci, [_vp, _ci, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_ci), ctypes.POINTER(_ci), ctypes.POINTER(_cd),
                                 ctypes.POINTER(_ci), ctypes.POINTER(_cd), ctypes.POINTER(Opts),
                                 _vp, ctypes.POINTER(Stats)]),
    "bhx_extend_fields": (_ci, [_vp, _ci, _vp, ctypes.POINTER(_vp), _ci, _ci, _cd, _ci, _cd,
                                ctypes.POINTER(Opts), _vp, ctypes.POINTER(Stats)]),
    "bhx_workspace_bytes": (ctypes.c_size_t, [_ci, _ci, _ci, ctypes.POINTER(Opts)]),
    "bhx_extend3d": (_ci, [_vp, _vp, _vp, _ci, _ci, _ci, _cd, _ci, _cd, ctypes.POINTER(Opts), _vp,
                           ctypes.POINTER(Stats)]),
    "bhx_workspace_bytes3d": (ctypes.c_size_t, [_ci, _ci, _ci, _ci, ctypes.POINTER(Opts)]),
    "bhx_debug_apply3d": (_ci, [_vp, _ci, _vp, _vp, _vp, _ci, _ci, _ci, _ci, _ci, _vp]),
    "bhx_engine_create": (_ci, [ctypes.POINTER(_vp), _ci, ctypes.c_size_t, _ci,
                                ctypes.POINTER(Opts)]),
    "bhx_engine_submit": (_ci, [_vp, _vp, _vp, _ci, _ci, _cd, _ci, _cd,
                                ctypes.POINTER(ctypes.c_uint64)]),
    "bhx_engine_poll": (_ci, [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(Stats), _ci,
                              ctypes.POINTER(_ci)]),
    "bhx_engine_inflight": (_ci, [_vp]),
    "bhx_engine_profile": (_ci, [_vp, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 _ci]),
    "bhx_engine_destroy": (None, [_vp]),
    "bhx_status_string": (ctypes.c_char_p, [_ci]),
    "bhx_version": (ctypes.c_char_p, []),
    "bhx_last_error": (ctypes.c_char_p, []),
    "bhx_debug_apply": (_ci, [_vp, _ci, _vp, _vp, _vp, _ci, _ci, _ci, _ci, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_functions(path: str = HEADER_PATH) -> list:
    """Names of the functions declared in include/bhx.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bhx_[a-z0-9_]+)\s*\(", text)) - {"bhx_BC"})


def exported(name: str) -> bool:
    try:
        getattr(_lib, name)
        return True
    except AttributeError:
        return False


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(x):
    """Device address of a torch tensor (checked) or an int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch tensor or a device address")
    if x.dtype != torch.float64 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("arrays must be contiguous float64 device tensors")
    return x.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _dims(a):
    if hasattr(a, "shape") and len(a.shape) == 2:
        return int(a.shape[1]), int(a.shape[0])
    raise ValueError("pass (ny, nx) arrays or explicit sizes")


def _dims3(a):
    if hasattr(a, "shape") and len(a.shape) == 3:
        return int(a.shape[2]), int(a.shape[1]), int(a.shape[0])
    raise ValueError("pass (nz, ny, nx) arrays or explicit sizes")


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.bhx_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def status_string(s: int) -> str:
    return _lib.bhx_status_string(int(s)).decode()


def version() -> str:
    return _lib.bhx_version().decode()


def last_error() -> str:
    return _lib.bhx_last_error().decode()


class BhxError(RuntimeError):
    def __init__(self, status):
        extra = f" ({last_error()})" if status == ERR_HIP else ""
        super().__init__(f"bhx status {status}: {status_string(status)}{extra}")
        self.status = status


def create(device: int = 0) -> int:
    h = _vp()
    s = _lib.bhx_create(ctypes.byref(h), int(device))
    if s != OK:
        raise BhxError(s)
    return h.value


def destroy(handle: int) -> None:
    _lib.bhx_destroy(handle)


# Objects that own library resources (handles, engines) and are still open.
# They are closed explicitly by an exit hook that runs while the HIP runtime
# (and a profiler attached to it) is still up: engines first (their worker
# threads are joined), then handles.  A finaliser that runs during interpreter
# shutdown releases nothing, since the runtime may already be gone then.
_open = weakref.WeakValueDictionary()
_open_seq = itertools.count()


def _register(obj) -> int:
    key = next(_open_seq)
    _open[key] = obj
    return key


def close_all() -> None:
    """Close every open engine, then every open handle (idempotent)."""
    objs = list(_open.values())
    for o in objs:
        if getattr(o, "is_engine", False):
            o.close()
    for o in objs:
        o.close()


atexit.register(close_all)


class Handle:
    """Owning wrapper of a ``bhx_handle``.  Call ``close()`` when done (or use
    it as a context manager); open handles are closed at interpreter exit."""

    is_engine = False

    def __init__(self, device: int = 0):
        self.device = device
        self.ptr = create(device)
        self._key = _register(self)

    def close(self):
        if self.ptr:
            ptr, self.ptr = self.ptr, None
            _open.pop(self._key, None)
            destroy(ptr)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass


def extend(phi, F, nx=None, ny=None, h=1.0, bc=0, tol=1e-8) -> int:
    """``bhx_extend``: default handle, null stream, FP64 PCG; returns the status."""
    if nx is None:
        nx, ny = _dims(phi)
    return _lib.bhx_extend(_ptr(phi), _ptr(F), nx, ny, float(h), int(bc), float(tol))


def extend_ex(handle, phi, F, nx=None, ny=None, h=1.0, bc=0, tol=1e-8, opts=None,
              stream=None):
    """``bhx_extend_ex``; returns (status, Stats)."""
    if nx is None:
        nx, ny = _dims(phi)
    hp = handle.ptr if isinstance(handle, Handle) else handle
    st = Stats()
    s = _lib.bhx_extend_ex(hp, _ptr(phi), _ptr(F), nx, ny, float(h), int(bc), float(tol),
                           ctypes.byref(opts) if opts is not None else None, _stream(stream),
                           ctypes.byref(st))
    return s, st


def extend_noalloc(handle, phi, F, nx=None, ny=None, h=1.0, bc=0, tol=1e-8, opts=None,
                   stream=None):
    """``bhx_extend_noalloc`` (no device allocation: the library's static
    scratch array); returns (status, Stats)."""
    if nx is None:
        nx, ny = _dims(phi)
    hp = handle.ptr if isinstance(handle, Handle) else handle
    st = Stats()
    s = _lib.bhx_extend_noalloc(hp, _ptr(phi), _ptr(F), nx, ny, float(h), int(bc),
                                float(tol), ctypes.byref(opts) if opts is not None else None,
                                _stream(stream), ctypes.byref(st))
    return s, st


def extend_batched(handle, phis, Fs, hs, bcs, tols, opts=None, stream=None, sizes=None):
    """``bhx_extend_batched``; returns (status, [Stats])."""
    n = len(phis)
    if sizes is None:
        sizes = [_dims(p) for p in phis]
    hp = handle.ptr if isinstance(handle, Handle) else handle
    P = (_vp * n)(*[_ptr(p) for p in phis])
    Fp = (_vp * n)(*[_ptr(f) for f in Fs])
    NX = (_ci * n)(*[s[0] for s in sizes])
    NY = (_ci * n)(*[s[1] for s in sizes])
    H = (_cd * n)(*[float(x) for x in hs])
    B = (_ci * n)(*[int(x) for x in bcs])
    T = (_cd * n)(*[float(x) for x in tols])
    st = (Stats * n)()
    s = _lib.bhx_extend_batched(hp, n, P, Fp, NX, NY, H, B, T,
                                ctypes.byref(opts) if opts is not None else None,
                                _stream(stream), st)
    return s, list(st)


def extend_fields(handle, phi, Fs, h=1.0, bc=0, tol=1e-8, opts=None, stream=None, nx=None,
                  ny=None):
    """``bhx_extend_fields``: several fields known on one region; returns
    (status, [Stats])."""
    if nx is None:
        nx, ny = _dims(phi)
    n = len(Fs)
    hp = handle.ptr if isinstance(handle, Handle) else handle
    Fp = (_vp * n)(*[_ptr(f) for f in Fs])
    st = (Stats * n)()
    s = _lib.bhx_extend_fields(hp, n, _ptr(phi), Fp, nx, ny, float(h), int(bc), float(tol),
                               ctypes.byref(opts) if opts is not None else None,
                               _stream(stream), st)
    return s, list(st)


def extend3d(handle, phi, F, nx=None, ny=None, nz=None, h=1.0, bc=0, tol=1e-8, opts=None,
             stream=None):
    """``bhx_extend3d``; arrays (nz, ny, nx); returns (status, Stats)."""
    if nx is None:
        nx, ny, nz = _dims3(phi)
    hp = handle.ptr if isinstance(handle, Handle) else handle
    st = Stats()
    s = _lib.bhx_extend3d(hp, _ptr(phi), _ptr(F), nx, ny, nz, float(h), int(bc), float(tol),
                          ctypes.byref(opts) if opts is not None else None, _stream(stream),
                          ctypes.byref(st))
    return s, st


def workspace_bytes3d(nx, ny, nz, bc, opts=None) -> int:
    return int(_lib.bhx_workspace_bytes3d(nx, ny, nz, bc,
                                          ctypes.byref(opts) if opts is not None else None))


def debug_apply3d(handle, op, phi, x, out, nx=None, ny=None, nz=None, bc=0, precision=0,
                  stream=None):
    """``bhx_debug_apply3d``: op 0 masked 25-point operator, op 1 preconditioner."""
    if nx is None:
        nx, ny, nz = _dims3(phi)
    hp = handle.ptr if isinstance(handle, Handle) else handle
    return _lib.bhx_debug_apply3d(hp, int(op), _ptr(phi), _ptr(x), _ptr(out), nx, ny, nz,
                                  int(bc), int(precision), _stream(stream))


def workspace_bytes(nx, ny, bc, opts=None) -> int:
    return int(_lib.bhx_workspace_bytes(nx, ny, bc,
                                        ctypes.byref(opts) if opts is not None else None))


def debug_apply(handle, op, phi, x, out, nx=None, ny=None, bc=0, precision=0, stream=None,
                transform=0):
    """``bhx_debug_apply``: op 0 masked operator, op 1 preconditioner
    (``transform`` as bhx_opts.transform)."""
    if nx is None:
        nx, ny = _dims(phi)
    hp = handle.ptr if isinstance(handle, Handle) else handle
    return _lib.bhx_debug_apply(hp, int(op), _ptr(phi), _ptr(x), _ptr(out), nx, ny, int(bc),
                                int(precision) | (int(transform) << 4), _stream(stream))


# ---------------------------------------------------------------------------
# engine
# ---------------------------------------------------------------------------

def engine_create(device: int, hbm_budget: int, max_slots: int, opts=None) -> int:
    e = _vp()
    s = _lib.bhx_engine_create(ctypes.byref(e), int(device), int(hbm_budget), int(max_slots),
                               ctypes.byref(opts) if opts is not None else None)
    if s != OK:
        raise BhxError(s)
    return e.value


def engine_submit(engine, phi, F, nx=None, ny=None, h=1.0, bc=0, tol=1e-8):
    """Returns (status, request id)."""
    if nx is None:
        nx, ny = _dims(phi)
    rid = ctypes.c_uint64(0)
    s = _lib.bhx_engine_submit(engine, _ptr(phi), _ptr(F), nx, ny, float(h), int(bc), float(tol),
                               ctypes.byref(rid))
    return s, rid.value


def engine_poll(engine, max_n: int = 256):
    """Returns a list of (request id, Stats) of finished requests."""
    ids = (ctypes.c_uint64 * max_n)()
    st = (Stats * max_n)()
    n = _ci(0)
    s = _lib.bhx_engine_poll(engine, ids, st, max_n, ctypes.byref(n))
    if s != OK:
        raise BhxError(s)
    return [(ids[i], st[i]) for i in range(n.value)]


def engine_inflight(engine) -> int:
    return int(_lib.bhx_engine_inflight(engine))


def engine_profile(engine, reset: bool = False) -> dict:
    """``bhx_engine_profile``: per-pass kernel time, launches and node sums."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_longlong * 4)()
    u = (ctypes.c_double * 4)()
    a = (ctypes.c_double * 4)()
    s = _lib.bhx_engine_profile(engine, ms, n, u, a, int(reset))
    if s != OK:
        raise BhxError(s)
    return {"ms": list(ms), "launches": list(n), "unknown_nodes": list(u), "nodes": list(a)}


def engine_destroy(engine) -> None:
    _lib.bhx_engine_destroy(engine)
