"""Python binding of the shfmm C ABI (``include/shfmm.h``): argument marshalling only.

Every computation runs in the HIP library ``libshfmm.so`` built for gfx950 (see
``build.py``); the functions here carry the C names and forward to them via ctypes.
Device arrays are passed as torch tensors on the GPU (their ``data_ptr()``) or as raw
integer addresses.  There is no CPU fallback: if the library is missing, importing
works but every call raises ``LibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshfmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "shfmm.h")

SH_OK, SH_EINVAL, SH_EORDER, SH_ESHIFT, SH_ENOMEM, SH_EDEVICE, SH_EBUSY = 0, -1, -2, -3, -4, -5, -6
SH_M2M, SH_M2L, SH_L2L = 0, 1, 2
SH_F64, SH_F32 = 0, 1
SH_ACCUMULATE = 1
SH_SINGLE_HEIGHT = 2  # single-height M2L (p_in = p_out)
SH_FMM_NO_GRAPH = 1
SH_FMM_MAX_LEVELS = 6
SH_PLAN_AUTOTUNE = 2
SH_PLAN_NO_GRAPH = 4
SH_SHARED_FP32 = 1
SH_SHARED_BF16X3 = 3
SH_SHARED_BF16X6 = 6
SH_MAX_ORDER = 64
SH_NOALLOC_SCRATCH_BYTES = 66816  # staging array of sh_translate_single_noalloc
OPS = {"m2m": SH_M2M, "m2l": SH_M2L, "l2l": SH_L2L}


class LibraryMissing(RuntimeError):
    pass


class ShError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {sh_strerror(status)} ({status})")


_lib = None

_c_i32, _c_i64, _c_u32, _vp = ctypes.c_int, ctypes.c_int64, ctypes.c_uint, ctypes.c_void_p
_SIGS = {
    "sh_strerror": (ctypes.c_char_p, [_c_i32]),
    "sh_create": (_c_i32, [ctypes.POINTER(_vp), _c_i32, _c_i32]),
    "sh_destroy": (None, [_vp]),
    "sh_max_order": (_c_i32, [_vp]),
    "sh_device": (_c_i32, [_vp]),
    "sh_device_error": (_c_i32, [_vp]),
    "sh_translate_batch": (_c_i32, [_vp, _c_i32, _c_i32, _c_i32, _c_i32, _c_i64, _vp, _vp, _c_i64, _vp, _c_i64, _c_u32, _vp]),
    "sh_translate_indexed": (_c_i32, [_vp, _c_i32, _c_i32, _c_i32, _c_i32, _c_i64, _vp, _vp, _vp, _c_i64, _vp, _vp, _c_i64, _c_u32, _vp]),
    "sh_translate_indexed_checked": (_c_i32, [_vp, _c_i32, _c_i32, _c_i32, _c_i32, _c_i64, _vp, _vp, _vp, _c_i64, _c_i64,
                                              _vp, _vp, _c_i64, _c_i64, _c_u32, _vp]),
    "sh_m2l_naive_batch_f64": (_c_i32, [_vp, _c_i32, _c_i32, _c_i64, _vp, _vp, _c_i64, _vp, _c_i64, _c_u32, _vp]),
    "sh_p2m_batch_f64": (_c_i32, [_vp, _c_i32, _c_i64, _vp, _c_i64, _vp, _vp, _vp, _c_i64, _vp]),
    "sh_l2p_batch_f64": (_c_i32, [_vp, _c_i32, _c_i64, _vp, _c_i64, _vp, _vp, _c_i64, _vp, _c_u32, _vp]),
    "sh_fmm_create": (_c_i32, [_vp, _c_i32, _c_i32, _vp, ctypes.c_double, _c_i64, _vp]),
    "sh_fmm_create_orders": (_c_i32, [_vp, _c_i32, _vp, _vp, ctypes.c_double, _c_i64, _vp]),
    "sh_fmm_destroy": (None, [_vp]),
    "sh_fmm_orders_for_tolerance": (_c_i32, [ctypes.c_double, _c_i32, _vp]),
    "sh_fmm_evaluate": (_c_i32, [_vp, _vp, _vp, _vp, _c_u32, _vp]),
    "sh_fmm_describe": (_c_i32, [_vp, _vp]),
    "sh_swap_matrix_f64": (_c_i32, [_c_i32, _c_i32, _c_i32, _vp]),
    "sh_normalise_f64": (_c_i32, [_c_i32, _c_i32, _c_i64, _vp, _c_i64]),
    "sh_denormalise_f64": (_c_i32, [_c_i32, _c_i32, _c_i64, _vp, _c_i64]),
    "sh_plan_create": (_c_i32, [_vp, _c_i32, _vp, _c_i64, _c_u32, ctypes.POINTER(_vp)]),
    "sh_plan_execute": (_c_i32, [_vp, _vp, _c_i64, _vp, _c_i64, _vp]),
    "sh_plan_describe": (_c_i32, [_vp, _vp, _c_i64, ctypes.POINTER(_c_i64)]),
    "sh_plan_destroy": (None, [_vp]),
    "sh_translate_list": (_c_i32, [_vp, _c_i32, _vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_u32, _vp]),
    "sh_shared_create": (_c_i32, [_vp, _c_i32, _c_i32, _c_i32, _c_i32, _vp, _c_i32, ctypes.POINTER(_vp)]),
    "sh_shared_execute": (_c_i32, [_vp, _c_i64, _vp, _vp, _c_i64, _vp, _c_i64, _c_u32, _vp]),
    "sh_shared_bytes": (_c_i64, [_vp]),
    "sh_shared_destroy": (None, [_vp]),
    "sh_server_create": (_c_i32, [_vp, _vp, ctypes.POINTER(_vp)]),
    "sh_server_destroy": (None, [_vp]),
    "sh_server_tree_create": (_c_i32, [_vp, _c_i32, _c_i32, _c_i64, _c_i32, _c_i64, ctypes.POINTER(ctypes.c_int32)]),
    "sh_server_tree_write": (_c_i32, [_vp, ctypes.c_int32, _c_i32, _c_i64, _c_i64, _vp]),
    "sh_server_tree_read": (_c_i32, [_vp, ctypes.c_int32, _c_i32, _c_i64, _c_i64, _vp]),
    "sh_server_tree_destroy": (_c_i32, [_vp, ctypes.c_int32]),
    "sh_server_submit": (_c_i32, [_vp, _vp, ctypes.POINTER(_c_i64)]),
    "sh_server_wait": (_c_i32, [_vp, _c_i64, ctypes.POINTER(ctypes.c_double)]),
    "sh_server_drain": (_c_i32, [_vp]),
    "sh_server_stats_get": (_c_i32, [_vp, _vp]),
    "sh_server_stats_reset": (_c_i32, [_vp]),
    "sh_translate_single_noalloc": (_c_i32, [_vp, _c_i32, _c_i32, _c_i32, _c_i32, _vp, _vp, _vp]),
}
for _op in ("m2l", "m2m", "l2l"):
    for _dt in ("f64", "f32"):
        _SIGS[f"sh_{_op}_batch_{_dt}"] = (_c_i32, [_vp, _c_i32, _c_i32, _c_i64, _vp, _vp, _c_i64, _vp, _c_i64, _c_u32, _vp])
        _SIGS[f"sh_{_op}_{_dt}"] = (_c_i32, [_vp, _c_i32, _c_i32, _vp, _vp, _vp])


def lib():
    """The loaded ctypes library (raises LibraryMissing if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname (libamdhip64.so.7); loading
        # torch first makes this library bind to that runtime, so that torch's device
        # memory, streams, events and synchronisation are the ones the kernels use.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - C-only environments
            pass
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Names of every function the C header declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(sh_\w+)\s*\(", text, re.M)))


def sh_strerror(status: int) -> str:
    return lib().sh_strerror(int(status)).decode()


def _check(st: int, where: str) -> None:
    if st != SH_OK:
        raise ShError(st, where)


def _ptr(x):
    """Device/host address of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s):
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # pragma: no cover - torch without GPU
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Context:
    """Owning wrapper of an ``sh_ctx*`` (sh_create / sh_destroy)."""

    def __init__(self, max_order: int = 32, device: int = 0):
        h = _vp()
        _check(lib().sh_create(ctypes.byref(h), int(max_order), int(device)), "sh_create")
        self._h = h
        self.max_order = max_order
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().sh_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    def device_error(self) -> int:
        return lib().sh_device_error(self._h)


def sh_create(max_order: int = 32, device: int = 0) -> Context:
    return Context(max_order, device)


def sh_destroy(ctx: Context) -> None:
    ctx.close()


def sh_device_error(ctx: Context) -> int:
    return ctx.device_error()


def sh_max_order(ctx) -> int:
    return lib().sh_max_order(_h(ctx))


def sh_device(ctx) -> int:
    return lib().sh_device(_h(ctx))


def _h(ctx):
    return ctx.handle if isinstance(ctx, Context) else ctx


def sh_translate_batch(ctx, op, dtype, p_in, p_out, count, r, inp, ld_in, out, ld_out, flags=0, stream=None):
    _check(lib().sh_translate_batch(_h(ctx), OPS.get(op, op), dtype, p_in, p_out, count, _ptr(r), _ptr(inp),
                                    ld_in, _ptr(out), ld_out, flags, _stream(stream)), "sh_translate_batch")


def sh_translate_indexed(ctx, op, dtype, p_in, p_out, count, r, src, in_pool, ld_in, dst, out_pool, ld_out,
                         flags=0, stream=None):
    _check(lib().sh_translate_indexed(_h(ctx), OPS.get(op, op), dtype, p_in, p_out, count, _ptr(r), _ptr(src),
                                      _ptr(in_pool), ld_in, _ptr(dst), _ptr(out_pool), ld_out, flags,
                                      _stream(stream)), "sh_translate_indexed")


def sh_translate_indexed_checked(ctx, op, dtype, p_in, p_out, count, r, src, in_pool, ld_in, n_in, dst, out_pool,
                                 ld_out, n_out, flags=0, stream=None):
    _check(lib().sh_translate_indexed_checked(_h(ctx), OPS.get(op, op), dtype, p_in, p_out, count, _ptr(r), _ptr(src),
                                              _ptr(in_pool), ld_in, n_in, _ptr(dst), _ptr(out_pool), ld_out, n_out,
                                              flags, _stream(stream)), "sh_translate_indexed_checked")


def _make_batch(name):
    def f(ctx, p_in, p_out, count, r, inp, ld_in, out, ld_out, flags=0, stream=None):
        _check(getattr(lib(), name)(_h(ctx), p_in, p_out, count, _ptr(r), _ptr(inp), ld_in, _ptr(out), ld_out,
                                    flags, _stream(stream)), name)
    f.__name__ = name
    f.__doc__ = f"Forwards to the C function {name} (device pointers, stream-ordered)."
    return f


def _make_single(name, dtype):
    def f(ctx, p_in, p_out, r, C):
        """Single translation on host arrays (synchronous); returns the output solid."""
        r = np.ascontiguousarray(r, dtype=dtype)
        C = np.ascontiguousarray(C, dtype=dtype)
        out = np.zeros(p_out * (p_out + 1), dtype)
        _check(getattr(lib(), name)(_h(ctx), p_in, p_out, r.ctypes.data, C.ctypes.data, out.ctypes.data), name)
        return out
    f.__name__ = name
    return f


for _op in ("m2l", "m2m", "l2l"):
    for _dt, _npdt in (("f64", np.float64), ("f32", np.float32)):
        globals()[f"sh_{_op}_batch_{_dt}"] = _make_batch(f"sh_{_op}_batch_{_dt}")
        globals()[f"sh_{_op}_{_dt}"] = _make_single(f"sh_{_op}_{_dt}", _npdt)
sh_m2l_naive_batch_f64 = _make_batch("sh_m2l_naive_batch_f64")


def sh_translate_single_noalloc(ctx, op, dtype, p_in, p_out, r, C):
    """Single translation on host arrays through the library's fixed staging array (no
    device allocation); returns the output solid."""
    npdt = np.float64 if dtype == SH_F64 else np.float32
    r = np.ascontiguousarray(r, dtype=npdt)
    C = np.ascontiguousarray(C, dtype=npdt)
    out = np.zeros(p_out * (p_out + 1), npdt)
    _check(lib().sh_translate_single_noalloc(_h(ctx), OPS.get(op, op), dtype, p_in, p_out, r.ctypes.data,
                                             C.ctypes.data, out.ctypes.data), "sh_translate_single_noalloc")
    return out


def sh_p2m_batch_f64(ctx, P, count, centres, npts, pts, q, M, ldM, stream=None):
    _check(lib().sh_p2m_batch_f64(_h(ctx), P, count, _ptr(centres), npts, _ptr(pts), _ptr(q), _ptr(M), ldM,
                                  _stream(stream)), "sh_p2m_batch_f64")


def sh_l2p_batch_f64(ctx, P, count, centres, npts, pts, L, ldL, out, flags=0, stream=None):
    _check(lib().sh_l2p_batch_f64(_h(ctx), P, count, _ptr(centres), npts, _ptr(pts), _ptr(L), ldL, _ptr(out),
                                  flags, _stream(stream)), "sh_l2p_batch_f64")


def sh_swap_matrix_f64(n: int, which: int, normalised: bool = False) -> np.ndarray:
    out = np.zeros((n + 1, n + 1))
    _check(lib().sh_swap_matrix_f64(n, which, int(bool(normalised)), out.ctypes.data), "sh_swap_matrix_f64")
    return out


def sh_normalise_f64(kind: int, P: int, solids: np.ndarray) -> np.ndarray:
    a = np.array(solids, dtype=np.float64, copy=True, order="C")
    a2 = a.reshape(-1, a.shape[-1])
    _check(lib().sh_normalise_f64(kind, P, a2.shape[0], a2.ctypes.data, a2.shape[1]), "sh_normalise_f64")
    return a


def sh_denormalise_f64(kind: int, P: int, solids: np.ndarray) -> np.ndarray:
    a = np.array(solids, dtype=np.float64, copy=True, order="C")
    a2 = a.reshape(-1, a.shape[-1])
    _check(lib().sh_denormalise_f64(kind, P, a2.shape[0], a2.ctypes.data, a2.shape[1]), "sh_denormalise_f64")
    return a


# ---------------- mixed work lists ----------------

# numpy image of the C struct sh_item (56 bytes)
SH_ITEM = np.dtype([("op", "<i4"), ("p_in", "<i4"), ("p_out", "<i4"), ("reserved", "<i4"),
                    ("in_off", "<i8"), ("out_off", "<i8"), ("r", "<f8", (3,))], align=True)
assert SH_ITEM.itemsize == 56


def make_items(op, p_in, p_out, in_off, out_off, r) -> np.ndarray:
    """Packs per-item arrays (broadcast) into an sh_item array."""
    op = np.asarray(op)
    n = np.broadcast(op, np.asarray(p_in), np.asarray(p_out), np.asarray(in_off), np.asarray(out_off)).shape
    n = int(np.prod(n)) if n else 1
    it = np.zeros(n, SH_ITEM)
    it["op"] = op
    it["p_in"] = p_in
    it["p_out"] = p_out
    it["in_off"] = in_off
    it["out_off"] = out_off
    it["r"] = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    return it


class Plan:
    """Owning wrapper of an ``sh_plan*`` (sh_plan_create / sh_plan_destroy)."""

    def __init__(self, ctx, dtype: int, items: np.ndarray, flags: int = 0):
        items = np.ascontiguousarray(items, dtype=SH_ITEM)
        h = _vp()
        _check(lib().sh_plan_create(_h(ctx), dtype, items.ctypes.data if len(items) else None, len(items), flags,
                                    ctypes.byref(h)), "sh_plan_create")
        self._h = h.value
        self.ctx = ctx
        self.dtype = dtype

    @property
    def handle(self):
        if not self._h:
            raise ValueError("plan destroyed")
        return self._h

    def execute(self, arena_in, in_reals, arena_out, out_reals, stream=None):
        _check(lib().sh_plan_execute(self.handle, _ptr(arena_in), in_reals, _ptr(arena_out), out_reals,
                                     _stream(stream)), "sh_plan_execute")

    def describe(self) -> dict:
        import json
        need = _c_i64()
        _check(lib().sh_plan_describe(self.handle, None, 0, ctypes.byref(need)), "sh_plan_describe")
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().sh_plan_describe(self.handle, buf, need.value, None), "sh_plan_describe")
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            lib().sh_plan_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


def sh_plan_create(ctx, dtype, items, flags=0) -> Plan:
    return Plan(ctx, dtype, items, flags)


def sh_plan_execute(plan: Plan, arena_in, in_reals, arena_out, out_reals, stream=None) -> None:
    plan.execute(arena_in, in_reals, arena_out, out_reals, stream)


def sh_plan_describe(plan: Plan) -> dict:
    return plan.describe()


def sh_plan_destroy(plan: Plan) -> None:
    plan.close()


def sh_translate_list(ctx, dtype, items, arena_in, in_reals, arena_out, out_reals, flags=0, stream=None):
    items = np.ascontiguousarray(items, dtype=SH_ITEM)
    _check(lib().sh_translate_list(_h(ctx), dtype, items.ctypes.data if len(items) else None, len(items),
                                   _ptr(arena_in), in_reals, _ptr(arena_out), out_reals, flags, _stream(stream)),
           "sh_translate_list")


# ---------------- shared-shift operators (matrix cores) ----------------

class Shared:
    """Owning wrapper of an ``sh_shared*`` (sh_shared_create / sh_shared_destroy)."""

    def __init__(self, ctx, op, p_in, p_out, shifts, precision=SH_SHARED_BF16X6):
        shifts = np.ascontiguousarray(np.reshape(shifts, (-1, 3)), dtype=np.float64)
        h = _vp()
        _check(lib().sh_shared_create(_h(ctx), OPS.get(op, op), p_in, p_out, shifts.shape[0], shifts.ctypes.data,
                                      precision, ctypes.byref(h)), "sh_shared_create")
        self._h = h.value
        self.nclass = shifts.shape[0]
        self.p_in, self.p_out = p_in, p_out

    @property
    def handle(self):
        if not self._h:
            raise ValueError("shared operators destroyed")
        return self._h

    def execute(self, count, class_start, inp, ld_in, out, ld_out, flags=0, stream=None):
        _check(lib().sh_shared_execute(self.handle, count, _ptr(class_start), _ptr(inp), ld_in, _ptr(out), ld_out,
                                       flags, _stream(stream)), "sh_shared_execute")

    def nbytes(self) -> int:
        return int(lib().sh_shared_bytes(self.handle))

    def close(self):
        if self._h:
            lib().sh_shared_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


def sh_shared_create(ctx, op, p_in, p_out, shifts, precision=SH_SHARED_BF16X6) -> Shared:
    return Shared(ctx, op, p_in, p_out, shifts, precision)


def sh_shared_execute(shared: Shared, count, class_start, inp, ld_in, out, ld_out, flags=0, stream=None) -> None:
    shared.execute(count, class_start, inp, ld_in, out, ld_out, flags, stream)


def sh_shared_bytes(shared: Shared) -> int:
    return shared.nbytes()


def sh_shared_destroy(shared: Shared) -> None:
    shared.close()


# ---------------- serving ----------------

class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("staging_bytes", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("max_batch_jobs", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_int32), ("op", ctypes.c_int32), ("count", ctypes.c_int64),
                ("r", ctypes.c_void_p), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("jobs_done", "jobs_failed", "translations_done", "batches",
                                              "queue_peak", "staging_peak_bytes", "pool_used_bytes",
                                              "jobs_deferred")] + \
               [(n, ctypes.c_double) for n in ("mean_batch_jobs", "elapsed_s", "p50_s", "p99_s", "mean_s", "max_s")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Server:
    """Owning wrapper of an ``sh_server*`` (sh_server_create / sh_server_destroy)."""

    def __init__(self, ctx, pool_bytes, staging_bytes=64 << 20, streams=2, max_batch_jobs=64):
        cfg = ServerConfig(pool_bytes, staging_bytes, streams, max_batch_jobs)
        h = _vp()
        _check(lib().sh_server_create(_h(ctx), ctypes.byref(cfg), ctypes.byref(h)), "sh_server_create")
        self._h = h.value
        self.ctx = ctx

    @property
    def handle(self):
        if not self._h:
            raise ValueError("server destroyed")
        return self._h

    def tree_create(self, dtype, p_m, n_m, p_l, n_l) -> int:
        t = ctypes.c_int32()
        _check(lib().sh_server_tree_create(self.handle, dtype, p_m, n_m, p_l, n_l, ctypes.byref(t)),
               "sh_server_tree_create")
        return t.value

    def tree_write(self, tree, pool, first, solids: np.ndarray):
        a = np.ascontiguousarray(solids)
        _check(lib().sh_server_tree_write(self.handle, tree, pool, first, a.shape[0], a.ctypes.data),
               "sh_server_tree_write")

    def tree_read(self, tree, pool, first, n, P, dtype=np.float64) -> np.ndarray:
        out = np.zeros((n, P * (P + 1)), dtype)
        _check(lib().sh_server_tree_read(self.handle, tree, pool, first, n, out.ctypes.data), "sh_server_tree_read")
        return out

    def tree_destroy(self, tree):
        _check(lib().sh_server_tree_destroy(self.handle, tree), "sh_server_tree_destroy")

    def submit(self, tree, op, r, src, dst, flags=0) -> int:
        r = np.ascontiguousarray(np.reshape(r, (-1, 3)), dtype=np.float64)
        src = np.ascontiguousarray(src, dtype=np.int64)
        dst = np.ascontiguousarray(dst, dtype=np.int64)
        n = len(src)
        if r.shape[0] != n or len(dst) != n:
            raise ValueError("r, src and dst must describe the same number of translations")
        job = Job(tree, OPS.get(op, op), n, r.ctypes.data if n else None, src.ctypes.data if n else None,
                  dst.ctypes.data if n else None, flags, 0)
        jid = _c_i64()
        _check(lib().sh_server_submit(self.handle, ctypes.byref(job), ctypes.byref(jid)), "sh_server_submit")
        return jid.value

    def wait(self, job_id) -> float:
        lat = ctypes.c_double()
        _check(lib().sh_server_wait(self.handle, job_id, ctypes.byref(lat)), "sh_server_wait")
        return lat.value

    def drain(self):
        _check(lib().sh_server_drain(self.handle), "sh_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().sh_server_stats_get(self.handle, ctypes.byref(st)), "sh_server_stats_get")
        return st.as_dict()

    def stats_reset(self):
        _check(lib().sh_server_stats_reset(self.handle), "sh_server_stats_reset")

    def close(self):
        if self._h:
            lib().sh_server_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


def sh_server_create(ctx, pool_bytes, staging_bytes=64 << 20, streams=2, max_batch_jobs=64) -> Server:
    return Server(ctx, pool_bytes, staging_bytes, streams, max_batch_jobs)


def sh_server_destroy(server: Server) -> None:
    server.close()


def sh_server_tree_create(server: Server, dtype, p_m, n_m, p_l, n_l) -> int:
    return server.tree_create(dtype, p_m, n_m, p_l, n_l)


def sh_server_tree_write(server: Server, tree, pool, first, solids) -> None:
    server.tree_write(tree, pool, first, solids)


def sh_server_tree_read(server: Server, tree, pool, first, n, P, dtype=np.float64) -> np.ndarray:
    return server.tree_read(tree, pool, first, n, P, dtype)


def sh_server_tree_destroy(server: Server, tree) -> None:
    server.tree_destroy(tree)


def sh_server_submit(server: Server, tree, op, r, src, dst, flags=0) -> int:
    return server.submit(tree, op, r, src, dst, flags)


def sh_server_wait(server: Server, job_id) -> float:
    return server.wait(job_id)


def sh_server_drain(server: Server) -> None:
    server.drain()


def sh_server_stats_get(server: Server) -> dict:
    return server.stats()


def sh_server_stats_reset(server: Server) -> None:
    server.stats_reset()


def sh_fmm_create(ctx, P, levels, origin, width, npts):
    """Returns the sh_fmm handle (a ctypes.c_void_p)."""
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    h = ctypes.c_void_p()
    _check(lib().sh_fmm_create(_h(ctx), int(P), int(levels), o, float(width), int(npts), ctypes.byref(h)),
           "sh_fmm_create")
    return h


def sh_fmm_create_orders(ctx, levels, orders, origin, width, npts):
    """Per-level orders: orders[l - 2] for level l = 2..levels.  Returns the sh_fmm handle."""
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    ords = (ctypes.c_int * len(orders))(*[int(v) for v in orders])
    if len(orders) != int(levels) - 1:
        raise ValueError("orders needs one entry per level 2..levels")
    h = ctypes.c_void_p()
    _check(lib().sh_fmm_create_orders(_h(ctx), int(levels), ords, o, float(width), int(npts), ctypes.byref(h)),
           "sh_fmm_create_orders")
    return h


def sh_fmm_orders_for_tolerance(tol, levels):
    """Orders of levels 2..levels for a relative potential error target (host only)."""
    out = (ctypes.c_int * (int(levels) - 1))() if int(levels) >= 2 else (ctypes.c_int * 1)()
    _check(lib().sh_fmm_orders_for_tolerance(float(tol), int(levels), out), "sh_fmm_orders_for_tolerance")
    return list(out)


def sh_fmm_destroy(h):
    lib().sh_fmm_destroy(h)


def sh_fmm_evaluate(h, pts, q, out, flags=0, stream=None):
    _check(lib().sh_fmm_evaluate(h, _ptr(pts), _ptr(q), _ptr(out), flags, _stream(stream)), "sh_fmm_evaluate")


def sh_fmm_describe(h):
    """[M2M, M2L, L2L translations per evaluation, translation calls, leaves]."""
    c = (ctypes.c_int64 * 5)()
    _check(lib().sh_fmm_describe(h, c), "sh_fmm_describe")
    return list(c)


class Fmm:
    """Uniform-octree FMM handle (sh_fmm_*): P2M, M2M, M2L, L2L, L2P and P2P on the device."""

    def __init__(self, ctx, P, levels, origin, width, npts, orders=None):
        """orders (optional): the order of each level 2..levels; P is then ignored."""
        self._ctx = ctx
        self._h = None
        if orders is None:
            self._h = sh_fmm_create(ctx, P, levels, origin, width, npts)
        else:
            self._h = sh_fmm_create_orders(ctx, levels, orders, origin, width, npts)
            P = orders[-1]
        self.P, self.levels, self.npts = int(P), int(levels), int(npts)
        self.n_particles = 8 ** self.levels * self.npts

    def evaluate(self, pts, q, out, flags=0, stream=None):
        sh_fmm_evaluate(self._h, pts, q, out, flags, stream)

    def describe(self):
        c = sh_fmm_describe(self._h)
        return {"m2m": c[0], "m2l": c[1], "l2l": c[2], "calls": c[3], "leaves": c[4]}

    def close(self):
        if self._h:
            sh_fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
