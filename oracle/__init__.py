"""CPU reference oracle for the solid-harmonic translations -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``oracle.c`` (plain FP64 definitions of the regular and
singular harmonics, P2M/P2L, the double-height M2L sum, M2M, L2L and evaluation;
see the header of ``oracle.c`` for the passages of the paper each routine follows).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.

Parity status: every routine here is pinned by ``tests/test_oracle_pins.py``
against closed forms, the paper's z-axis formulas, direct summation and
exact-arithmetic identities; no routine is "parity unpinned".

Layout of a solid of order P: ``P*(P+1)`` reals, ``Re C_n^m`` at ``n*(n+1)+2*m`` and
``Im C_n^m`` right after it (m = 0..n).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIBS = {
    "double": os.path.join(_HERE, "liboracle_f64.so"),
    "longdouble": os.path.join(_HERE, "liboracle_ld.so"),
}
_FLAGS = {
    "double": [],
    "longdouble": ["-DREAL=long double", "-DORACLE_LONG_DOUBLE"],
}


def build(force: bool = True) -> None:
    """Compile the oracle (both precisions) with gcc.  No fast-math: IEEE semantics."""
    for kind, out in _LIBS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
               *_FLAGS[kind], _SRC, "-o", out + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def compile_variant(src: str, out: str, kind: str = "double") -> None:
    """Compile an arbitrary copy of the oracle source (used by the planted-mistake tests)."""
    cmd = ["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c99", *_FLAGS[kind],
           src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)


class Oracle:
    """One loaded oracle library (double or long double arithmetic)."""

    def __init__(self, kind: str = "double", path: str | None = None):
        if path is None:
            path = _LIBS[kind]
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
                build(force=True)
        self.kind = kind
        self.dtype = np.float64 if kind == "double" else np.longdouble
        ct = ctypes.c_double if kind == "double" else ctypes.c_longdouble
        self._ct = ct
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(ct)
        i32, i64 = ctypes.c_int, ctypes.c_int64
        sig = {
            "or_regular": (None, [P, i32, P]),
            "or_singular": (None, [P, i32, P]),
            "or_p2m": (None, [i32, P, i64, P, P, P]),
            "or_p2l": (None, [i32, P, i64, P, P, P]),
            "or_m2l": (None, [i32, i32, P, P, P]),
            "or_m2m": (None, [i32, i32, P, P, P]),
            "or_l2l": (None, [i32, i32, P, P, P]),
            "or_eval_m": (ct, [i32, P, P, P]),
            "or_eval_l": (ct, [i32, P, P, P]),
            "or_direct": (ct, [i64, P, P, P]),
            "or_l2p": (None, [i32, P, P, P, P]),
            "or_m2l_single": (None, [i32, P, P, P]),
            "or_m2l_single_batch": (None, [i64, i32, P, P, i64, P, i64, i32]),
            "or_l2p_batch": (None, [i64, i32, P, i64, P, P, i64, P, i32]),
            "or_translate_batch": (None, [i32, i64, i32, i32, P, P, i64, P, i64, i32]),
            "or_p2m_batch": (None, [i64, i32, P, i64, P, P, P, i64, i32]),
            "or_p2l_batch": (None, [i64, i32, P, i64, P, P, P, i64, i32]),
            "or_real_size": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        self._lib = lib
        self._P = P
        assert lib.or_real_size() == np.dtype(self.dtype).itemsize

    # -- marshalling helpers -------------------------------------------------
    def _arr(self, a):
        a = np.ascontiguousarray(a, dtype=self.dtype)
        return a, a.ctypes.data_as(self._P)

    @staticmethod
    def size(P: int) -> int:
        return P * (P + 1)

    # -- harmonics -------------------------------------------------------------
    def regular(self, r, P):
        r, rp = self._arr(r)
        out = np.zeros(self.size(P), self.dtype)
        self._lib.or_regular(rp, P, out.ctypes.data_as(self._P))
        return out

    def singular(self, r, P):
        r, rp = self._arr(r)
        out = np.zeros(self.size(P), self.dtype)
        self._lib.or_singular(rp, P, out.ctypes.data_as(self._P))
        return out

    # -- particle <-> expansion ----------------------------------------------
    def p2m(self, P, centre, pts, q):
        c, cp = self._arr(centre)
        pts, pp = self._arr(np.reshape(pts, (-1, 3)))
        q, qp = self._arr(q)
        out = np.zeros(self.size(P), self.dtype)
        self._lib.or_p2m(P, cp, len(q), pp, qp, out.ctypes.data_as(self._P))
        return out

    def p2l(self, P, centre, pts, q):
        c, cp = self._arr(centre)
        pts, pp = self._arr(np.reshape(pts, (-1, 3)))
        q, qp = self._arr(q)
        out = np.zeros(self.size(P), self.dtype)
        self._lib.or_p2l(P, cp, len(q), pp, qp, out.ctypes.data_as(self._P))
        return out

    def _p2x_batch(self, fn, P, centres, pts, q, nthreads):
        centres, cp = self._arr(np.reshape(centres, (-1, 3)))
        count = centres.shape[0]
        pts, pp = self._arr(np.reshape(pts, (count, -1, 3)))
        npts = pts.shape[1]
        q, qp = self._arr(np.reshape(q, (count, npts)))
        out = np.zeros((count, self.size(P)), self.dtype)
        fn(count, P, cp, npts, pp, qp, out.ctypes.data_as(self._P), self.size(P), nthreads)
        return out

    def p2m_batch(self, P, centres, pts, q, nthreads=1):
        return self._p2x_batch(self._lib.or_p2m_batch, P, centres, pts, q, nthreads)

    def p2l_batch(self, P, centres, pts, q, nthreads=1):
        return self._p2x_batch(self._lib.or_p2l_batch, P, centres, pts, q, nthreads)

    # -- translations ----------------------------------------------------------
    def _tr(self, fn, p_in, p_out, r, C):
        r, rp = self._arr(r)
        C, Cp = self._arr(C)
        assert C.size >= self.size(p_in)
        out = np.zeros(self.size(p_out), self.dtype)
        fn(p_in, p_out, rp, Cp, out.ctypes.data_as(self._P))
        return out

    def m2l(self, p_in, p_out, r, M):
        return self._tr(self._lib.or_m2l, p_in, p_out, r, M)

    def m2l_single(self, P, r, M):
        """Single-height M2L (eq. m2lkernels, left) at one order P."""
        r, rp = self._arr(r)
        M, Mp = self._arr(M)
        assert M.size >= self.size(P)
        out = np.zeros(self.size(P), self.dtype)
        self._lib.or_m2l_single(P, rp, Mp, out.ctypes.data_as(self._P))
        return out

    def m2l_single_batch(self, P, r, C, nthreads=1):
        r, rp = self._arr(np.reshape(r, (-1, 3)))
        count = r.shape[0]
        C, Cp = self._arr(np.reshape(C, (count, -1)))
        out = np.zeros((count, self.size(P)), self.dtype)
        self._lib.or_m2l_single_batch(count, P, rp, Cp, C.shape[1], out.ctypes.data_as(self._P), self.size(P),
                                      nthreads)
        return out

    def m2m(self, p_in, p_out, r, M):
        return self._tr(self._lib.or_m2m, p_in, p_out, r, M)

    def l2l(self, p_in, p_out, r, L):
        return self._tr(self._lib.or_l2l, p_in, p_out, r, L)

    OPS = {"m2m": 0, "m2l": 1, "l2l": 2}

    def translate_batch(self, op, p_in, p_out, r, C, nthreads=1):
        """Batched translation: C has shape (count, >= p_in(p_in+1)), r shape (count, 3)."""
        r, rp = self._arr(np.reshape(r, (-1, 3)))
        count = r.shape[0]
        C, Cp = self._arr(np.reshape(C, (count, -1)))
        out = np.zeros((count, self.size(p_out)), self.dtype)
        self._lib.or_translate_batch(self.OPS[op], count, p_in, p_out, rp, Cp, C.shape[1],
                                     out.ctypes.data_as(self._P), self.size(p_out), nthreads)
        return out

    # -- evaluation --------------------------------------------------------------
    def eval_m(self, P, centre, M, x):
        c, cp = self._arr(centre)
        M, Mp = self._arr(M)
        x, xp = self._arr(x)
        return self._lib.or_eval_m(P, cp, Mp, xp)

    def eval_l(self, P, centre, L, x):
        c, cp = self._arr(centre)
        L, Lp = self._arr(L)
        x, xp = self._arr(x)
        return self._lib.or_eval_l(P, cp, Lp, xp)

    def l2p(self, P, centre, L, x):
        """{Phi_L(x), grad Phi_L(x)} of one local expansion at one point."""
        c, cp = self._arr(centre)
        L, Lp = self._arr(L)
        x, xp = self._arr(x)
        out = np.zeros(4, self.dtype)
        self._lib.or_l2p(P, cp, Lp, xp, out.ctypes.data_as(self._P))
        return out

    def l2p_batch(self, P, centres, pts, L, nthreads=1):
        """Boxes of npts targets each: returns (count, npts, 4) = {Phi, grad Phi} per target."""
        centres, cp = self._arr(np.reshape(centres, (-1, 3)))
        count = centres.shape[0]
        pts, pp = self._arr(np.reshape(pts, (count, -1, 3)))
        npts = pts.shape[1]
        L, Lp = self._arr(np.reshape(L, (count, -1)))
        out = np.zeros((count, npts, 4), self.dtype)
        self._lib.or_l2p_batch(count, P, cp, npts, pp, Lp, L.shape[1], out.ctypes.data_as(self._P), nthreads)
        return out

    def direct(self, pts, q, x):
        pts, pp = self._arr(np.reshape(pts, (-1, 3)))
        q, qp = self._arr(q)
        x, xp = self._arr(x)
        return self._lib.or_direct(len(q), pp, qp, xp)


_CACHE: dict = {}


def get(kind: str = "double") -> Oracle:
    if kind not in _CACHE:
        _CACHE[kind] = Oracle(kind)
    return _CACHE[kind]
