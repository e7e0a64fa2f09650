"""CPU FP64 oracle for findpts / findpts_eval, in three dimensions
(OracleMesh) and two (OracleMesh2) (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``findpts_oracle.c`` through
ctypes and shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
        L.or_gll.argtypes = [C.c_int, dp, dp]
        L.or_lagrange.argtypes = [C.c_int, C.c_double, dp, dp]
        L.or_bernstein_inverse.argtypes = [C.c_int, dp]
        L.or_setup.restype = vp
        L.or_setup.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, ip, dp]
        L.or_free.argtypes = [vp]
        L.or_get_bbox.argtypes = [vp, dp, dp]
        L.or_get_hash.argtypes = [vp, ip, dp, dp, ip]
        L.or_map.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or_candidates.argtypes = [vp, dp, C.c_int, ip, C.c_int]
        L.or_newton.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or_newton_from.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or_findpts.argtypes = [vp, C.c_int, dp, ip, ip, ip, dp, dp,
                                 C.POINTER(C.c_longlong), C.c_int]
        L.or_brute.argtypes = [vp, C.c_int, dp, ip, C.c_int, C.c_int, C.c_int,
                               ip, ip, dp, dp, C.c_int]
        L.or_eval.argtypes = [vp, C.c_int, ip, ip, dp, C.c_int,
                              C.POINTER(dp), dp, C.c_int]
        L.or_threads.argtypes = [C.c_int]
        L.or2_setup.restype = vp
        L.or2_setup.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, ip, dp]
        L.or2_free.argtypes = [vp]
        L.or2_get_bbox.argtypes = [vp, dp, dp]
        L.or2_map.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or2_candidates.argtypes = [vp, dp, C.c_int, ip, C.c_int]
        L.or2_newton.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or2_newton_from.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or2_findpts.argtypes = [vp, C.c_int, dp, ip, ip, ip, dp, dp,
                                  C.POINTER(C.c_longlong), C.c_int]
        L.or2_brute.argtypes = [vp, C.c_int, dp, ip, C.c_int, C.c_int, C.c_int,
                                ip, ip, dp, dp, C.c_int]
        L.or2_eval.argtypes = [vp, C.c_int, ip, ip, dp, C.c_int,
                               C.POINTER(dp), dp, C.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def gll(N):
    z, w = np.zeros(N + 1), np.zeros(N + 1)
    if lib().or_gll(N, _d(z), _d(w)):
        raise ValueError("N out of range")
    return z, w


def lagrange(N, r):
    h, dh = np.zeros(N + 1), np.zeros(N + 1)
    if lib().or_lagrange(N, float(r), _d(h), _d(dh)):
        raise ValueError("N out of range")
    return h, dh


def bernstein_inverse(N):
    B = np.zeros((N + 1) * (N + 1))
    lib().or_bernstein_inverse(N, _d(B))
    return B.reshape(N + 1, N + 1)


class OracleMesh:
    """Oracle state for one mesh (keeps host copies of its inputs alive)."""

    def __init__(self, x, y, z, N, tol=1e-12, session=None, delta=None):
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        self.N = int(N)
        n1 = self.N + 1
        self.V = n1 ** 3
        self.E = self.x.size // self.V
        self.session = None if session is None else _i32(session)
        self.delta = None if delta is None else _f64(delta)
        self.tol = float(tol)
        h = lib().or_setup(self.E, self.N, _d(self.x), _d(self.y), _d(self.z),
                           self.tol,
                           None if self.session is None else _i(self.session),
                           None if self.delta is None else _d(self.delta))
        if not h:
            raise ValueError("oracle setup rejected the mesh")
        self._h = C.c_void_p(h)

    @classmethod
    def from_mesh(cls, mesh, tol=1e-12):
        hd = mesh.host()
        return cls(hd["x"], hd["y"], hd["z"], mesh.N, tol, hd["session"], hd["delta"])

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_free(self._h)
            self._h = None

    # ------------------------------------------------------------------
    def bbox(self):
        b, h = np.zeros(6 * self.E), np.zeros(self.E)
        lib().or_get_bbox(self._h, _d(b), _d(h))
        return b.reshape(self.E, 6), h

    def hash_info(self):
        nc, lo, dx, nnz = (C.c_int * 3)(), np.zeros(3), np.zeros(3), C.c_int()
        lib().or_get_hash(self._h, nc, _d(lo), _d(dx), C.byref(nnz))
        return list(nc), lo, dx, nnz.value

    def map(self, e, r):
        r = _f64(r); x = np.zeros(3); J = np.zeros(9)
        lib().or_map(self._h, int(e), _d(r), _d(x), _d(J))
        return x, J.reshape(3, 3)

    def candidates(self, p, psess=-1):
        p = _f64(p); out = np.zeros(self.E, np.int32)
        n = lib().or_candidates(self._h, _d(p), int(psess), _i(out), self.E)
        return out[:n].copy()

    def newton(self, e, p, r0=None):
        p = _f64(p); r = np.zeros(3) if r0 is None else _f64(r0).copy(); d2 = np.zeros(1)
        if r0 is None:
            it = lib().or_newton(self._h, int(e), _d(p), _d(r), _d(d2))
        else:
            it = lib().or_newton_from(self._h, int(e), _d(p), _d(r), _d(d2))
        return r, float(d2[0]), it

    def findpts(self, pts, psess=None, nthreads=0):
        pts = _f64(pts).reshape(-1, 3)
        n = pts.shape[0]
        code, el = np.zeros(n, np.int32), np.zeros(n, np.int32)
        rst, d2 = np.zeros((n, 3)), np.zeros(n)
        st = (C.c_longlong * 2)()
        ps = None if psess is None else _i32(psess)
        lib().or_findpts(self._h, n, _d(pts), None if ps is None else _i(ps),
                         _i(code), _i(el), _d(rst), _d(d2), st, int(nthreads))
        self.last_stats = (st[0], st[1])
        return code, el, rst, d2

    def brute(self, pts, psess=None, grid=3, all_nodes=False, only_boxes=False,
              nthreads=0):
        pts = _f64(pts).reshape(-1, 3)
        n = pts.shape[0]
        code, el = np.zeros(n, np.int32), np.zeros(n, np.int32)
        rst, d2 = np.zeros((n, 3)), np.zeros(n)
        ps = None if psess is None else _i32(psess)
        lib().or_brute(self._h, n, _d(pts), None if ps is None else _i(ps),
                       int(grid), int(bool(all_nodes)), int(bool(only_boxes)),
                       _i(code), _i(el), _d(rst), _d(d2), int(nthreads))
        return code, el, rst, d2

    def eval(self, code, el, rst, fields, nthreads=0):
        code, el, rst = _i32(code), _i32(el), _f64(rst)
        n = code.size
        fl = [_f64(f) for f in fields]
        arr = (C.POINTER(C.c_double) * len(fl))(*[_d(f) for f in fl])
        out = np.zeros((len(fl), n))
        lib().or_eval(self._h, n, _i(code), _i(el), _d(rst), len(fl), arr,
                      _d(out), int(nthreads))
        return out


class OracleMesh2:
    """Oracle state for one two-dimensional mesh (quadrilateral elements,
    x and y of E*(N+1)^2 nodes each)."""

    def __init__(self, x, y, N, tol=1e-12, session=None, delta=None):
        self.x, self.y = _f64(x), _f64(y)
        self.N = int(N)
        self.V = (self.N + 1) ** 2
        self.E = self.x.size // self.V
        self.session = None if session is None else _i32(session)
        self.delta = None if delta is None else _f64(delta)
        self.tol = float(tol)
        h = lib().or2_setup(self.E, self.N, _d(self.x), _d(self.y), self.tol,
                            None if self.session is None else _i(self.session),
                            None if self.delta is None else _d(self.delta))
        if not h:
            raise ValueError("oracle setup rejected the mesh")
        self._h = C.c_void_p(h)

    @classmethod
    def from_mesh(cls, mesh, tol=1e-12):
        hd = mesh.host()
        return cls(hd["x"], hd["y"], mesh.N, tol, hd["session"], hd["delta"])

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or2_free(self._h)
            self._h = None

    def bbox(self):
        b, h = np.zeros(4 * self.E), np.zeros(self.E)
        lib().or2_get_bbox(self._h, _d(b), _d(h))
        return b.reshape(self.E, 4), h

    def map(self, e, r):
        r = _f64(r); x = np.zeros(2); J = np.zeros(4)
        lib().or2_map(self._h, int(e), _d(r), _d(x), _d(J))
        return x, J.reshape(2, 2)

    def candidates(self, p, psess=-1):
        p = _f64(p); out = np.zeros(self.E, np.int32)
        n = lib().or2_candidates(self._h, _d(p), int(psess), _i(out), self.E)
        return out[:n].copy()

    def newton(self, e, p, r0=None):
        p = _f64(p); r = np.zeros(2) if r0 is None else _f64(r0).copy(); d2 = np.zeros(1)
        if r0 is None:
            it = lib().or2_newton(self._h, int(e), _d(p), _d(r), _d(d2))
        else:
            it = lib().or2_newton_from(self._h, int(e), _d(p), _d(r), _d(d2))
        return r, float(d2[0]), it

    def findpts(self, pts, psess=None, nthreads=0):
        pts = _f64(pts).reshape(-1, 2)
        n = pts.shape[0]
        code, el = np.zeros(n, np.int32), np.zeros(n, np.int32)
        rs, d2 = np.zeros((n, 2)), np.zeros(n)
        st = (C.c_longlong * 2)()
        ps = None if psess is None else _i32(psess)
        lib().or2_findpts(self._h, n, _d(pts), None if ps is None else _i(ps),
                          _i(code), _i(el), _d(rs), _d(d2), st, int(nthreads))
        self.last_stats = (st[0], st[1])
        return code, el, rs, d2

    def brute(self, pts, psess=None, grid=3, all_nodes=False, only_boxes=False,
              nthreads=0):
        pts = _f64(pts).reshape(-1, 2)
        n = pts.shape[0]
        code, el = np.zeros(n, np.int32), np.zeros(n, np.int32)
        rs, d2 = np.zeros((n, 2)), np.zeros(n)
        ps = None if psess is None else _i32(psess)
        lib().or2_brute(self._h, n, _d(pts), None if ps is None else _i(ps),
                        int(grid), int(bool(all_nodes)), int(bool(only_boxes)),
                        _i(code), _i(el), _d(rs), _d(d2), int(nthreads))
        return code, el, rs, d2

    def eval(self, code, el, rs, fields, nthreads=0):
        code, el, rs = _i32(code), _i32(el), _f64(rs)
        n = code.size
        fl = [_f64(f) for f in fields]
        arr = (C.POINTER(C.c_double) * len(fl))(*[_d(f) for f in fl])
        out = np.zeros((len(fl), n))
        lib().or2_eval(self._h, n, _i(code), _i(el), _d(rs), len(fl), arr,
                       _d(out), int(nthreads))
        return out


def threads(n=0):
    return lib().or_threads(int(n))
