"""Thin ctypes binding of libfindpts.so (the gfx950 findpts library).

Same names as the C ABI in include/findpts.h.  This module only marshals
arguments (torch CUDA tensors -> device pointers, the current torch stream ->
hipStream_t) and allocates output tensors when the caller does not pass
them; every step of point location and interpolation runs in the library's
HIP kernels.  There is no fallback: if the library is not built, or a tensor
is not a contiguous CUDA tensor of the right dtype, a call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfindpts.so")

FP_OK, FP_EINVAL, FP_ENOMEM, FP_EHIP, FP_ESTATE, FP_ERANGE, FP_EBUSY = 0, -1, -2, -3, -4, -5, -6
FP_INSIDE, FP_BORDER, FP_NOT_FOUND = 0, 1, 2
FP_PREC_FP64, FP_PREC_MIXED = 0, 1

# Every symbol the C ABI exports (checked against include/findpts.h by tests).
SYMBOLS = ("findpts_setup", "findpts_update", "findpts", "findpts_eval", "findpts_eval_noalloc",
           "findpts_set_precision",
           "findpts_stats", "findpts_timing", "findpts_timing_read",
           "findpts_get_bbox", "findpts_get_hash", "findpts_get_cells",
           "findpts_footprint", "findpts_free", "fp_last_error", "fp_copy",
           "fp_flux_correct", "fp_extrapolate",
           "fps_create", "fps_add_mesh", "fps_submit", "fps_wait", "fps_latency",
           "fps_destroy",
           "findpts2_setup", "findpts2", "findpts2_eval", "findpts2_stats",
           "findpts2_get_bbox", "findpts2_free")

FP_FLUX_WORK = 1024


class FindptsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libfindpts.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1811_04891_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp, llp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_longlong)
    L.findpts_setup.argtypes = [C.POINTER(vp), vp, vp, vp, C.c_int, C.c_int, C.c_double,
                                vp, vp, C.c_int, C.c_int, vp]
    L.findpts_update.argtypes = [vp, vp, vp, vp, vp, vp]
    L.findpts.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
    L.findpts_eval.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int, C.POINTER(vp), vp, vp]
    L.findpts_eval_noalloc.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int, C.POINTER(vp), vp, vp]
    L.findpts_set_precision.argtypes = [vp, C.c_int]
    L.findpts_stats.argtypes = [vp, llp, C.c_int]
    L.findpts_timing.argtypes = [vp, C.c_int]
    L.findpts_timing_read.argtypes = [vp, dp, llp]
    L.findpts_get_bbox.argtypes = [vp, dp, dp]
    L.findpts_get_hash.argtypes = [vp, ip, dp, dp, llp]
    L.findpts_get_cells.argtypes = [vp, ip, ip]
    L.findpts_footprint.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.findpts_free.argtypes = [vp]
    L.fp_last_error.restype = C.c_char_p
    L.fp_last_error.argtypes = []
    L.fp_copy.argtypes = [vp, vp, C.c_size_t, vp]
    L.fp_flux_correct.argtypes = [C.c_int, vp, vp, C.c_longlong, vp, vp, C.c_longlong, vp, vp]
    L.fp_extrapolate.argtypes = [C.c_longlong, C.c_int, C.POINTER(vp), vp, vp]
    L.fps_create.argtypes = [C.POINTER(vp), C.c_size_t, C.c_int]
    L.fps_add_mesh.argtypes = [vp, vp, C.POINTER(vp), C.c_int, ip]
    L.fps_submit.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_int, ip, vp, vp, vp, vp, vp, llp]
    L.fps_wait.argtypes = [vp, C.c_longlong, C.c_double]
    L.fps_latency.argtypes = [vp, dp, dp, dp, llp, C.c_int]
    L.fps_destroy.argtypes = [vp]
    L.findpts2_setup.argtypes = [C.POINTER(vp), vp, vp, C.c_int, C.c_int, C.c_double, vp, vp,
                                 C.c_int, vp]
    L.findpts2.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
    L.findpts2_eval.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int, C.POINTER(vp), vp, vp]
    L.findpts2_stats.argtypes = [vp, llp, C.c_int]
    L.findpts2_get_bbox.argtypes = [vp, dp, dp]
    L.findpts2_free.argtypes = [vp]
    for name in SYMBOLS:
        if name != "fp_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != FP_OK:
        raise FindptsError(rc, f"{what}: {lib().fp_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor], dtype, name: str, numel: Optional[int] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Handle:
    """Owns an fp_handle*; freed with findpts_free."""

    def __init__(self, ptr: C.c_void_p, E: int, N: int, device: torch.device):
        self.ptr, self.E, self.N, self.device = ptr, E, N, device
        self.n1 = N + 1
        self.V = self.n1 ** 3

    def free(self):
        if self.ptr is not None and self.ptr.value:
            _check(lib().findpts_free(self.ptr), "findpts_free")
        self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def findpts_setup(x: torch.Tensor, y: torch.Tensor, z: torch.Tensor, N: int,
                  tol: float = 1e-12, elem_session: Optional[torch.Tensor] = None,
                  delta: Optional[torch.Tensor] = None, max_points: int = 1 << 20,
                  precision: int = FP_PREC_FP64, stream=None) -> Handle:
    n1 = N + 1
    V = n1 ** 3
    if x.numel() % V:
        raise ValueError("coordinate arrays must hold E*(N+1)^3 values")
    E = x.numel() // V
    h = C.c_void_p()
    rc = lib().findpts_setup(C.byref(h), _ptr(x, torch.float64, "x", E * V),
                             _ptr(y, torch.float64, "y", E * V),
                             _ptr(z, torch.float64, "z", E * V), E, N, float(tol),
                             _ptr(elem_session, torch.int32, "elem_session", E),
                             _ptr(delta, torch.float64, "delta", E * V),
                             int(max_points), int(precision), _stream(stream))
    _check(rc, "findpts_setup")
    return Handle(h, E, N, x.device)


def findpts_update(h: Handle, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor,
                   delta: Optional[torch.Tensor] = None, stream=None):
    """New node coordinates of the same mesh (moving or deforming meshes)."""
    n = h.E * h.V
    _check(lib().findpts_update(h.ptr, _ptr(x, torch.float64, "x", n),
                                _ptr(y, torch.float64, "y", n), _ptr(z, torch.float64, "z", n),
                                _ptr(delta, torch.float64, "delta", n), _stream(stream)),
           "findpts_update")


def findpts(h: Handle, pts: torch.Tensor, pt_session: Optional[torch.Tensor] = None,
            code=None, el=None, rst=None, dist2=None, stream=None):
    """Locate pts (npts x 3, float64).  Returns (code, el, rst, dist2)."""
    n = pts.numel() // 3
    dev = pts.device
    code = torch.empty(n, dtype=torch.int32, device=dev) if code is None else code
    el = torch.empty(n, dtype=torch.int32, device=dev) if el is None else el
    rst = torch.empty((n, 3), dtype=torch.float64, device=dev) if rst is None else rst
    dist2 = torch.empty(n, dtype=torch.float64, device=dev) if dist2 is None else dist2
    rc = lib().findpts(h.ptr, n, _ptr(pts, torch.float64, "pts", 3 * n),
                       _ptr(pt_session, torch.int32, "pt_session", n),
                       _ptr(code, torch.int32, "code", n), _ptr(el, torch.int32, "el", n),
                       _ptr(rst, torch.float64, "rst", 3 * n),
                       _ptr(dist2, torch.float64, "dist2", n), _stream(stream))
    _check(rc, "findpts")
    return code, el, rst, dist2


def findpts_eval(h: Handle, code: torch.Tensor, el: torch.Tensor, rst: torch.Tensor,
                 fields: Sequence[torch.Tensor], out: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    """Interpolate fields (each E*(N+1)^3 float64) at located points.
    Returns out (nfields x npts)."""
    n = code.numel()
    nf = len(fields)
    if out is None:
        out = torch.empty((nf, n), dtype=torch.float64, device=code.device)
    arr = (C.c_void_p * max(nf, 1))(*[_ptr(f, torch.float64, f"fields[{i}]", h.E * h.V)
                                       for i, f in enumerate(fields)])
    rc = lib().findpts_eval(h.ptr, n, _ptr(code, torch.int32, "code", n),
                            _ptr(el, torch.int32, "el", n),
                            _ptr(rst, torch.float64, "rst", 3 * n), nf, arr,
                            _ptr(out, torch.float64, "out", nf * n), _stream(stream))
    _check(rc, "findpts_eval")
    return out


def findpts_eval_noalloc(h: Handle, code: torch.Tensor, el: torch.Tensor, rst: torch.Tensor,
                         fields: Sequence[torch.Tensor], out: torch.Tensor,
                         stream=None) -> torch.Tensor:
    """findpts_eval through the entry point that allocates nothing: the
    caller passes out (nfields x npts float64); the grouping arrays live in
    the library's per-GPU scratch array (calls on one GPU must not overlap)."""
    n = code.numel()
    nf = len(fields)
    arr = (C.c_void_p * max(nf, 1))(*[_ptr(f, torch.float64, f"fields[{i}]", h.E * h.V)
                                       for i, f in enumerate(fields)])
    rc = lib().findpts_eval_noalloc(h.ptr, n, _ptr(code, torch.int32, "code", n),
                                    _ptr(el, torch.int32, "el", n),
                                    _ptr(rst, torch.float64, "rst", 3 * n), nf, arr,
                                    _ptr(out, torch.float64, "out", nf * n), _stream(stream))
    _check(rc, "findpts_eval_noalloc")
    return out


def findpts_set_precision(h: Handle, precision: int):
    _check(lib().findpts_set_precision(h.ptr, int(precision)), "findpts_set_precision")


def findpts_stats(h: Handle, reset: bool = False, first_pass: bool = False):
    """(pairs solved, Newton iterations, points located, method candidates)
    since setup/reset; with first_pass, also (pairs, iterations) of the
    first-pass Newton launches."""
    v = (C.c_longlong * 6)()
    _check(lib().findpts_stats(h.ptr, v, int(bool(reset))), "findpts_stats")
    return tuple(v) if first_pass else tuple(v)[:4]


def findpts_timing(h: Handle, enable: bool = True):
    _check(lib().findpts_timing(h.ptr, int(bool(enable))), "findpts_timing")


def findpts_timing_read(h: Handle):
    """{phase: (total ms, launches)} for the first-pass locate kernel, eval
    kernel, findpts, findpts_eval and the second-pass locate kernel."""
    ms, n = (C.c_double * 5)(), (C.c_longlong * 5)()
    _check(lib().findpts_timing_read(h.ptr, ms, n), "findpts_timing_read")
    names = ("locate_kernel", "eval_kernel", "findpts", "findpts_eval", "locate_kernel_2")
    return {names[i]: (ms[i], n[i]) for i in range(5)}


def findpts_get_bbox(h: Handle):
    import numpy as np
    b, s = np.zeros(6 * h.E), np.zeros(h.E)
    _check(lib().findpts_get_bbox(h.ptr, b.ctypes.data_as(C.POINTER(C.c_double)),
                                  s.ctypes.data_as(C.POINTER(C.c_double))), "findpts_get_bbox")
    return b.reshape(h.E, 6), s


def findpts_get_hash(h: Handle):
    import numpy as np
    nc, lo, dx, meta = (C.c_int * 3)(), np.zeros(3), np.zeros(3), (C.c_longlong * 3)()
    _check(lib().findpts_get_hash(h.ptr, nc, lo.ctypes.data_as(C.POINTER(C.c_double)),
                                  dx.ctypes.data_as(C.POINTER(C.c_double)), meta),
           "findpts_get_hash")
    return list(nc), lo, dx, tuple(meta)


def findpts_get_cells(h: Handle):
    import numpy as np
    _, _, _, (ncell, nnz, _) = findpts_get_hash(h)
    off, cel = np.zeros(ncell + 1, np.int32), np.zeros(max(nnz, 1), np.int32)
    _check(lib().findpts_get_cells(h.ptr, off.ctypes.data_as(C.POINTER(C.c_int)),
                                   cel.ctypes.data_as(C.POINTER(C.c_int))), "findpts_get_cells")
    return off, cel[:nnz]


def findpts_footprint(h: Handle) -> int:
    v = C.c_size_t()
    _check(lib().findpts_footprint(h.ptr, C.byref(v)), "findpts_footprint")
    return v.value


def fp_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    _check(lib().fp_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                         nbytes, _stream(stream)), "fp_copy")


def fp_flux_correct(w: torch.Tensor, n: torch.Tensor, u: torch.Tensor,
                    iface: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    """Mass-flux correction of u (3, P) in place; returns the work buffer
    (work[0] = gamma).  n and u may be (3, P) views with a row stride (e.g.
    a column slice of findpts_eval's output)."""
    P = w.numel()
    if work is None:
        work = torch.empty(FP_FLUX_WORK, dtype=torch.float64, device=w.device)
    for name, t in (("n", n), ("u", u)):
        if (t.dim() != 2 or t.shape[0] < 3 or t.shape[1] != P or t.stride(1) != 1
                or t.dtype != torch.float64 or t.device.type != "cuda"):
            raise ValueError(f"{name} must be a (3, {P}) float64 CUDA tensor with unit column stride")
    _check(lib().fp_flux_correct(int(P), _ptr(w, torch.float64, "w", P),
                                 C.c_void_p(n.data_ptr()), C.c_longlong(n.stride(0)),
                                 _ptr(iface, torch.int32, "iface", P),
                                 C.c_void_p(u.data_ptr()), C.c_longlong(u.stride(0)),
                                 _ptr(work, torch.float64, "work", FP_FLUX_WORK),
                                 _stream(stream)), "fp_flux_correct")
    return work


def fp_extrapolate(hist: Sequence[torch.Tensor], order: int, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """m-th order time extrapolation; hist most recent first."""
    n = hist[0].numel()
    if out is None:
        out = torch.empty_like(hist[0])
    arr = (C.c_void_p * max(1, len(hist)))(
        *[_ptr(t, torch.float64, f"hist[{i}]", n).value for i, t in enumerate(hist)])
    _check(lib().fp_extrapolate(C.c_longlong(n), int(order), arr,
                                _ptr(out, torch.float64, "out", n), _stream(stream)),
           "fp_extrapolate")
    return out


class Request:
    """Outputs of one served request (valid once Server.wait returned)."""

    def __init__(self, ticket: int, code, el, rst, dist2, out, keep):
        self.ticket, self.code, self.el, self.rst, self.dist2, self.out = (
            ticket, code, el, rst, dist2, out)
        self._keep = keep  # inputs stay alive until the request completed


class Server:
    """The serving layer (fps_*): resident meshes, HBM-budgeted admission,
    `slots` concurrent HIP streams, p50/p99 latency.  Keeps the registered
    handles and fields alive for its own lifetime."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4):
        p = C.c_void_p()
        _check(lib().fps_create(C.byref(p), int(hbm_budget_bytes), int(slots)), "fps_create")
        self.ptr = p
        self._meshes = []

    def add_mesh(self, h: Handle, fields: Sequence[torch.Tensor] = ()) -> int:
        for i, f in enumerate(fields):
            _ptr(f, torch.float64, f"fields[{i}]", h.E * h.V)
        arr = (C.c_void_p * max(1, len(fields)))(*[f.data_ptr() for f in fields])
        mid = C.c_int()
        _check(lib().fps_add_mesh(self.ptr, h.ptr, arr, len(fields), C.byref(mid)),
               "fps_add_mesh")
        self._meshes.append((h, list(fields)))
        return mid.value

    def submit(self, mesh_id: int, pts: torch.Tensor, field_ids: Sequence[int] = (),
               pt_session: Optional[torch.Tensor] = None, out=None) -> Request:
        """Queue a request; `pts` must be ready (its stream synchronised)."""
        P = pts.shape[0] if pts.dim() == 2 else pts.numel() // 3
        dev = pts.device
        nf = len(field_ids)
        if out is None:
            code = torch.empty(P, dtype=torch.int32, device=dev)
            el = torch.empty(P, dtype=torch.int32, device=dev)
            rst = torch.empty((P, 3), dtype=torch.float64, device=dev)
            d2 = torch.empty(P, dtype=torch.float64, device=dev)
            vals = torch.empty((nf, P), dtype=torch.float64, device=dev) if nf else None
        else:
            code, el, rst, d2, vals = out
        ids = (C.c_int * max(1, nf))(*[int(i) for i in field_ids])
        t = C.c_longlong()
        _check(lib().fps_submit(self.ptr, int(mesh_id), int(P),
                                _ptr(pts, torch.float64, "pts", 3 * P),
                                _ptr(pt_session, torch.int32, "pt_session", P), nf, ids,
                                _ptr(code, torch.int32, "code", P), _ptr(el, torch.int32, "el", P),
                                _ptr(rst, torch.float64, "rst", 3 * P),
                                _ptr(d2, torch.float64, "dist2", P),
                                _ptr(vals, torch.float64, "out", nf * P) if nf else None,
                                C.byref(t)), "fps_submit")
        return Request(t.value, code, el, rst, d2, vals, (pts, pt_session))

    def wait(self, req, timeout_s: float = -1.0) -> int:
        """FP_OK when done, FP_EBUSY on timeout; raises on a failed request."""
        ticket = req.ticket if isinstance(req, Request) else int(req)
        rc = lib().fps_wait(self.ptr, C.c_longlong(ticket), float(timeout_s))
        if rc == FP_EBUSY:
            return rc
        _check(rc, "fps_wait")
        return rc

    def latency(self, reset: bool = False) -> dict:
        p50, p99, rate = C.c_double(), C.c_double(), C.c_double()
        info = (C.c_longlong * 6)()
        _check(lib().fps_latency(self.ptr, C.byref(p50), C.byref(p99), C.byref(rate), info,
                                 int(reset)), "fps_latency")
        return {"p50_s": p50.value, "p99_s": p99.value, "points_per_s": rate.value,
                "completed": info[0], "waiting": info[1], "running": info[2],
                "peak_concurrent": info[3], "peak_arena_bytes": info[4],
                "waited_admissions": info[5]}

    def destroy(self):
        if self.ptr is not None and self.ptr.value:
            _check(lib().fps_destroy(self.ptr), "fps_destroy")
        self.ptr = None
        self._meshes = []

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Two dimensions (quadrilateral elements): findpts2_*.
# ---------------------------------------------------------------------------
class Handle2:
    """Owns an fp2_handle*; freed with findpts2_free."""

    def __init__(self, ptr: C.c_void_p, E: int, N: int, device: torch.device):
        self.ptr, self.E, self.N, self.device = ptr, E, N, device
        self.n1 = N + 1
        self.V = self.n1 ** 2

    def free(self):
        if self.ptr is not None and self.ptr.value:
            _check(lib().findpts2_free(self.ptr), "findpts2_free")
        self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def findpts2_setup(x: torch.Tensor, y: torch.Tensor, N: int, tol: float = 1e-12,
                   elem_session: Optional[torch.Tensor] = None,
                   delta: Optional[torch.Tensor] = None, max_points: int = 1 << 20,
                   stream=None) -> Handle2:
    V = (N + 1) ** 2
    if x.numel() % V:
        raise ValueError("coordinate arrays must hold E*(N+1)^2 values")
    E = x.numel() // V
    h = C.c_void_p()
    rc = lib().findpts2_setup(C.byref(h), _ptr(x, torch.float64, "x", E * V),
                              _ptr(y, torch.float64, "y", E * V), E, N, float(tol),
                              _ptr(elem_session, torch.int32, "elem_session", E),
                              _ptr(delta, torch.float64, "delta", E * V), int(max_points),
                              _stream(stream))
    _check(rc, "findpts2_setup")
    return Handle2(h, E, N, x.device)


def findpts2(h: Handle2, pts: torch.Tensor, pt_session: Optional[torch.Tensor] = None,
             code=None, el=None, rs=None, dist2=None, stream=None):
    """Locate pts (npts x 2, float64).  Returns (code, el, rs, dist2)."""
    n = pts.numel() // 2
    dev = pts.device
    code = torch.empty(n, dtype=torch.int32, device=dev) if code is None else code
    el = torch.empty(n, dtype=torch.int32, device=dev) if el is None else el
    rs = torch.empty((n, 2), dtype=torch.float64, device=dev) if rs is None else rs
    dist2 = torch.empty(n, dtype=torch.float64, device=dev) if dist2 is None else dist2
    rc = lib().findpts2(h.ptr, n, _ptr(pts, torch.float64, "pts", 2 * n),
                        _ptr(pt_session, torch.int32, "pt_session", n),
                        _ptr(code, torch.int32, "code", n), _ptr(el, torch.int32, "el", n),
                        _ptr(rs, torch.float64, "rs", 2 * n),
                        _ptr(dist2, torch.float64, "dist2", n), _stream(stream))
    _check(rc, "findpts2")
    return code, el, rs, dist2


def findpts2_eval(h: Handle2, code: torch.Tensor, el: torch.Tensor, rs: torch.Tensor,
                  fields: Sequence[torch.Tensor], out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Interpolate fields (each E*(N+1)^2 float64) at located points.
    Returns out (nfields x npts)."""
    n = code.numel()
    nf = len(fields)
    if out is None:
        out = torch.empty((nf, n), dtype=torch.float64, device=code.device)
    arr = (C.c_void_p * max(nf, 1))(*[_ptr(f, torch.float64, f"fields[{i}]", h.E * h.V)
                                       for i, f in enumerate(fields)])
    rc = lib().findpts2_eval(h.ptr, n, _ptr(code, torch.int32, "code", n),
                             _ptr(el, torch.int32, "el", n),
                             _ptr(rs, torch.float64, "rs", 2 * n), nf, arr,
                             _ptr(out, torch.float64, "out", nf * n), _stream(stream))
    _check(rc, "findpts2_eval")
    return out


def findpts2_stats(h: Handle2, reset: bool = False):
    """(pairs solved, Newton iterations, method candidates) since setup/reset."""
    v = (C.c_longlong * 3)()
    _check(lib().findpts2_stats(h.ptr, v, int(bool(reset))), "findpts2_stats")
    return tuple(v)


def findpts2_get_bbox(h: Handle2):
    import numpy as np
    b, s = np.zeros(4 * h.E), np.zeros(h.E)
    _check(lib().findpts2_get_bbox(h.ptr, b.ctypes.data_as(C.POINTER(C.c_double)),
                                   s.ctypes.data_as(C.POINTER(C.c_double))), "findpts2_get_bbox")
    return b.reshape(h.E, 4), s
