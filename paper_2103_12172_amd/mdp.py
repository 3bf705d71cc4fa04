"""Thin Python binding of libmdp (include/mdp.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
arguments to the C-ABI's plain pointers and sizes.  Device buffers are torch
tensors on the GPU (their data_ptr() is passed through), streams are torch
streams.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdp.so")

MDP_OK, MDP_ERR_ARG, MDP_ERR_HIP, MDP_ERR_OOM, MDP_ERR_SINGULAR, MDP_ERR_NONFINITE, MDP_ERR_NODEVICE = 0, -1, -2, -3, -4, -5, -6
MDP_C128, MDP_C64, MDP_C64_REFINED = 0, 1, 2
PRECISIONS = {"c128": MDP_C128, "c64": MDP_C64, "c64r": MDP_C64_REFINED}

STATUS_NAMES = {0: "MDP_OK", -1: "MDP_ERR_ARG", -2: "MDP_ERR_HIP", -3: "MDP_ERR_OOM", -4: "MDP_ERR_SINGULAR",
                -5: "MDP_ERR_NONFINITE", -6: "MDP_ERR_NODEVICE"}

EXPORTED = ["mdp_create", "mdp_destroy", "mdp_last_error", "mdp_build_projector", "mdp_build_projectors",
            "mdp_projector_info",
            "mdp_projector_release", "mdp_solve_interface", "mdp_reconstruct", "mdp_ap_solve", "mdp_cheb_points",
            "mdp_cheb_coeffs", "mdp_version", "mdp_cache_clear", "mdp_profile_enable", "mdp_profile_report",
            "mdp_set_projector_path", "mdp_set_interface_path", "mdp_profile_select", "mdp_projector_gamma_feet", "mdp_ap_grid",
            "mdp_dd_gradient", "mdp_set_autotune", "mdp_set_fused_schedule", "mdp_fused_schedule_used",
            "mdp_ap_solve_noalloc"]
MDP_PATH_AUTO, MDP_PATH_DENSE = 0, 1
PROJECTOR_PATHS = {"auto": MDP_PATH_AUTO, "dense": MDP_PATH_DENSE}
INTERFACE_PATHS = {"auto": 0, "dense": 1, "multifrontal": 2}


class MdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class C128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Subdomain(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("k", ctypes.c_double), ("n", ctypes.c_int)]


class Source(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("jet", ctypes.c_void_p)]


class Side(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("d", ctypes.POINTER(C128)), ("nbr", ctypes.c_int), ("nbr_side", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmdp.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmdp.so not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.mdp_create.argtypes = [ctypes.POINTER(vp), ip]
    lib.mdp_create.restype = ip
    lib.mdp_destroy.argtypes = [vp]
    lib.mdp_destroy.restype = None
    lib.mdp_last_error.argtypes = [vp]
    lib.mdp_last_error.restype = ctypes.c_char_p
    lib.mdp_build_projector.argtypes = [vp, ctypes.POINTER(Subdomain), ip, ip, vp, ctypes.POINTER(vp)]
    lib.mdp_build_projector.restype = ip
    lib.mdp_build_projectors.argtypes = [vp, ip, ctypes.POINTER(Subdomain), ip, ip, vp, ctypes.POINTER(vp)]
    lib.mdp_build_projectors.restype = ip
    lib.mdp_projector_info.argtypes = [vp, ctypes.POINTER(ip), ctypes.POINTER(ctypes.POINTER(ip)), ctypes.POINTER(vp)]
    lib.mdp_projector_info.restype = ip
    lib.mdp_projector_release.argtypes = [vp]
    lib.mdp_projector_release.restype = None
    lib.mdp_solve_interface.argtypes = [vp, ip, ctypes.POINTER(Subdomain), ctypes.POINTER(vp), ctypes.POINTER(Side),
                                        ip, ctypes.POINTER(Source), vp, vp, ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.mdp_solve_interface.restype = ip
    lib.mdp_dd_gradient.argtypes = [vp, ip, ctypes.POINTER(Subdomain), ctypes.POINTER(vp), ctypes.POINTER(Side), ip,
                                    ip, ctypes.POINTER(ip), ctypes.POINTER(ip), vp, vp, ctypes.POINTER(dp), vp]
    lib.mdp_dd_gradient.restype = ip
    lib.mdp_reconstruct.argtypes = [vp, ip, ctypes.POINTER(vp), vp, ctypes.POINTER(Source), vp, vp]
    lib.mdp_projector_gamma_feet.argtypes = [vp, ctypes.POINTER(Subdomain), ctypes.POINTER(dp), ctypes.POINTER(ip)]
    lib.mdp_projector_gamma_feet.restype = ip
    lib.mdp_ap_grid.argtypes = [ctypes.POINTER(Subdomain), ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.mdp_ap_grid.restype = ip
    lib.mdp_reconstruct.restype = ip
    lib.mdp_ap_solve.argtypes = [vp, ip, dp, dp, ip, ip, vp, vp, vp]
    lib.mdp_ap_solve.restype = ip
    lib.mdp_ap_solve_noalloc.argtypes = [vp, ip, dp, dp, ip, ip, vp, vp, vp]
    lib.mdp_ap_solve_noalloc.restype = ip
    lib.mdp_cheb_points.argtypes = [ip, ctypes.POINTER(dp)]
    lib.mdp_cheb_points.restype = ip
    lib.mdp_cheb_coeffs.argtypes = [ip, ctypes.POINTER(C128), ctypes.POINTER(C128)]
    lib.mdp_cheb_coeffs.restype = ip
    lib.mdp_profile_select.argtypes = [vp, ctypes.c_char_p]
    lib.mdp_profile_select.restype = ip
    lib.mdp_set_projector_path.argtypes = [vp, ip]
    lib.mdp_set_projector_path.restype = ip
    lib.mdp_set_interface_path.argtypes = [vp, ip]
    lib.mdp_set_interface_path.restype = ip
    lib.mdp_set_autotune.argtypes = [vp, ip]
    lib.mdp_set_autotune.restype = ip
    lib.mdp_set_fused_schedule.argtypes = [vp, ip]
    lib.mdp_set_fused_schedule.restype = ip
    lib.mdp_fused_schedule_used.argtypes = [vp]
    lib.mdp_fused_schedule_used.restype = ip
    lib.mdp_cache_clear.argtypes = [vp]
    lib.mdp_cache_clear.restype = ip
    lib.mdp_profile_enable.argtypes = [vp, ip]
    lib.mdp_profile_enable.restype = ip
    lib.mdp_profile_report.argtypes = [vp, ctypes.c_char_p, ip]
    lib.mdp_profile_report.restype = ip
    lib.mdp_version.argtypes = []
    lib.mdp_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """Owns an mdp_ctx on one device."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.mdp_create(ctypes.byref(h), device)
        if rc != MDP_OK:
            raise MdpError(rc, lib.mdp_last_error(None).decode())
        self.handle = h
        self.lib = lib
        self.device = device

    def check(self, rc: int):
        if rc != MDP_OK:
            raise MdpError(rc, self.lib.mdp_last_error(self.handle).decode())

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mdp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """__cuda_array_interface__ view of library-owned device memory."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 3, "strides": None}


class Projector:
    """A reference to a cached mdp_projector (released on close/garbage collection)."""

    def __init__(self, ctx: Context, handle: ctypes.c_void_p, m_star: int):
        self.ctx, self.handle, self.m_star = ctx, handle, m_star

    def info(self):
        ng = ctypes.c_int()
        gmq = ctypes.POINTER(ctypes.c_int)()
        q = ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.mdp_projector_info(self.handle, ctypes.byref(ng), ctypes.byref(gmq),
                                                       ctypes.byref(q)))
        n = ng.value
        mq = np.ctypeslib.as_array(gmq, shape=(2 * n,)).reshape(n, 2).copy()
        return n, mq, q.value

    def q_tensor(self):
        """Q as a torch complex128 tensor (n_gamma x 8M*), copied from the library's buffer."""
        import torch
        n, _, ptr = self.info()
        view = _DeviceArray(ptr, (8 * self.m_star, n), "<c16")
        t = torch.as_tensor(view, device="cuda:%d" % self.ctx.device)
        return t.T.clone()

    def release(self):
        if self.handle:
            self.ctx.lib.mdp_projector_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def mdp_create(device: int = 0) -> Context:
    return Context(device)


def mdp_build_projector(ctx: Context, sd: Subdomain, m_star: int, precision, stream=None) -> Projector:
    prec = PRECISIONS.get(precision, precision)
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.mdp_build_projector(ctx.handle, ctypes.byref(sd), m_star, prec,
                                          ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)))
    return Projector(ctx, h, m_star)


def mdp_build_projectors(ctx: Context, sds: Sequence[Subdomain], m_star: int, precision, stream=None):
    """Projectors of all subdomains in one call (batched launches over every new projector)."""
    prec = PRECISIONS.get(precision, precision)
    n = len(sds)
    arr = (Subdomain * n)(*sds)
    hs = (ctypes.c_void_p * n)()
    ctx.check(ctx.lib.mdp_build_projectors(ctx.handle, n, arr, m_star, prec, ctypes.c_void_p(_stream_ptr(stream)),
                                           hs))
    return [Projector(ctx, ctypes.c_void_p(hs[i]), m_star) for i in range(n)]


# numpy view of an mdp_side array (the same field offsets), for setting the d pointers in one step
_SIDE_DT = np.dtype({"names": ["kind", "alpha", "beta", "d", "nbr", "nbr_side"],
                     "formats": [np.int32, np.float64, np.float64, np.uintp, np.int32, np.int32],
                     "offsets": [Side.kind.offset, Side.alpha.offset, Side.beta.offset, Side.d.offset,
                                 Side.nbr.offset, Side.nbr_side.offset],
                     "itemsize": ctypes.sizeof(Side)})


def make_sides(sides: Sequence[Side], d_arrays: Sequence[Optional[np.ndarray]]):
    """Side structs with their boundary coefficient arrays attached (kept alive by the returned holder).
    A ctypes array of Side (as dd.side_structs returns) is copied in one move; the boundary
    coefficients go into one contiguous buffer whose pieces the d pointers address."""
    if len(d_arrays) != len(sides):
        raise ValueError("one coefficient entry (array or None) per side")
    n = len(sides)
    arr = (Side * n)()
    if isinstance(sides, ctypes.Array) and sides._type_ is Side:
        ctypes.memmove(arr, sides, ctypes.sizeof(arr))
    else:
        for i, s in enumerate(sides):
            arr[i] = s
    rec = np.frombuffer(arr, dtype=_SIDE_DT)
    rec["d"] = 0
    idx = [i for i, d in enumerate(d_arrays) if d is not None]
    if not idx:
        return arr, []
    bufs = [np.ascontiguousarray(d_arrays[i], dtype=np.complex128).reshape(-1) for i in idx]   # C128 pairs
    flat = np.concatenate(bufs)
    offs = np.zeros(len(bufs), dtype=np.uint64)
    np.cumsum([b.size for b in bufs[:-1]], out=offs[1:])
    rec["d"][idx] = np.uint64(flat.ctypes.data) + np.uint64(16) * offs
    return arr, [flat]


def make_sources(sources):
    """mdp_source array from per-subdomain (f, jet) device tensors or None (None overall: no source)."""
    if sources is None:
        return None
    arr = (Source * len(sources))()
    for i, src in enumerate(sources):
        if src is None:
            arr[i].f, arr[i].jet = None, None
        else:
            f, jet = src
            arr[i].f, arr[i].jet = f.data_ptr(), jet.data_ptr()
    return arr


def mdp_solve_interface(ctx: Context, subs: Sequence[Subdomain], projectors: Sequence[Projector], sides,
                        d_arrays, m_star: int, c_out, stream=None, want_cond: bool = True, sources=None):
    """sources: None or, per subdomain, None or (f, jet) complex128 device tensors (see mdp_source)."""
    n = len(subs)
    sub_arr = (Subdomain * n)(*subs)
    parr = (ctypes.c_void_p * n)(*[p.handle.value for p in projectors])
    side_arr, keep = make_sides(sides, d_arrays)
    src_arr = make_sources(sources)
    rel = ctypes.c_double()
    cond = ctypes.c_double()
    ctx.check(ctx.lib.mdp_solve_interface(ctx.handle, n, sub_arr, parr, side_arr, m_star, src_arr,
                                          ctypes.c_void_p(_stream_ptr(stream)), ctypes.c_void_p(c_out.data_ptr()),
                                          ctypes.byref(rel), ctypes.byref(cond) if want_cond else None))
    del keep
    return rel.value, (cond.value if want_cond else None)


def mdp_dd_gradient(ctx: Context, subs: Sequence[Subdomain], projectors: Sequence[Projector], sides, d_arrays,
                    m_star: int, rcv_sub, rcv_node, ubar, stream=None):
    """Gradient of Phi = Re sum_t conj(ubar_t) u(receiver t): (dPhi/dk^2 per subdomain,
    dPhi/dd as complex [n_sub, 4, M*] (zero on interface sides))."""
    n = len(subs)
    sub_arr = (Subdomain * n)(*subs)
    parr = (ctypes.c_void_p * n)(*[p.handle.value for p in projectors])
    side_arr, keep = make_sides(sides, d_arrays)
    rs = np.ascontiguousarray(rcv_sub, dtype=np.int32)
    rn = np.ascontiguousarray(rcv_node, dtype=np.int32)
    ub = np.ascontiguousarray(ubar, dtype=np.complex128)
    gk = np.zeros(n, dtype=np.float64)
    gd = np.zeros((n, 4, m_star), dtype=np.complex128)
    ip_ = ctypes.POINTER(ctypes.c_int)
    ctx.check(ctx.lib.mdp_dd_gradient(ctx.handle, n, sub_arr, parr, side_arr, m_star, int(rs.size),
                                      rs.ctypes.data_as(ip_), rn.ctypes.data_as(ip_), ctypes.c_void_p(ub.ctypes.data),
                                      ctypes.c_void_p(_stream_ptr(stream)),
                                      gk.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.c_void_p(gd.ctypes.data)))
    del keep
    return gk, gd


def mdp_reconstruct(ctx: Context, projectors: Sequence[Projector], c, u_out, stream=None, sources=None):
    n = len(projectors)
    parr = (ctypes.c_void_p * n)(*[p.handle.value for p in projectors])
    ctx.check(ctx.lib.mdp_reconstruct(ctx.handle, n, parr, ctypes.c_void_p(c.data_ptr()), make_sources(sources),
                                      ctypes.c_void_p(_stream_ptr(stream)), ctypes.c_void_p(u_out.data_ptr())))


def mdp_projector_gamma_feet(P: "Projector", sub: Subdomain):
    """(xy [n_gamma, 2], side [n_gamma]) foot points of gamma on the rectangle sub."""
    lib = load()
    ng = ctypes.c_int()
    P.ctx.check(lib.mdp_projector_info(P.handle, ctypes.byref(ng), None, None))
    xy = np.zeros((ng.value, 2))
    side = np.zeros(ng.value, dtype=np.int32)
    rc = lib.mdp_projector_gamma_feet(P.handle, ctypes.byref(sub), xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      side.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_projector_gamma_feet")
    return xy, side


def mdp_ap_grid(sub: Subdomain):
    """(xa, ya, h) of the auxiliary grid of the rectangle sub."""
    lib = load()
    xa, ya, h = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib.mdp_ap_grid(ctypes.byref(sub), ctypes.byref(xa), ctypes.byref(ya), ctypes.byref(h))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_ap_grid")
    return xa.value, ya.value, h.value


def mdp_ap_solve(ctx: Context, n: int, h: float, k: float, precision, g, u, stream=None):
    prec = PRECISIONS.get(precision, precision)
    batch = g.numel() // ((n + 1) * (n + 1))
    ctx.check(ctx.lib.mdp_ap_solve(ctx.handle, n, float(h), float(k), prec, batch, ctypes.c_void_p(g.data_ptr()),
                                   ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))))


def mdp_ap_solve_noalloc(ctx: Context, n: int, h: float, k: float, precision, g, u, stream=None):
    """mdp_ap_solve with the batch buffers in the library's static device scratch array (allocates
    nothing; the plan of (n, h, k) must exist: an earlier mdp_ap_solve with those values creates it)."""
    prec = PRECISIONS.get(precision, precision)
    batch = g.numel() // ((n + 1) * (n + 1))
    ctx.check(ctx.lib.mdp_ap_solve_noalloc(ctx.handle, n, float(h), float(k), prec, batch,
                                           ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(_stream_ptr(stream))))


def mdp_cheb_points(m_star: int) -> np.ndarray:
    lib = load()
    t = (ctypes.c_double * m_star)()
    rc = lib.mdp_cheb_points(m_star, t)
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_cheb_points")
    return np.array(t[:])


def mdp_cheb_coeffs(samples: np.ndarray) -> np.ndarray:
    lib = load()
    m = len(samples)
    s = (C128 * m)(*[C128(float(v.real), float(v.imag)) for v in samples])
    d = (C128 * m)()
    rc = lib.mdp_cheb_coeffs(m, s, d)
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_cheb_coeffs")
    return np.array([complex(v.re, v.im) for v in d])


def mdp_cache_clear(ctx: Context):
    ctx.check(ctx.lib.mdp_cache_clear(ctx.handle))


def mdp_set_projector_path(ctx: Context, path):
    """Route of later projector builds: "auto" (fused support-in / gamma-out
    sweep for complex128) or "dense" (full AP solves + gather)."""
    ctx.check(ctx.lib.mdp_set_projector_path(ctx.handle, PROJECTOR_PATHS.get(path, path)))


def mdp_set_interface_path(ctx: Context, path):
    """Route of later interface solves: "auto" (dense up to 4096 unknowns),
    "dense" (dense Gram Cholesky) or "multifrontal" (nested dissection over the
    subdomain layout)."""
    ctx.check(ctx.lib.mdp_set_interface_path(ctx.handle, INTERFACE_PATHS.get(path, path)))


def mdp_set_autotune(ctx: Context, enable: bool = True):
    """Pick the sine GEMM's tile shape per (precision, n, rows) and the fused sweep's columns per lane
    per (precision, widest n, batch size) by timing at first use (process-wide; results change only by
    rounding)."""
    ctx.check(ctx.lib.mdp_set_autotune(ctx.handle, 1 if enable else 0))


def mdp_set_fused_schedule(ctx: Context, cols_per_lane: int = 0):
    """Mode columns per lane of the fused projector sweep (1, 2, 4; 0 = chosen per batch)."""
    ctx.check(ctx.lib.mdp_set_fused_schedule(ctx.handle, int(cols_per_lane)))


def mdp_fused_schedule_used(ctx: Context) -> int:
    return int(ctx.lib.mdp_fused_schedule_used(ctx.handle))


def mdp_profile_enable(ctx: Context, enable: bool = True):
    ctx.check(ctx.lib.mdp_profile_enable(ctx.handle, 1 if enable else 0))


def mdp_profile_select(ctx: Context, classes=None):
    """Record only these kernel classes (list or comma-separated string; None = all)."""
    if classes is not None and not isinstance(classes, str):
        classes = ",".join(classes)
    ctx.check(ctx.lib.mdp_profile_select(ctx.handle, classes.encode() if classes else None))


def mdp_profile_report(ctx: Context) -> dict:
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    ctx.check(ctx.lib.mdp_profile_report(ctx.handle, buf, len(buf)))
    return json.loads(buf.value.decode())


def version() -> str:
    return load().mdp_version().decode()
