"""FP64 CPU oracle for visual-sphere perspective-map rasterization.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The arithmetic lives in
``vsr_oracle.c`` (plain C, double precision, one pixel x one triangle at a
time); this module compiles it with gcc and marshals numpy arrays.  It
imports nothing from the HIP library and the HIP library imports nothing
from here.

Per-pixel flags returned by :func:`render`:
  FLAG_EDGE    a triangle whose depth is within 1e-5 of the winner's (or
               that could be hit from behind) passes within 1e-6 rad of one
               of its edge planes: the id there may legitimately differ in
               FP32.
  FLAG_DEPTH   best and second-best covered depths differ by <= 2e-5 * r.
  FLAG_INVALID the pixel has no view direction (outside the projection).
  FLAG_DOMAIN  the pixel lies within 1e-6 of the projection's domain edge
               (k < 0, |sin(k*Omega/2)*R| within 1e-6 of 1): it may have a
               direction in one precision and none in another.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vsr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NO_HIT = 0xFFFFFFFF
FLAG_EDGE, FLAG_DEPTH, FLAG_INVALID, FLAG_DOMAIN = 1, 2, 4, 8

_lock = threading.Lock()
_lib = None


def build_sanitized(out: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) into ``out``; a process loads it in place of the
    normal build when ORACLE_LIB names it (and libasan is preloaded)."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", out, _SRC, "-lm", "-lpthread"])
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction).
    With ORACLE_LIB set, that library is used as it is."""
    if os.environ.get("ORACLE_LIB"):
        return os.environ["ORACLE_LIB"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _View(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("aov", ctypes.c_int32),
                ("k", ctypes.c_double), ("l", ctypes.c_double), ("s", ctypes.c_double),
                ("omega_deg", ctypes.c_double), ("rot", ctypes.c_double * 9),
                ("lens", ctypes.c_int32), ("lens_n", ctypes.c_int32), ("lp", ctypes.c_double * 8)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("ORACLE_LIB") or _LIB
            if path == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
                build(force=True)
            lib = ctypes.CDLL(path)
            dp = ctypes.POINTER(ctypes.c_double)
            lib.orc_limits.argtypes = [dp, dp, dp, dp]
            lib.orc_view_coord.argtypes = [ctypes.c_int32] * 5 + [dp, dp]
            lib.orc_direction.argtypes = [ctypes.c_double] * 6 + [dp]
            lib.orc_direction.restype = ctypes.c_int
            lib.orc_pixel_direction.argtypes = [ctypes.POINTER(_View), ctypes.c_int32, ctypes.c_int32, dp]
            lib.orc_pixel_direction.restype = ctypes.c_int
            lib.orc_map.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_void_p]
            lib.orc_inverse.argtypes = [dp] + [ctypes.c_double] * 4 + [dp, dp]
            lib.orc_triangle.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, dp]
            lib.orc_cap.argtypes = [dp, dp, dp, dp]
            lib.orc_render.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32]
            lib.orc_render.restype = ctypes.c_int
            lib.orc_lens_direction.argtypes = [ctypes.POINTER(_View), ctypes.c_double, ctypes.c_double, dp,
                                               ctypes.POINTER(ctypes.c_int32)]
            lib.orc_lens_direction.restype = ctypes.c_int
            lib.orc_wireframe.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
            lib.orc_wireframe.restype = ctypes.c_int
            lib.orc_particles.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, dp, dp, dp, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32]
            lib.orc_particles.restype = ctypes.c_int
            lib.orc_delta.argtypes = [ctypes.POINTER(_View), ctypes.c_int32, ctypes.c_int32]
            lib.orc_delta.restype = ctypes.c_double
            lib.orc_aa_render.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, dp, dp, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32]
            lib.orc_aa_render.restype = ctypes.c_int
            lib.orc_fragments.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, dp, dp]
            lib.orc_pair.argtypes = [ctypes.POINTER(_View), ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, dp]
            _lib = lib
    return _lib


def _cview(view) -> _View:
    v = _View()
    v.width, v.height, v.aov = int(view.width), int(view.height), int(view.aov)
    v.k, v.l, v.s, v.omega_deg = float(view.k), float(view.l), float(view.s), float(view.omega_deg)
    for i, r in enumerate(view.rot):
        v.rot[i] = float(r)
    v.lens = int(getattr(view, "lens", 0))
    v.lens_n = int(getattr(view, "lens_n", 1))
    for i, x in enumerate(tuple(getattr(view, "lens_p", ()))[:8]):
        v.lp[i] = float(x)
    return v


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def limits(k: float, l: float, s: float, omega_deg: float):
    """Section 2.1.1 parameter limits: returns (k, l, s, omega_deg) clamped."""
    lib = _load()
    a = [ctypes.c_double(float(x)) for x in (k, l, s, omega_deg)]
    lib.orc_limits(*[ctypes.byref(x) for x in a])
    return tuple(x.value for x in a)


def view_coord(i: int, j: int, width: int, height: int, aov: int = 0):
    lib = _load()
    x, y = ctypes.c_double(), ctypes.c_double()
    lib.orc_view_coord(i, j, width, height, aov, ctypes.byref(x), ctypes.byref(y))
    return x.value, y.value


def direction(x: float, y: float, k: float, l: float, s: float, omega_deg: float):
    """Section 2.1.2 for already-limited parameters: (unit vector, valid)."""
    lib = _load()
    out = np.zeros(3)
    ok = lib.orc_direction(x, y, k, l, s, omega_deg, _dp(out))
    return out, bool(ok)


def inverse(v: Sequence[float], k: float, l: float, s: float, omega_deg: float):
    """Section 2.1.3 for already-limited parameters: camera vector -> (x, y)."""
    lib = _load()
    vv = np.ascontiguousarray(v, dtype=np.float64)
    x, y = ctypes.c_double(), ctypes.c_double()
    lib.orc_inverse(_dp(vv), k, l, s, omega_deg, ctypes.byref(x), ctypes.byref(y))
    return x.value, y.value


def perspective_map(view):
    """World-space map: (float64[H, W, 3], bool[H, W] valid)."""
    lib = _load()
    d = np.zeros((view.height, view.width, 3), dtype=np.float64)
    ok = np.zeros((view.height, view.width), dtype=np.uint8)
    cv = _cview(view)
    lib.orc_map(ctypes.byref(cv), d.ctypes.data, ok.ctypes.data)
    return d, ok.astype(bool)


def triangle(tris: np.ndarray, t: int) -> dict:
    """Per-triangle quantities of sections 1.1 and 1.1.4 for triangle t."""
    lib = _load()
    tris = np.ascontiguousarray(tris, dtype=np.float32)
    out = np.zeros(14)
    lib.orc_triangle(tris.ctypes.data, tris.shape[1], t, _dp(out))
    return {"n": out[0:9].reshape(3, 3), "N": out[9:12], "d": out[12], "live": bool(out[13])}


def cap(a, b, c):
    """Section 1.1.2 smallest circle: (S_hat[3], |S|)."""
    lib = _load()
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c)]
    out = np.zeros(4)
    lib.orc_cap(_dp(arr[0]), _dp(arr[1]), _dp(arr[2]), _dp(out))
    return out[:3].copy(), float(out[3])


@dataclass
class RenderResult:
    id: np.ndarray       # uint32, NO_HIT where nothing is covered
    depth: np.ndarray    # float64, +inf where nothing is covered
    depth2: np.ndarray   # float64 second-nearest covered depth
    cover: np.ndarray    # uint32 number of covering triangles
    flags: np.ndarray    # uint8 FLAG_* bits


def render(view, tris: np.ndarray, pixels: Optional[np.ndarray] = None,
           threads: Optional[int] = None) -> RenderResult:
    """Brute-force FP64 render of the listed flat pixel indices (j*W+i), or
    of the whole frame (arrays shaped [H, W]) when ``pixels`` is None."""
    lib = _load()
    tris = np.ascontiguousarray(tris, dtype=np.float32)
    assert tris.ndim == 2 and tris.shape[0] == 9
    ntri = tris.shape[1]
    if pixels is None:
        n = view.width * view.height
        pix_ptr = None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pixels.shape[0]
        pix_ptr = pixels.ctypes.data
    ids = np.empty(n, dtype=np.uint32)
    depth = np.empty(n, dtype=np.float64)
    depth2 = np.empty(n, dtype=np.float64)
    cover = np.empty(n, dtype=np.uint32)
    flags = np.empty(n, dtype=np.uint8)
    threads = threads or os.cpu_count() or 1
    cv = _cview(view)
    rc = lib.orc_render(ctypes.byref(cv), tris.ctypes.data, ntri, pix_ptr, n, ids.ctypes.data,
                        depth.ctypes.data, depth2.ctypes.data, cover.ctypes.data, flags.ctypes.data,
                        int(threads))
    if rc != 0:
        raise MemoryError("oracle render failed")
    res = RenderResult(ids, depth, depth2, cover, flags)
    if pixels is None:
        for f in ("id", "depth", "depth2", "cover", "flags"):
            setattr(res, f, getattr(res, f).reshape(view.height, view.width))
    return res


def pair(view, tris: np.ndarray, t: int, p: int):
    """(oriented edge values[3], r, pixel valid) of one pixel-triangle pair."""
    lib = _load()
    tris = np.ascontiguousarray(tris, dtype=np.float32)
    out = np.zeros(5)
    cv = _cview(view)
    lib.orc_pair(ctypes.byref(cv), tris.ctypes.data, tris.shape[1], int(t), int(p), _dp(out))
    return out[0:3].copy(), float(out[3]), bool(out[4])


def fragments(view, tris: np.ndarray, attr: np.ndarray, pixels: np.ndarray, ids: np.ndarray,
              normalize3: bool = False):
    """Section 1.1.4 fragment data of the listed pixels with winners ``ids``:
    (b [n, 3] barycentric weights of A, B, C; f [n, nattr] interpolated
    vertex data, attr shaped [3, nattr, T])."""
    lib = _load()
    tris = np.ascontiguousarray(tris, dtype=np.float32)
    attr = np.ascontiguousarray(attr, dtype=np.float32)
    assert attr.ndim == 3 and attr.shape[0] == 3 and attr.shape[2] == tris.shape[1]
    nattr = attr.shape[1]
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n = pixels.shape[0]
    b = np.zeros((n, 3))
    f = np.zeros((n, max(nattr, 1)))
    cv = _cview(view)
    lib.orc_fragments(ctypes.byref(cv), tris.ctypes.data, tris.shape[1], attr.ctypes.data, nattr,
                      int(bool(normalize3)), pixels.ctypes.data, ids.ctypes.data, n, _dp(b), _dp(f))
    return b, f[:, :nattr]


def lens_direction(view, fs: float, ft: float):
    """Camera-frame direction of texture coordinate (fs, ft) for the view's
    map generator (section 2.1 or 2.2): (unit vector, has direction,
    picture segment)."""
    lib = _load()
    cv = _cview(view)
    out = np.zeros(3)
    seg = ctypes.c_int32(0)
    ok = lib.orc_lens_direction(ctypes.byref(cv), float(fs), float(ft), _dp(out), ctypes.byref(seg))
    return out, bool(ok), int(seg.value)


def delta(view, i: int, j: int) -> float:
    """Section 1.1.1 global delta of pixel (i, j): 1 / max_c fwidth(G_c) of
    the camera-frame map (central differences, one-sided at borders)."""
    lib = _load()
    cv = _cview(view)
    return float(lib.orc_delta(ctypes.byref(cv), int(i), int(j)))


@dataclass
class AAResult:
    cov: np.ndarray      # float64 coverage in [0, 1]
    depth: np.ndarray    # float64 depth pass: sum of clipped mask x depth
    dom: np.ndarray      # uint32 id with the largest clipped mask, NO_HIT if none
    margin: np.ndarray   # largest clipped mask minus the second largest
    gap: np.ndarray      # smallest relative depth step between fragments taken
    n_near: np.ndarray   # fragments taken + the first left out
    sum_r: np.ndarray    # their summed depth
    sum_rg: np.ndarray   # their summed depth / cos(ray, plane normal)


def aa_render(view, tris: np.ndarray, pixels: Optional[np.ndarray] = None,
              threads: Optional[int] = None) -> AAResult:
    """Aliasing-free render (sections 1.1.1, 1.1.2, 1.4) of the listed flat
    pixel indices, or of the whole frame ([H, W] arrays) when ``pixels`` is
    None."""
    lib = _load()
    tris = np.ascontiguousarray(tris, dtype=np.float32)
    ntri = tris.shape[1]
    if pixels is None:
        n, pix_ptr = view.width * view.height, None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n, pix_ptr = pixels.shape[0], pixels.ctypes.data
    cov, depth = np.empty(n), np.empty(n)
    dom = np.empty(n, dtype=np.uint32)
    aux = np.empty((n, 5))
    cv = _cview(view)
    rc = lib.orc_aa_render(ctypes.byref(cv), tris.ctypes.data, ntri, pix_ptr, n, _dp(cov), _dp(depth),
                           dom.ctypes.data, aux.ctypes.data, int(threads or os.cpu_count() or 1))
    if rc != 0:
        raise MemoryError("oracle aa render failed")
    res = AAResult(cov, depth, dom, *(aux[:, c].copy() for c in range(5)))
    if pixels is None:
        for f in ("cov", "depth", "dom", "margin", "gap", "n_near", "sum_r", "sum_rg"):
            setattr(res, f, getattr(res, f).reshape(view.height, view.width))
    return res


@dataclass
class WireResult:
    cov: np.ndarray      # float64 largest line mask over the triangles' sides
    dom: np.ndarray      # uint32 triangle of that side (ties: lower id), NO_HIT if none
    second: np.ndarray   # largest mask of any other triangle


def wireframe(view, tris: np.ndarray, pixels: Optional[np.ndarray] = None,
              threads: Optional[int] = None) -> WireResult:
    """Aliasing-free wire frame of the triangles' sides (section 1.2)."""
    lib = _load()
    tris = np.ascontiguousarray(tris, dtype=np.float32)
    if pixels is None:
        n, pix_ptr = view.width * view.height, None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n, pix_ptr = pixels.shape[0], pixels.ctypes.data
    cov, second = np.empty(n), np.empty(n)
    dom = np.empty(n, dtype=np.uint32)
    cv = _cview(view)
    rc = lib.orc_wireframe(ctypes.byref(cv), tris.ctypes.data, tris.shape[1], pix_ptr, n, _dp(cov),
                           dom.ctypes.data, second.ctypes.data, int(threads or os.cpu_count() or 1))
    if rc != 0:
        raise MemoryError("oracle wireframe failed")
    res = WireResult(cov, dom, second)
    if pixels is None:
        for f in ("cov", "dom", "second"):
            setattr(res, f, getattr(res, f).reshape(view.height, view.width))
    return res


@dataclass
class ParticleResult:
    cov: np.ndarray
    depth: np.ndarray    # depth pass
    uv: np.ndarray       # texture-coordinate pass [..., 2]
    dom: np.ndarray
    margin: np.ndarray
    gap: np.ndarray
    n_near: np.ndarray
    sum_r: np.ndarray


def particles(view, pr: np.ndarray, pixels: Optional[np.ndarray] = None,
              threads: Optional[int] = None) -> ParticleResult:
    """Aliasing-free particles (section 1.3) combined front to back (1.4);
    pr = float32[4, n] (x, y, z, radius)."""
    lib = _load()
    pr = np.ascontiguousarray(pr, dtype=np.float32)
    if pixels is None:
        n, pix_ptr = view.width * view.height, None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n, pix_ptr = pixels.shape[0], pixels.ctypes.data
    cov, depth = np.empty(n), np.empty(n)
    uv = np.empty((n, 2))
    dom = np.empty(n, dtype=np.uint32)
    aux = np.empty((n, 4))
    cv = _cview(view)
    rc = lib.orc_particles(ctypes.byref(cv), pr.ctypes.data, pr.shape[1], pix_ptr, n, _dp(cov), _dp(depth),
                           _dp(uv), dom.ctypes.data, aux.ctypes.data, int(threads or os.cpu_count() or 1))
    if rc != 0:
        raise MemoryError("oracle particles failed")
    res = ParticleResult(cov, depth, uv, dom, *(aux[:, c].copy() for c in range(4)))
    if pixels is None:
        H, W = view.height, view.width
        for f in ("cov", "depth", "dom", "margin", "gap", "n_near", "sum_r"):
            setattr(res, f, getattr(res, f).reshape(H, W))
        res.uv = res.uv.reshape(H, W, 2)
    return res
