"""Python binding of libvsr (include/vsr.h): argument marshalling only.

Every function has the name and arguments of its C entry point; device
buffers are torch tensors on the GPU (their ``data_ptr()`` is passed) and
the stream defaults to torch's current stream.  Errors raise
:class:`VsrError` with the library's message.  There is no fallback: if
``libvsr.so`` has not been built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvsr.so")

VSR_OK, VSR_E_ARG, VSR_E_SPACE, VSR_E_RANGE, VSR_E_HIP = 0, -1, -2, -3, -4
VSR_MAP_F32, VSR_MAP_OCT16 = 0, 1
VSR_STRICT = 1
VSR_MAP_AA = 2
VSR_MAP_AA_LINES = 4
(VSR_LENS_UNIVERSAL, VSR_LENS_EQUIRECT, VSR_LENS_CUBE, VSR_LENS_SCREENS, VSR_LENS_VR, VSR_LENS_PANORAMA,
 VSR_LENS_DOME) = range(7)
VSR_BIN_ALL = 1
VSR_BIN_BLOCKS, VSR_BIN_SUPERTILES, VSR_BIN_TILE16 = 2, 4, 8
VSR_NO_HIT = 0xFFFFFFFF
VSR_SUBMIT_BINNED, VSR_SUBMIT_FUSED = 0, 1
VSR_SUBMIT_TABLE_READY = 0x100
VSR_SUBMIT_BIN_BLOCKS, VSR_SUBMIT_BIN_SUPERTILES, VSR_SUBMIT_BIN_TILE16 = 0x200, 0x400, 0x800
VSR_SUBMIT_PERSISTENT = 0x1000
VSR_TILE = 8
VSR_RESOLVE_NORMALIZE3 = 1
VSR_AOV_HORIZONTAL, VSR_AOV_DIAGONAL, VSR_AOV_VERTICAL, VSR_AOV_HORIZONTAL_4X3 = 0, 1, 2, 3

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libvsr.so not built at {LIB_PATH}: run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)


class VsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class vsr_view(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("aov", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("k", ctypes.c_float), ("l", ctypes.c_float),
                ("s", ctypes.c_float), ("omega_deg", ctypes.c_float), ("rot", ctypes.c_float * 9)]


class vsr_lens(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("n", ctypes.c_int32), ("p", ctypes.c_float * 8)]


class vsr_job(ctypes.Structure):
    _fields_ = [("view", vsr_view), ("setup", ctypes.c_void_p), ("ntri", ctypes.c_int64),
                ("tri_id", ctypes.c_void_p), ("depth", ctypes.c_void_p)]


_vp, _i32, _i64, _u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
_lib.vsr_map_bytes.argtypes = [_i32, _i32, _i32]
_lib.vsr_map_bytes.restype = _i64
_lib.vsr_setup_bytes.argtypes = [_i64]
_lib.vsr_setup_bytes.restype = _i64
_lib.vsr_bin_bytes.argtypes = [_i32, _i32, _i32]
_lib.vsr_bin_bytes.restype = _i64
_lib.vsr_build_map.argtypes = [ctypes.POINTER(vsr_view), _i32, _u32, _vp, _i64, ctypes.POINTER(vsr_view), _vp]
_lib.vsr_build_map_lens.argtypes = [ctypes.POINTER(vsr_view), ctypes.POINTER(vsr_lens), _i32, _u32, _vp, _i64,
                                    ctypes.POINTER(vsr_view), _vp]
_lib.vsr_map_unpack.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _vp]
_lib.vsr_setup_tris.argtypes = [_vp, _i64, _vp, _i64, _vp]
_lib.vsr_bin.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _i32, _u32, _vp, _i64, _vp]
_lib.vsr_raster.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp]
_lib.vsr_raster_stats.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _i32,
                                  _vp]
_lib.vsr_render_bytes.argtypes = [_i32, _i32]
_lib.vsr_render_bytes.restype = _i64
_lib.vsr_render.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp]
_lib.vsr_render_noalloc.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _vp, _vp]
_lib.vsr_resolve.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _vp, _i32, _u32, _vp, _vp, _vp]
_lib.vsr_aa_map_bytes.argtypes = [_i32, _i32, _i32]
_lib.vsr_aa_map_bytes.restype = _i64
_lib.vsr_aa_raster.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp, _vp]
_lib.vsr_aa_raster_stats.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp,
                                     _vp, _i32, _vp]
_lib.vsr_setup_particles.argtypes = [_vp, _i64, _vp, _i64, _vp]
_lib.vsr_aa_particles.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                  _vp]
_lib.vsr_aa_particles_stats.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _i32, _vp]
_lib.vsr_wire_bytes.argtypes = [_i64]
_lib.vsr_wire_bytes.restype = _i64
_lib.vsr_setup_wire.argtypes = [_vp, _vp, _i64, _vp, _i64, _vp]
_lib.vsr_aa_wireframe.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp]
_lib.vsr_aa_wireframe_stats.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp,
                                        _vp, _vp]
_lib.vsr_resolve_pack_bytes.argtypes = [_i64, _i32]
_lib.vsr_resolve_pack_bytes.restype = _i64
_lib.vsr_resolve_pack.argtypes = [_vp, _vp, _i64, _i32, _vp, _i64, _vp]
_lib.vsr_resolve_packed.argtypes = [ctypes.POINTER(vsr_view), _i32, _vp, _vp, _i64, _i32, _vp, _u32, _vp, _vp, _vp]
_lib.vsr_submit_bytes.argtypes = [ctypes.POINTER(vsr_job), _i32, _i32, _i32, _i32]
_lib.vsr_submit_bytes.restype = _i64
_lib.vsr_submit.argtypes = [ctypes.POINTER(vsr_job), _i32, _i32, _i32, _i32, _vp, _i64, _vp]
_lib.vsr_submit_timed.argtypes = [ctypes.POINTER(vsr_job), _i32, _i32, _i32, _i32, _vp, _i64,
                                  ctypes.POINTER(ctypes.c_void_p), _i32, _vp]
_lib.vsr_submit_table_bytes.argtypes = [_i32]
_lib.vsr_submit_table_bytes.restype = _i64
_lib.vsr_submit_table_offset.argtypes = []
_lib.vsr_submit_table_offset.restype = _i64
_lib.vsr_submit_table.argtypes = [ctypes.POINTER(vsr_job), _i32, _i32, _i32, _i32, _vp, _vp, _i64]
_lib.vsr_bin_overflow.argtypes = [_vp, _i32, ctypes.POINTER(_i64)]
_lib.vsr_calib_copy.argtypes = [_vp, _vp, _i64, _vp]
_lib.vsr_calib_fma.argtypes = [_vp, _i64, _i32, _vp]
_lib.vsr_strerror.argtypes = [ctypes.c_int]
_lib.vsr_strerror.restype = ctypes.c_char_p
_lib.vsr_last_error.restype = ctypes.c_char_p
for _f in ("vsr_build_map", "vsr_map_unpack", "vsr_setup_tris", "vsr_bin", "vsr_raster", "vsr_raster_stats", "vsr_render", "vsr_render_noalloc", "vsr_submit",
           "vsr_submit_timed", "vsr_submit_table", "vsr_bin_overflow", "vsr_calib_copy", "vsr_calib_fma"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTS = ("vsr_map_bytes", "vsr_setup_bytes", "vsr_bin_bytes", "vsr_build_map", "vsr_build_map_lens", "vsr_map_unpack", "vsr_setup_tris", "vsr_bin",
           "vsr_raster", "vsr_raster_stats", "vsr_render_bytes", "vsr_render", "vsr_render_noalloc", "vsr_resolve", "vsr_resolve_pack_bytes", "vsr_resolve_pack",
           "vsr_resolve_packed", "vsr_aa_map_bytes",
           "vsr_aa_raster", "vsr_aa_raster_stats", "vsr_setup_particles", "vsr_aa_particles",
           "vsr_aa_particles_stats", "vsr_wire_bytes", "vsr_setup_wire", "vsr_aa_wireframe", "vsr_aa_wireframe_stats", "vsr_submit_bytes",
           "vsr_submit_table_bytes", "vsr_submit_table_offset", "vsr_submit_table", "vsr_submit", "vsr_submit_timed", "vsr_bin_overflow", "vsr_calib_copy", "vsr_calib_fma",
           "vsr_strerror", "vsr_last_error")


def _check(rc: int) -> None:
    if rc != VSR_OK:
        raise VsrError(rc, _lib.vsr_last_error().decode() or _lib.vsr_strerror(rc).decode())


def _size(rc: int, what: str) -> int:
    if rc < 0:
        raise VsrError(int(rc), f"{what}: invalid arguments")
    return int(rc)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _nbytes(t) -> int:
    return 0 if t is None else int(t.numel() * t.element_size())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def make_view(view) -> vsr_view:
    """vsr_view from any object with width, height, aov, k, l, s, omega_deg, rot."""
    v = vsr_view()
    v.width, v.height, v.aov, v.reserved = int(view.width), int(view.height), int(view.aov), 0
    v.k, v.l, v.s, v.omega_deg = float(view.k), float(view.l), float(view.s), float(view.omega_deg)
    for q, r in enumerate(view.rot):
        v.rot[q] = float(r)
    return v


def vsr_map_bytes(width: int, height: int, fmt: int = VSR_MAP_F32) -> int:
    return _size(_lib.vsr_map_bytes(width, height, fmt), "vsr_map_bytes")


def vsr_setup_bytes(ntri: int) -> int:
    return _size(_lib.vsr_setup_bytes(ntri), "vsr_setup_bytes")


def vsr_bin_bytes(width: int, height: int, bin_depth: int) -> int:
    return _size(_lib.vsr_bin_bytes(width, height, bin_depth), "vsr_bin_bytes")


def vsr_build_map(view, fmt: int, flags: int, map_buf, stream=None) -> vsr_view:
    v = make_view(view)
    eff = vsr_view()
    _check(_lib.vsr_build_map(ctypes.byref(v), fmt, flags, _ptr(map_buf), _nbytes(map_buf), ctypes.byref(eff),
                              _stream(stream)))
    return eff


def make_lens(view) -> vsr_lens:
    """vsr_lens from a view's optional ``lens``, ``lens_n`` and ``lens_p``."""
    ln = vsr_lens()
    ln.type = int(getattr(view, "lens", VSR_LENS_UNIVERSAL))
    ln.n = int(getattr(view, "lens_n", 1))
    for q, x in enumerate(tuple(getattr(view, "lens_p", ()))[:8]):
        ln.p[q] = float(x)
    return ln


def has_lens(view) -> bool:
    """True when the view asks for another generator or lens distortion."""
    return int(getattr(view, "lens", VSR_LENS_UNIVERSAL)) != VSR_LENS_UNIVERSAL or any(
        float(x) != 0.0 for x in tuple(getattr(view, "lens_p", ())))


def vsr_build_map_lens(view, fmt: int, flags: int, map_buf, stream=None) -> vsr_view:
    v = make_view(view)
    ln = make_lens(view)
    eff = vsr_view()
    _check(_lib.vsr_build_map_lens(ctypes.byref(v), ctypes.byref(ln), fmt, flags, _ptr(map_buf), _nbytes(map_buf),
                                   ctypes.byref(eff), _stream(stream)))
    return eff


def vsr_map_unpack(view, fmt: int, map_buf, out, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_map_unpack(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(out), _stream(stream)))


def vsr_setup_tris(xyz, setup_buf, stream=None) -> None:
    assert xyz.dim() == 2 and xyz.shape[0] == 9 and xyz.is_contiguous()
    _check(_lib.vsr_setup_tris(_ptr(xyz), int(xyz.shape[1]), _ptr(setup_buf), _nbytes(setup_buf), _stream(stream)))


def vsr_bin(view, fmt: int, map_buf, setup_buf, ntri: int, bin_depth: int, flags: int, bins, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_bin(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, bin_depth, flags, _ptr(bins),
                        _nbytes(bins), _stream(stream)))


def vsr_raster(view, fmt: int, map_buf, setup_buf, ntri: int, bins, bin_depth: int, tri_id, depth,
               stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_raster(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, _ptr(bins), bin_depth,
                           _ptr(tri_id), _ptr(depth), _stream(stream)))


def vsr_raster_stats(view, fmt: int, map_buf, setup_buf, ntri: int, bins, bin_depth: int, tri_id, depth, stats,
                     no_early_exit: bool = False, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_raster_stats(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, _ptr(bins), bin_depth,
                                 _ptr(tri_id), _ptr(depth), _ptr(stats), int(bool(no_early_exit)), _stream(stream)))


def make_jobs(jobs: Sequence[tuple]):
    """ctypes array from (view, setup_buf, ntri, tri_id, depth) tuples."""
    arr = (vsr_job * len(jobs))()
    for q, (view, setup_buf, ntri, tri_id, depth) in enumerate(jobs):
        arr[q].view = make_view(view)
        arr[q].setup = _ptr(setup_buf)
        arr[q].ntri = int(ntri)
        arr[q].tri_id = _ptr(tri_id)
        arr[q].depth = _ptr(depth)
    return arr


def vsr_render_bytes(width: int, height: int) -> int:
    return _size(_lib.vsr_render_bytes(width, height), "vsr_render_bytes")


def vsr_render(view, fmt: int, map_buf, setup_buf, ntri: int, scratch, tri_id, depth, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_render(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, _ptr(scratch),
                           _nbytes(scratch), _ptr(tri_id), _ptr(depth), _stream(stream)))


def vsr_render_noalloc(view, fmt: int, map_buf, setup_buf, ntri: int, tri_id, depth, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_render_noalloc(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, _ptr(tri_id),
                                   _ptr(depth), _stream(stream)))


def vsr_resolve(view, fmt: int, map_buf, xyz, ntri: int, tri_id, vattr, nattr: int, flags: int, bary, attr,
                stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_resolve(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(xyz), ntri, _ptr(tri_id), _ptr(vattr), nattr,
                            flags, _ptr(bary), _ptr(attr), _stream(stream)))


def vsr_resolve_pack_bytes(ntri: int, nattr: int) -> int:
    return _size(_lib.vsr_resolve_pack_bytes(ntri, nattr), "vsr_resolve_pack_bytes")


def vsr_resolve_pack(xyz, vattr, ntri: int, nattr: int, packed, stream=None) -> None:
    _check(_lib.vsr_resolve_pack(_ptr(xyz), _ptr(vattr), ntri, nattr, _ptr(packed), _nbytes(packed),
                                 _stream(stream)))


def vsr_resolve_packed(view, fmt: int, map_buf, packed, ntri: int, nattr: int, tri_id, flags: int, bary, attr,
                       stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_resolve_packed(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(packed), ntri, nattr, _ptr(tri_id),
                                   flags, _ptr(bary), _ptr(attr), _stream(stream)))


def vsr_aa_map_bytes(width: int, height: int, fmt: int = VSR_MAP_F32) -> int:
    return _size(_lib.vsr_aa_map_bytes(width, height, fmt), "vsr_aa_map_bytes")


def vsr_aa_raster(view, fmt: int, map_buf, setup_buf, ntri: int, bins, bin_depth: int, coverage, depth_pass,
                  dominant, lost=None, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_aa_raster(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, _ptr(bins), bin_depth,
                              _ptr(coverage), _ptr(depth_pass), _ptr(dominant), _ptr(lost), _stream(stream)))


def vsr_aa_raster_stats(view, fmt: int, map_buf, setup_buf, ntri: int, bins, bin_depth: int, coverage, depth_pass,
                        dominant, lost, stats, no_skip: bool = False, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_aa_raster_stats(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), ntri, _ptr(bins),
                                    bin_depth, _ptr(coverage), _ptr(depth_pass), _ptr(dominant), _ptr(lost),
                                    _ptr(stats), int(bool(no_skip)), _stream(stream)))


def vsr_setup_particles(pr, setup_buf, stream=None) -> None:
    assert pr.dim() == 2 and pr.shape[0] == 4 and pr.is_contiguous()
    _check(_lib.vsr_setup_particles(_ptr(pr), int(pr.shape[1]), _ptr(setup_buf), _nbytes(setup_buf),
                                    _stream(stream)))


def vsr_aa_particles(view, fmt: int, map_buf, setup_buf, n: int, bins, bin_depth: int, coverage, depth_pass, uv,
                     dominant, lost=None, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_aa_particles(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), n, _ptr(bins), bin_depth,
                                 _ptr(coverage), _ptr(depth_pass), _ptr(uv), _ptr(dominant), _ptr(lost),
                                 _stream(stream)))


def vsr_aa_particles_stats(view, fmt: int, map_buf, setup_buf, n: int, bins, bin_depth: int, coverage, depth_pass,
                           uv, dominant, lost, stats, no_skip: bool = False, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_aa_particles_stats(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), n, _ptr(bins),
                                       bin_depth, _ptr(coverage), _ptr(depth_pass), _ptr(uv), _ptr(dominant),
                                       _ptr(lost), _ptr(stats), int(bool(no_skip)), _stream(stream)))


def vsr_wire_bytes(ntri: int) -> int:
    return _size(_lib.vsr_wire_bytes(ntri), "vsr_wire_bytes")


def vsr_setup_wire(setup_buf, xyz, ntri: int, wire, stream=None) -> None:
    _check(_lib.vsr_setup_wire(_ptr(setup_buf), _ptr(xyz), ntri, _ptr(wire), _nbytes(wire), _stream(stream)))


def vsr_aa_wireframe(view, fmt: int, map_buf, setup_buf, wire, ntri: int, bins, bin_depth: int, coverage, dominant,
                     stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_aa_wireframe(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), _ptr(wire), ntri, _ptr(bins),
                                 bin_depth, _ptr(coverage), _ptr(dominant), _stream(stream)))


def vsr_aa_wireframe_stats(view, fmt: int, map_buf, setup_buf, wire, ntri: int, bins, bin_depth: int, coverage,
                           dominant, stats, stream=None) -> None:
    v = make_view(view)
    _check(_lib.vsr_aa_wireframe_stats(ctypes.byref(v), fmt, _ptr(map_buf), _ptr(setup_buf), _ptr(wire), ntri,
                                       _ptr(bins), bin_depth, _ptr(coverage), _ptr(dominant), _ptr(stats),
                                       _stream(stream)))


def vsr_submit_bytes(jobs, fmt: int, mode: int = 0, bin_depth: int = 1024) -> int:
    return _size(_lib.vsr_submit_bytes(jobs, len(jobs), fmt, mode, bin_depth), "vsr_submit_bytes")


def vsr_submit(jobs, fmt: int, mode: int, bin_depth: int, workspace, stream=None) -> None:
    _check(_lib.vsr_submit(jobs, len(jobs), fmt, mode, bin_depth, _ptr(workspace), _nbytes(workspace),
                           _stream(stream)))


def vsr_submit_timed(jobs, fmt: int, mode: int, bin_depth: int, workspace, events, stream=None) -> None:
    """events: four recorded-once torch.cuda.Event objects (or raw hipEvent_t
    handles) that the library records between the stages."""
    handles = [int(e.cuda_event) if hasattr(e, "cuda_event") else int(e) for e in events]
    arr = (ctypes.c_void_p * len(handles))(*handles)
    _check(_lib.vsr_submit_timed(jobs, len(jobs), fmt, mode, bin_depth, _ptr(workspace), _nbytes(workspace), arr,
                                 len(handles), _stream(stream)))


def vsr_submit_table_bytes(njobs: int) -> int:
    return _size(_lib.vsr_submit_table_bytes(njobs), "vsr_submit_table_bytes")


def vsr_submit_table_offset() -> int:
    return int(_lib.vsr_submit_table_offset())


def vsr_submit_table(jobs, fmt: int, mode: int, bin_depth: int, workspace, host_table) -> None:
    """host_table: a host (CPU) uint8 tensor or numpy array."""
    ptr = host_table.data_ptr() if hasattr(host_table, "data_ptr") else host_table.ctypes.data
    n = host_table.numel() if hasattr(host_table, "numel") else host_table.nbytes
    _check(_lib.vsr_submit_table(jobs, len(jobs), fmt, mode, bin_depth, _ptr(workspace), ptr, n))


def vsr_bin_overflow(bins_or_ws, is_workspace: bool = False) -> int:
    out = ctypes.c_int64(0)
    _check(_lib.vsr_bin_overflow(_ptr(bins_or_ws), int(bool(is_workspace)), ctypes.byref(out)))
    return int(out.value)


def vsr_calib_copy(src, dst, stream=None) -> None:
    _check(_lib.vsr_calib_copy(_ptr(src), _ptr(dst), min(_nbytes(src), _nbytes(dst)) // 16 * 16, _stream(stream)))


def vsr_calib_fma(out, iters: int, stream=None) -> None:
    _check(_lib.vsr_calib_fma(_ptr(out), int(out.numel()), int(iters), _stream(stream)))


def vsr_strerror(code: int) -> str:
    return _lib.vsr_strerror(code).decode()


def vsr_last_error() -> str:
    return _lib.vsr_last_error().decode()
