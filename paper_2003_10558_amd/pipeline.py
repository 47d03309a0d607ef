"""Device-memory plumbing around the C ABI: resident scenes and view buffers.

Nothing here computes any part of the method; it allocates the buffers the
vsr_* calls need (torch tensors on the GPU) and chains the calls.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import vsr

DEFAULT_BIN_DEPTH = 256


def _buffer(nbytes: int, device) -> torch.Tensor:
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def build_map(view, fmt: int, flags: int, map_buf, stream=None):
    """vsr_build_map, or vsr_build_map_lens when the view names another
    generator or a lens distortion."""
    if vsr.has_lens(view):
        return vsr.vsr_build_map_lens(view, fmt, flags, map_buf, stream)
    return vsr.vsr_build_map(view, fmt, flags, map_buf, stream)


class Scene:
    """Triangles resident on the GPU with their setup (vsr_setup_tris)."""

    def __init__(self, xyz: np.ndarray | torch.Tensor, device="cuda", stream=None):
        if isinstance(xyz, np.ndarray):
            xyz = torch.from_numpy(np.ascontiguousarray(xyz, dtype=np.float32))
        self.xyz = xyz.to(device=device, dtype=torch.float32).contiguous()
        assert self.xyz.dim() == 2 and self.xyz.shape[0] == 9
        self.ntri = int(self.xyz.shape[1])
        self.device = self.xyz.device
        self.setup = _buffer(vsr.vsr_setup_bytes(self.ntri), self.device)
        self.wire = None  # side caps for wire frames, made on first use
        self.refresh(stream)

    def refresh(self, stream=None) -> None:
        """Re-run the per-triangle setup (e.g. after the vertices moved)."""
        vsr.vsr_setup_tris(self.xyz, self.setup, stream)
        if self.wire is not None:
            vsr.vsr_setup_wire(self.setup, self.xyz, self.ntri, self.wire, stream)

    def wire_caps(self, stream=None) -> torch.Tensor:
        """The side caps of vsr_setup_wire (kept in step with refresh())."""
        if self.wire is None:
            self.wire = _buffer(vsr.vsr_wire_bytes(self.ntri), self.device)
            vsr.vsr_setup_wire(self.setup, self.xyz, self.ntri, self.wire, stream)
        return self.wire


@dataclass
class Frame:
    tri_id: torch.Tensor   # uint32 as int32 storage, [H, W]
    depth: torch.Tensor    # float32 [H, W]
    map: torch.Tensor
    bins: torch.Tensor
    view_eff: object


def alloc_outputs(view, device) -> Tuple[torch.Tensor, torch.Tensor]:
    ids = torch.empty((view.height, view.width), dtype=torch.int32, device=device)
    dep = torch.empty((view.height, view.width), dtype=torch.float32, device=device)
    return ids, dep


def render(scene: Scene, view, fmt: int = vsr.VSR_MAP_F32, bin_depth: int = DEFAULT_BIN_DEPTH,
           bin_flags: int = 0, stream=None, frame: Optional[Frame] = None) -> Frame:
    """build_map -> bin -> raster for one view (plain per-view path)."""
    dev = scene.device
    if frame is None:
        ids, dep = alloc_outputs(view, dev)
        frame = Frame(ids, dep, _buffer(vsr.vsr_map_bytes(view.width, view.height, fmt), dev),
                      _buffer(vsr.vsr_bin_bytes(view.width, view.height, bin_depth), dev), None)
    frame.view_eff = build_map(view, fmt, 0, frame.map, stream)
    vsr.vsr_bin(view, fmt, frame.map, scene.setup, scene.ntri, bin_depth, bin_flags, frame.bins, stream)
    vsr.vsr_raster(view, fmt, frame.map, scene.setup, scene.ntri, frame.bins, bin_depth, frame.tri_id,
                   frame.depth, stream)
    return frame


def render_fused(scene: Scene, view, fmt: int = vsr.VSR_MAP_F32, stream=None,
                 frame: Optional[Frame] = None) -> Frame:
    """build_map -> fused depth-sliced bin + raster (vsr_render) for one view."""
    dev = scene.device
    if frame is None:
        ids, dep = alloc_outputs(view, dev)
        frame = Frame(ids, dep, _buffer(vsr.vsr_map_bytes(view.width, view.height, fmt), dev),
                      _buffer(vsr.vsr_render_bytes(view.width, view.height), dev), None)
    frame.view_eff = build_map(view, fmt, 0, frame.map, stream)
    vsr.vsr_render(view, fmt, frame.map, scene.setup, scene.ntri, frame.bins, frame.tri_id, frame.depth, stream)
    return frame


def pack_resolve(scene: Scene, vattr: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, int]:
    """Packed copy of the scene's vertices and per-vertex data [3, K, T] for
    resolve(..., packed=...); returns (buffer, K)."""
    dev = scene.device
    nattr = 0 if vattr is None else int(vattr.shape[1])
    if nattr:
        vattr = vattr.to(device=dev, dtype=torch.float32).contiguous()
        assert vattr.shape == (3, nattr, scene.ntri)
    buf = _buffer(vsr.vsr_resolve_pack_bytes(scene.ntri, nattr), dev)
    vsr.vsr_resolve_pack(scene.xyz, vattr, scene.ntri, nattr, buf, stream)
    return buf, nattr


def resolve(scene: Scene, view, frame: Frame, vattr: Optional[torch.Tensor] = None, normalize3: bool = False,
            fmt: int = vsr.VSR_MAP_F32, stream=None,
            packed: Optional[Tuple[torch.Tensor, int]] = None) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    """Fragment data of a rendered frame: barycentric weights [3, H, W] and,
    with per-vertex data ``vattr`` [3, K, T], the interpolated data [K, H, W]
    (the first three normalised when ``normalize3``).  With ``packed`` (from
    pack_resolve) the packed copy is read instead of the arrays."""
    if packed is not None:
        buf, nattr = packed
        dev = scene.device
        bary = torch.empty((3, view.height, view.width), dtype=torch.float32, device=dev)
        attr = torch.empty((nattr, view.height, view.width), dtype=torch.float32, device=dev) if nattr else None
        vsr.vsr_resolve_packed(view, fmt, frame.map, buf, scene.ntri, nattr, frame.tri_id,
                               vsr.VSR_RESOLVE_NORMALIZE3 if normalize3 else 0, bary, attr, stream)
        return bary, attr
    dev = scene.device
    bary = torch.empty((3, view.height, view.width), dtype=torch.float32, device=dev)
    nattr = 0 if vattr is None else int(vattr.shape[1])
    attr = None
    if nattr:
        vattr = vattr.to(device=dev, dtype=torch.float32).contiguous()
        assert vattr.shape == (3, nattr, scene.ntri)
        attr = torch.empty((nattr, view.height, view.width), dtype=torch.float32, device=dev)
    vsr.vsr_resolve(view, fmt, frame.map, scene.xyz, scene.ntri, frame.tri_id, vattr, nattr,
                    vsr.VSR_RESOLVE_NORMALIZE3 if normalize3 else 0, bary, attr, stream)
    return bary, attr


@dataclass
class AAFrame:
    coverage: torch.Tensor    # float32 [H, W], m_b in [0, 1]
    depth_pass: torch.Tensor  # float32 [H, W], sum of m_fc * r
    dominant: torch.Tensor    # uint32 as int32 storage, [H, W]
    lost: torch.Tensor        # int32 [1]: pixels whose fragment list overflowed
    map: torch.Tensor
    bins: torch.Tensor
    view_eff: object


def render_aa(scene: Scene, view, fmt: int = vsr.VSR_MAP_F32, bin_depth: int = DEFAULT_BIN_DEPTH,
              bin_flags: int = 0, stream=None, frame: Optional[AAFrame] = None,
              stats: Optional[torch.Tensor] = None, no_skip: bool = False) -> AAFrame:
    """Aliasing-free frame: build_map (VSR_MAP_AA) -> bin -> vsr_aa_raster."""
    dev = scene.device
    H, W = view.height, view.width
    if frame is None:
        frame = AAFrame(torch.empty((H, W), dtype=torch.float32, device=dev),
                        torch.empty((H, W), dtype=torch.float32, device=dev),
                        torch.empty((H, W), dtype=torch.int32, device=dev),
                        torch.empty(1, dtype=torch.int32, device=dev),
                        _buffer(vsr.vsr_aa_map_bytes(W, H, fmt), dev),
                        _buffer(vsr.vsr_bin_bytes(W, H, bin_depth), dev), None)
    frame.view_eff = build_map(view, fmt, vsr.VSR_MAP_AA, frame.map, stream)
    vsr.vsr_bin(view, fmt, frame.map, scene.setup, scene.ntri, bin_depth, bin_flags, frame.bins, stream)
    if stats is None:
        vsr.vsr_aa_raster(view, fmt, frame.map, scene.setup, scene.ntri, frame.bins, bin_depth, frame.coverage,
                          frame.depth_pass, frame.dominant, frame.lost, stream)
    else:
        vsr.vsr_aa_raster_stats(view, fmt, frame.map, scene.setup, scene.ntri, frame.bins, bin_depth,
                                frame.coverage, frame.depth_pass, frame.dominant, frame.lost, stats, no_skip,
                                stream)
    return frame


@dataclass
class WireFrame:
    coverage: torch.Tensor    # float32 [H, W], largest line mask
    dominant: torch.Tensor    # uint32 as int32 storage, [H, W]
    map: torch.Tensor
    bins: torch.Tensor
    view_eff: object


def render_wireframe(scene: Scene, view, fmt: int = vsr.VSR_MAP_F32, bin_depth: int = DEFAULT_BIN_DEPTH,
                     bin_flags: int = 0, stream=None, frame: Optional[WireFrame] = None,
                     stats: Optional[torch.Tensor] = None) -> WireFrame:
    """Aliasing-free wire frame of the scene's triangle sides:
    build_map (VSR_MAP_AA_LINES) -> bin -> vsr_aa_wireframe."""
    dev = scene.device
    H, W = view.height, view.width
    if frame is None:
        frame = WireFrame(torch.empty((H, W), dtype=torch.float32, device=dev),
                          torch.empty((H, W), dtype=torch.int32, device=dev),
                          _buffer(vsr.vsr_aa_map_bytes(W, H, fmt), dev),
                          _buffer(vsr.vsr_bin_bytes(W, H, bin_depth), dev), None)
    frame.view_eff = build_map(view, fmt, vsr.VSR_MAP_AA_LINES, frame.map, stream)
    vsr.vsr_bin(view, fmt, frame.map, scene.setup, scene.ntri, bin_depth, bin_flags, frame.bins, stream)
    wire = scene.wire_caps(stream)
    if stats is None:
        vsr.vsr_aa_wireframe(view, fmt, frame.map, scene.setup, wire, scene.ntri, frame.bins, bin_depth,
                             frame.coverage, frame.dominant, stream)
    else:
        vsr.vsr_aa_wireframe_stats(view, fmt, frame.map, scene.setup, wire, scene.ntri, frame.bins, bin_depth,
                                   frame.coverage, frame.dominant, stats, stream)
    return frame


class ParticleScene:
    """Particles (float[4][n]: x, y, z, radius) resident on the GPU with their
    setup (vsr_setup_particles)."""

    def __init__(self, pr: np.ndarray | torch.Tensor, device="cuda", stream=None):
        if isinstance(pr, np.ndarray):
            pr = torch.from_numpy(np.ascontiguousarray(pr, dtype=np.float32))
        self.pr = pr.to(device=device, dtype=torch.float32).contiguous()
        assert self.pr.dim() == 2 and self.pr.shape[0] == 4
        self.ntri = self.n = int(self.pr.shape[1])
        self.device = self.pr.device
        self.setup = _buffer(vsr.vsr_setup_bytes(self.n), self.device)
        self.refresh(stream)

    def refresh(self, stream=None) -> None:
        vsr.vsr_setup_particles(self.pr, self.setup, stream)


@dataclass
class ParticleFrame:
    coverage: torch.Tensor
    depth_pass: torch.Tensor
    uv: torch.Tensor          # float32 [2, H, W] texture-coordinate pass
    dominant: torch.Tensor
    lost: torch.Tensor
    map: torch.Tensor
    bins: torch.Tensor
    view_eff: object


def render_particles(scene: ParticleScene, view, fmt: int = vsr.VSR_MAP_F32, bin_depth: int = DEFAULT_BIN_DEPTH,
                     bin_flags: int = 0, stream=None, frame: Optional[ParticleFrame] = None,
                     stats: Optional[torch.Tensor] = None, no_skip: bool = False) -> ParticleFrame:
    """Aliasing-free particles: build_map (VSR_MAP_AA) -> bin -> vsr_aa_particles."""
    dev = scene.device
    H, W = view.height, view.width
    if frame is None:
        frame = ParticleFrame(torch.empty((H, W), dtype=torch.float32, device=dev),
                              torch.empty((H, W), dtype=torch.float32, device=dev),
                              torch.empty((2, H, W), dtype=torch.float32, device=dev),
                              torch.empty((H, W), dtype=torch.int32, device=dev),
                              torch.empty(1, dtype=torch.int32, device=dev),
                              _buffer(vsr.vsr_aa_map_bytes(W, H, fmt), dev),
                              _buffer(vsr.vsr_bin_bytes(W, H, bin_depth), dev), None)
    frame.view_eff = build_map(view, fmt, vsr.VSR_MAP_AA, frame.map, stream)
    vsr.vsr_bin(view, fmt, frame.map, scene.setup, scene.n, bin_depth, bin_flags, frame.bins, stream)
    if stats is None:
        vsr.vsr_aa_particles(view, fmt, frame.map, scene.setup, scene.n, frame.bins, bin_depth, frame.coverage,
                             frame.depth_pass, frame.uv, frame.dominant, frame.lost, stream)
    else:
        vsr.vsr_aa_particles_stats(view, fmt, frame.map, scene.setup, scene.n, frame.bins, bin_depth,
                                   frame.coverage, frame.depth_pass, frame.uv, frame.dominant, frame.lost, stats,
                                   no_skip, stream)
    return frame


class Batch:
    """Workspace + outputs for vsr_submit over a fixed list of (scene, view)."""

    def __init__(self, items: Sequence[Tuple[Scene, object]], fmt: int = vsr.VSR_MAP_F32,
                 mode: int = vsr.VSR_SUBMIT_BINNED, bin_depth: int = DEFAULT_BIN_DEPTH):
        assert len(items) > 0
        if any(vsr.has_lens(v) for _, v in items):
            raise ValueError("vsr_submit takes Universal Perspective views only; render other generators with "
                             "render() / render_aa()")
        self.items = list(items)
        self.fmt, self.mode, self.bin_depth = fmt, mode, bin_depth
        dev = items[0][0].device
        self.outputs = [alloc_outputs(v, dev) for _, v in self.items]
        self.jobs = vsr.make_jobs([(v, s.setup, s.ntri, o[0], o[1])
                                   for (s, v), o in zip(self.items, self.outputs)])
        self.workspace = _buffer(vsr.vsr_submit_bytes(self.jobs, fmt, mode, bin_depth), dev)

    def submit(self, stream=None, events=None) -> List[Tuple[torch.Tensor, torch.Tensor]]:
        """One vsr_submit; with ``events`` (four torch.cuda.Event) the stage
        boundaries are recorded on the stream (vsr_submit_timed)."""
        if events is None:
            vsr.vsr_submit(self.jobs, self.fmt, self.mode, self.bin_depth, self.workspace, stream)
        else:
            vsr.vsr_submit_timed(self.jobs, self.fmt, self.mode, self.bin_depth, self.workspace, events, stream)
        return self.outputs


class GraphBatch:
    """A batch captured once in a HIP graph and replayed with new view
    parameters.  Shapes (view sizes, scenes) are fixed at capture; between
    replays set_views() rewrites the job table in device memory with one
    host-to-device copy on the capture stream."""

    def __init__(self, items: Sequence[Tuple[Scene, object]], fmt: int = vsr.VSR_MAP_F32,
                 mode: int = vsr.VSR_SUBMIT_BINNED, bin_depth: int = DEFAULT_BIN_DEPTH, stream=None):
        self.batch = Batch(items, fmt=fmt, mode=mode, bin_depth=bin_depth)
        self.stream = stream or torch.cuda.Stream(device=self.batch.workspace.device)
        nb = vsr.vsr_submit_table_bytes(len(self.batch.jobs))
        off = vsr.vsr_submit_table_offset()
        self.table_host = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
        self.table_dev = self.batch.workspace[off:off + nb]
        self.set_views([v for _, v in items])
        self.stream.synchronize()
        # warm-up launch outside the capture, then capture
        with torch.cuda.stream(self.stream):
            self._launch()
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._launch()

    def _launch(self):
        b = self.batch
        vsr.vsr_submit(b.jobs, b.fmt, b.mode | vsr.VSR_SUBMIT_TABLE_READY, b.bin_depth, b.workspace,
                       torch.cuda.current_stream())

    def set_views(self, views: Sequence[object]) -> None:
        b = self.batch
        assert len(views) == len(b.jobs)
        for q, v in enumerate(views):
            old = b.jobs[q].view
            assert (int(v.width), int(v.height)) == (old.width, old.height), "view sizes are fixed at capture"
            b.jobs[q].view = vsr.make_view(v)
        self.stream.synchronize()  # the previous replay may still read the table
        vsr.vsr_submit_table(b.jobs, b.fmt, b.mode, b.bin_depth, b.workspace, self.table_host)
        with torch.cuda.stream(self.stream):
            self.table_dev.copy_(self.table_host, non_blocking=True)

    def replay(self) -> List[Tuple[torch.Tensor, torch.Tensor]]:
        with torch.cuda.stream(self.stream):
            self.graph.replay()
        return self.batch.outputs


def ids_u32(t: torch.Tensor) -> np.ndarray:
    """Device int32 id image -> host uint32 array."""
    return t.cpu().numpy().view(np.uint32)
