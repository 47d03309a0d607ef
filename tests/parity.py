"""Comparison of a GPU (tri_id, depth) image with the FP64 oracle.

Rule (per pixel, from the oracle's flags):
  * clean pixels (no flag): the GPU triangle id equals the oracle's, bit for
    bit, and the FP32 depth is within 1e-5 relative of the FP64 depth.  For
    a pixel whose depth is off by more, the grazing-incidence factor
    kappa = 1/|g . N_hat| is reported beside it (FP32 rounding of the view
    direction and the plane grows as 1/cos(incidence)) but excuses nothing;
  * flagged pixels (EDGE, DEPTH) are excused from the id comparison, but the
    GPU's choice must still be valid: no hit only where the oracle has none
    or an edge is within the band, otherwise a triangle that passes every
    edge test within the band and whose FP64 depth is within 2e-5 of the
    oracle's winner;
  * DOMAIN pixels (within 1e-6 of the projection's domain edge) are excused
    and counted apart from the edge band;
  * INVALID pixels must be NO_HIT on the GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

import oracle

BAND = math.sin(1e-6)


@dataclass
class ParityStats:
    pixels: int = 0
    clean: int = 0
    hits: int = 0
    edge_excused: int = 0
    depth_excused: int = 0
    domain_excused: int = 0
    invalid: int = 0
    id_mismatch: int = 0
    depth_bad: int = 0
    kappa_max: float = 0.0  # largest grazing factor among pixels off by more than 1e-5 (report only)
    max_rel_depth: float = 0.0
    excused_invalid_choice: int = 0
    notes: list = field(default_factory=list)

    def ok(self) -> bool:
        return self.id_mismatch == 0 and self.depth_bad == 0 and self.excused_invalid_choice == 0

    def line(self) -> str:
        return (f"pixels={self.pixels} clean={self.clean} hits={self.hits} edge_excused={self.edge_excused} "
                f"depth_excused={self.depth_excused} domain_excused={self.domain_excused} invalid={self.invalid} "
                f"id_mismatch={self.id_mismatch} depth_bad={self.depth_bad} kappa_max={self.kappa_max:.1f} "
                f"max_rel_depth={self.max_rel_depth:.3e} bad_excused_choice={self.excused_invalid_choice}")


def _plane_normals(tris: np.ndarray) -> np.ndarray:
    a = tris[0:3].T.astype(np.float64)
    b = tris[3:6].T.astype(np.float64)
    c = tris[6:9].T.astype(np.float64)
    n = np.cross(a - b, c - b)
    ln = np.linalg.norm(n, axis=1, keepdims=True)
    return n / np.where(ln > 0, ln, 1.0)


def compare(view, tris: np.ndarray, gpu_ids: np.ndarray, gpu_depth: np.ndarray, ref: oracle.RenderResult,
            pixels: np.ndarray | None = None, check_excused: int = 2000) -> ParityStats:
    """gpu_ids/gpu_depth: full [H, W] images.  ref: oracle result for
    ``pixels`` (flat indices) or the full frame when pixels is None."""
    W, H = view.width, view.height
    if pixels is None:
        pixels = np.arange(W * H, dtype=np.int64)
        rid, rdep, rfl = ref.id.reshape(-1), ref.depth.reshape(-1), ref.flags.reshape(-1)
    else:
        rid, rdep, rfl = ref.id, ref.depth, ref.flags
    gid = gpu_ids.reshape(-1)[pixels]
    gdep = gpu_depth.reshape(-1)[pixels].astype(np.float64)
    st = ParityStats(pixels=len(pixels))
    inv = (rfl & oracle.FLAG_INVALID) != 0
    edge = (rfl & oracle.FLAG_EDGE) != 0
    dflag = (rfl & oracle.FLAG_DEPTH) != 0
    dom = (rfl & oracle.FLAG_DOMAIN) != 0
    clean = rfl == 0
    st.invalid = int((inv & ~dom).sum())
    st.domain_excused = int(dom.sum())
    st.edge_excused = int((edge & ~inv & ~dom).sum())
    st.depth_excused = int((dflag & ~edge & ~inv & ~dom).sum())
    st.clean = int(clean.sum())
    # invalid pixels are never covered on the GPU either
    bad_inv = inv & ~dom & (gid != oracle.NO_HIT)
    st.id_mismatch += int(bad_inv.sum())
    mism = clean & (gid != rid)
    st.id_mismatch += int(mism.sum())
    if mism.any():
        q = np.nonzero(mism)[0][:5]
        st.notes.append(f"first id mismatches at pixels {pixels[q].tolist()}: gpu {gid[q].tolist()} "
                        f"oracle {rid[q].tolist()}")
    hit = clean & (rid != oracle.NO_HIT) & (gid == rid)
    st.hits = int(hit.sum())
    if hit.any():
        rel = np.abs(gdep[hit] - rdep[hit]) / rdep[hit]
        st.max_rel_depth = float(rel.max())
        over = rel > 1e-5
        if over.any():
            dirs, _ = oracle.perspective_map(view) if W * H <= 4_000_000 else (None, None)
            idx = np.nonzero(hit)[0][over]
            nrm = _plane_normals(tris)
            for k, p in zip(idx, pixels[idx]):
                if dirs is not None:
                    g = dirs.reshape(-1, 3)[p]
                else:
                    g = _pixel_dir(view, int(p))
                kappa = 1.0 / max(abs(float(g @ nrm[rid[k]])), 1e-300)
                r = abs(gdep[k] - rdep[k]) / rdep[k]
                st.depth_bad += 1
                st.kappa_max = max(st.kappa_max, kappa)
                if len(st.notes) < 8:
                    st.notes.append(f"depth pixel {p}: gpu {gdep[k]!r} oracle {rdep[k]!r} rel {r:.2e} "
                                    f"kappa {kappa:.1f}")
    # excused pixels: the GPU's choice must be a valid one
    exc = np.nonzero((edge | dflag) & ~inv & ~dom)[0]
    if len(exc) > check_excused:
        exc = np.random.default_rng(0).choice(exc, size=check_excused, replace=False)
    for k in exc:
        p = int(pixels[k])
        g_id = int(gid[k])
        if g_id == int(rid[k]):
            continue
        if g_id == oracle.NO_HIT:
            if not edge[k]:
                st.excused_invalid_choice += 1
            continue
        e, r, valid = oracle.pair(view, tris, g_id, p)
        near = bool(np.all(e > -BAND))
        depth_ok = rid[k] == oracle.NO_HIT or r <= rdep[k] * (1 + 2e-5) or r <= 0
        if not (valid and near and depth_ok):
            st.excused_invalid_choice += 1
            if len(st.notes) < 8:
                st.notes.append(f"excused pixel {p}: gpu chose {g_id} (edges {e}, r {r}) oracle {int(rid[k])} "
                                f"r {rdep[k]}")
    return st


def _pixel_dir(view, p: int) -> np.ndarray:
    i, j = p % view.width, p // view.width
    g, _, _ = oracle.lens_direction(view, (i + 0.5) / view.width, (j + 0.5) / view.height)
    return view.rot_matrix() @ g
