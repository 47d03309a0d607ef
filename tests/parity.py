"""Comparison of a GPU (tri_id, depth) image with the FP64 oracle.

Rule (per pixel, from the oracle's flags):
  * clean pixels (no flag): the GPU triangle id equals the oracle's, bit for
    bit, and the FP32 depth is within 1e-5 relative of the FP64 depth.  The
    one exception is grazing incidence: the depth r = A.N / g.N moves by
    kappa * delta (relative) when the direction g moves by delta radians,
    kappa = 1/|g . N_hat| (section 1.1.4), so no FP32 map meets 1e-5 where
    kappa is large (a direction rounded to FP32 is already off by up to
    6e-8 rad).  A pixel whose winner is seen at kappa > KAPPA_GRAZING may
    instead be off by up to kappa * GRAZING_PER_KAPPA: the map's direction
    bound (1e-6 rad, asserted by the map parity test) plus 6 units of FP32
    rounding for the plane normal and the two dot products.  Such pixels are
    counted (`grazing`) and reported with the largest kappa and error/kappa;
  * flagged pixels (EDGE, DEPTH) are excused from the id comparison, but the
    GPU's choice must still be valid: no hit only where the oracle has none
    or an edge is within the band, otherwise a triangle that passes every
    edge test within the band and whose FP64 depth is within 2e-5 of the
    oracle's winner -- or of the winner once the triangles that lie within
    the band at this pixel (which FP32 may leave uncovered) are set aside,
    one after another;
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
DEPTH_REL = 1e-5
KAPPA_GRAZING = 20.0  # incidence beyond 87.1 degrees
GRAZING_PER_KAPPA = 1e-6 + 6 * 2.0 ** -24


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
    grazing: int = 0  # clean id-matching pixels off by more than 1e-5 within the grazing bound
    grazing_hits: int = 0  # clean id-matching pixels whose winner is seen at kappa > KAPPA_GRAZING
    kappa_max: float = 0.0  # largest kappa among pixels off by more than 1e-5
    err_per_kappa_max: float = 0.0  # largest (relative error / kappa) among them
    max_rel_depth: float = 0.0
    excused_invalid_choice: int = 0
    notes: list = field(default_factory=list)

    def ok(self) -> bool:
        return self.id_mismatch == 0 and self.depth_bad == 0 and self.excused_invalid_choice == 0

    def line(self) -> str:
        return (f"pixels={self.pixels} clean={self.clean} hits={self.hits} edge_excused={self.edge_excused} "
                f"depth_excused={self.depth_excused} domain_excused={self.domain_excused} invalid={self.invalid} "
                f"id_mismatch={self.id_mismatch} depth_bad={self.depth_bad} grazing={self.grazing} "
                f"(of {self.grazing_hits} hits at kappa>{KAPPA_GRAZING:.0f}; kappa_max={self.kappa_max:.1f} "
                f"err/kappa_max={self.err_per_kappa_max:.2e}) max_rel_depth={self.max_rel_depth:.3e} "
                f"bad_excused_choice={self.excused_invalid_choice}")


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
        hk = np.nonzero(hit)[0]
        kap = _kappa(view, tris, pixels[hk], rid[hk])
        st.grazing_hits = int((kap > KAPPA_GRAZING).sum())
        rel = np.abs(gdep[hk] - rdep[hk]) / rdep[hk]
        st.max_rel_depth = float(rel.max())
        for j in np.nonzero(rel > DEPTH_REL)[0]:
            k, p, kappa, r = hk[j], int(pixels[hk[j]]), float(kap[j]), float(rel[j])
            st.kappa_max = max(st.kappa_max, kappa)
            st.err_per_kappa_max = max(st.err_per_kappa_max, r / kappa)
            if kappa > KAPPA_GRAZING and r <= kappa * GRAZING_PER_KAPPA:
                st.grazing += 1
                continue
            st.depth_bad += 1
            if len(st.notes) < 6:
                st.notes.append(f"depth pixel {p}: gpu {gdep[k]!r} oracle {rdep[k]!r} rel {r:.2e} "
                                f"kappa {kappa:.1f}")
    # excused pixels: the GPU's choice must be a valid one
    exc = np.nonzero((edge | dflag) & ~inv & ~dom)[0]
    if len(exc) > check_excused:
        exc = np.random.default_rng(0).choice(exc, size=check_excused, replace=False)
    enotes = []
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
        if valid and near and not depth_ok:
            depth_ok = _behind_band_triangles(view, tris, p, int(rid[k]), g_id, r)
        if not (valid and near and depth_ok):
            st.excused_invalid_choice += 1
            if len(enotes) < 6:
                g = _pixel_dir(view, p)
                kap = [1.0 / max(abs(float(g @ _plane_normal(tris, t))), 1e-300)
                       for t in (g_id, int(rid[k])) if t != oracle.NO_HIT]
                enotes.append(f"excused pixel {p} (flags {int(rfl[k])}): gpu chose {g_id} (edges {e}, r {r!r}) "
                              f"oracle {int(rid[k])} r {rdep[k]!r}; gpu depth {gdep[k]!r}; kappa "
                              + " / ".join(f"{x:.1f}" for x in kap))
    st.notes += enotes
    return st


def _plane_normal(tris: np.ndarray, t: int) -> np.ndarray:
    return _plane_normals(tris[:, t:t + 1])[0]


def _kappa(view, tris: np.ndarray, pixels: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """kappa = 1/|g . N_hat| of each (pixel, winner) pair, FP64."""
    W, H = view.width, view.height
    if W * H <= 4_000_000:
        dirs, _ = oracle.perspective_map(view)
        g = dirs.reshape(-1, 3)[pixels]
    else:
        g = np.stack([_pixel_dir(view, int(p)) for p in pixels]) if len(pixels) else np.zeros((0, 3))
    n = _plane_normals(tris[:, ids.astype(np.int64)])
    return 1.0 / np.maximum(np.abs(np.einsum("ij,ij->i", g, n)), 1e-300)


def _behind_band_triangles(view, tris: np.ndarray, p: int, winner: int, choice: int, r_choice: float,
                           rounds: int = 8) -> bool:
    """Is `choice` (depth r_choice) the nearest triangle at pixel p, within
    2e-5, once triangles that lie within the edge band at p are set aside?
    The oracle's winner, and each next winner in turn while it too lies
    within the band, is removed (made degenerate, so it covers nothing) and
    the pixel rendered again."""
    t = np.array(tris, dtype=np.float32, copy=True)
    w = winner
    for _ in range(rounds):
        e, _, _ = oracle.pair(view, tris, w, p)
        if not np.any(np.abs(e) < BAND):
            return False  # a triangle clearly covering p lies in front
        t[:, w] = 0.0
        ref = oracle.render(view, t, np.array([p], dtype=np.int64))
        w = int(ref.id[0])
        if w == choice or (w != oracle.NO_HIT and r_choice <= float(ref.depth[0]) * (1 + 2e-5)):
            return True
        if w == oracle.NO_HIT:
            return False
    return False


def _pixel_dir(view, p: int) -> np.ndarray:
    i, j = p % view.width, p // view.width
    g, _, _ = oracle.lens_direction(view, (i + 0.5) / view.width, (j + 0.5) / view.height)
    return view.rot_matrix() @ g
