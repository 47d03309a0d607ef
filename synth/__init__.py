"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and builds input arrays (vertex
positions, view parameters, pixel samples, arrival times).  It holds none of
the rasterization method's arithmetic: no perspective map, no edge planes, no
depth.  Every array is drawn in float64 with numpy's PCG64 generator
(``numpy.random.default_rng(seed)``) and rounded once to float32.

Triangle arrays are structure-of-arrays ``float32[9, T]`` with rows
``ax, ay, az, bx, by, bz, cx, cy, cz``; vertices are relative to the
projection origin O.  A triangle's id is its column index.  Scenes put the
enclosing icosphere first (ids 0..1279) and the random triangles after it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# Views
# ----------------------------------------------------------------------------

AOV_HORIZONTAL, AOV_DIAGONAL, AOV_VERTICAL, AOV_HORIZONTAL_4X3 = 0, 1, 2, 3


LENS_UNIVERSAL, LENS_EQUIRECT, LENS_CUBE, LENS_SCREENS, LENS_VR, LENS_PANORAMA, LENS_DOME = 0, 1, 2, 3, 4, 5, 6


@dataclasses.dataclass
class View:
    """View request (camera frame: +x right, +y down, +z forward; ``rot`` is
    the row-major camera->world rotation).  ``lens`` selects the map
    generator (LENS_*; k, l, s, omega_deg and aov belong to the Universal
    Perspective one), ``lens_n`` and ``lens_p`` are its parameters."""

    width: int
    height: int
    k: float
    l: float
    s: float
    omega_deg: float
    aov: int = AOV_HORIZONTAL
    rot: Tuple[float, ...] = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    lens: int = LENS_UNIVERSAL
    lens_n: int = 1
    lens_p: Tuple[float, ...] = ()

    def rot_matrix(self) -> np.ndarray:
        return np.asarray(self.rot, dtype=np.float64).reshape(3, 3)


def yaw_pitch_rotation(yaw: float, pitch: float) -> Tuple[float, ...]:
    """Camera->world rotation: pitch about the camera x axis, then yaw about
    the world y axis (row-major, float32-representable values)."""
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    ry = np.array([[cy, 0.0, sy], [0.0, 1.0, 0.0], [-sy, 0.0, cy]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, cp, -sp], [0.0, sp, cp]])
    m = (ry @ rx).astype(np.float32).astype(np.float64)
    return tuple(float(v) for v in m.reshape(-1))


def view_small() -> View:
    """256x256 map, k=0.32, l=0.62, s=0.86, horizontal 270 degrees."""
    return View(256, 256, 0.32, 0.62, 0.86, 270.0)


def views_1080p_sweep() -> List[View]:
    """1920x1080, l=0.5, s=1; k=1 at 90 degrees, k in {0.5, 0, -0.5} at 180."""
    out = [View(1920, 1080, 1.0, 0.5, 1.0, 90.0)]
    for k in (0.5, 0.0, -0.5):
        out.append(View(1920, 1080, k, 0.5, 1.0, 180.0))
    return out


def views_1080p_batch(n: int = 64) -> List[View]:
    """The benchmark's batch: view q has the lens of views_1080p_sweep()[q % 4]
    (4 distinct lenses), yaw 2 pi (q // 4) / (n // 4) and pitch asin(U[-0.5,
    0.5]) (seed 1234)."""
    sweep = views_1080p_sweep()
    rng = np.random.default_rng(1234)
    out = []
    for q in range(n):
        base = sweep[q % 4]
        yaw = 2 * math.pi * (q // 4) / max(1, n // 4)
        pitch = math.asin(rng.uniform(-0.5, 0.5))
        out.append(View(base.width, base.height, base.k, base.l, base.s, base.omega_deg, base.aov,
                        yaw_pitch_rotation(yaw, pitch)))
    return out


def view_4k() -> View:
    """3840x2160 map with the 256x256 case's lens parameters."""
    return View(3840, 2160, 0.32, 0.62, 0.86, 270.0)


BATCH_RESOLUTIONS = ((512, 512), (1024, 768), (1920, 1080), (2048, 1024))
SERVE_RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080), (4096, 2048))


def random_views(n: int, seed: int, resolutions=BATCH_RESOLUTIONS) -> List[View]:
    """Views with a random resolution from ``resolutions``, k~U[-1,1],
    l~U[0,1], s~U[0,1], omega~U[90,360] degrees, yaw~U[0,2pi),
    pitch=asin(U[-1,1]), no roll.  Parameters are NOT clamped here."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        k = float(np.float32(rng.uniform(-1.0, 1.0)))
        l = float(np.float32(rng.uniform(0.0, 1.0)))
        s = float(np.float32(rng.uniform(0.0, 1.0)))
        om = float(np.float32(rng.uniform(90.0, 360.0)))
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        pitch = math.asin(rng.uniform(-1.0, 1.0))
        out.append(View(w, h, k, l, s, om, AOV_HORIZONTAL, yaw_pitch_rotation(yaw, pitch)))
    return out


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: exponential gaps."""
    rng = np.random.default_rng(seed)
    n_guess = int(rate_hz * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_guess))
    while t[-1] < duration_s:
        more = t[-1] + np.cumsum(rng.exponential(1.0 / rate_hz, size=n_guess))
        t = np.concatenate([t, more])
    return t[t < duration_s]


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------

def _to_soa(a: np.ndarray, b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Stack [T,3] float64 vertex arrays into float32[9, T] (one rounding)."""
    out = np.empty((9, a.shape[0]), dtype=np.float32)
    out[0:3] = a.T
    out[3:6] = b.T
    out[6:9] = c.T
    return out


def icosphere(subdivisions: int = 3, radius: float = 10.0) -> np.ndarray:
    """Regular icosahedron, each face split 4-way ``subdivisions`` times with
    the new vertices pushed to the sphere.  Vertices are shared by index, so
    a shared edge has bit-identical endpoints in both faces; faces are wound
    consistently.  Returns float32[9, 20*4**subdivisions]."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
             (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
             (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdivisions):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    v = (np.array(verts) * radius).astype(np.float32).astype(np.float64)
    f = np.array(faces)
    return _to_soa(v[f[:, 0]], v[f[:, 1]], v[f[:, 2]])


def icosphere_vertex_count(subdivisions: int = 3) -> int:
    return 10 * 4 ** subdivisions + 2


def _unit_vectors(rng, n: int) -> np.ndarray:
    u = rng.normal(size=(n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def shell_triangles(n: int, seed: int, r_min: float = 1.0, r_max: float = 8.0,
                    sigma: float = 0.25) -> np.ndarray:
    """Random triangles: centroid direction uniform on the sphere, centroid
    radius uniform in the volume of the shell r_min..r_max, each vertex the
    centroid plus an isotropic N(0, sigma^2) offset.  float32[9, n]."""
    rng = np.random.default_rng(seed)
    u = _unit_vectors(rng, n)
    q = rng.uniform(0.0, 1.0, size=n)
    rho = np.cbrt(r_min ** 3 + q * (r_max ** 3 - r_min ** 3))
    c = u * rho[:, None]
    offs = rng.normal(0.0, sigma, size=(3, n, 3))
    return _to_soa(c + offs[0], c + offs[1], c + offs[2])


def small_triangles(n: int, seed: int, d_min: float = 1.0, d_max: float = 50.0,
                    edge_mean: float = 0.02, edge_sd: float = 0.005) -> np.ndarray:
    """Small near-equilateral triangles of angular edge ~N(edge_mean,
    edge_sd^2) rad (clipped at 1e-3), at a distance uniform in d_min..d_max,
    facing direction uniform on the sphere, random in-plane rotation."""
    rng = np.random.default_rng(seed)
    u = _unit_vectors(rng, n)
    d = rng.uniform(d_min, d_max, size=n)
    e = np.maximum(rng.normal(edge_mean, edge_sd, size=n), 1e-3)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, size=n)
    # tangent basis: cross with the axis least aligned with u
    ax = np.zeros_like(u)
    ax[np.arange(n), np.argmin(np.abs(u), axis=1)] = 1.0
    t1 = np.cross(u, ax)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(u, t1)
    rad = np.tan(e / math.sqrt(3.0))
    vs = []
    for j in range(3):
        ang = phi0 + 2.0 * math.pi * j / 3.0
        v = u + rad[:, None] * (np.cos(ang)[:, None] * t1 + np.sin(ang)[:, None] * t2)
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        vs.append(v * d[:, None])
    return _to_soa(vs[0], vs[1], vs[2])


def scene(n_random: int, seed: int, kind: str = "shell", sphere_radius: float = 10.0) -> np.ndarray:
    """Icosphere (subdivision 3) of ``sphere_radius`` followed by ``n_random``
    triangles of the given kind ("shell" or "small")."""
    ico = icosphere(3, sphere_radius)
    if n_random == 0:
        return ico
    if kind == "shell":
        rnd = shell_triangles(n_random, seed)
    elif kind == "small":
        rnd = small_triangles(n_random, seed)
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(np.concatenate([ico, rnd], axis=1))


def scene_small() -> np.ndarray:
    """Radius-10 icosphere + 500 shell triangles, seed 0 (1,780 triangles)."""
    return scene(500, 0, "shell", 10.0)


def scene_1m() -> np.ndarray:
    """Radius-100 icosphere + 1,000,000 small triangles, seed 1."""
    return scene(1_000_000, 1, "small", 100.0)


def scene_4m() -> np.ndarray:
    """Radius-10 icosphere + 4,000,000 shell triangles, seed 2."""
    return scene(4_000_000, 2, "shell", 10.0)


def scene_500k() -> np.ndarray:
    """Radius-10 icosphere + 500,000 shell triangles, seed 3."""
    return scene(500_000, 3, "shell", 10.0)


SERVE_SCENE_SIZES = (100_000, 1_000_000, 2_000_000)
SERVE_SCENE_SEEDS = (5, 6, 7)
SERVE_ARRIVAL_SEED = 8


def serve_scenes() -> List[np.ndarray]:
    return [scene(n, s, "shell", 10.0) for n, s in zip(SERVE_SCENE_SIZES, SERVE_SCENE_SEEDS)]


# ----------------------------------------------------------------------------
# Pixel samples for parity at full size
# ----------------------------------------------------------------------------

def particles(n: int, seed: int, d_min: float = 1.0, d_max: float = 50.0,
              ang_mean: float = 0.02, ang_sd: float = 0.005) -> np.ndarray:
    """float32[4, n] spheres (x, y, z, radius): direction uniform on the
    sphere, distance U(d_min, d_max), angular diameter ~N(ang_mean, ang_sd^2)
    clipped at 1e-3 rad (the small-triangle recipe's angular size)."""
    rng = np.random.default_rng(seed)
    u = _unit_vectors(rng, n)
    d = rng.uniform(d_min, d_max, size=n)
    e = np.maximum(rng.normal(ang_mean, ang_sd, size=n), 1e-3)
    out = np.empty((4, n))
    out[0:3] = (u * d[:, None]).T
    out[3] = d * np.sin(e / 2)
    return out.astype(np.float32)


def particles_1m() -> np.ndarray:
    """10^6 particles, seed 9 (the 1080p particle workload)."""
    return particles(1_000_000, 9)


def vertex_attributes(n_tri: int, seed: int) -> np.ndarray:
    """Per-vertex data ``float32[3, 5, T]`` (vertex, attribute, triangle):
    attributes 0..2 a unit normal per vertex (a random direction per
    triangle plus a per-vertex random offset of 0.3, renormalised), 3..4 a
    texture coordinate uniform in [0, 1]^2."""
    rng = np.random.default_rng(seed)
    base = rng.normal(size=(n_tri, 3))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    out = np.empty((3, 5, n_tri), dtype=np.float64)
    for v in range(3):
        nv = base + 0.3 * rng.normal(size=(n_tri, 3))
        nv /= np.linalg.norm(nv, axis=1, keepdims=True)
        out[v, 0:3] = nv.T
        out[v, 3:5] = rng.uniform(0.0, 1.0, size=(2, n_tri))
    return out.astype(np.float32)


def pixel_sample(width: int, height: int, seed: int, n_tiles: int = 64, tile: int = 16,
                 n_pixels: int = 16384) -> np.ndarray:
    """Sorted unique flat pixel indices (j*W+i): every pixel of ``n_tiles``
    random tile x tile blocks plus ``n_pixels`` random pixels."""
    rng = np.random.default_rng(seed)
    idx = []
    tx_n, ty_n = max(1, width // tile), max(1, height // tile)
    for _ in range(n_tiles):
        tx, ty = int(rng.integers(tx_n)), int(rng.integers(ty_n))
        ii, jj = np.meshgrid(np.arange(tx * tile, min(width, tx * tile + tile)),
                             np.arange(ty * tile, min(height, ty * tile + tile)))
        idx.append((jj * width + ii).reshape(-1))
    idx.append(rng.integers(0, width * height, size=n_pixels))
    return np.unique(np.concatenate(idx).astype(np.int64))
