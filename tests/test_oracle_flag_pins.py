"""Pins of the oracle's ambiguity flags, the rule that decides which pixels
are excused from the bit-exact triangle-id comparison.

The flags are built from geometry constructed around one pixel whose view
direction is known in closed form: a 16x16 pinhole view (k = 1, l = s = 1,
horizontal angle of view 90 degrees, section 2.1.2) looks along
g = (x, y, 1)/|(x, y, 1)| with x = (2i + 1 - W)/W, y = (2j + 1 - H)/W.  A
triangle is placed so that one of its edge planes passes at a chosen angle
from g; the angle and the depths are then recomputed here in FP64 from the
FP32-rounded vertices (not by the oracle), and the flags must follow:

  * EDGE   when a triangle whose depth is within 1e-5 of the winner's (or
           with no winner) passes within 1e-6 rad of one of its edge
           planes, on either side, and within the band of the other two;
  * DEPTH  when the two nearest covered depths differ by at most 2e-5 r;
  * DOMAIN within 1e-6 of the edge of a k < 0 projection's domain,
           |sin(k Omega/2) R| = 1 (section 2.1.2), reported apart from EDGE;
  * INVALID where the projection gives no direction.

A band ten times too wide or too narrow, a depth window of 1e-4 instead of
1e-5, an edge test on one side only, or a domain test on R instead of
|sin(k Omega/2) R| each fails one of these pins.
"""
import math

import numpy as np
import pytest

import synth

W = H = 16
PIX = (5, 9)  # column i, row j


def _view():
    return synth.View(W, H, 1.0, 1.0, 1.0, 90.0, 0)


def _g(i=PIX[0], j=PIX[1]):
    x, y = (2 * i + 1 - W) / W, (2 * j + 1 - H) / W
    v = np.array([x, y, 1.0])
    return v / np.linalg.norm(v)


def _edge_triangle(g, eps, R, shift=0.0):
    """Vertices A, B on the plane through O whose unit normal n satisfies
    n . g = sin(eps) (g on the positive side for eps > 0), C on that side.
    With shift > 0.3 the edge AB, and the triangle, end before reaching g
    (g then lies near AB's great circle but beyond the segment)."""
    u = np.cross(g, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    w = np.cross(g, u)
    m = -math.sin(eps) * u + math.cos(eps) * g  # in the plane, next to g
    a = R * (m + (shift + 0.3) * w)
    b = R * (m + (shift - 0.3) * w)
    c = R * (g + shift * w + 0.3 * u)
    return np.concatenate([a, b, c])


def _background(z0):
    """A large triangle in the plane z = z0 around the view axis."""
    return np.array([-50, -40, z0, 60, -30, z0, 0, 70, z0], dtype=np.float64)


def _soa(*tris):
    return np.ascontiguousarray(np.stack(tris, axis=1).astype(np.float32))


def _measure(tris32, t, g):
    """FP64 signed angle of g from triangle t's nearest edge plane (positive
    inside), the smaller signed angle of the other two, and the ray-plane
    depth, from the rounded vertices."""
    v = tris32[:, t].astype(np.float64)
    a, b, c = v[0:3], v[3:6], v[6:9]
    sig = np.sign(np.dot(a, np.cross(b, c)))
    ang = []
    for p, q in ((a, b), (b, c), (c, a)):
        n = sig * np.cross(p, q)
        ang.append(math.asin(np.dot(n, g) / np.linalg.norm(n)))
    nn = np.cross(a - b, c - b)
    r = np.dot(a, nn) / np.dot(g, nn)
    near = min(ang, key=abs)
    others = sorted(ang, key=abs)[1:]
    return near, min(others), r


def _flags(oracle_lib, tris32):
    p = PIX[1] * W + PIX[0]
    res = oracle_lib.render(_view(), tris32, np.array([p], dtype=np.int64))
    return int(res.flags[0]), int(res.id[0]), float(res.depth[0])


def test_pinhole_direction_closed_form(oracle_lib):
    dirs, ok = oracle_lib.perspective_map(_view())
    assert ok.all()
    assert np.allclose(dirs[PIX[1], PIX[0]], _g(), atol=1e-15)


@pytest.mark.parametrize("eps,covered,flagged", [
    (0.5e-6, True, True), (2e-6, True, False), (-0.5e-6, False, True), (-2e-6, False, False),
    (0.09e-6, True, True), (12e-6, True, False)])
def test_edge_band_of_the_winner(oracle_lib, eps, covered, flagged):
    g = _g()
    tris = _soa(_edge_triangle(g, eps, 3.0))
    ang, second, r = _measure(tris, 0, g)
    # the rounded vertices keep the designed angle to a few 1e-8 rad, and
    # the other two edges are far from g
    assert abs(ang - eps) < 0.05e-6 and second > 1e-3
    f, tid, _ = _flags(oracle_lib, tris)
    assert (tid == 0) == covered
    assert bool(f & oracle_lib.FLAG_EDGE) == flagged
    assert not f & (oracle_lib.FLAG_DEPTH | oracle_lib.FLAG_DOMAIN | oracle_lib.FLAG_INVALID)


@pytest.mark.parametrize("eps,gap,edge,depth_flag", [
    (0.5e-6, 0.3e-5, True, True),    # covering competitor just behind: both
    (-0.5e-6, 0.3e-5, True, False),  # missing it by 0.5e-6 rad, just behind
    (0.5e-6, 0.8e-5, True, True),    # inside the 1e-5 window
    (2e-6, 0.3e-5, False, True),     # outside the band: only the depth tie
    (0.5e-6, 3e-5, False, False),    # farther than 1e-5 (and 2e-5): never
    (-0.5e-6, 1.5e-5, False, False),  # farther than 1e-5, missing
    (0.5e-6, 1.5e-5, False, True),   # band, but farther than 1e-5; depth tie within 2e-5
])
def test_edge_band_of_a_competitor(oracle_lib, eps, gap, edge, depth_flag):
    g = _g()
    z0 = 4.0
    r0 = z0 / g[2]
    # the competitor's depth along g is R (1 + O(eps)): place it at the gap
    tris = _soa(_background(z0), _edge_triangle(g, eps, r0 * (1 + gap)))
    _, _, r0m = _measure(tris, 0, g)
    ang, _, r1 = _measure(tris, 1, g)
    assert abs(ang - eps) < 0.05e-6
    assert abs((r1 - r0m) / r0m - gap) < 0.05e-5
    f, tid, d = _flags(oracle_lib, tris)
    assert tid == 0 and d == pytest.approx(r0m, rel=1e-12)
    assert bool(f & oracle_lib.FLAG_EDGE) == edge
    assert bool(f & oracle_lib.FLAG_DEPTH) == depth_flag
    assert not f & (oracle_lib.FLAG_DOMAIN | oracle_lib.FLAG_INVALID)


@pytest.mark.parametrize("eps", [0.5e-6, -0.5e-6])
def test_edge_band_needs_the_segment(oracle_lib, eps):
    """Near the great circle of an edge but beyond its end (far outside
    another edge of the triangle): no flag."""
    g = _g()
    tris = _soa(_edge_triangle(g, eps, 3.0, shift=0.5))
    ang, second, _ = _measure(tris, 0, g)
    # AB's great circle passes 0.5e-6 rad from g, and g is far outside
    # another edge
    assert abs(ang - eps) < 0.05e-6 and second < -1e-2
    f, tid, _ = _flags(oracle_lib, tris)
    assert tid == oracle_lib.NO_HIT and f == 0


def test_competitor_in_front_in_the_band_wins_and_flags(oracle_lib):
    g = _g()
    z0 = 4.0
    r0 = z0 / g[2]
    tris = _soa(_background(z0), _edge_triangle(g, 0.5e-6, 0.5 * r0))
    f, tid, _ = _flags(oracle_lib, tris)
    assert tid == 1 and f & oracle_lib.FLAG_EDGE
    tris = _soa(_background(z0), _edge_triangle(g, 3e-6, 0.5 * r0))
    f, tid, _ = _flags(oracle_lib, tris)
    assert tid == 1 and f == 0
    # a near competitor missing by 0.5e-6 rad: the winner behind it could
    # lose to it in FP32
    tris = _soa(_background(z0), _edge_triangle(g, -0.5e-6, 0.5 * r0))
    f, tid, _ = _flags(oracle_lib, tris)
    assert tid == 0 and f & oracle_lib.FLAG_EDGE


def _domain_view(delta, k=-1.0, om=180.0, kq=None):
    """16x16 view, s = 1, l chosen so that the four corner pixels have
    |sin(kq Omega/2)| R = 1 + delta (kq = k unless given)."""
    kq = k if kq is None else kq
    x = y = (W - 1) / W
    R = (1.0 + delta) / abs(math.sin(kq * math.radians(om) / 2))
    l = (R * R - x * x) / (y * y)
    assert 0.0 <= l <= 1.0
    return synth.View(W, H, k, l, 1.0, om, 0), l


def _domain_q(l, k=-1.0, om=180.0):
    i, j = np.meshgrid(np.arange(W), np.arange(H))
    x, y = (2 * i + 1 - W) / W, (2 * j + 1 - H) / W
    return math.sin(k * math.radians(om) / 2) * np.sqrt(x * x + l * y * y)


@pytest.mark.parametrize("k,om", [(-1.0, 180.0), (-0.5, 270.0)])
@pytest.mark.parametrize("delta,flagged", [(0.5e-6, True), (-0.5e-6, True), (0.09e-6, True),
                                           (2e-6, False), (-2e-6, False), (-12e-6, False)])
def test_domain_edge_flag(oracle_lib, delta, flagged, k, om):
    view, l = _domain_view(delta, k, om)
    q = _domain_q(l, k, om)
    near = np.abs(np.abs(q) - 1.0) < 1e-6
    res = oracle_lib.render(view, np.zeros((9, 0), np.float32))
    f = res.flags.reshape(H, W)
    dom = (f & oracle_lib.FLAG_DOMAIN) != 0
    assert np.array_equal(dom, near)
    corners = np.zeros((H, W), bool)
    corners[[0, 0, -1, -1], [0, -1, 0, -1]] = True
    assert np.array_equal(dom, corners if flagged else np.zeros_like(corners))
    # invalid exactly where |q| > 1, and the domain flag is not an edge flag
    assert np.array_equal((f & oracle_lib.FLAG_INVALID) != 0, np.abs(q) > 1.0)
    assert not np.any(f & oracle_lib.FLAG_EDGE)


def test_domain_edge_flag_needs_negative_k(oracle_lib):
    # the same picture geometry at k = 0 (equidistant: every pixel valid)
    view, l = _domain_view(0.5e-6, k=0.0, kq=-1.0)
    res = oracle_lib.render(view, np.zeros((9, 0), np.float32))
    assert not np.any(res.flags & (oracle_lib.FLAG_DOMAIN | oracle_lib.FLAG_INVALID))
