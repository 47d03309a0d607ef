"""Pins of the oracle's wire-frame (section 1.2) and particle (section 1.3)
rasterization, aliasing-free with the global delta (1.1.1), particles
combined front to back (1.4).

Expected values come from outside the oracle: the exact overlap of a
one-pixel strip with a pixel square (a tent), the box coverage of a
pinhole-projected disc by supersampling, the disc's area, the geometry of a
sphere's silhouette cone, invariance under vertex order, and
min(1, sum of masks).
"""
import math

import numpy as np
import pytest

import synth

NO_HIT = 0xFFFFFFFF


def _tri(*verts):
    return np.concatenate([np.asarray(v, dtype=np.float64) for v in verts]).astype(np.float32).reshape(9, 1)


def _tris(*tris):
    return np.ascontiguousarray(np.concatenate(tris, axis=1))


def _pinhole(W, H, om=40.0):
    return synth.View(W, H, 1.0, 0.5, 1.0, om), math.tan(math.radians(om) / 2)


# -------------------------------------------------------------- wire frame

@pytest.mark.parametrize("frac", [0.0, 0.3, 0.5, -0.65])
def test_line_along_a_column_is_a_one_pixel_strip(oracle_lib, frac):
    """A side along a picture column: each pixel gets the overlap of a
    one-pixel-wide strip centred on the line with its square,
    1 - min(|i + 1/2 - u|, 1) (the pixel-smooth line step), near the centre
    of a pinhole view; the other two sides are out of view."""
    W = H = 64
    view, t_f = _pinhole(W, H)
    u = W / 2 + frac
    X = (2 * u / W - 1) * t_f
    res = oracle_lib.wireframe(view, _tri((X, -5, 1), (X, 5, 1), (X + 5, 0, 1)))
    cols = np.arange(W // 2 - 4, W // 2 + 4)
    want = 1 - np.minimum(np.abs(cols + 0.5 - u), 1.0)
    for row in range(H // 2 - 2, H // 2 + 2):
        assert np.allclose(res.cov[row, cols], want, atol=5e-3), (row, res.cov[row, cols], want)
    assert np.all(res.dom[res.cov > 0] == 0) and np.all(res.dom[res.cov == 0] == NO_HIT)


def test_segment_ends_at_its_end_points(oracle_lib):
    """The cap around the segment cuts the line at its end points: a pixel
    centred 1.2 px beyond an end on the line gets nothing (its square does
    not reach the segment), one 2 px inside the segment gets the full strip."""
    W = H = 64
    view, t_f = _pinhole(W, H)
    Z = 2.0

    def P(u, v):
        return ((2 * u / W - 1) * t_f * Z, (v - H / 2) * 2 / W * t_f * Z, Z)

    a, b = (20.0, 32.5), (44.3, 32.5)   # horizontal side, through the centres of row 32
    tri = _tri(P(*a), P(*b), P(32.0, 5.0))
    res = oracle_lib.wireframe(view, tri)
    assert res.cov[32, 45] == 0.0          # centre 45.5: 1.2 px beyond the end at 44.3
    assert res.cov[32, 42] == pytest.approx(1.0, abs=1e-3)
    assert res.cov[32, 21] == pytest.approx(1.0, abs=1e-3)


def test_wire_interior_is_empty_and_order_free(oracle_lib):
    """Pixels more than a pixel from every side get nothing; the image does
    not depend on the vertex order or winding; a shared side is drawn once
    (the lower id)."""
    W = H = 48
    view, t_f = _pinhole(W, H, 50.0)
    A, B, C = (-0.3, -0.25, 1.5), (0.35, -0.2, 1.6), (0.0, 0.3, 1.4)
    r0 = oracle_lib.wireframe(view, _tri(A, B, C))
    for perm in ((B, C, A), (A, C, B), (C, B, A)):
        r1 = oracle_lib.wireframe(view, _tri(*perm))
        assert np.allclose(r0.cov, r1.cov, atol=1e-12)
    # interior: rasterized coverage of the triangle two pixels inside
    hard = oracle_lib.render(view, _tri(A, B, C))
    dirs, _ = oracle_lib.perspective_map(view)
    far = 0
    for j in range(H):
        for i in range(W):
            if hard.id[j, i] != 0:
                continue
            g = dirs[j, i]
            d = oracle_lib.delta(view, i, j)
            # angular distance to each side's great circle, in pixels
            V = [np.array(x) / np.linalg.norm(x) for x in (A, B, C)]
            dist = min(abs(g @ (np.cross(V[k], V[(k + 1) % 3]) / np.linalg.norm(np.cross(V[k], V[(k + 1) % 3]))))
                       for k in range(3)) * d
            if dist > 1.05:
                far += 1
                assert r0.cov[j, i] == 0.0
    assert far > 50
    # D shares side B-C with the first triangle
    D = (0.5, 0.35, 1.5)
    two = oracle_lib.wireframe(view, _tris(_tri(A, B, C), _tri(C, B, D)))
    rd = oracle_lib.wireframe(view, _tri(C, B, D))
    assert np.array_equal(two.cov, np.maximum(r0.cov, rd.cov))
    tie = (r0.cov == rd.cov) & (r0.cov > 0)          # pixels whose largest mask is the shared side
    assert tie.sum() > 10 and np.all(two.dom[tie] == 0)
    assert np.all(two.dom[rd.cov > r0.cov] == 1)


# ---------------------------------------------------------------- particles

def _disc_box_coverage(W, H, t_f, R_img, ss=16):
    """Box-filter coverage of the image disc of radius R_img (pixels) centred
    in the picture, by ss x ss supersampling of each pixel square."""
    o = (np.arange(ss) + 0.5) / ss
    cov = np.zeros((H, W))
    cx, cy = W / 2, H / 2
    for j in range(H):
        for i in range(W):
            u = i + o[None, :] - cx
            v = j + o[:, None] - cy
            cov[j, i] = np.mean(u * u + v * v < R_img * R_img)
    return cov


def test_particle_is_the_projected_disc(oracle_lib):
    """A sphere on the axis of a pinhole view projects to a circle of radius
    f tan(rho), sin(rho) = r/|P|: each pixel's mask is close to the box
    coverage of that disc and the masks add up to its area."""
    W = H = 96
    view, t_f = _pinhole(W, H, 50.0)
    P, r = 5.0, 0.6
    rho = math.asin(r / P)
    R_img = (W / 2) * math.tan(rho) / t_f
    pr = np.array([[0.0], [0.0], [P], [r]], dtype=np.float32)
    res = oracle_lib.particles(view, pr)
    box = _disc_box_coverage(W, H, t_f, R_img)
    assert np.max(np.abs(res.cov - box)) < 0.06
    assert res.cov.sum() == pytest.approx(math.pi * R_img ** 2, rel=0.01)
    assert np.all(res.dom[res.cov > 0] == 0)


def test_particle_texture_coordinates(oracle_lib):
    """The texture plane is perpendicular to P: |uv - (1/2, 1/2)| equals
    sin(angle(g, P)) |P| / (2r), so the silhouette (sin = r/|P|) maps to the
    circle inscribed in the unit square; the centre direction maps to the
    square's centre; uv turns with g around P from the X axis
    (P_z, 0, -P_x)."""
    W, H = 81, 61
    view = synth.View(W, H, 0.5, 0.5, 1.0, 120.0, 0, synth.yaw_pitch_rotation(0.4, -0.3))
    Rm = view.rot_matrix()
    Pdir = Rm @ np.array([0.0, 0.0, 1.0])             # the centre pixel's direction
    P = 7.0 * Pdir
    r = 2.0
    pr = np.array([[P[0]], [P[1]], [P[2]], [r]], dtype=np.float32)
    res = oracle_lib.particles(view, pr)
    Pf = pr[:3, 0].astype(np.float64)
    Ph = Pf / np.linalg.norm(Pf)
    X = np.array([Pf[2], 0.0, -Pf[0]])
    X /= np.linalg.norm(X)
    Y = np.cross(X, Ph)
    dirs, _ = oracle_lib.perspective_map(view)
    inside = res.cov > 0.999
    assert inside.sum() > 200
    for j, i in zip(*np.nonzero(inside)):
        g = dirs[j, i]
        d = res.uv[j, i] - 0.5
        sin_a = np.linalg.norm(np.cross(g, Ph))
        assert np.linalg.norm(d) == pytest.approx(sin_a * np.linalg.norm(Pf) / (2 * r), abs=1e-9)
        assert np.linalg.norm(d) <= 0.5 + 1e-9
        if sin_a > 1e-3:
            perp = g - (g @ Ph) * Ph
            assert math.atan2(d[1], d[0]) == pytest.approx(math.atan2(perp @ Y, perp @ X), abs=1e-9)
    c = res.uv[H // 2, W // 2]
    assert np.allclose(c, [0.5, 0.5], atol=1e-6)


def test_nearer_particle_hides_the_farther(oracle_lib):
    """Two particles on one axis: where both cover fully the pixel is the
    nearer one's (coverage 1, its plane depth |P| / (g . P_hat), its texture
    coordinates), whatever the ids; coverage is min(1, sum of the single
    masks) everywhere."""
    W = H = 64
    view, t_f = _pinhole(W, H, 40.0)
    near = [0.0, 0.0, 4.0, 0.5]
    far = [0.05, 0.0, 6.0, 0.9]
    dirs, _ = oracle_lib.perspective_map(view)
    for order in ((far, near), (near, far)):
        pr = np.array(order, dtype=np.float32).T.copy()
        res = oracle_lib.particles(view, pr)
        nid = order.index(near)
        single = [oracle_lib.particles(view, pr[:, k:k + 1]) for k in range(2)]
        assert np.allclose(res.cov, np.minimum(1.0, single[0].cov + single[1].cov), atol=1e-12)
        both = (single[0].cov == 1.0) & (single[1].cov == 1.0)
        assert both.sum() > 50
        Pn = np.array(near[:3], dtype=np.float32).astype(np.float64)
        for j, i in zip(*np.nonzero(both)):
            g = dirs[j, i]
            assert res.dom[j, i] == nid
            assert res.depth[j, i] == pytest.approx(np.linalg.norm(Pn) ** 2 / (g @ Pn), rel=1e-12)
            assert np.allclose(res.uv[j, i], single[nid].uv[j, i], atol=1e-12)


def test_skipped_particles(oracle_lib):
    view, _ = _pinhole(16, 16)
    pr = np.array([[0, 0, 5, 0.0], [0, 0, 0.5, 1.0], [0, 0, 5, -1.0]], dtype=np.float32).T.copy()
    res = oracle_lib.particles(view, pr)
    assert not res.cov.any() and np.all(res.dom == NO_HIT)


def test_duplicate_particles_tie_to_lower_id(oracle_lib):
    """Two copies of one particle: equal depths and masks; the lower id goes
    first, so where m < 1/2 both get the same share and the lower id is
    dominant; coverage is min(1, 2m)."""
    view, _ = _pinhole(48, 48, 50.0)
    one = oracle_lib.particles(view, np.array([[0.1], [0.0], [5.0], [0.7]], dtype=np.float32))
    two = oracle_lib.particles(view, np.array([[0.1, 0.1], [0.0, 0.0], [5.0, 5.0], [0.7, 0.7]], dtype=np.float32))
    assert np.allclose(two.cov, np.minimum(1.0, 2 * one.cov), atol=1e-15)
    fringe = (one.cov > 0) & (one.cov < 0.5)
    assert fringe.sum() > 10 and np.all(two.dom[one.cov > 0] == 0)
