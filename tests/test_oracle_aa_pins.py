"""Pins of the oracle's aliasing-free coverage (sections 1.1.1, 1.1.2, 1.4).

The expected values come from outside the oracle: the derivative of the
textbook projections (pixel pitch of the map), the box-filter coverage of a
pixel square by an axis-aligned half-plane, perspective-projected areas
(shoelace), ray-plane depths by LAPACK, and invariants that any correct
front-to-back combination has (a closed surface covers every pixel, shared
edges sum to one, coverage is min(1, sum of masks)).
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NO_HIT = 0xFFFFFFFF


def _radial(name, theta):
    """Textbook image radius of a named azimuthal projection (r'(0) = 1)."""
    return {
        "gnomonic": math.tan(theta),
        "stereographic": 2 * math.tan(theta / 2),
        "equidistant": theta,
        "equisolid": 2 * math.sin(theta / 2),
        "orthographic": math.sin(theta),
    }[name]


def _angle(name, rho, omega):
    """Textbook angle from the axis at image radius rho (rho = 1 at Omega/2)."""
    return {
        "gnomonic": lambda: math.atan(rho * math.tan(omega / 2)),
        "stereographic": lambda: 2 * math.atan(rho * math.tan(omega / 4)),
        "equidistant": lambda: rho * omega / 2,
        "equisolid": lambda: 2 * math.asin(rho * math.sin(omega / 4)),
        "orthographic": lambda: math.asin(rho * math.sin(omega / 2)),
    }[name]()


def _tri(*verts):
    return np.concatenate([np.asarray(v, dtype=np.float64) for v in verts]).astype(np.float32).reshape(9, 1)


def _tris(*tris):
    return np.ascontiguousarray(np.concatenate(tris, axis=1))


def _pinhole_xy(W, t_f, u, v, H, Z=1.0):
    """3D point at depth Z seen at pixel position (u, v) of a horizontal-AOV
    pinhole view (pixel centres at i + 1/2)."""
    return np.array([(2 * u / W - 1) * Z * t_f, (v - H / 2) * 2 / W * Z * t_f, Z])


# ------------------------------------------------------------ global delta --

@pytest.mark.parametrize("omega_deg", [60.0, 120.0, 170.0])
def test_delta_is_reciprocal_pixel_pitch_at_centre(oracle_lib, omega_deg):
    """At the centre pixel of an odd-sized named projection the horizontal
    neighbours look at angle theta(2/W) left and right, the vertical ones
    up and down, so the central differences of G_x and G_y are
    sin(theta(2/W)) and that of G_z is 0: delta = 1 / sin(theta(2/W)).  For
    fine pixels this is the reciprocal of the angular pixel pitch
    (2/W) r(Omega/2)."""
    with open(os.path.join(GOLD, "projection_types.json")) as f:
        types = json.load(f)["types"]
    W = H = 101
    for row in types:
        _, _, _, om = oracle_lib.limits(row["k"], 1.0, 1.0, omega_deg)
        view = synth.View(W, H, row["k"], 1.0, 1.0, om)
        exact = 1.0 / math.sin(_angle(row["name"], 2.0 / W, math.radians(om)))
        assert oracle_lib.delta(view, 50, 50) == pytest.approx(exact, rel=1e-9), row
        pitch = W / (2 * _radial(row["name"], math.radians(om) / 2))
        assert oracle_lib.delta(view, 50, 50) == pytest.approx(pitch, rel=3e-2), row
    fine = synth.View(1001, 1001, 0.0, 1.0, 1.0, 90.0)
    assert oracle_lib.delta(fine, 500, 500) == pytest.approx(1001 / (math.pi / 2), rel=1e-6)


def test_delta_matches_pinhole_jacobian(oracle_lib):
    """k=1 is a pinhole: G = v/|v|, v = (x, y, cot); the derivative per pixel
    is (I - G G^T) dv/|v| with dv = 2/W along either axis; delta is
    1 / max_c (|dG_c/di| + |dG_c/dj|).  Central differences agree to O(h^2)
    inside the picture, one-sided ones to O(h) on its border."""
    W, H, om = 121, 91, 70.0
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    cot = 1.0 / math.tan(math.radians(om) / 2)
    rng = np.random.default_rng(2)
    pts = [(int(rng.integers(1, W - 1)), int(rng.integers(1, H - 1))) for _ in range(60)]
    border = [(0, 0), (W - 1, 45), (60, 0), (60, H - 1), (W - 1, H - 1)]
    for i, j in pts + border:
        v = np.array([(2 * i + 1 - W) / W, (2 * j + 1 - H) / W, cot])
        n = np.linalg.norm(v)
        G = v / n
        P = (np.eye(3) - np.outer(G, G)) / n
        di, dj = P @ np.array([2 / W, 0, 0]), P @ np.array([0, 2 / W, 0])
        want = 1.0 / np.max(np.abs(di) + np.abs(dj))
        tol = 3e-2 if (i, j) in border else 2e-3
        assert oracle_lib.delta(view, i, j) == pytest.approx(want, rel=tol), (i, j)


def test_delta_is_zero_without_direction(oracle_lib):
    # orthographic, 180 degrees: the frame's corners are outside the domain
    view = synth.View(64, 64, -1.0, 1.0, 1.0, 180.0)
    assert oracle_lib.delta(view, 0, 0) == 0.0
    assert oracle_lib.delta(view, 32, 32) > 0.0


# ---------------------------------------------------------- pixel step ramp --

@pytest.mark.parametrize("frac", [0.0, 0.25, 0.5, 0.8, -0.35])
def test_axis_aligned_edge_is_box_filter_coverage(oracle_lib, frac):
    """An edge along a picture column of a pinhole view: the pixel step gives
    each pixel the fraction of its square on the covered side,
    clamp(i + 1 - u_edge, 0, 1) (exact box filter for an axis-aligned edge),
    near the view centre where the perspective is locally affine."""
    W = H = 64
    om = 40.0
    t_f = math.tan(math.radians(om) / 2)
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    u_e = W / 2 + frac
    X = (2 * u_e / W - 1) * t_f
    right = _tri((X, -5, 1), (X, 5, 1), (X + 5, 0, 1))
    flipped = _tri((X, 5, 1), (X, -5, 1), (X + 5, 0, 1))      # other winding
    left = _tri((X, -5, 1), (X, 5, 1), (X - 5, 0, 1))
    rows = slice(H // 2 - 2, H // 2 + 2)
    cols = np.arange(W // 2 - 4, W // 2 + 4)
    want = np.clip(cols + 1 - u_e, 0, 1)
    a = oracle_lib.aa_render(view, right)
    b = oracle_lib.aa_render(view, flipped)
    c = oracle_lib.aa_render(view, left)
    for row in range(rows.start, rows.stop):
        assert np.allclose(a.cov[row, cols], want, atol=5e-3), (row, a.cov[row, cols], want)
        assert np.allclose(c.cov[row, cols], 1 - want, atol=5e-3)
    assert np.array_equal(a.cov, b.cov)
    # a horizontal edge: the same along rows
    v_e = H / 2 + frac
    Y = (v_e - H / 2) * 2 / W * t_f
    down = oracle_lib.aa_render(view, _tri((-5, Y, 1), (5, Y, 1), (0, Y + 5, 1)))
    rows_i = np.arange(H // 2 - 4, H // 2 + 4)
    want_v = np.clip(rows_i + 1 - v_e, 0, 1)
    for col in range(W // 2 - 2, W // 2 + 2):
        assert np.allclose(down.cov[rows_i, col], want_v, atol=5e-3)


def test_coverage_mass_is_projected_area(oracle_lib):
    """The ramps are odd about each edge, so the summed coverage of a
    triangle equals its area in pixels (pinhole projection maps it to a 2D
    triangle, shoelace area) up to corner terms of a fraction of a pixel."""
    W, H, om = 96, 80, 50.0
    t_f = math.tan(math.radians(om) / 2)
    view = synth.View(W, H, 1.0, 0.7, 1.0, om)
    rng = np.random.default_rng(8)
    n = 0
    while n < 12:
        Z = rng.uniform(2, 5, size=3)
        uv = np.stack([rng.uniform(20, W - 20, size=3), rng.uniform(18, H - 18, size=3)], axis=1)
        area = 0.5 * abs((uv[1, 0] - uv[0, 0]) * (uv[2, 1] - uv[0, 1]) - (uv[2, 0] - uv[0, 0]) * (uv[1, 1] - uv[0, 1]))
        sides = [np.linalg.norm(uv[a] - uv[b]) for a, b in ((0, 1), (1, 2), (2, 0))]
        if area < 150 or min(sides) < 12:
            continue
        verts = [_pinhole_xy(W, t_f, uv[q, 0], uv[q, 1], H, Z[q]) for q in range(3)]
        tris = _tri(*verts)
        # projected area of the float32-rounded vertices
        v32 = tris[:, 0].astype(np.float64).reshape(3, 3)
        p = np.array([[(W / 2) * (1 + x / (z * t_f)), H / 2 + (W / 2) * y / (z * t_f)] for x, y, z in v32])
        area = 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1]))
        res = oracle_lib.aa_render(view, tris)
        assert res.cov.sum() == pytest.approx(area, rel=0.015, abs=1.0), (n, area)
        n += 1


# ------------------------------------------------------------- miter mask --

def test_miter_cuts_a_sliver_tip(oracle_lib):
    """An isosceles sliver with an 8 degree apex: the apex lies on the
    smallest circle's rim with the axis along the radius, so a pixel centred
    1.2 px beyond the apex on the axis gets no coverage (its square does not
    reach the triangle: box coverage 0).  The edge steps alone would give it
    about 0.4.  Well inside the sliver the coverage is 1."""
    W, H, om = 96, 64, 40.0
    t_f = math.tan(math.radians(om) / 2)
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    pi, pj = 70, 31
    apex = (pi + 0.5 - 1.2, pj + 0.5)
    L, half = 40.0, math.radians(4.0)
    b1 = (apex[0] - L, apex[1] - L * math.tan(half))
    b2 = (apex[0] - L, apex[1] + L * math.tan(half))
    verts = [_pinhole_xy(W, t_f, u, v, H, 3.0) for u, v in (apex, b1, b2)]
    res = oracle_lib.aa_render(view, _tri(*verts))
    assert res.cov[pj, pi] == 0.0
    # what the three edge steps alone give there (delta at the pixel)
    d = oracle_lib.delta(view, pi, pj)
    dirs, _ = oracle_lib.perspective_map(view)
    g = dirs[pj, pi]
    vs = [np.asarray(v) for v in verts]
    steps = []
    for a, b in ((0, 1), (1, 2), (2, 0)):
        n = np.cross(vs[a], vs[b])
        n *= np.sign(np.linalg.det(np.stack(vs))) / np.linalg.norm(n)
        steps.append(min(1.0, max(0.0, d * (n @ g) + 0.5)))
    assert min(steps) > 0.3
    # interior: at two thirds of the length the sliver is 3.7 px wide
    ci, cj = int(apex[0] - 2 * L / 3), pj
    assert res.cov[cj, ci] == pytest.approx(1.0, abs=1e-12)


# ------------------------------------------------------ front-to-back (1.4) --

def _plane_depth(tris, t, g):
    m = np.stack([tris[0:3, t], tris[3:6, t], tris[6:9, t]], axis=1).astype(np.float64)
    return 1.0 / np.linalg.solve(m, g).sum()


def test_full_cover_layers(oracle_lib):
    """Two triangles each covering the whole view: coverage 1, the depth and
    the dominant id of the nearer plane, whatever the id order."""
    W, H, om = 40, 30, 60.0
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    back = _tri((-20, -20, 3), (20, -20, 3.5), (0, 30, 2.5))
    front = _tri((-20, -20, 2), (20, -20, 2.2), (0, 30, 1.6))
    dirs, _ = oracle_lib.perspective_map(view)
    for tris, front_id in ((_tris(back, front), 1), (_tris(front, back), 0)):
        res = oracle_lib.aa_render(view, tris)
        assert np.all(res.cov == 1.0)
        assert np.all(res.dom == front_id)
        for j in range(0, H, 5):
            for i in range(0, W, 5):
                assert res.depth[j, i] == pytest.approx(_plane_depth(tris, front_id, dirs[j, i]), rel=1e-12)


@pytest.mark.parametrize("frac", [0.2, 0.7])
def test_partial_front_over_full_back(oracle_lib, frac):
    """A front triangle whose edge crosses a pixel with box coverage m1 over
    a full back triangle: coverage 1, depth m1 r1 + (1 - m1) r2, dominant id
    the larger share.  Swapped depths: the full triangle in front hides the
    partial one completely."""
    W = H = 64
    om = 40.0
    t_f = math.tan(math.radians(om) / 2)
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    u_e = W / 2 + frac
    X = (2 * u_e / W - 1) * t_f
    dirs, _ = oracle_lib.perspective_map(view)
    for zf, zb in ((2.0, 4.0), (4.0, 2.0)):
        part = _tri((X * zf, -5, zf), (X * zf, 5, zf), (X * zf + 5, 0, zf))
        full = _tri((-20, -20, zb), (20, -20, zb), (0, 30, zb))
        tris = _tris(full, part)
        res = oracle_lib.aa_render(view, tris)
        for j in range(H // 2 - 2, H // 2 + 2):
            for i in range(W // 2 - 3, W // 2 + 4):
                m1 = min(1.0, max(0.0, i + 1 - u_e))
                r1, r2 = _plane_depth(tris, 1, dirs[j, i]), _plane_depth(tris, 0, dirs[j, i])
                assert res.cov[j, i] == pytest.approx(1.0, abs=1e-12)
                if zf < zb:
                    assert res.depth[j, i] == pytest.approx(m1 * r1 + (1 - m1) * r2, abs=5e-3 * (r2 - r1))
                    assert res.dom[j, i] == (1 if m1 > 0.5 else 0)
                else:
                    assert res.depth[j, i] == pytest.approx(r2, rel=1e-12)
                    assert res.dom[j, i] == 0


def test_coverage_is_min_one_sum_of_masks(oracle_lib):
    """Whatever the depth order, m_b after all fragments is min(1, sum of the
    fragment masks); each mask is what the triangle covers alone."""
    view = synth.View(48, 40, 0.4, 0.7, 0.9, 160.0, 0, synth.yaw_pitch_rotation(0.3, -0.2))
    rng = np.random.default_rng(17)
    Rm = view.rot_matrix()
    cols = []
    for _ in range(40):
        # a triangle of about 0.6 rad a few units in front of the camera
        c = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.6, 0.6), 1.0]) * rng.uniform(2, 6)
        verts = [Rm @ (c + rng.normal(0, 0.3 * np.linalg.norm(c), 3)) for _ in range(3)]
        cols.append(_tri(*verts))
    tris = _tris(*cols)
    total = np.zeros((view.height, view.width))
    for t in range(tris.shape[1]):
        one = oracle_lib.aa_render(view, np.ascontiguousarray(tris[:, t:t + 1]))
        assert np.all((one.cov == 0) | (one.dom == 0))
        total += one.cov
    res = oracle_lib.aa_render(view, tris)
    assert np.allclose(res.cov, np.minimum(1.0, total), atol=1e-12)
    assert (total > 1.0).sum() > 20 and ((total > 0) & (total < 1)).sum() > 20


def test_shared_edge_is_seamless(oracle_lib):
    """Two coplanar triangles sharing a diagonal: their masks sum to one
    across it, so pixels away from the outer outline get coverage 1 and the
    plane's depth; one triangle alone is fractional along the diagonal."""
    W, H, om = 64, 64, 50.0
    t_f = math.tan(math.radians(om) / 2)
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    Z = 3.0
    c = [(10.0, 12.0), (54.0, 9.0), (57.0, 50.0), (8.0, 55.0)]
    P = [_pinhole_xy(W, t_f, u, v, H, Z) for u, v in c]
    t1, t2 = _tri(P[0], P[1], P[2]), _tri(P[0], P[2], P[3])
    both = oracle_lib.aa_render(view, _tris(t1, t2))
    one = oracle_lib.aa_render(view, t1)
    dirs, _ = oracle_lib.perspective_map(view)
    inner = 0
    diag_frac = 0
    for j in range(H):
        for i in range(W):
            u, v = i + 0.5, j + 0.5
            # distance to the outer outline (pixel units, straight lines in a pinhole view)
            dist = min(_line_dist(c[a], c[(a + 1) % 4], (u, v)) for a in range(4))
            if not _inside(c, (u, v)) or dist < 3.0:
                continue
            inner += 1
            assert both.cov[j, i] == pytest.approx(1.0, abs=1e-12)
            assert both.depth[j, i] == pytest.approx(Z / dirs[j, i][2], rel=1e-6)
            if _line_dist(c[0], c[2], (u, v)) < 0.3:
                diag_frac += 1
                assert 0.05 < one.cov[j, i] < 0.95
    assert inner > 1000 and diag_frac > 10


def _line_dist(a, b, p):
    ax, ay = a
    bx, by = b
    px, py = p
    return abs((bx - ax) * (py - ay) - (by - ay) * (px - ax)) / math.hypot(bx - ax, by - ay)


def _inside(poly, p):
    s = []
    for a in range(len(poly)):
        (ax, ay), (bx, by) = poly[a], poly[(a + 1) % len(poly)]
        s.append((bx - ax) * (p[1] - ay) - (by - ay) * (p[0] - ax))
    return all(x > 0 for x in s) or all(x < 0 for x in s)


def test_closed_surface_covers_every_pixel(oracle_lib):
    """An icosphere around O (consistent winding, shared edges): every pixel
    with a direction farther than three pixel pitches from a vertex is fully
    covered (the summed shared-edge masks), away from edges the dominant id
    is the hard render's winner and the depth its depth where one fragment
    covers fully."""
    R = 10.0
    ico = synth.icosphere(1, R)
    view = synth.View(128, 96, -0.5, 0.6, 0.9, 220.0, 0, synth.yaw_pitch_rotation(0.8, 0.5))
    res = oracle_lib.aa_render(view, ico)
    hard = oracle_lib.render(view, ico)
    dirs, ok = oracle_lib.perspective_map(view)
    vdir = ico.astype(np.float64).reshape(3, 3, -1).transpose(0, 2, 1).reshape(-1, 3)
    vdir /= np.linalg.norm(vdir, axis=1, keepdims=True)
    n_far = n_clean = 0
    for j in range(view.height):
        for i in range(view.width):
            if not ok[j, i]:
                assert res.cov[j, i] == 0.0 and res.dom[j, i] == NO_HIT and res.depth[j, i] == 0.0
                continue
            d = oracle_lib.delta(view, i, j)
            ang = math.acos(min(1.0, float(np.max(vdir @ dirs[j, i]))))
            if ang * d < 3.0:
                continue
            n_far += 1
            assert res.cov[j, i] == pytest.approx(1.0, abs=1e-12), (i, j)
            if res.margin[j, i] == 1.0:   # one fragment, fully covering
                n_clean += 1
                assert res.dom[j, i] == hard.id[j, i]
                assert res.depth[j, i] == pytest.approx(hard.depth[j, i], rel=1e-12)
    assert n_far > 0.6 * ok.sum() and n_clean > 0.3 * ok.sum()


def test_empty_scene(oracle_lib):
    view = synth.View(16, 12, 0.2, 0.5, 0.9, 200.0)
    res = oracle_lib.aa_render(view, np.zeros((9, 0), dtype=np.float32))
    assert np.all(res.cov == 0) and np.all(res.depth == 0) and np.all(res.dom == NO_HIT)


def test_duplicate_triangles_tie_to_lower_id(oracle_lib):
    """Two copies of one triangle: equal depth, equal masks.  The lower id
    goes first, so coverage is min(1, 2m) and, where m < 1/2 gives both
    copies the same clipped share, the dominant id is the lower one."""
    view = synth.View(48, 40, 1.0, 0.5, 1.0, 60.0)
    t = _tri((-0.3, -0.2, 2.0), (0.4, -0.25, 2.2), (0.05, 0.35, 1.9))
    one = oracle_lib.aa_render(view, t)
    two = oracle_lib.aa_render(view, _tris(t, t))
    assert np.allclose(two.cov, np.minimum(1.0, 2 * one.cov), atol=1e-15)
    fringe = (one.cov > 0) & (one.cov < 0.5)
    assert fringe.sum() > 20
    assert np.all(two.dom[fringe] == 0) and np.all(two.dom[one.cov > 0] == 0)
