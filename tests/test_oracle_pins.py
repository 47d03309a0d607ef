"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against one of: values the paper states
(tests/golden), textbook closed forms of the named azimuthal projections, the
paper's second (rectilinear) formula, the paper's 3D->2D inverse, a LAPACK
linear solve, the classic 2D edge-function rasterizer on pinhole-projected
vertices, and invariances every correct renderer has.  None of them re-types
the oracle's own formula.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- limits --

def test_limits_match_paper_table(oracle_lib):
    g = _gold("limits.json")
    for row in g["omega_max_deg"]:
        k, l, s, om = oracle_lib.limits(row["k"], 0.5, 0.9, 1e9)
        assert om == pytest.approx(row["omega_max"], abs=1e-12), row
    for row in g["clamps"]:
        out = oracle_lib.limits(*row["in"])
        assert np.allclose(out, row["out"], atol=1e-12), (row, out)


# ------------------------------------------------------------------- map --

def test_map_unit_length(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(40):
        k, l, s = rng.uniform(-1, 1), rng.uniform(0, 1), rng.uniform(0, 1)
        om = rng.uniform(20, 360)
        w, h = int(rng.integers(3, 40)), int(rng.integers(3, 40))
        v = synth.View(w, h, k, l, s, om, int(rng.integers(0, 4)))
        d, ok = oracle_lib.perspective_map(v)
        n = np.linalg.norm(d, axis=-1)
        assert np.all(np.abs(n[ok] - 1.0) < 1e-14)
        assert np.all(n[~ok] == 0.0)
        # a float32-rounded rotation is orthonormal to ~1e-7
        v.rot = synth.yaw_pitch_rotation(rng.uniform(0, 6), rng.uniform(-1.5, 1.5))
        d2, ok2 = oracle_lib.perspective_map(v)
        assert np.array_equal(ok, ok2)
        assert np.all(np.abs(np.linalg.norm(d2, axis=-1)[ok] - 1.0) < 3e-7)


def _rectilinear(fs, ft, a, omega_deg, aov):
    """Rectilinear map of section 2.2.1 (its own formula, per AOV type)."""
    cot = 1.0 / math.tan(math.radians(omega_deg) / 2)
    if aov == synth.AOV_HORIZONTAL:
        v = np.array([2 * fs - 1, (2 * ft - 1) / a, cot])
    elif aov == synth.AOV_DIAGONAL:
        q = math.sqrt(a * a + 1)
        v = np.array([a * (2 * fs - 1) / q, (2 * ft - 1) / q, cot])
    else:
        v = np.array([a * (2 * fs - 1), 2 * ft - 1, cot])
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("aov", [synth.AOV_HORIZONTAL, synth.AOV_DIAGONAL, synth.AOV_VERTICAL])
@pytest.mark.parametrize("omega", [40.0, 90.0, 150.0, 178.0])
def test_k1_is_the_rectilinear_map(oracle_lib, aov, omega):
    w, h = 37, 23
    for l in (0.0, 0.3, 1.0):
        v = synth.View(w, h, 1.0, l, 1.0, omega, aov)
        d, ok = oracle_lib.perspective_map(v)
        assert ok.all()
        for j in range(h):
            for i in range(0, w, 5):
                ref = _rectilinear((i + 0.5) / w, (j + 0.5) / h, w / h, omega, aov)
                assert np.max(np.abs(d[j, i] - ref)) < 1e-13


def _fisheye(name, rho, omega):
    """Textbook angle from the axis for image radius rho (rho=1 at Omega/2)."""
    if name == "gnomonic":
        return math.atan(rho * math.tan(omega / 2))
    if name == "stereographic":
        return 2 * math.atan(rho * math.tan(omega / 4))
    if name == "equidistant":
        return rho * omega / 2
    if name == "equisolid":
        return 2 * math.asin(rho * math.sin(omega / 4))
    if name == "orthographic":
        return math.asin(rho * math.sin(omega / 2))
    raise KeyError(name)


@pytest.mark.parametrize("omega_deg", [60.0, 120.0, 170.0])
def test_named_projections_closed_forms(oracle_lib, omega_deg):
    rng = np.random.default_rng(3)
    for row in _gold("projection_types.json")["types"]:
        k, name = row["k"], row["name"]
        _, _, _, om = oracle_lib.limits(k, 1.0, 1.0, omega_deg)
        for _ in range(200):
            x, y = rng.uniform(-1, 1, size=2)
            rho = math.hypot(x, y)
            if rho > 1.0:
                continue
            g, ok = oracle_lib.direction(x, y, k, 1.0, 1.0, om)
            assert ok
            want = _fisheye(name, rho, math.radians(om))
            assert math.acos(max(-1.0, min(1.0, g[2]))) == pytest.approx(want, abs=1e-12)
            assert math.atan2(g[1], g[0]) == pytest.approx(math.atan2(y, x), abs=1e-12)


def test_orthographic_outside_domain_is_invalid(oracle_lib):
    # k=-1, Omega=180: sin(Omega/2)*R > 1 for R > 1 (corner of a wide frame)
    g, ok = oracle_lib.direction(1.2, 0.5, -1.0, 1.0, 1.0, 180.0)
    assert not ok and np.all(g == 0)
    g, ok = oracle_lib.direction(0.6, 0.5, -1.0, 1.0, 1.0, 180.0)
    assert ok


def test_round_trip_through_paper_inverse(oracle_lib):
    """Section 2.1.3 inverts 2.1.2 when l(1-s)+s = 1 (s=1 here), any l."""
    rng = np.random.default_rng(5)
    n = 0
    for _ in range(600):
        k = rng.uniform(-1, 1)
        l = rng.uniform(0, 1)
        kk, ll, ss, om = oracle_lib.limits(k, l, 1.0, rng.uniform(30, 300))
        x, y = rng.uniform(-1, 1), rng.uniform(-0.6, 0.6)
        g, ok = oracle_lib.direction(x, y, kk, ll, ss, om)
        if not ok or math.acos(max(-1, min(1, g[2] / math.sqrt(g[0]**2 + ll * g[1]**2 + g[2]**2)))) > 3.1:
            continue
        xx, yy = oracle_lib.inverse(g, kk, ll, ss, om)
        assert xx == pytest.approx(x, abs=1e-9) and yy == pytest.approx(y, abs=1e-9), (kk, ll, om, x, y)
        n += 1
    assert n > 300


def test_cylindrical_meridians_and_anamorphic_scale(oracle_lib):
    """l=0 is cylindrical: a column of the picture lies on one great circle
    through the vertical poles; s rescales the vertical coordinate only."""
    rng = np.random.default_rng(9)
    up = np.array([0.0, 1.0, 0.0])
    for _ in range(100):
        k = rng.uniform(-1, 1)
        kk, ll, ss, om = oracle_lib.limits(k, 0.0, rng.uniform(0.8, 1.0), rng.uniform(30, 170))
        x = rng.uniform(-0.9, 0.9)
        y1, y2 = rng.uniform(-0.8, 0.8, size=2)
        g1, ok1 = oracle_lib.direction(x, y1, kk, ll, ss, om)
        g2, ok2 = oracle_lib.direction(x, y2, kk, ll, ss, om)
        assert ok1 and ok2
        assert abs(np.linalg.det(np.stack([g1, g2, up]))) < 1e-13
        h, okh = oracle_lib.direction(x, y1 / ss, kk, ll, 1.0, om)
        assert okh and np.max(np.abs(h - g1)) < 1e-13


def test_spherical_ignores_anamorphic(oracle_lib):
    """With l = 1 there is no anamorphic correction: s has no effect."""
    rng = np.random.default_rng(10)
    for _ in range(100):
        kk, ll, _, om = oracle_lib.limits(rng.uniform(-1, 1), 1.0, 1.0, rng.uniform(30, 300))
        x, y = rng.uniform(-0.7, 0.7, size=2)
        a, oka = oracle_lib.direction(x, y, kk, 1.0, 1.0, om)
        b, okb = oracle_lib.direction(x, y, kk, 1.0, 0.8, om)
        assert oka == okb
        assert np.max(np.abs(a - b)) < 1e-15


def test_horizontal_4x3_at_4x3_aspect(oracle_lib):
    """'Horizontal 4x3' on a 4:3 picture is the horizontal AOV."""
    for i, j in [(0, 0), (7, 3), (15, 11), (3, 9)]:
        a = oracle_lib.view_coord(i, j, 16, 12, synth.AOV_HORIZONTAL)
        b = oracle_lib.view_coord(i, j, 16, 12, synth.AOV_HORIZONTAL_4X3)
        assert a == pytest.approx(b, abs=1e-15)


# ---------------------------------------------------- coverage and depth --

def _solve_weights(tri, g):
    """Weights w with [A B C] w = g (LAPACK via numpy.linalg.solve)."""
    m = np.stack([tri[0:3], tri[3:6], tri[6:9]], axis=1).astype(np.float64)
    return np.linalg.solve(m, g)


def test_coverage_and_depth_match_linear_solve(oracle_lib):
    """g lies inside the triangle's cone iff g = aA + bB + cC with a,b,c > 0,
    and then the ray hits the triangle at r = 1/(a+b+c)."""
    rng = np.random.default_rng(21)
    tris = synth.shell_triangles(40, 77)
    view = synth.View(160, 120, 0.4, 0.7, 0.9, 300.0, 0,
                      synth.yaw_pitch_rotation(0.7, -0.3))
    dirs, ok = oracle_lib.perspective_map(view)
    checked = covered = 0
    flat = dirs.reshape(-1, 3)
    for t in range(tris.shape[1]):
        cen = tris[:, t].astype(np.float64).reshape(3, 3).sum(axis=0)
        near = np.argsort(-(flat @ cen))[:30]  # pixels looking at the triangle
        for p in np.concatenate([near, rng.integers(0, view.width * view.height, size=30)]):
            e, r, valid = oracle_lib.pair(view, tris, t, p)
            g = dirs.reshape(-1, 3)[p]
            w = _solve_weights(tris[:, t], g)
            inside = bool(np.all(w > 0))
            if np.min(np.abs(w)) < 1e-9:
                continue
            assert (np.all(e > 0)) == inside
            checked += 1
            if inside:
                covered += 1
                assert r == pytest.approx(1.0 / w.sum(), rel=1e-10)
    assert checked > 1000 and covered > 20


def test_winner_matches_linear_solve_bruteforce(oracle_lib):
    tris = synth.shell_triangles(25, 31)
    view = synth.View(20, 16, -0.3, 0.5, 0.85, 250.0, 0, synth.yaw_pitch_rotation(2.0, 0.4))
    res = oracle_lib.render(view, tris)
    dirs, ok = oracle_lib.perspective_map(view)
    for j in range(view.height):
        for i in range(view.width):
            g = dirs[j, i]
            best, best_t = math.inf, 0xFFFFFFFF
            for t in range(tris.shape[1]):
                w = _solve_weights(tris[:, t], g)
                if np.all(w > 0):
                    r = 1.0 / w.sum()
                    if r < best:
                        best, best_t = r, t
            assert res.id[j, i] == best_t
            if best_t != 0xFFFFFFFF:
                assert res.depth[j, i] == pytest.approx(best, rel=1e-10)


def test_pinhole_edge_functions_at_k1(oracle_lib):
    """k=1, s=1 is a pinhole camera: coverage equals the 2D edge-function
    test on the perspective-projected vertices (all in front, z > 0)."""
    W, H, om = 64, 36, 90.0
    view = synth.View(W, H, 1.0, 0.5, 1.0, om)
    rng = np.random.default_rng(4)
    t_f = math.tan(math.radians(om) / 2)
    n_checked = 0
    for trial in range(30):
        c = np.array([rng.uniform(-1, 1), rng.uniform(-0.5, 0.5), rng.uniform(2, 4)])
        tri = np.concatenate([c + rng.normal(0, 0.6, 3) for _ in range(3)])
        tri[2::3] = np.abs(tri[2::3]) + 0.5
        tris = np.ascontiguousarray(tri.astype(np.float32).reshape(9, 1))
        res = oracle_lib.render(view, tris)
        verts = tris[:, 0].astype(np.float64).reshape(3, 3)
        uv = [((W / 2) * (1 + X / (Z * t_f)), H / 2 + (W / 2) * Y / (Z * t_f)) for X, Y, Z in verts]

        def edge(a, b, p):
            return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])

        for j in range(H):
            for i in range(W):
                p = (i + 0.5, j + 0.5)
                e = [edge(uv[0], uv[1], p), edge(uv[1], uv[2], p), edge(uv[2], uv[0], p)]
                if min(abs(x) for x in e) < 1e-6:
                    continue
                inside = all(x > 0 for x in e) or all(x < 0 for x in e)
                assert (res.cover[j, i] == 1) == inside, (trial, i, j)
                n_checked += 1
    assert n_checked > 60000


def test_icosphere_covers_every_pixel_exactly_once(oracle_lib):
    """A closed, consistently wound surface around O: every pixel outside
    the edge band is covered by exactly one face, and the depth is the
    distance to that face's plane, between the inner and outer radius."""
    R = 10.0
    ico = synth.icosphere(3, R)
    for view in (synth.view_small(), synth.View(96, 64, -0.5, 0.2, 0.9, 360.0, 0,
                                                 synth.yaw_pitch_rotation(1.1, 0.6))):
        res = oracle_lib.render(view, ico)
        valid = (res.flags & oracle_lib.FLAG_INVALID) == 0
        clean = valid & ((res.flags & oracle_lib.FLAG_EDGE) == 0)
        assert np.all(res.cover[clean] == 1)
        assert clean.sum() > 0.99 * valid.sum()
        # inner radius: distance from O to the nearest face plane
        a = ico[0:3].T.astype(np.float64)
        b = ico[3:6].T.astype(np.float64)
        c = ico[6:9].T.astype(np.float64)
        n = np.cross(b - a, c - a)
        inner = np.min(np.abs(np.einsum("ij,ij->i", a, n)) / np.linalg.norm(n, axis=1))
        d = res.depth[clean]
        assert np.all(d <= R * (1 + 1e-6)) and np.all(d >= inner * (1 - 1e-12))
        dirs, _ = oracle_lib.perspective_map(view)
        hit = dirs[clean] * d[:, None]
        tid = res.id[clean].astype(np.int64)
        w = np.einsum("ij,ij->i", hit - a[tid], n[tid])
        assert np.max(np.abs(w) / np.linalg.norm(n[tid], axis=1)) < 1e-9


def test_plane_depth_closed_form(oracle_lib):
    """A big triangle in the plane z = z0 around the view axis: every
    covered pixel has r = z0 / g_z."""
    z0 = 3.0
    tri = np.array([-50, -40, z0, 60, -30, z0, 0, 70, z0], dtype=np.float32).reshape(9, 1)
    view = synth.View(40, 30, 0.5, 1.0, 1.0, 120.0)
    res = oracle_lib.render(view, tri)
    dirs, _ = oracle_lib.perspective_map(view)
    assert np.all(res.id == 0)
    assert np.allclose(res.depth, z0 / dirs[..., 2], rtol=1e-13)


def test_invariances(oracle_lib):
    tris = synth.shell_triangles(600, 8)
    view = synth.View(96, 80, 0.2, 0.6, 0.9, 260.0, 0, synth.yaw_pitch_rotation(0.3, 0.2))
    base = oracle_lib.render(view, tris)
    valid = (base.flags & (oracle_lib.FLAG_EDGE | oracle_lib.FLAG_DEPTH)) == 0
    assert (base.id != oracle_lib.NO_HIT).sum() > 400
    # 1. rotate the scene and the view together (non-symmetric rotation)
    q = np.array(synth.yaw_pitch_rotation(1.3, -0.7)).reshape(3, 3)
    rt = np.empty_like(tris, dtype=np.float64)
    for v in range(3):
        rt[3 * v:3 * v + 3] = q @ tris[3 * v:3 * v + 3].astype(np.float64)
    view_r = synth.View(view.width, view.height, view.k, view.l, view.s, view.omega_deg, 0,
                        tuple((q @ view.rot_matrix()).reshape(-1)))
    # the rotated vertices are rounded to float32; compare loosely on depth
    rot = oracle_lib.render(view_r, rt.astype(np.float32))
    same = valid & (rot.flags & (oracle_lib.FLAG_EDGE | oracle_lib.FLAG_DEPTH) == 0)
    assert np.mean(rot.id[same] == base.id[same]) > 0.999
    hit = same & (base.id != oracle_lib.NO_HIT) & (rot.id == base.id)
    assert np.allclose(rot.depth[hit], base.depth[hit], rtol=1e-6)
    # 2. uniform scale: same ids, depth scales exactly (power of two)
    sc = oracle_lib.render(view, (tris * np.float32(4.0)))
    assert np.array_equal(sc.id, base.id)
    h = base.id != oracle_lib.NO_HIT
    assert np.allclose(sc.depth[h], 4.0 * base.depth[h], rtol=1e-14)
    # 3. vertex order: cyclic shift and reversed winding change nothing
    cyc = np.concatenate([tris[3:9], tris[0:3]])
    rev = np.concatenate([tris[0:3], tris[6:9], tris[3:6]])
    for t2 in (cyc, rev):
        r2 = oracle_lib.render(view, np.ascontiguousarray(t2))
        assert np.array_equal(r2.id[valid], base.id[valid])
        assert np.allclose(r2.depth[h & valid], base.depth[h & valid], rtol=1e-12)


def test_depth_ties_go_to_lower_id(oracle_lib):
    tri = synth.shell_triangles(3, 2)
    tri[:, 1] = [-50, -40, 3, 60, -30, 3, 0, 70, 3]  # big, in front of the camera
    dup = np.ascontiguousarray(np.concatenate([tri, tri[:, 1:2]], axis=1))  # id 3 == id 1
    view = synth.View(40, 40, 0.0, 1.0, 1.0, 360.0)
    res = oracle_lib.render(view, dup)
    assert not np.any(res.id == 3)
    assert np.any(res.id == 1)
    assert np.all(res.flags[res.id == 1] & oracle_lib.FLAG_DEPTH)


def test_degenerate_triangles_cover_nothing(oracle_lib):
    # a triangle whose plane contains O, and one with two equal vertices
    t1 = np.array([1, 0, 0, 0, 1, 0, 1, 1, 0], dtype=np.float32)
    t2 = np.array([1, 2, 3, 1, 2, 3, -1, 0, 2], dtype=np.float32)
    tris = np.ascontiguousarray(np.stack([t1, t2], axis=1))
    res = oracle_lib.render(synth.View(32, 32, 0.0, 1.0, 1.0, 360.0), tris)
    assert np.all(res.id == oracle_lib.NO_HIT)


# ---------------------------------------------------------- bounding cap --

def test_smallest_circle_cap_contains_spherical_triangle(oracle_lib):
    """Section 1.1.2 cap: every vertex direction and every direction inside
    the spherical triangle lies in the cap; the rim passes through all three
    vertices (acute) or through the longest edge's endpoints (obtuse)."""
    rng = np.random.default_rng(12)
    tris = synth.shell_triangles(300, 13).astype(np.float64)
    for t in range(tris.shape[1]):
        A, B, C = tris[0:3, t], tris[3:6, t], tris[6:9, t]
        S, cosr = oracle_lib.cap(A, B, C)
        assert 0.0 < cosr <= 1.0 and abs(np.linalg.norm(S) - 1) < 1e-14
        units = [x / np.linalg.norm(x) for x in (A, B, C)]
        dots = np.array([u @ S for u in units])
        assert np.all(dots >= cosr - 1e-12)
        on_rim = np.abs(dots - cosr) < 1e-9
        assert on_rim.sum() >= 2
        w = rng.dirichlet([1, 1, 1], size=64)
        inner = w @ np.stack(units)
        inner /= np.linalg.norm(inner, axis=1, keepdims=True)
        assert np.all(inner @ S >= cosr - 1e-12)


# -------------------------------------------------------- fragment data --

def test_fragment_barycentrics_match_linear_solve(oracle_lib):
    """Section 1.1.4 fragment data against LAPACK: with [A B C] w = g, the
    ray meets the plane at P = g / sum(w) = sum(w_i V_i) / sum(w), so the
    barycentric weights are w / sum(w); an attribute that is an affine
    function of position interpolates to its value at P; the normal pass is
    unit length."""
    tris = synth.scene(60, 41)
    view = synth.View(96, 72, 0.3, 0.6, 0.9, 260.0, 0, synth.yaw_pitch_rotation(0.4, 0.2))
    res = oracle_lib.render(view, tris)
    pix = np.flatnonzero(res.id.reshape(-1) != 0xFFFFFFFF)
    ids = res.id.reshape(-1)[pix]
    rng = np.random.default_rng(5)
    T = tris.shape[1]
    verts = tris.astype(np.float64).reshape(3, 3, T)            # [vertex, xyz, t]
    M, c = rng.normal(size=(2, 3)), rng.normal(size=2)
    aff = np.einsum("kx,vxt->vkt", M, verts) + c[None, :, None]  # affine in position
    attr = np.concatenate([synth.vertex_attributes(T, 7).astype(np.float64), aff], axis=1)
    b, f = oracle_lib.fragments(view, tris, attr.astype(np.float32), pix, ids, normalize3=True)
    b2, f2 = oracle_lib.fragments(view, tris, aff.astype(np.float32), pix, ids)
    dirs, ok = oracle_lib.perspective_map(view)
    flat = dirs.reshape(-1, 3)
    a32 = aff.astype(np.float32).astype(np.float64)
    for q in range(0, len(pix), 7):
        t, g = int(ids[q]), flat[pix[q]]
        w = _solve_weights(tris[:, t], g)
        assert np.allclose(b[q], w / w.sum(), rtol=1e-9, atol=1e-9), (q, b[q], w / w.sum())
        assert b[q].sum() == pytest.approx(1.0, abs=1e-11)
        assert b[q].min() > -1e-11                      # covered: inside the triangle
        P = g / w.sum()
        assert np.allclose(b[q] @ verts[:, :, t], P, rtol=1e-9, atol=1e-9)
        exp = a32[:, :, t].T @ b[q]                      # same weights on the float32 data
        assert np.allclose(f2[q], exp, rtol=1e-9, atol=1e-9)
        assert np.allclose(f2[q], M @ P + c, rtol=1e-5, atol=1e-5)  # float32 rounding of the data
        assert np.linalg.norm(f[q, 0:3]) == pytest.approx(1.0, abs=1e-12)
    assert len(pix) > 2000


def test_fragment_at_a_vertex_is_that_vertex(oracle_lib):
    """A pixel looking straight at vertex A gets b = (1, 0, 0) and A's data."""
    view = synth.View(64, 48, -0.2, 0.8, 0.9, 200.0, 0)
    dirs, ok = oracle_lib.perspective_map(view)
    p = 23 * 64 + 40
    g = dirs.reshape(-1, 3)[p]
    A = 7.0 * g
    B = A + np.array([1.0, 0.2, 0.1])
    C = A + np.array([0.1, 1.0, 0.3])
    tris = np.concatenate([A, B, C]).reshape(9, 1).astype(np.float32)
    attr = synth.vertex_attributes(1, 3)
    b, f = oracle_lib.fragments(view, tris, attr, np.array([p]), np.array([0], dtype=np.uint32))
    assert np.allclose(b[0], [1.0, 0.0, 0.0], atol=1e-6)
    assert np.allclose(f[0], attr[0, :, 0], atol=1e-6)
    # no hit, or a pixel without direction: zeros
    b, f = oracle_lib.fragments(view, tris, attr, np.array([p]), np.array([0xFFFFFFFF], dtype=np.uint32))
    assert not b.any() and not f.any()
