"""Pins of the oracle's other map generators (sections 2.2.2, 2.2.4,
2.2.7-2.2.9) and the Brown-Conrady distortion (section 2.3).

Expected values come from geometry outside the generators' formulas:
meridians and parallels of a sphere, the six-face partition of a cube map,
reductions to the rectilinear Universal map (pinned on its own against the
paper's separate rectilinear formula), proper rotations recovered by an SVD
(Kabsch), continuity at screen seams, mirror symmetry of the two eyes, and
the paper's 3D->2D inverse of section 2.1.3.
"""
import math

import numpy as np
import pytest

import synth


def _map(oracle_lib, view):
    d, ok = oracle_lib.perspective_map(view)
    return d, ok


def _kabsch(P, Q):
    """Rotation R (det +1 if proper) minimising |R P_i - Q_i|; returns R and
    the largest residual."""
    U, S, Vt = np.linalg.svd(Q.T @ P)
    R = U @ Vt
    return R, float(np.max(np.linalg.norm(P @ R.T - Q, axis=1)))


# ----------------------------------------------------------- equirectangular

def test_equirect_meridians_parallels_and_longitude(oracle_lib):
    """Columns are meridians (great circles through the poles +-y), rows are
    parallels (constant y), longitude grows linearly by 2 pi / W per column
    from -pi at the left edge, the polar angle from -y by pi / H per row."""
    W, H = 64, 32
    v = synth.View(W, H, 0, 0, 0, 0, lens=synth.LENS_EQUIRECT)
    d, ok = _map(oracle_lib, v)
    assert ok.all()
    up = np.array([0.0, 1.0, 0.0])
    for i in range(W):
        col = d[:, i]
        for j in range(1, H):
            assert abs(np.linalg.det(np.stack([col[0], col[j], up]))) < 1e-14
        lon = math.atan2(col[H // 2][0], col[H // 2][2])
        want = -math.pi + 2 * math.pi * (i + 0.5) / W
        assert abs(math.remainder(lon - want, 2 * math.pi)) < 1e-13
    for j in range(H):
        assert np.ptp(d[j, :, 1]) < 1e-15
        assert math.acos(-d[j, 0, 1]) == pytest.approx(math.pi * (j + 0.5) / H, abs=1e-13)
    # the full sphere: the pixels' solid angles (sin(polar) dlon dpolar) sum to 4 pi
    polar = np.arccos(-d[:, 0, 1])
    assert np.sum(np.sin(polar)) * (2 * math.pi / W) * (math.pi / H) * W == pytest.approx(4 * math.pi, rel=1e-3)


# ------------------------------------------------------------------- cube

def test_cube_faces_partition_the_sphere(oracle_lib):
    """Six faces side by side: each face's centre is a distinct axis
    direction, and every pixel lies in the cone of its face's axis (its
    largest component is along that axis, with its sign)."""
    F = 16
    v = synth.View(6 * F, F, 0, 0, 0, 0, lens=synth.LENS_CUBE)
    d, ok = _map(oracle_lib, v)
    assert ok.all()
    axes = []
    for f in range(6):
        g, okc, seg = oracle_lib.lens_direction(v, (f + 0.5) / 6, 0.5)
        assert okc and seg == f
        ax = int(np.argmax(np.abs(g)))
        assert abs(abs(g[ax]) - 1.0) < 1e-15
        axes.append((ax, np.sign(g[ax])))
        block = d[:, f * F:(f + 1) * F].reshape(-1, 3)
        assert np.all(np.argmax(np.abs(block), axis=1) == ax)
        assert np.all(np.sign(block[:, ax]) == np.sign(g[ax]))
    assert len(set(axes)) == 6


def test_cube_faces_are_rotations_of_the_forward_pinhole(oracle_lib):
    """Face 3 is a 90-degree square rectilinear view (the Universal map at
    k = 1, Omega = 90 on an F x F picture); every other face is that view
    turned by a proper rotation (recovered by SVD, det +1, exact)."""
    F = 12
    v = synth.View(6 * F, F, 0, 0, 0, 0, lens=synth.LENS_CUBE)
    d, _ = _map(oracle_lib, v)
    front, _ = _map(oracle_lib, synth.View(F, F, 1.0, 0.5, 1.0, 90.0))
    assert np.max(np.abs(d[:, 3 * F:4 * F] - front)) < 1e-15
    P = front.reshape(-1, 3)
    for f in range(6):
        Q = d[:, f * F:(f + 1) * F].reshape(-1, 3)
        R, res = _kabsch(P, Q)
        assert res < 1e-13 and np.linalg.det(R) == pytest.approx(1.0, abs=1e-12), f


# --------------------------------------------------------- screen array

def test_one_screen_is_the_rectilinear_map(oracle_lib):
    for om in (40.0, 75.0, 120.0):
        a = synth.View(48, 30, 0, 0, 0, 0, lens=synth.LENS_SCREENS, lens_n=1, lens_p=(om,))
        b = synth.View(48, 30, 1.0, 0.5, 1.0, om)
        da, _ = _map(oracle_lib, a)
        db, _ = _map(oracle_lib, b)
        assert np.max(np.abs(da - db)) < 1e-15


@pytest.mark.parametrize("n", [2, 3, 5])
def test_screen_array_seams_and_turns(oracle_lib, n):
    """n flat screens in a ring: neighbouring screens meet at a common edge
    direction (continuity at the seam), screen s looks at azimuth
    (s - (n-1)/2) Omega, and each screen is the one-screen map of its own
    size turned about the vertical axis."""
    om = 50.0
    Ws, H = 20, 30
    v = synth.View(n * Ws, H, 0, 0, 0, 0, lens=synth.LENS_SCREENS, lens_n=n, lens_p=(om,))
    for s in range(1, n):
        for ft in (0.1, 0.5, 0.77):
            g0, _, s0 = oracle_lib.lens_direction(v, s / n - 1e-12, ft)
            g1, _, s1 = oracle_lib.lens_direction(v, s / n + 1e-12, ft)
            assert (s0, s1) == (s - 1, s)
            assert np.max(np.abs(g0 - g1)) < 1e-10
    d, _ = _map(oracle_lib, v)
    one, _ = _map(oracle_lib, synth.View(Ws, H, 0, 0, 0, 0, lens=synth.LENS_SCREENS, lens_n=1, lens_p=(om,)))
    for s in range(n):
        g, _, _ = oracle_lib.lens_direction(v, (s + 0.5) / n, 0.5)
        assert math.degrees(math.atan2(g[0], g[2])) == pytest.approx((s - (n - 1) / 2) * om, abs=1e-11)
        R, res = _kabsch(one.reshape(-1, 3), d[:, s * Ws:(s + 1) * Ws].reshape(-1, 3))
        assert res < 1e-13 and np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
        assert np.allclose(R @ np.array([0.0, 1.0, 0.0]), [0.0, 1.0, 0.0], atol=1e-13)  # about y


# ---------------------------------------------------------- virtual reality

def test_vr_eyes_mirror_and_reduce_to_rectilinear(oracle_lib):
    """The two eyes are mirror images (x -> -x); with IPD d = 1/2 and no lens
    distortion each eye is the rectilinear Universal map with vertical angle
    of view of its half of the picture; the lens axis of the left eye sits
    at fs = (1 - d)/2."""
    W, H = 64, 40
    for om, d_ipd, k1, k2 in [(90.0, 0.5, 0.0, 0.0), (100.0, 0.42, 0.22, 0.05)]:
        v = synth.View(W, H, 0, 0, 0, 0, lens=synth.LENS_VR, lens_p=(om, d_ipd, k1, k2))
        dm, ok = _map(oracle_lib, v)
        assert ok.all()
        mirror = dm[:, ::-1] * np.array([-1.0, 1.0, 1.0])
        assert np.max(np.abs(dm - mirror)) < 1e-15
        g, _, seg = oracle_lib.lens_direction(v, (1 - d_ipd) / 2, 0.5)
        assert seg == 0 and np.max(np.abs(g - [0.0, 0.0, 1.0])) < 1e-15
        if k1 == 0.0 and d_ipd == 0.5:
            eye, _ = _map(oracle_lib, synth.View(W // 2, H, 1.0, 0.5, 1.0, om, synth.AOV_VERTICAL))
            assert np.max(np.abs(dm[:, :W // 2] - eye)) < 1e-15


def test_vr_radial_distortion_scales_the_tangent_plane_radius(oracle_lib):
    """On the tangent plane at distance cot(Omega/2) the distorted point is
    the undistorted one scaled by (1 + k1 R^2 + k2 R^4)/(1 + k1 + k2)
    (radial polynomial lens model); at R = 1 nothing moves."""
    om, dd, k1, k2 = 96.0, 0.47, 0.3, -0.04
    plain = synth.View(80, 50, 0, 0, 0, 0, lens=synth.LENS_VR, lens_p=(om, dd, 0.0, 0.0))
    dist = synth.View(80, 50, 0, 0, 0, 0, lens=synth.LENS_VR, lens_p=(om, dd, k1, k2))
    cot = 1 / math.tan(math.radians(om) / 2)
    rng = np.random.default_rng(3)
    for _ in range(100):
        fs, ft = rng.uniform(0, 1), rng.uniform(0, 1)
        a, _, _ = oracle_lib.lens_direction(plain, fs, ft)
        b, _, _ = oracle_lib.lens_direction(dist, fs, ft)
        pa, pb = a[:2] / a[2] * cot, b[:2] / b[2] * cot
        R2 = pa @ pa
        assert np.allclose(pb, pa * (1 + k1 * R2 + k2 * R2 * R2) / (1 + k1 + k2), atol=1e-13)
    # R = 1: the vertical edge of the lens axis column
    a, _, _ = oracle_lib.lens_direction(plain, (1 - dd) / 2, 0.0)
    b, _, _ = oracle_lib.lens_direction(dist, (1 - dd) / 2, 0.0)
    assert np.max(np.abs(a - b)) < 1e-15


# ----------------------------------------------------------- curved panorama

def test_panorama_is_a_unit_cylinder(oracle_lib):
    """A cylinder of radius 1 around the vertical axis: azimuth is linear
    across the picture (Omega (fs - 1/2)), columns are meridians, and the
    height on the cylinder, v_y / hypot(v_x, v_z), is linear down the
    picture with the same scale (square pixels at the centre)."""
    W, H, om = 90, 30, 200.0
    v = synth.View(W, H, 0, 0, 0, 0, lens=synth.LENS_PANORAMA, lens_p=(om,))
    d, ok = _map(oracle_lib, v)
    assert ok.all()
    omr = math.radians(om)
    up = np.array([0.0, 1.0, 0.0])
    for i in range(0, W, 7):
        for j in range(H):
            g = d[j, i]
            assert math.atan2(g[0], g[2]) == pytest.approx(omr * ((i + 0.5) / W - 0.5), abs=1e-13)
            h = g[1] / math.hypot(g[0], g[2])
            # height scale: the same angle per pixel as across, Omega / W
            assert h == pytest.approx(omr / W * (j + 0.5 - H / 2), abs=1e-13)
            assert abs(np.linalg.det(np.stack([d[0, i], g, up]))) < 1e-14


# --------------------------------------------------------------- distortion

def test_zero_distortion_is_the_plain_map(oracle_lib):
    base = synth.View(40, 30, 0.3, 0.6, 0.9, 200.0, 1)
    dist = synth.View(40, 30, 0.3, 0.6, 0.9, 200.0, 1, lens_p=(0, 0, 0, 0, 0, 0))
    a, _ = _map(oracle_lib, base)
    b, _ = _map(oracle_lib, dist)
    assert np.array_equal(a, b)


def test_distortion_acts_on_view_coordinates(oracle_lib):
    """The paper's 3D->2D inverse (section 2.1.3, exact at s = 1) recovers
    the view coordinates the 2D->3D transform received: they are the
    Brown-Conrady image of the pixel's view coordinates (radial k1, k2; thin
    prism p; decentering q) for every angle-of-view type."""
    rng = np.random.default_rng(6)
    for aov in (0, 1, 2):
        for _ in range(4):
            k = rng.uniform(-0.6, 0.9)
            c = (rng.uniform(-0.2, 0.2), rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05),
                 rng.uniform(-0.05, 0.05), rng.uniform(-0.03, 0.03), rng.uniform(-0.03, 0.03))
            v = synth.View(36, 24, k, 0.7, 1.0, 120.0, aov, lens_p=c)
            kk, ll, ss, om = oracle_lib.limits(k, 0.7, 1.0, 120.0)
            for _ in range(20):
                i, j = int(rng.integers(0, 36)), int(rng.integers(0, 24))
                x, y = oracle_lib.view_coord(i, j, 36, 24, aov)
                g, ok, _ = oracle_lib.lens_direction(v, (i + 0.5) / 36, (j + 0.5) / 24)
                if not ok:
                    continue
                r2 = x * x + y * y
                rad = 1 + c[0] * r2 + c[1] * r2 * r2
                pr = c[2] * x + c[3] * y
                want = (x * rad + pr * x + c[4] * r2, y * rad + pr * y + c[5] * r2)
                got = oracle_lib.inverse(g, kk, ll, ss, om)
                assert got == pytest.approx(want, abs=1e-9), (aov, k, c, i, j)


# ----------------------------------------------------- global delta at seams

def test_delta_does_not_difference_across_cube_seams(oracle_lib):
    """Pixels beside a cube-face seam take one-sided differences within
    their face: their delta stays within a few percent of the next pixel in,
    instead of collapsing by the jump to an unrelated face."""
    F = 32
    v = synth.View(6 * F, F, 0, 0, 0, 0, lens=synth.LENS_CUBE)
    for f in range(6):
        for j in (3, F // 2, F - 4):
            edge = oracle_lib.delta(v, f * F, j)
            inner = oracle_lib.delta(v, f * F + 1, j)
            assert edge == pytest.approx(inner, rel=0.08), (f, j, edge, inner)


# ---------------------------------------------------------------- full dome

def test_dome_is_an_equidistant_fisheye_about_the_zenith(oracle_lib):
    """Full dome, no offset or tilt: the angle from the zenith (+y) grows
    linearly with the distance from the picture centre, reaching 90 degrees
    + compression at the inscribed circle, azimuth preserved; outside the
    circle no direction."""
    W = H = 64
    for comp in (0.0, 30.0, -20.0):
        v = synth.View(W, H, 0, 0, 0, 0, lens=synth.LENS_DOME, lens_p=(comp, 0.0, 0.0))
        d, ok = oracle_lib.perspective_map(v)
        for j in range(H):
            for i in range(W):
                x, y = 2 * (i + 0.5) / W - 1, 1 - 2 * (j + 0.5) / H
                R = math.hypot(x, y)
                assert ok[j, i] == (R <= 1.0)
                if R > 1.0:
                    continue
                g = d[j, i]
                assert math.acos(max(-1, min(1, g[1]))) == pytest.approx(R * math.radians(90 + comp), abs=1e-12)
                if math.sin(R * math.radians(90 + comp)) > 1e-6:
                    assert math.atan2(g[2], g[0]) == pytest.approx(math.atan2(y, x), abs=1e-9)


def test_dome_offset_and_tilt(oracle_lib):
    """The offset moves the viewpoint: the direction is the unit dome point
    seen from -o along z; the tilt turns the whole map about x (a proper
    rotation fixing x, recovered by SVD)."""
    rng = np.random.default_rng(2)
    base = synth.View(48, 48, 0, 0, 0, 0, lens=synth.LENS_DOME, lens_p=(10.0, 0.0, 0.0))
    off = synth.View(48, 48, 0, 0, 0, 0, lens=synth.LENS_DOME, lens_p=(10.0, 0.0, 0.35))
    tilt = synth.View(48, 48, 0, 0, 0, 0, lens=synth.LENS_DOME, lens_p=(10.0, 25.0, 0.0))
    for _ in range(50):
        fs, ft = rng.uniform(0.2, 0.8, size=2)
        a, oka, _ = oracle_lib.lens_direction(base, fs, ft)
        b, okb, _ = oracle_lib.lens_direction(off, fs, ft)
        assert oka and okb
        w = a + np.array([0.0, 0.0, 0.35])
        assert np.allclose(b, w / np.linalg.norm(w), atol=1e-14)
    da, oka = oracle_lib.perspective_map(base)
    dt, okt = oracle_lib.perspective_map(tilt)
    assert np.array_equal(oka, okt)
    R, res = _kabsch(da[oka], dt[okt])
    assert res < 1e-13 and np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
    assert np.allclose(R @ [1.0, 0.0, 0.0], [1.0, 0.0, 0.0], atol=1e-13)
    assert math.degrees(math.acos(R[1, 1])) == pytest.approx(25.0, abs=1e-9)
