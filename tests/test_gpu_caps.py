"""Tile, super-tile and block caps of the map (GPU).

Binning is exact only if every cap the map stores contains the directions
of all of its pixels, with the safety margin the binner's FP32 tests rely
on.  This checks that property directly, in FP64 on the host, for the
Universal Perspective lenses of the benchmark and the other map generators
(section 2.2), on ragged sizes, for both map formats and for plain,
aliasing-free and wire-frame maps: every pixel direction, widened by its
fringe (aliasing-free maps: asin(1/(2 delta)) for triangles, asin(5/(4
delta)) for lines, delta the pixel's global delta of section 1.1.1), lies at
least half the absolute margin inside its tile cap, every tile cap inside
its super-tile cap and every super-tile cap inside its block cap.
"""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CAP_WIDE, CAP_EMPTY = 1.0, 2.0
# Tile caps are widened by 2e-5 rad in radius (plus 1e-6 relative): a pixel
# (with its fringe) must sit at least half of that inside.
TILE_INSIDE = 1e-5
FRINGE = {"plain": 0.0, "aa": 0.5, "lines": 1.25}


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_10558_amd import pipeline, vsr
    return torch, pipeline, vsr


def _align(x):
    return (x + 255) // 256 * 256


def _views(vsr):
    return {
        "k1_90": synth.View(333, 205, 1.0, 0.5, 1.0, 90.0),
        "k0.5_180": synth.View(333, 205, 0.5, 0.5, 1.0, 180.0),
        "k0_180": synth.View(320, 200, 0.0, 0.5, 1.0, 180.0),
        "k-0.5_180": synth.View(333, 205, -0.5, 0.5, 1.0, 180.0),
        "k-0.9_300": synth.View(301, 177, -0.9, 0.7, 0.9, 300.0),
        "equirect": synth.View(512, 256, 0, 0, 1, 90, 0, lens=vsr.VSR_LENS_EQUIRECT),
        "cube": synth.View(864, 144, 0, 0, 1, 90, 0, lens=vsr.VSR_LENS_CUBE),
        "screens3": synth.View(480, 270, 0, 0, 1, 90, 0, lens=vsr.VSR_LENS_SCREENS, lens_n=3, lens_p=(60.0,)),
        "vr": synth.View(480, 270, 0, 0, 1, 90, 0, lens=vsr.VSR_LENS_VR, lens_p=(100.0, 0.42, 0.22, 0.05)),
        "panorama": synth.View(480, 270, 0, 0, 1, 90, 0, lens=vsr.VSR_LENS_PANORAMA, lens_p=(270.0,)),
        "distorted": synth.View(333, 205, 0.5, 0.5, 1.0, 180.0,
                                lens_p=(0.12, -0.03, 0.01, -0.01, 0.005, -0.005)),
    }


def _rho(sh):
    return 2.0 * np.arcsin(np.minimum(1.0, sh))


def _angle(a, b):
    """Angle between two directions from the chord of their FP64-normalised
    vectors (acos of the dot product loses ~1e-5 rad at these angles when the
    stored centres are unit only to FP32 rounding)."""
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    return 2.0 * math.atan2(float(np.linalg.norm(a - b)), float(np.linalg.norm(a + b)))


def _check_children(parent0, parent1, child0, child1, nx, ny, what):
    """Every non-empty child cap (2x2 children per parent, row-major grids)
    lies inside its parent's cap.  Caps as float64 arrays [n, 4]."""
    npx = (nx + 1) // 2
    for p in range(len(parent0)):
        px, py = p % npx, p // npx
        kids = [(2 * py + b) * nx + 2 * px + a for b in (0, 1) for a in (0, 1)
                if 2 * px + a < nx and 2 * py + b < ny]
        live = [k for k in kids if child1[k, 2] != 0.0]  # flag: 0 empty for super/block children
        if what == "tile":
            live = [k for k in kids if child1[k, 2] != CAP_EMPTY]
        if not live:
            assert parent1[p, 2] == 0.0, f"{what} children empty but parent {p} not"
            continue
        assert parent1[p, 2] == 1.0, f"parent {p} of live {what} caps marked empty"
        if parent1[p, 3] != 0.0:  # wide parent
            continue
        cs = parent0[p, :3]
        rs = _rho(parent0[p, 3])
        for k in live:
            wide = child1[k, 2] == CAP_WIDE if what == "tile" else child1[k, 3] != 0.0
            assert not wide, f"wide {what} cap {k} under a narrow parent {p}"
            ang = _angle(cs, child0[k, :3])
            assert ang + _rho(child0[k, 3]) <= rs + 1e-6, (what, p, k, ang, _rho(child0[k, 3]), rs)


@pytest.mark.parametrize("name", ["k1_90", "k0.5_180", "k0_180", "k-0.5_180", "k-0.9_300", "equirect", "cube",
                                  "screens3", "vr", "panorama", "distorted"])
@pytest.mark.parametrize("fmt", [0, 1], ids=["f32", "oct16"])
@pytest.mark.parametrize("kind", ["plain", "aa", "lines"])
def test_caps_contain_their_pixels(gpu, name, fmt, kind):
    torch, pipeline, vsr = gpu
    view = _views(vsr)[name]
    _say(f"[caps] {name} fmt={fmt} {kind} {view.width}x{view.height}")
    W, H = view.width, view.height
    flags = {"plain": 0, "aa": vsr.VSR_MAP_AA, "lines": vsr.VSR_MAP_AA_LINES}[kind]
    nbytes = vsr.vsr_map_bytes(W, H, fmt) if kind == "plain" else vsr.vsr_aa_map_bytes(W, H, fmt)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    pipeline.build_map(view, fmt, flags, buf)
    dirs = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    vsr.vsr_map_unpack(view, fmt, buf, dirs)  # identity rotation: camera frame, as the caps are stored
    torch.cuda.synchronize()
    g = dirs.cpu().numpy().astype(np.float64)
    raw = buf.cpu().numpy()

    ntx, nty = (W + 7) // 8, (H + 7) // 8
    ntiles = ntx * nty
    nsx, nsy = (ntx + 1) // 2, (nty + 1) // 2
    nbx, nby = (ntx + 3) // 4, (nty + 3) // 4
    caps_off = _align(ntiles * 64 * (12 if fmt == 0 else 4))
    sups_off = caps_off + _align(ntiles * 32)
    blks_off = sups_off + _align(nsx * nsy * 32)
    delta_off = blks_off + _align(nbx * nby * 32)  # aliasing-free maps: one float per pixel, tile-major

    def caps_at(off, n):
        a = raw[off:off + 32 * n].view(np.float32).astype(np.float64).reshape(n, 2, 4)
        return a[:, 0], a[:, 1]

    t0, t1 = caps_at(caps_off, ntiles)
    s0, s1 = caps_at(sups_off, nsx * nsy)
    b0, b1 = caps_at(blks_off, nbx * nby)

    # pixel directions per tile, [nty, ntx, 64, 3]; a zero vector has no direction
    pad = np.zeros((nty * 8, ntx * 8, 3))
    pad[:H, :W] = g
    tg = pad.reshape(nty, 8, ntx, 8, 3).transpose(0, 2, 1, 3, 4).reshape(ntiles, 64, 3)
    valid = np.linalg.norm(tg, axis=-1) > 0.5
    assert valid.any()

    flag = t1[:, 2]
    has = valid.any(axis=1)
    assert np.all(flag[~has] == CAP_EMPTY) and np.all(flag[has] != CAP_EMPTY)
    narrow = has & (flag == 0.0)
    assert narrow.sum() > 0.5 * has.sum()  # most tiles are usable for culling
    # tile caps: unit centre, consistent sine/cosine fields, pixels well inside
    c = t0[narrow, :3]
    sh, chh, srho = t0[narrow, 3], t1[narrow, 0], t1[narrow, 1]
    assert np.all(np.abs(np.linalg.norm(c, axis=1) - 1.0) < 1e-6)
    assert np.all(np.abs(sh * sh + chh * chh - 1.0) < 1e-6)
    assert np.all(srho >= np.sin(_rho(sh)) - 1e-7)
    cu = c / np.linalg.norm(c, axis=1, keepdims=True)
    chord = np.linalg.norm(tg[narrow] - cu[:, None, :], axis=-1)
    ang = 2.0 * np.arcsin(np.minimum(1.0, 0.5 * chord))
    if kind != "plain":
        delta = raw[delta_off:delta_off + 4 * 64 * ntiles].view(np.float32).astype(np.float64).reshape(ntiles, 64)
        d = delta[narrow]
        assert np.all(d[valid[narrow]] > 0.0)
        with np.errstate(divide="ignore"):
            ang = ang + np.arcsin(np.minimum(1.0, np.where(np.isinf(d), 0.0, FRINGE[kind] / d)))
    ang = np.where(valid[narrow], ang, 0.0)
    worst = (ang - _rho(sh)[:, None]).max()
    assert worst <= -TILE_INSIDE, f"a pixel lies {worst:.3g} rad from its tile cap's rim"

    _check_children(s0, s1, t0, t1, ntx, nty, "tile")
    _check_children(b0, b1, s0, s1, nsx, nsy, "super")
    _say(f"[caps] {name}: {int(narrow.sum())} narrow tile caps of {ntiles}, margin {-worst:.3g}")
