"""GPU parity of the aliasing-free coverage step (sections 1.1.1, 1.1.2, 1.4;
vsr_build_map with VSR_MAP_AA, vsr_bin, vsr_aa_raster) against the FP64
oracle.

Tolerance, per pixel, from a first-order error model of the FP32 path:
  - a direction of the FP32 map is within 1e-6 rad of the exact one, so an
    edge or miter value n.G is off by at most EPS_E = 2e-6;
  - the global delta is a difference quotient of FP32 directions: relative
    error at most EPS_D = 4e-6 * delta + 1e-5 (checked below);
  - a mask m = clamp(delta x + 1/2) therefore moves by at most
    DM = delta * EPS_E + EPS_D / 2 (|delta x| <= 1/2 on the ramp);
  - coverage = min(1, sum of masks) moves by at most n * DM over the n
    fragments that take part (oracle: fragments taken + the first left out);
  - a depth r = d / (G.N) moves by r (EPS_E / cos + 4 ulp); the depth pass
    sum m_fc r by at most 2 DM sum(r) + EPS_E sum(r / cos) + 1e-6 sum(r);
    two fragments whose depths are within those errors may swap order, which
    moves the depth pass by no more than the same bound;
  - the dominant id may differ only where the oracle's largest share leads
    the second by less than 2 n DM, or two fragments' depths are within
    rounding (relative step below 4e-6 / cos).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
NO_HIT = 0xFFFFFFFF
EPS_E = 2e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_10558_amd import pipeline, vsr
    oracle.build(force=False)
    return torch, pipeline, vsr


def _delta_plane(gpu, frame, view, fmt=0):
    """The AA map's delta plane (tile-major after the plain map) as [H, W]."""
    torch, pipeline, vsr = gpu
    W, H = view.width, view.height
    off = vsr.vsr_map_bytes(W, H, fmt)
    ntx, nty = (W + 7) // 8, (H + 7) // 8
    raw = frame.map[off:off + ntx * nty * 64 * 4].cpu().numpy().view(np.float32)
    d = raw.reshape(nty, ntx, 8, 8).transpose(0, 2, 1, 3).reshape(nty * 8, ntx * 8)
    return d[:H, :W].astype(np.float64)


def _eps_delta(delta):
    return 4e-6 * delta + 1e-5


def _compare(gpu, view, tris, fr, pix=None, tag=""):
    """Per-pixel parity of one AA frame with the oracle (whole frame or the
    listed flat pixel indices); returns (cov err / tol, depth err / tol)."""
    torch, pipeline, vsr = gpu
    torch.cuda.synchronize()
    cov = fr.coverage.cpu().numpy().astype(np.float64).reshape(-1)
    dp = fr.depth_pass.cpu().numpy().astype(np.float64).reshape(-1)
    dom = pipeline.ids_u32(fr.dominant).reshape(-1)
    lost = int(fr.lost.cpu().item())
    assert lost == 0, (tag, lost)
    ref = oracle.aa_render(view, tris, pix)
    if pix is None:
        pix = np.arange(view.width * view.height)
        flat = lambda a: a.reshape(-1)  # noqa: E731
    else:
        flat = lambda a: a  # noqa: E731
    delta = _delta_plane(gpu, fr, view).reshape(-1)[pix]
    dm = delta * EPS_E + 0.5 * _eps_delta(delta)
    n_near = flat(ref.n_near)
    tol_c = n_near * dm + 1e-6
    tol_d = 2 * dm * flat(ref.sum_r) + EPS_E * flat(ref.sum_rg) + 1e-6 * flat(ref.sum_r) + 1e-6
    ec = np.abs(cov[pix] - flat(ref.cov))
    ed = np.abs(dp[pix] - flat(ref.depth))
    bad_c = np.flatnonzero(ec > tol_c)
    bad_d = np.flatnonzero(ed > tol_d)
    assert bad_c.size == 0, (tag, pix[bad_c[:5]], cov[pix][bad_c[:5]], flat(ref.cov)[bad_c[:5]], tol_c[bad_c[:5]])
    assert bad_d.size == 0, (tag, pix[bad_d[:5]], dp[pix][bad_d[:5]], flat(ref.depth)[bad_d[:5]], tol_d[bad_d[:5]])
    diff = np.flatnonzero(dom[pix] != flat(ref.dom))
    if diff.size:
        sum_r = np.maximum(flat(ref.sum_r)[diff], 1e-300)
        near_tie = flat(ref.margin)[diff] <= 2 * tol_c[diff]
        order = flat(ref.gap)[diff] <= 4e-6 * np.maximum(1.0, flat(ref.sum_rg)[diff] / sum_r)
        unexplained = diff[~(near_tie | order)]
        assert unexplained.size == 0, (tag, pix[unexplained[:5]], dom[pix][unexplained[:5]],
                                       flat(ref.dom)[unexplained[:5]], flat(ref.margin)[unexplained[:5]])
    _say(f"  {tag}: {len(pix)} px, coverage err/tol max {np.max(ec / tol_c):.3f}, depth err/tol max "
         f"{np.max(ed / tol_d):.3f}, dominant differs at {diff.size} (explained)")
    return np.max(ec / tol_c), np.max(ed / tol_d)


def _views_small():
    return [
        synth.View(128, 96, 0.32, 0.62, 0.86, 270.0, 0, synth.yaw_pitch_rotation(0.3, 0.2)),
        synth.View(120, 88, 1.0, 0.5, 1.0, 90.0, 0, synth.yaw_pitch_rotation(1.0, -0.4)),
        synth.View(100, 100, -0.5, 0.8, 0.9, 200.0, 1, synth.yaw_pitch_rotation(2.5, 0.7)),
        synth.View(117, 61, 0.0, 0.3, 0.8, 180.0, 2, synth.yaw_pitch_rotation(-1.2, 0.1)),
    ]


def test_delta_plane_matches_oracle(gpu):
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(np.zeros((9, 0), dtype=np.float32))
    rng = np.random.default_rng(3)
    views = _views_small() + [synth.View(37, 23, -1.0, 1.0, 1.0, 180.0), synth.View(1, 5, 0.5, 0.5, 0.9, 60.0),
                              synth.View(1920, 1080, 0.3, 0.6, 0.9, 250.0)]
    for view in views:
        _say(f"delta plane {view.width}x{view.height} k={view.k}")
        fr = pipeline.render_aa(scene, view)
        d = _delta_plane(gpu, fr, view)
        for _ in range(200):
            i, j = int(rng.integers(0, view.width)), int(rng.integers(0, view.height))
            want = oracle.delta(view, i, j)
            if want == 0.0:
                assert d[j, i] == 0.0
            elif np.isinf(want):
                assert np.isinf(d[j, i])
            else:
                assert abs(d[j, i] - want) <= _eps_delta(want) * want, (view, i, j, d[j, i], want)


@pytest.mark.parametrize("vi", range(4))
def test_aa_frames_match_oracle(gpu, vi):
    torch, pipeline, vsr = gpu
    view = _views_small()[vi]
    tris = synth.scene(3000, 70 + vi)
    _say(f"aa frame view {vi}: {view}")
    scene = pipeline.Scene(tris)
    fr = pipeline.render_aa(scene, view)
    _compare(gpu, view, tris, fr, tag=f"view {vi}")


def test_aa_pinhole_pins_scene(gpu):
    """The oracle pins' geometry on the GPU: layered, shared-edge and sliver
    triangles in a pinhole view."""
    torch, pipeline, vsr = gpu
    W = H = 64
    view = synth.View(W, H, 1.0, 0.5, 1.0, 40.0)
    t_f = np.tan(np.radians(20.0))

    def P(u, v, Z):
        return [(2 * u / W - 1) * Z * t_f, (v - H / 2) * 2 / W * Z * t_f, Z]

    quad = [(10.0, 12.0), (54.0, 9.0), (57.0, 50.0), (8.0, 55.0)]
    t1 = P(*quad[0], 3) + P(*quad[1], 3) + P(*quad[2], 3)
    t2 = P(*quad[0], 3) + P(*quad[2], 3) + P(*quad[3], 3)
    back = [-20, -20, 5, 20, -20, 5.5, 0, 30, 4.5]
    apex = (40.3, 31.5)
    sl = P(*apex, 2) + P(apex[0] - 30, apex[1] - 2.1, 2) + P(apex[0] - 30, apex[1] + 2.1, 2)
    tris = np.array([t1, t2, back, sl], dtype=np.float32).T.copy()
    scene = pipeline.Scene(tris)
    fr = pipeline.render_aa(scene, view)
    _compare(gpu, view, tris, fr, tag="pins scene")


@pytest.mark.parametrize("size", [(1, 1), (8, 8), (9, 9), (37, 23), (5, 70)])
def test_aa_ragged_sizes(gpu, size):
    torch, pipeline, vsr = gpu
    W, H = size
    view = synth.View(W, H, 0.4, 0.7, 0.9, 160.0, 0, synth.yaw_pitch_rotation(0.2, 0.1))
    tris = synth.scene(800, 5)
    scene = pipeline.Scene(tris)
    fr = pipeline.render_aa(scene, view)
    _compare(gpu, view, tris, fr, tag=f"{W}x{H}")


def test_aa_empty_and_degenerate(gpu):
    torch, pipeline, vsr = gpu
    view = synth.View(40, 30, 0.2, 0.5, 0.9, 200.0)
    fr = pipeline.render_aa(pipeline.Scene(np.zeros((9, 0), dtype=np.float32)), view)
    torch.cuda.synchronize()
    assert not fr.coverage.any().item() and not fr.depth_pass.any().item()
    assert np.all(pipeline.ids_u32(fr.dominant) == NO_HIT)
    # zero-area and plane-through-O triangles cover nothing; one live triangle
    tris = np.array([[0, 0, 1, 0, 0, 1, 0, 0, 1],
                     [1, 0, 2, 2, 0, 4, 3, 0, 6],
                     [-1, -1, 3, 1, -1, 3, 0, 1, 3]], dtype=np.float32).T.copy()
    fr = pipeline.render_aa(pipeline.Scene(tris), view)
    _compare(gpu, view, tris, fr, tag="degenerate")
    dom = pipeline.ids_u32(fr.dominant)
    assert set(np.unique(dom)) <= {2, NO_HIT}


def test_aa_overflow_and_binner_paths_identical(gpu):
    """Bin overflow (the tile gathers its own candidates) and the block /
    super-tile binners list the same triangles in other orders: the sorted
    per-pixel lists and so the images are bit-identical."""
    torch, pipeline, vsr = gpu
    view = _views_small()[0]
    tris = synth.scene(20000, 9)
    scene = pipeline.Scene(tris)
    base = pipeline.render_aa(scene, view, bin_depth=256)
    torch.cuda.synchronize()
    ref = [base.coverage.clone(), base.depth_pass.clone(), base.dominant.clone()]
    for depth, flags in [(4, 0), (256, vsr.VSR_BIN_BLOCKS), (256, vsr.VSR_BIN_SUPERTILES), (256, vsr.VSR_BIN_ALL)]:
        fr = pipeline.render_aa(scene, view, bin_depth=depth, bin_flags=flags)
        torch.cuda.synchronize()
        if depth == 4:
            assert vsr.vsr_bin_overflow(fr.bins) > 0
        for a, b in zip(ref, [fr.coverage, fr.depth_pass, fr.dominant]):
            assert torch.equal(a, b), (depth, flags)


def test_aa_fragment_list_overflow_is_counted(gpu):
    """Twelve nested triangles whose edges all cross one pixel column with
    small masks: pixels meeting more than eight unsaturated fragments are
    counted as lost; every other pixel still matches the oracle."""
    torch, pipeline, vsr = gpu
    W = H = 32
    view = synth.View(W, H, 1.0, 0.5, 1.0, 40.0)
    t_f = np.tan(np.radians(20.0))
    rows = []
    for q in range(12):
        Z = 2.0 + 0.1 * q
        X = (2 * 16.95 / W - 1) * t_f * Z  # 0.45 px right of column 16's centre: mask 0.05
        rows.append([X, -5, Z, X, 5, Z, X + 5, 0, Z])
    tris = np.array(rows, dtype=np.float32).T.copy()
    fr = pipeline.render_aa(pipeline.Scene(tris), view)
    torch.cuda.synchronize()
    lost = int(fr.lost.cpu().item())
    ref = oracle.aa_render(view, tris)
    over = (ref.n_near > 8) & (ref.cov < 1.0 - 1e-9)
    assert lost == int(over.sum()) and lost > 0
    ok = ~over.reshape(-1)
    cov = fr.coverage.cpu().numpy().reshape(-1).astype(np.float64)
    assert np.allclose(cov[ok], ref.cov.reshape(-1)[ok], atol=1e-4)


def test_aa_1080p_1m_sampled(gpu):
    """Full size: 1080p view of the 1M-triangle scene, sampled pixels."""
    torch, pipeline, vsr = gpu
    view = synth.views_1080p_sweep()[1]
    tris = synth.scene_1m()
    _say("aa 1080p x 1M: render")
    scene = pipeline.Scene(tris)
    fr = pipeline.render_aa(scene, view)
    pix = synth.pixel_sample(view.width, view.height, 11, n_tiles=4, tile=8, n_pixels=300)
    _say(f"aa 1080p x 1M: oracle on {len(pix)} pixels")
    _compare(gpu, view, tris, fr, pix=pix, tag="1080p x 1M")
