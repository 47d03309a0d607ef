"""GPU parity of the aliasing-free coverage step (sections 1.1.1, 1.1.2, 1.4;
vsr_build_map with VSR_MAP_AA, vsr_bin, vsr_aa_raster) against the FP64
oracle, with the per-pixel tolerance model of tests/aa_parity.py."""
import sys

import numpy as np
import pytest

import oracle
import synth
from aa_parity import compare_aa, delta_plane, eps_delta

pytestmark = pytest.mark.gpu
NO_HIT = 0xFFFFFFFF


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
        d = delta_plane(fr, view)
        for _ in range(200):
            i, j = int(rng.integers(0, view.width)), int(rng.integers(0, view.height))
            want = oracle.delta(view, i, j)
            if want == 0.0:
                assert d[j, i] == 0.0
            elif np.isinf(want):
                assert np.isinf(d[j, i])
            else:
                assert abs(d[j, i] - want) <= eps_delta(want) * want, (view, i, j, d[j, i], want)


@pytest.mark.parametrize("vi", range(4))
def test_aa_frames_match_oracle(gpu, vi):
    torch, pipeline, vsr = gpu
    view = _views_small()[vi]
    tris = synth.scene(3000, 70 + vi)
    _say(f"aa frame view {vi}: {view}")
    scene = pipeline.Scene(tris)
    fr = pipeline.render_aa(scene, view)
    compare_aa(gpu, view, tris, fr, tag=f"view {vi}")


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
    compare_aa(gpu, view, tris, fr, tag="pins scene")


@pytest.mark.parametrize("size", [(1, 1), (8, 8), (9, 9), (37, 23), (5, 70)])
def test_aa_ragged_sizes(gpu, size):
    torch, pipeline, vsr = gpu
    W, H = size
    view = synth.View(W, H, 0.4, 0.7, 0.9, 160.0, 0, synth.yaw_pitch_rotation(0.2, 0.1))
    tris = synth.scene(800, 5)
    scene = pipeline.Scene(tris)
    fr = pipeline.render_aa(scene, view)
    compare_aa(gpu, view, tris, fr, tag=f"{W}x{H}")


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
    compare_aa(gpu, view, tris, fr, tag="degenerate")
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
    for depth, flags in [(4, 0), (256, vsr.VSR_BIN_BLOCKS), (256, vsr.VSR_BIN_SUPERTILES), (256, vsr.VSR_BIN_ALL),
                         (256, vsr.VSR_BIN_TILE16)]:
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
    compare_aa(gpu, view, tris, fr, pix=pix, tag="1080p x 1M")
