"""GPU parity of the wire-frame (section 1.2) and particle (section 1.3)
steps against the FP64 oracle.

Tolerances follow the first-order model of tests/aa_parity.py: a mask or
line step moves by at most DM = delta * EPS_E + EPS_D/2 (|delta x| <= 1 on
the line tent, so the line step moves by delta * EPS_E + EPS_D); a wire
pixel keeps one side's mask, so its error is that bound; the dominant
triangle may differ only where the oracle's best and second masks are
within twice the bound.  Particle coverage and depth pass as for
triangles; the texture-coordinate pass moves by 2 n DM (uv within [-1, 2]
in the fringe) plus scale * 4e-6 for the FP32 texture axes, scale =
|P|/(2r) <= the largest over the scene.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from aa_parity import EPS_E, delta_plane, eps_delta

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


VIEWS = [
    synth.View(128, 96, 0.32, 0.62, 0.86, 270.0, 0, synth.yaw_pitch_rotation(0.3, 0.2)),
    synth.View(120, 88, 1.0, 0.5, 1.0, 90.0, 0, synth.yaw_pitch_rotation(1.0, -0.4)),
    synth.View(37, 23, -0.5, 0.8, 0.9, 200.0, 1, synth.yaw_pitch_rotation(2.5, 0.7)),
    synth.View(96, 48, 0, 0, 1, 90, 0, synth.yaw_pitch_rotation(0.5, 0.1), lens=synth.LENS_EQUIRECT),
]


def _compare_wire(gpu, view, tris, fr, pix=None, tag=""):
    torch, pipeline, vsr = gpu
    torch.cuda.synchronize()
    cov = fr.coverage.cpu().numpy().astype(np.float64).reshape(-1)
    dom = pipeline.ids_u32(fr.dominant).reshape(-1)
    ref = oracle.wireframe(view, tris, pix)
    if pix is None:
        pix = np.arange(view.width * view.height)
    rc, rd, rs = ref.cov.reshape(-1), ref.dom.reshape(-1), ref.second.reshape(-1)
    delta = delta_plane(fr, view).reshape(-1)[pix]
    tol = delta * EPS_E + eps_delta(delta) + 1e-6
    err = np.abs(cov[pix] - rc)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, (tag, pix[bad[:5]], cov[pix][bad[:5]], rc[bad[:5]], tol[bad[:5]])
    diff = np.flatnonzero(dom[pix] != rd)
    unexplained = diff[~(rc[diff] - rs[diff] <= 2 * tol[diff])]
    assert unexplained.size == 0, (tag, pix[unexplained[:5]], dom[pix][unexplained[:5]], rd[unexplained[:5]])
    _say(f"  {tag}: {len(pix)} px, drawn {int((rc > 0).sum())}, coverage err/tol max {np.max(err / tol):.3f}, "
         f"dominant differs at {diff.size} (near ties)")


def _compare_particles(gpu, view, pr, fr, pix=None, tag=""):
    torch, pipeline, vsr = gpu
    torch.cuda.synchronize()
    cov = fr.coverage.cpu().numpy().astype(np.float64).reshape(-1)
    dp = fr.depth_pass.cpu().numpy().astype(np.float64).reshape(-1)
    uv = fr.uv.cpu().numpy().astype(np.float64).reshape(2, -1)
    dom = pipeline.ids_u32(fr.dominant).reshape(-1)
    assert int(fr.lost.cpu().item()) == 0, tag
    ref = oracle.particles(view, pr, pix)
    if pix is None:
        pix = np.arange(view.width * view.height)
    f = lambda a: a.reshape(-1)  # noqa: E731
    delta = delta_plane(fr, view).reshape(-1)[pix]
    dm = delta * EPS_E + 0.5 * eps_delta(delta)
    n = f(ref.n_near)
    p64 = pr.astype(np.float64)
    dist = np.linalg.norm(p64[:3], axis=0)
    ok = (p64[3] > 0) & (dist > p64[3])
    scale_max = float(np.max(dist[ok] / (2 * p64[3][ok]))) if ok.any() else 0.0
    tol_c = n * dm + 1e-6
    tol_d = 2 * dm * f(ref.sum_r) + 2 * EPS_E * f(ref.sum_r) + 1e-6
    tol_uv = 2 * n * dm * 2 + 4e-6 * scale_max * np.minimum(1.0, f(ref.cov) + n * dm) + 1e-6
    ec = np.abs(cov[pix] - f(ref.cov))
    ed = np.abs(dp[pix] - f(ref.depth))
    eu = np.max(np.abs(uv[:, pix].T - ref.uv.reshape(-1, 2)), axis=1)
    for name, e, t in (("coverage", ec, tol_c), ("depth", ed, tol_d), ("uv", eu, tol_uv)):
        bad = np.flatnonzero(e > t)
        assert bad.size == 0, (tag, name, pix[bad[:5]], e[bad[:5]], t[bad[:5]])
    diff = np.flatnonzero(dom[pix] != f(ref.dom))
    if diff.size:
        near_tie = f(ref.margin)[diff] <= 2 * tol_c[diff]
        order = f(ref.gap)[diff] <= 1e-5
        unexplained = diff[~(near_tie | order)]
        assert unexplained.size == 0, (tag, pix[unexplained[:5]])
    _say(f"  {tag}: {len(pix)} px, covered {int((f(ref.cov) > 0).sum())}, err/tol max coverage "
         f"{np.max(ec / tol_c):.3f} depth {np.max(ed / tol_d):.3f} uv {np.max(eu / tol_uv):.3f}, dominant differs "
         f"at {diff.size} (explained)")


@pytest.mark.parametrize("vi", range(len(VIEWS)))
def test_wireframe_matches_oracle(gpu, vi):
    torch, pipeline, vsr = gpu
    view = VIEWS[vi]
    tris = synth.scene(1500, 40 + vi)
    _say(f"wire view {vi}")
    fr = pipeline.render_wireframe(pipeline.Scene(tris), view)
    _compare_wire(gpu, view, tris, fr, tag=f"wire view {vi}")


def test_wireframe_binning_paths_identical(gpu):
    torch, pipeline, vsr = gpu
    view = VIEWS[0]
    scene = pipeline.Scene(synth.scene(20000, 9))
    ref = pipeline.render_wireframe(scene, view, bin_depth=256)
    torch.cuda.synchronize()
    rc, rd = ref.coverage.clone(), ref.dominant.clone()
    for depth, flags in [(4, 0), (256, vsr.VSR_BIN_BLOCKS), (256, vsr.VSR_BIN_SUPERTILES), (256, vsr.VSR_BIN_ALL),
                         (256, vsr.VSR_BIN_TILE16)]:
        fr = pipeline.render_wireframe(scene, view, bin_depth=depth, bin_flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(fr.coverage, rc) and torch.equal(fr.dominant, rd), (depth, flags)


@pytest.mark.parametrize("vi", range(len(VIEWS)))
def test_particles_match_oracle(gpu, vi):
    torch, pipeline, vsr = gpu
    view = VIEWS[vi]
    pr = synth.particles(3000, 50 + vi, d_min=1.0, d_max=8.0, ang_mean=0.15, ang_sd=0.05)
    _say(f"particles view {vi}")
    fr = pipeline.render_particles(pipeline.ParticleScene(pr), view)
    _compare_particles(gpu, view, pr, fr, tag=f"particles view {vi}")


def test_particles_edge_cases(gpu):
    """Skipped particles (r <= 0, camera inside), a vertical particle (the
    texture x axis falls back to +x), an empty set, ragged sizes."""
    torch, pipeline, vsr = gpu
    pr = np.array([[0, 0, 5, 0.0], [0, 0, 0.5, 1.0], [0, -4, 0, 0.8], [0.3, 0.2, 3.0, 0.4],
                   [0.3, 0.2, 3.0, 0.4]], dtype=np.float32).T.copy()
    for view in (synth.View(33, 17, 0.5, 0.5, 0.9, 200.0, 0, synth.yaw_pitch_rotation(0.1, -1.2)),
                 synth.View(8, 8, 1.0, 0.5, 1.0, 90.0), synth.View(1, 1, 0.2, 0.5, 0.9, 120.0)):
        fr = pipeline.render_particles(pipeline.ParticleScene(pr), view)
        _compare_particles(gpu, view, pr, fr, tag=f"edge {view.width}x{view.height}")
    fr = pipeline.render_particles(pipeline.ParticleScene(np.zeros((4, 0), np.float32)), VIEWS[0])
    torch.cuda.synchronize()
    assert not fr.coverage.any().item() and np.all(pipeline.ids_u32(fr.dominant) == NO_HIT)


def test_particles_binning_paths_identical(gpu):
    torch, pipeline, vsr = gpu
    view = VIEWS[1]
    scene = pipeline.ParticleScene(synth.particles(30000, 7, d_max=10.0, ang_mean=0.05, ang_sd=0.02))
    ref = pipeline.render_particles(scene, view, bin_depth=256)
    torch.cuda.synchronize()
    base = [ref.coverage.clone(), ref.depth_pass.clone(), ref.uv.clone(), ref.dominant.clone()]
    for depth, flags in [(4, 0), (256, vsr.VSR_BIN_BLOCKS), (256, vsr.VSR_BIN_SUPERTILES), (256, vsr.VSR_BIN_ALL),
                         (256, vsr.VSR_BIN_TILE16)]:
        fr = pipeline.render_particles(scene, view, bin_depth=depth, bin_flags=flags)
        torch.cuda.synchronize()
        for a, b in zip(base, [fr.coverage, fr.depth_pass, fr.uv, fr.dominant]):
            assert torch.equal(a, b), (depth, flags)


def test_full_size_sampled(gpu):
    """1920x1080 (k = 0.5, 180 degrees): wire frame of the 1M-triangle scene
    and 10^6 particles, on sampled pixels."""
    torch, pipeline, vsr = gpu
    view = synth.views_1080p_sweep()[1]
    pix = synth.pixel_sample(view.width, view.height, 12, n_tiles=4, tile=8, n_pixels=300)
    tris = synth.scene_1m()
    _say("wire 1080p x 1M")
    fr = pipeline.render_wireframe(pipeline.Scene(tris), view)
    _compare_wire(gpu, view, tris, fr, pix=pix, tag="wire 1080p x 1M")
    pr = synth.particles_1m()
    _say("particles 1080p x 1M")
    fp = pipeline.render_particles(pipeline.ParticleScene(pr), view)
    _compare_particles(gpu, view, pr, fp, pix=pix, tag="particles 1080p x 1M")
