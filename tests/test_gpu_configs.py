"""GPU parity at the full sizes of the dense workloads.

* 3840x2160 view (k=0.32, l=0.62, s=0.86, 270 deg) of 4,000,000 shell
  triangles + radius-10 icosphere: FP32 map parity on the stratified sample
  (every pixel of 64 random 16x16 tiles + 16,384 random pixels), and the
  octahedral 2xfp16 map tier with its angular error and coverage-mismatch
  fraction against the FP64 oracle (reported, bounded).
* 64 views of mixed resolution and random parameters of a 500,000-triangle
  shell scene in one batched submit: every view identical to rendering it
  alone, parity against the oracle on the stratified sample of four views.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def scene_4m(gpu):
    torch, pipeline, vsr = gpu
    tris = synth.scene_4m()
    return tris, pipeline.Scene(tris)


def _angle(a, b):
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    d = np.einsum("...i,...i->...", a, b)
    return np.arctan2(c, d)


def test_4k_4m_fp32_sampled(gpu, scene_4m):
    torch, pipeline, vsr = gpu
    tris, scene = scene_4m
    view = synth.view_4k()
    _say("[4k] fused render, FP32 map")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    fr = pipeline.render_fused(scene, view)
    torch.cuda.synchronize()
    t0.record()
    pipeline.render_fused(scene, view, frame=fr)
    t1.record()
    torch.cuda.synchronize()
    _say(f"[4k] fused render {t0.elapsed_time(t1):.2f} ms")
    ids, dep = pipeline.ids_u32(fr.tri_id), fr.depth.cpu().numpy()
    pix = synth.pixel_sample(view.width, view.height, seed=300)
    _say(f"[4k] oracle on {len(pix)} sampled pixels x {tris.shape[1]} triangles")
    ref = oracle.render(view, tris, pix)
    st = compare(view, tris, ids, dep, ref, pix)
    _say("[4k] " + st.line() + " " + "; ".join(st.notes))
    assert st.ok(), st.notes


def test_4k_4m_oct16_tier(gpu, scene_4m):
    """Octahedral 2 x fp16 map: error and mismatch against FP64 (reported)."""
    torch, pipeline, vsr = gpu
    tris, scene = scene_4m
    view = synth.view_4k()
    fr = pipeline.render_fused(scene, view, fmt=vsr.VSR_MAP_OCT16)
    torch.cuda.synchronize()
    ids = pipeline.ids_u32(fr.tri_id)
    # map error over a sample of pixels
    out = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    vsr.vsr_map_unpack(view, vsr.VSR_MAP_OCT16, fr.map, out)
    torch.cuda.synchronize()
    g16 = out.cpu().numpy().reshape(-1, 3).astype(np.float64)
    pix = synth.pixel_sample(view.width, view.height, seed=301, n_tiles=4, n_pixels=1024)
    ref_dirs = np.stack([_dir(view, int(p)) for p in pix])
    err = _angle(g16[pix], ref_dirs)
    ref = oracle.render(view, tris, pix)
    mism = ids[np.unravel_index(pix, ids.shape)] != ref.id
    frac = float(mism.mean())
    _say(f"[4k-oct16] angular error mean {err.mean():.2e} p99 {np.quantile(err, 0.99):.2e} max {err.max():.2e} rad; "
         f"coverage mismatch {frac:.4f} of {len(pix)} sampled pixels")
    assert err.max() < 2e-3
    assert frac < 0.05


def _dir(view, p):
    x, y = oracle.view_coord(p % view.width, p // view.width, view.width, view.height, view.aov)
    k, l, s, om = oracle.limits(view.k, view.l, view.s, view.omega_deg)
    g, _ = oracle.direction(x, y, k, l, s, om)
    return view.rot_matrix() @ g


def test_batched_64_views_500k(gpu, tmp_path):
    """64 mixed views of the 500k shell scene in one submit, in the mode, bin
    tile size and depth the autotuner picks for them, and in every binned
    variant (8x8 and 16x16 bin tiles) and the fused one: each view identical
    to rendering it alone, sampled parity against the oracle."""
    torch, pipeline, vsr = gpu
    from paper_2003_10558_amd import autotune
    tris = synth.scene_500k()
    scene = pipeline.Scene(tris)
    views = synth.random_views(64, 3)
    tuner = autotune.Tuner(str(tmp_path / "tune.json"), reps=2)
    choice = tuner.choose(scene, views)
    _say(f"[batch64] autotuner: {autotune.describe(choice)}; candidates (ms) {next(iter(tuner.cache.values()))['ms']}")
    variants = [choice, (vsr.VSR_SUBMIT_BINNED, 1024), (vsr.VSR_SUBMIT_BINNED | vsr.VSR_SUBMIT_BIN_TILE16, 1024),
                (vsr.VSR_SUBMIT_FUSED, 1024)]
    results = []
    for mode, depth in variants:
        batch = pipeline.Batch([(scene, v) for v in views], mode=mode, bin_depth=depth)
        outs = batch.submit()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        batch.submit()
        t1.record()
        torch.cuda.synchronize()
        _say(f"[batch64] {autotune.describe((mode, depth))}: {t0.elapsed_time(t1):.2f} ms for 64 views")
        results.append([(pipeline.ids_u32(i), d.cpu().numpy().view(np.uint32).copy()) for i, d in outs])
    for r in results[1:]:
        for (ai, ad), (bi, bd) in zip(results[0], r):
            assert np.array_equal(ai, bi) and np.array_equal(ad, bd)
    outs = batch.outputs
    # identical to rendering each view alone (binned path, large depth) on a few views
    for q in (0, 17, 42):
        v = views[q]
        fr = pipeline.render(scene, v, bin_depth=2048)
        torch.cuda.synchronize()
        assert np.array_equal(pipeline.ids_u32(outs[q][0]), pipeline.ids_u32(fr.tri_id)), q
        assert np.array_equal(outs[q][1].cpu().numpy().view(np.uint32), fr.depth.cpu().numpy().view(np.uint32)), q
    # oracle parity on the stratified sample of four views
    for q in (1, 8, 33, 63):
        v = views[q]
        pix = synth.pixel_sample(v.width, v.height, seed=400 + q)
        ref = oracle.render(v, tris, pix)
        st = compare(v, tris, pipeline.ids_u32(outs[q][0]), outs[q][1].cpu().numpy(), ref, pix)
        _say(f"[batch64] view {q} {v.width}x{v.height} k={v.k:.2f} om={v.omega_deg:.0f}: " + st.line())
        assert st.ok(), st.notes
