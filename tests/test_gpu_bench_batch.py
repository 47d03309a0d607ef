"""Parity of the benchmark's own batch, at its full size and settings.

The headline step renders 64 views of 1920x1080 (four Universal Perspective
lenses, k = 1 at 90 degrees and k = 0.5, 0, -0.5 at 180 degrees, l = 0.5,
s = 1, each in 16 orientations) of the 1,000,000 small triangles + radius-100
icosphere in one binned vsr_submit (bin depth 256, automatic binner shape:
32x32 blocks at this size).  Here that exact batch is checked:

  * eight of its views (two per lens) are identical, ids and depth bit for
    bit, to the plain path vsr_build_map -> vsr_bin -> vsr_raster;
  * one view per lens matches the FP64 oracle on the stratified sample
    (every pixel of 64 random 16x16 tiles + 16,384 random pixels) under
    the parity rule (ids bit-exact outside the flagged pixels, depth within
    1e-5 relative);
  * the configuration the autotuner picks for the benchmark (16x16 bin
    tiles at depth 512), alone and run as the benchmark runs it (steps with
    their setup alternating between two streams, two scene buffers), gives
    all 64 images of the 8x8 batch bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare

pytestmark = pytest.mark.gpu

DEPTH = 256


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_10558_amd import pipeline, vsr
    oracle.build(force=False)
    tris = synth.scene_1m()
    scene = pipeline.Scene(tris)
    views = synth.views_1080p_batch(64)
    b = pipeline.Batch([(scene, v) for v in views], mode=vsr.VSR_SUBMIT_BINNED, bin_depth=DEPTH)
    _say("[bench-batch] 64 x 1920x1080 views of 1,001,280 triangles, binned submit, depth 256")
    outs = b.submit()
    torch.cuda.synchronize()
    ovf = vsr.vsr_bin_overflow(b.workspace, True)
    _say(f"[bench-batch] overflowed tiles {ovf}")
    return torch, pipeline, vsr, tris, scene, views, outs


@pytest.mark.parametrize("q", [0, 1, 2, 3, 36, 45, 58, 63])
def test_batched_view_equals_plain(batch, q):
    torch, pipeline, vsr, tris, scene, views, outs = batch
    fr = pipeline.render(scene, views[q], bin_depth=DEPTH)
    torch.cuda.synchronize()
    ids, dep = outs[q]
    n_id = int((ids != fr.tri_id).sum().item())
    n_dep = int((dep.view(torch.int32) != fr.depth.view(torch.int32)).sum().item())
    _say(f"[bench-batch] view {q} (k={views[q].k}): id mismatches {n_id}, depth mismatches {n_dep}")
    assert n_id == 0 and n_dep == 0


@pytest.mark.parametrize("q", [4, 9, 14, 19])
def test_batched_view_oracle_sample(batch, q):
    torch, pipeline, vsr, tris, scene, views, outs = batch
    v = views[q]
    pix = synth.pixel_sample(v.width, v.height, seed=300 + q)
    ids, dep = outs[q]
    _say(f"[bench-batch] view {q} (k={v.k}): oracle on {len(pix)} sampled pixels x {tris.shape[1]} triangles")
    ref = oracle.render(v, tris, pix)
    st = compare(v, tris, pipeline.ids_u32(ids), dep.cpu().numpy(), ref, pixels=pix)
    _say("[bench-batch] " + st.line())
    assert st.ok(), st.notes
    assert st.hits > 0.9 * st.pixels


def _same(torch, outs_a, outs_b):
    return [q for q, (a, b) in enumerate(zip(outs_a, outs_b))
            if not (torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32)))]


def test_tile16_batch_equals_tile8_batch(batch):
    torch, pipeline, vsr, tris, scene, views, outs = batch
    b16 = pipeline.Batch([(scene, v) for v in views], mode=vsr.VSR_SUBMIT_BINNED | vsr.VSR_SUBMIT_BIN_TILE16,
                         bin_depth=512)
    o16 = b16.submit()
    torch.cuda.synchronize()
    bad = _same(torch, outs, o16)
    _say(f"[bench-batch] 16x16 tiles, depth 512: {64 - len(bad)} of 64 views identical to the 8x8 batch; "
         f"overflowed tiles {vsr.vsr_bin_overflow(b16.workspace, True)}")
    assert not bad, bad


def test_two_stream_steps_equal_one_batch(batch):
    """Steps alternating between two streams, each refreshing its own scene
    buffer before its submit, while the other stream's step runs."""
    torch, pipeline, vsr, tris, scene, views, outs = batch
    mode = vsr.VSR_SUBMIT_BINNED | vsr.VSR_SUBMIT_BIN_TILE16
    scenes = [pipeline.Scene(scene.xyz), pipeline.Scene(scene.xyz)]
    batches = [pipeline.Batch([(s, v) for v in views], mode=mode, bin_depth=512) for s in scenes]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for k in range(6):
        q = k % 2
        scenes[q].refresh(streams[q])
        batches[q].submit(streams[q])
    torch.cuda.synchronize()
    for q in range(2):
        bad = _same(torch, outs, batches[q].outputs)
        _say(f"[bench-batch] two-stream steps, buffer {q}: {64 - len(bad)} of 64 views identical")
        assert not bad, bad
