"""vsr_render_noalloc (library-held scratch array) against vsr_render (caller
scratch): the same images, bit for bit, on two calls in a row, the second
smaller than the first; views above the array's tile limit are refused
before anything is enqueued."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_10558_amd import pipeline, vsr
    scene = pipeline.Scene(synth.scene(200_000, 11))
    return torch, pipeline, vsr, scene


def _compare(env, view):
    torch, pipeline, vsr, scene = env
    fmt = vsr.VSR_MAP_F32
    ref = pipeline.render_fused(scene, view, fmt=fmt)
    ids = torch.full((view.height, view.width), 0x5A5A5A5A, dtype=torch.int32, device=scene.device)
    dep = torch.full((view.height, view.width), -7.0, dtype=torch.float32, device=scene.device)
    vsr.vsr_render_noalloc(view, fmt, ref.map, scene.setup, scene.ntri, ids, dep)
    torch.cuda.synchronize()
    a_ids, b_ids = ref.tri_id.cpu().numpy(), ids.cpu().numpy()
    a_dep, b_dep = ref.depth.cpu().numpy(), dep.cpu().numpy()
    n_id = int(np.sum(a_ids != b_ids))
    n_dep = int(np.sum(a_dep.view(np.uint32) != b_dep.view(np.uint32)))
    hit = int(np.sum(a_ids != -1))
    _say(f"noalloc {view.width}x{view.height}: id mismatches {n_id}, depth mismatches {n_dep}, {hit} covered px")
    assert hit > 0
    assert n_id == 0 and n_dep == 0


def test_noalloc_matches_render_two_calls(env):
    torch, pipeline, vsr, scene = env
    views = synth.views_1080p_sweep()
    big = views[1]  # 1920x1080: 32,400 tiles, close to the array's limit
    small = synth.View(640, 480, 0.32, 0.62, 0.86, 270.0, 0, synth.yaw_pitch_rotation(0.7, 0.2))
    _say(f"noalloc: first call {big.width}x{big.height}, second {small.width}x{small.height}")
    _compare(env, big)
    _compare(env, small)


def test_noalloc_ragged_and_refusal(env):
    torch, pipeline, vsr, scene = env
    _compare(env, synth.View(37, 23, -0.5, 1.0, 1.0, 170.0, 1, synth.yaw_pitch_rotation(2.0, -0.3)))
    too_big = synth.View(2048, 1088, 0.5, 0.5, 1.0, 180.0, 0, synth.yaw_pitch_rotation(0.0, 0.0))  # 34,816 tiles
    ids = torch.empty((8, 8), dtype=torch.int32, device=scene.device)
    dep = torch.empty((8, 8), dtype=torch.float32, device=scene.device)
    mp = torch.empty(256, dtype=torch.uint8, device=scene.device)
    with pytest.raises(vsr.VsrError) as e:
        vsr.vsr_render_noalloc(too_big, vsr.VSR_MAP_F32, mp, scene.setup, scene.ntri, ids, dep)
    assert e.value.code == vsr.VSR_E_SPACE
