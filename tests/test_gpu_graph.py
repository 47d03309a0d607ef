"""HIP-graph replays of a batched submit with new view parameters, and the
autotuner."""
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
    from paper_2003_10558_amd import autotune, pipeline, vsr
    scene = pipeline.Scene(synth.scene(20000, 81))
    return torch, pipeline, vsr, autotune, scene


def _views(seed):
    vs = synth.random_views(6, seed, resolutions=((128, 96), (200, 120), (64, 64)))
    # fixed sizes across parameter sets: sizes from seed 1, parameters from `seed`
    base = synth.random_views(6, 1, resolutions=((128, 96), (200, 120), (64, 64)))
    for v, b in zip(vs, base):
        v.width, v.height = b.width, b.height
    return vs


@pytest.mark.parametrize("mode", [0x200, 0x400, 0xA00, 0xC00, 1],
                         ids=["binned-blocks", "binned-supertiles", "tile16-blocks", "tile16-supertiles", "fused"])
def test_graph_replays_match_eager(env, mode):
    torch, pipeline, vsr, autotune, scene = env
    g = pipeline.GraphBatch([(scene, v) for v in _views(1)], mode=mode, bin_depth=512)
    for rep, seed in enumerate((2, 3, 1, 4)):
        views = _views(seed)
        g.set_views(views)
        outs = g.replay()
        g.stream.synchronize()
        got = [(pipeline.ids_u32(i), d.cpu().numpy().copy()) for i, d in outs]
        # eager work between replays, then the same views eagerly
        eager = pipeline.Batch([(scene, v) for v in views], mode=mode, bin_depth=512).submit()
        torch.cuda.synchronize()
        for (gi, gd), (ei, ed) in zip(got, eager):
            assert np.array_equal(gi, pipeline.ids_u32(ei)), (rep, seed)
            assert np.array_equal(gd.view(np.uint32), ed.cpu().numpy().view(np.uint32)), (rep, seed)
        _say(f"[graph] mode {mode} replay {rep} (parameter seed {seed}) matches eager")


def test_autotuner_picks_a_candidate(env, tmp_path):
    torch, pipeline, vsr, autotune, scene = env
    t = autotune.Tuner(str(tmp_path / "tune.json"), reps=2)
    views = synth.random_views(4, 5, resolutions=((256, 256),))
    mode, depth = t.choose(scene, views)
    assert (mode, depth) in autotune.CANDIDATES
    t2 = autotune.Tuner(str(tmp_path / "tune.json"))
    assert t2.choose(scene, views) == (mode, depth)  # from the cache
    _say(f"[autotune] {t.cache}")
