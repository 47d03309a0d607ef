"""Serving: continuous batching gives every request the same images as
rendering it alone; admission respects the HBM budget."""
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
    from paper_2003_10558_amd import pipeline, serve, vsr
    scenes_np = [synth.scene(n, s) for n, s in ((5000, 51), (30000, 52), (80000, 53))]
    scenes = [pipeline.Scene(t) for t in scenes_np]
    return torch, pipeline, serve, vsr, scenes


RES = ((256, 256), (320, 240), (512, 256), (160, 96))


@pytest.mark.parametrize("mode", [0, 1], ids=["binned", "fused"])
def test_mix_equals_alone(env, mode):
    torch, pipeline, serve, vsr, scenes = env
    reqs = serve.make_requests(len(scenes), rate_hz=4000.0, duration_s=0.02, seed=61, view_seed=62,
                               resolutions=RES)
    assert len(reqs) >= 40
    srv = serve.Server(scenes, streams=3, max_batch=8, mode_for_scene=lambda s: (mode, 512))
    st = srv.run(reqs, keep={r.rid for r in reqs})
    _say(f"[serve] mode {mode}: {st.completed}/{st.offered} done in {st.batches} batches (mean {st.mean_batch:.1f}), "
         f"p50 {st.p50_ms:.2f} ms p99 {st.p99_ms:.2f} ms")
    assert st.completed == st.offered and st.dropped == 0
    assert st.batches > 1
    for r in reqs:
        fr = pipeline.render_fused(scenes[r.scene], r.view) if r.rid % 2 else \
            pipeline.render(scenes[r.scene], r.view, bin_depth=512)
        torch.cuda.synchronize()
        assert np.array_equal(r.result[0], pipeline.ids_u32(fr.tri_id)), r.rid
        assert np.array_equal(r.result[1].view(np.uint32), fr.depth.cpu().numpy().view(np.uint32)), r.rid


def test_admission_respects_budget(env):
    torch, pipeline, serve, vsr, scenes = env
    reqs = serve.make_requests(len(scenes), rate_hz=3000.0, duration_s=0.02, seed=71, view_seed=72,
                               resolutions=RES)
    one = max(serve.request_bytes(r.view, 0, 1, 1024) for r in reqs)
    budget = int(2.5 * one)
    srv = serve.Server(scenes, streams=4, max_batch=16, hbm_budget_bytes=budget)
    st = srv.run(reqs)
    _say(f"[serve-budget] budget {budget} B, max in flight {st.max_inflight_bytes} B, batches {st.batches}")
    assert st.completed == st.offered
    assert st.max_inflight_bytes <= budget
    assert st.mean_batch <= 2.5
