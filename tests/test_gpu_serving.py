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


def test_batches_on_two_streams_overlap_and_match_alone(env):
    """Two batches submitted on different streams run at the same time on
    the device: each alone leaves most of the chip idle (a few small views),
    so the pair finishes in clearly less than the two back to back; their
    device intervals (events around each submit) intersect; and every view
    equals its solo render."""
    torch, pipeline, serve, vsr, scenes = env
    va = synth.random_views(3, 81, resolutions=((256, 128), (192, 128)))
    vb = synth.random_views(3, 82, resolutions=((256, 128), (192, 128)))
    a = pipeline.Batch([(scenes[2], v) for v in va], mode=vsr.VSR_SUBMIT_BINNED, bin_depth=512)
    b = pipeline.Batch([(scenes[2], v) for v in vb], mode=vsr.VSR_SUBMIT_BINNED, bin_depth=512)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    reps = 40

    def run(pair):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sa.wait_event(e0)
        sb.wait_event(e0)
        marks = []
        for _ in range(reps):
            if pair:
                a0, a1, b0, b1 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
                a0.record(sa)
                a.submit(sa)
                a1.record(sa)
                b0.record(sb)
                b.submit(sb)
                b1.record(sb)
                marks.append((a0, a1, b0, b1))
                ea, eb = torch.cuda.Event(), torch.cuda.Event()
                ea.record(sa)
                eb.record(sb)
                sa.wait_event(eb)  # next round starts when both are done
                sb.wait_event(ea)
            else:
                a.submit(sa)
                b.submit(sa)
        ea, eb = torch.cuda.Event(), torch.cuda.Event()
        ea.record(sa)
        eb.record(sb)
        torch.cuda.current_stream().wait_event(ea)
        torch.cuda.current_stream().wait_event(eb)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), marks

    run(True)
    t_seq, _ = run(False)
    t_par, marks = run(True)
    inter = sum(1 for a0, a1, b0, b1 in marks if a0.elapsed_time(b1) > 0 and b0.elapsed_time(a1) > 0)
    _say(f"[serve-overlap] {reps} rounds: back to back {t_seq:.3f} ms, two streams {t_par:.3f} ms; "
         f"intervals intersecting in {inter} rounds")
    assert t_par < 0.85 * t_seq
    assert inter >= reps // 2
    torch.cuda.synchronize()
    for batch, views, sc in ((a, va, scenes[2]), (b, vb, scenes[2])):
        for (ids, dep), v in zip(batch.outputs, views):
            fr = pipeline.render(sc, v, bin_depth=512)
            torch.cuda.synchronize()
            assert torch.equal(ids, fr.tri_id) and torch.equal(dep.view(torch.int32), fr.depth.view(torch.int32))
