"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Run on an MI355X: python -u -m pytest -m gpu -x -v tests/
"""
import math
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


def _gpu_map(gpu, view, fmt=0):
    torch, pipeline, vsr = gpu
    buf = torch.empty(vsr.vsr_map_bytes(view.width, view.height, fmt), dtype=torch.uint8, device="cuda")
    eff = vsr.vsr_build_map(view, fmt, 0, buf)
    out = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    vsr.vsr_map_unpack(view, fmt, buf, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), eff


def _angle(a, b):
    """Angle between unit vectors, robust for tiny angles."""
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    d = np.einsum("...i,...i->...", a, b)
    return np.arctan2(c, d)


MAP_VIEWS = [
    ("small", synth.view_small()),
    ("1080p_k1", synth.views_1080p_sweep()[0]),
    ("1080p_k0.5", synth.views_1080p_sweep()[1]),
    ("1080p_k0", synth.views_1080p_sweep()[2]),
    ("1080p_k-0.5", synth.views_1080p_sweep()[3]),
    ("diag", synth.View(333, 121, -0.8, 0.3, 0.9, 150.0, synth.AOV_DIAGONAL, synth.yaw_pitch_rotation(0.4, 1.0))),
    ("vert", synth.View(100, 300, 0.7, 0.0, 0.8, 100.0, synth.AOV_VERTICAL, synth.yaw_pitch_rotation(2.0, -0.5))),
    ("4x3", synth.View(161, 97, -1.0, 1.0, 1.0, 180.0, synth.AOV_HORIZONTAL_4X3)),
    ("wide360", synth.View(200, 100, 0.0, 0.4, 0.85, 360.0, 0, synth.yaw_pitch_rotation(5.0, 0.2))),
]


@pytest.mark.parametrize("name,view", MAP_VIEWS, ids=[n for n, _ in MAP_VIEWS])
def test_map_matches_oracle(gpu, name, view):
    _say(f"[map] {name} {view.width}x{view.height} k={view.k}")
    g, eff = _gpu_map(gpu, view)
    ref, ok = oracle.perspective_map(view)
    k, l, s, om = oracle.limits(view.k, view.l, view.s, view.omega_deg)
    assert (eff.k, eff.omega_deg) == pytest.approx((k, om), rel=1e-6)
    gok = np.any(g != 0, axis=-1)
    # validity agrees except within 1e-6 of the domain edge
    diff = gok != ok
    if diff.any():
        js, is_ = np.nonzero(diff)
        for j, i in zip(js[:50], is_[:50]):
            assert oracle.render(view, np.zeros((9, 0), np.float32), np.array([j * view.width + i])).flags[0] & oracle.FLAG_DOMAIN
    both = gok & ok
    err = _angle(g[both], ref[both])
    _say(f"[map] {name}: max angular error {err.max():.3e} rad, p99 {np.quantile(err, 0.99):.3e}")
    assert err.max() < 1e-6
    assert np.all(np.abs(np.linalg.norm(g[both], axis=-1) - 1) < 1e-6)


def _render(gpu, tris, view, fmt=0, depth=1024, flags=0):
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(tris)
    fr = pipeline.render(scene, view, fmt=fmt, bin_depth=depth, bin_flags=flags)
    torch.cuda.synchronize()
    return pipeline.ids_u32(fr.tri_id), fr.depth.cpu().numpy(), vsr.vsr_bin_overflow(fr.bins)


@pytest.mark.parametrize("flags", [0, 8], ids=["tile8", "tile16"])
def test_small_full_frame(gpu, flags):
    view, tris = synth.view_small(), synth.scene_small()
    _say(f"[raster] 256x256 full frame vs oracle, bin flags {flags}")
    ids, dep, ovf = _render(gpu, tris, view, flags=flags)
    ref = oracle.render(view, tris)
    st = compare(view, tris, ids, dep, ref)
    _say("[raster] " + st.line() + " " + "; ".join(st.notes))
    assert st.ok(), st.notes
    assert ovf == 0


def test_binning_is_exact(gpu):
    """Real bins give the same bits as every triangle in every tile."""
    for name, view, tris in [("small", synth.view_small(), synth.scene_small()),
                             ("rot", synth.View(200, 150, -0.4, 0.3, 0.9, 300.0, 0, synth.yaw_pitch_rotation(1.0, 0.3)),
                              synth.scene(700, 17))]:
        _say(f"[bin-exact] {name}")
        b_ids, b_dep, ovf = _render(gpu, tris, view, depth=2048, flags=1)
        assert ovf == 0
        # automatic, 32x32 blocks, 16x16 super-tiles; then the same with 16x16 bin tiles
        for depth, shape in ((1024, 0), (256, 2), (256, 4), (1024, 8), (256, 8 | 2), (512, 8 | 2), (256, 8 | 4)):
            a_ids, a_dep, _ = _render(gpu, tris, view, depth=depth, flags=shape)
            assert np.array_equal(a_ids, b_ids), shape
            assert np.array_equal(a_dep.view(np.uint32), b_dep.view(np.uint32)), shape


@pytest.mark.parametrize("seed", list(range(6)))
def test_binning_is_exact_random_views(gpu, seed):
    """Random lenses up to 360 degrees, random orientation: culling never
    drops a triangle the rasterizer covers (bit-identical to no culling)."""
    views = synth.random_views(4, 500 + seed, resolutions=((200, 150), (96, 96), (311, 97)))
    tris = synth.scene(700, 600 + seed)
    for v in views:
        b_ids, b_dep, ovf = _render(gpu, tris, v, depth=2048, flags=1)
        assert ovf == 0
        for shape in (2, 4, 8 | 2, 8 | 4):  # 32x32 blocks, 16x16 super-tiles; 8x8 or 16x16 bin tiles
            a_ids, a_dep, _ = _render(gpu, tris, v, depth=256, flags=shape)
            assert np.array_equal(a_ids, b_ids), (v.k, v.omega_deg, shape)
            assert np.array_equal(a_dep.view(np.uint32), b_dep.view(np.uint32))


def _bin_lists(gpu, scene, view, depth, flags):
    """Per-tile counts, lists ([ntiles, depth] u32) and overflow count of one binning."""
    torch, pipeline, vsr = gpu
    fr = pipeline.render(scene, view, bin_depth=depth, bin_flags=flags)
    torch.cuda.synchronize()
    ntiles = ((view.width + 7) // 8) * ((view.height + 7) // 8)
    raw = fr.bins.cpu().numpy()
    counts = raw[256:256 + 4 * ntiles].view(np.uint32).copy()
    off = 256 + (ntiles * 4 + 255) // 256 * 256
    lists = raw[off:off + ntiles * depth * 4].view(np.uint32).reshape(ntiles, depth).copy()
    return counts, lists, vsr.vsr_bin_overflow(fr.bins)


def test_bin_lists_identical_across_shapes(gpu):
    """The 32x32-block and 16x16-super-tile binners give every tile the same
    count and, where the list fits, the same ranks in depth-bucket order: at
    depths 1, 2, 63-65 and at depths taken from the tiles' own counts, so
    that some lists are exactly full (kept) and the next longer ones
    overflow (counted)."""
    view = synth.View(200, 150, -0.4, 0.3, 0.9, 300.0, 0, synth.yaw_pitch_rotation(1.0, 0.3))
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(synth.scene(20000, 5))
    shift = 0
    while (256 << shift) < scene.ntri:
        shift += 1
    full, _, ovf_full = _bin_lists(gpu, scene, view, 2048, 4)
    assert ovf_full == 0
    seen = np.unique(full[(full > 0) & (full <= 256)])
    _say(f"[bin-lists] counts: max {int(full.max())}, {seen.size} distinct values <= 256")
    depths = sorted({1, 2, 63, 64, 65} | {int(seen[0]), int(seen[len(seen) // 2]), int(seen[-1])})
    for depth in depths:
        cb, lb, ob = _bin_lists(gpu, scene, view, depth, 2)
        cs, ls, os_ = _bin_lists(gpu, scene, view, depth, 4)
        assert np.array_equal(cb, full) and np.array_equal(cs, full), depth
        assert ob == os_ == int(np.sum(full > depth)), depth
        for t in np.flatnonzero((full > 0) & (full <= depth)):
            a, b = lb[t, :full[t]], ls[t, :full[t]]
            assert np.array_equal(np.sort(a), np.sort(b)), (depth, t)
            assert np.all(np.diff(a >> shift) >= 0) and np.all(np.diff(b >> shift) >= 0), (depth, t)


RAGGED = [
    (1, 1, 0), (7, 5, 0), (8, 8, 1), (9, 9, 2), (37, 23, 3), (129, 65, 0), (255, 257, 1),
]


@pytest.mark.parametrize("flags", [0, 8], ids=["tile8", "tile16"])
@pytest.mark.parametrize("w,h,aov", RAGGED)
def test_ragged_sizes(gpu, w, h, aov, flags):
    """Odd sizes: partial 8x8 tiles, and with 16x16 bin tiles partial strips
    and super-tiles (a strip whose right tile lies outside the image)."""
    rng = np.random.default_rng(w * 1000 + h)
    view = synth.View(w, h, float(rng.uniform(-1, 1)), float(rng.uniform(0, 1)), float(rng.uniform(0.8, 1)),
                      float(rng.uniform(60, 360)), aov, synth.yaw_pitch_rotation(rng.uniform(0, 6), rng.uniform(-1, 1)))
    tris = synth.scene(400, w + h)
    _say(f"[ragged] {w}x{h} aov={aov} k={view.k:.3f} bin flags {flags}")
    ids, dep, _ = _render(gpu, tris, view, flags=flags)
    st = compare(view, tris, ids, dep, oracle.render(view, tris))
    _say("[ragged] " + st.line())
    assert st.ok(), st.notes


def test_empty_and_degenerate(gpu):
    view = synth.View(64, 48, 0.2, 0.5, 0.9, 200.0)
    _say("[edge] empty scene")
    for flags in (0, 8):
        ids, dep, _ = _render(gpu, np.zeros((9, 0), np.float32), view, flags=flags)
        assert np.all(ids == 0xFFFFFFFF) and np.all(np.isinf(dep)), flags
    _say("[edge] degenerate triangles")
    t1 = [1, 0, 0, 0, 1, 0, 1, 1, 0]          # plane through O
    t2 = [1, 2, 3, 1, 2, 3, -1, 0, 2]         # two equal vertices
    t3 = [0, 0, 5, 0, 0, 5, 0, 0, 5]          # a point
    t4 = [-50, -40, 3, 60, -30, 3, 0, 70, 3]  # big, in front
    tris = np.ascontiguousarray(np.array([t1, t2, t3, t4], dtype=np.float32).T)
    ids, dep, _ = _render(gpu, tris, view)
    ref = oracle.render(view, tris)
    st = compare(view, tris, ids, dep, ref)
    assert st.ok(), st.notes
    assert set(np.unique(ids)) <= {3, 0xFFFFFFFF}


def test_winding_and_antipode(gpu):
    """Both windings cover the same pixels and nothing at the antipode."""
    view = synth.View(128, 64, 0.0, 1.0, 1.0, 360.0)
    tri = np.array([[-1, -1, 5, 1, -1, 5, 0, 1, 5]], dtype=np.float32).T
    rev = tri[[0, 1, 2, 6, 7, 8, 3, 4, 5]]
    a, da, _ = _render(gpu, np.ascontiguousarray(tri), view)
    b, db, _ = _render(gpu, np.ascontiguousarray(rev), view)
    ref = oracle.render(view, tri)
    assert np.array_equal(a, b)
    assert np.array_equal(a != 0xFFFFFFFF, ref.id != 0xFFFFFFFF)


@pytest.mark.parametrize("flags", [0, 8], ids=["tile8", "tile16"])
def test_overflow_falls_back(gpu, flags):
    """A tiny bin depth overflows; the rasterizer gathers itself: same bits."""
    view, tris = synth.view_small(), synth.scene_small()
    _say(f"[overflow] depth 4 vs 1024, bin flags {flags}")
    a_ids, a_dep, ovf_a = _render(gpu, tris, view, depth=1024)
    b_ids, b_dep, ovf_b = _render(gpu, tris, view, depth=4, flags=flags)
    assert ovf_a == 0 and ovf_b > 0
    assert np.array_equal(a_ids, b_ids)
    assert np.array_equal(a_dep.view(np.uint32), b_dep.view(np.uint32))


def test_tile16_lists_are_the_union_of_tile_lists(gpu):
    """A 16x16 bin tile's list holds every triangle of its four 8x8 tiles'
    lists, in depth-bucket order, on both binner shapes (the rasterizer
    keeps each tile's share with the 8x8 binner's own test)."""
    view = synth.View(200, 150, -0.4, 0.3, 0.9, 300.0, 0, synth.yaw_pitch_rotation(1.0, 0.3))
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(synth.scene(20000, 5))
    shift = 0
    while (256 << shift) < scene.ntri:
        shift += 1
    t8, l8, _ = _bin_lists(gpu, scene, view, 2048, 4)
    ntx = (view.width + 7) // 8
    nty = (view.height + 7) // 8
    nsx = (ntx + 1) // 2
    nsup = nsx * ((nty + 1) // 2)
    for shape in (2, 4):
        c16, l16, o16 = _bin_lists(gpu, scene, view, 1024, 8 | shape)
        assert o16 == int(np.sum(c16[:nsup] > 1024))  # overflowed lists are counted, not written
        for t in range(ntx * nty):
            tx, ty = t % ntx, t // ntx
            s_idx = (ty // 2) * nsx + tx // 2
            if c16[s_idx] > 1024:
                continue
            sup = set(l16[s_idx, :c16[s_idx]].tolist())
            assert set(l8[t, :t8[t]].tolist()) <= sup, (shape, t)
        for s_idx in range(nsup):
            if c16[s_idx] <= 1024:
                lst = l16[s_idx, :c16[s_idx]]
                assert np.all(np.diff(lst >> shift) >= 0), (shape, s_idx)
    _say(f"[tile16] lists: {int(t8.sum())} 8x8 entries, {int(c16[:nsup].sum())} 16x16 entries, {o16} overflowed")


@pytest.mark.parametrize("bin_flags", [0, 8], ids=["tile8", "tile16"])
def test_early_exit_is_exact(gpu, bin_flags):
    """The nearest-first early exit (stop once every pixel beats the depth
    lower bound of the current bucket) skips only triangles that cannot win:
    same bits as testing every listed triangle, on the 1920x1080 frames of
    the 1M-triangle scene where it skips most of the lists."""
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(synth.scene_1m())
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    ref8 = None
    for q, view in enumerate(synth.views_1080p_sweep()):
        fr = pipeline.render(scene, view, bin_flags=bin_flags)
        if bin_flags:
            ref8 = pipeline.render(scene, view)
            torch.cuda.synchronize()
            assert torch.equal(ref8.tri_id, fr.tri_id) and torch.equal(ref8.depth.view(torch.int32),
                                                                       fr.depth.view(torch.int32)), q
        ids = torch.empty_like(fr.tri_id)
        dep = torch.empty_like(fr.depth)
        vsr.vsr_raster_stats(view, 0, fr.map, scene.setup, scene.ntri, fr.bins, pipeline.DEFAULT_BIN_DEPTH, ids, dep,
                             stats, no_early_exit=True)
        torch.cuda.synchronize()
        assert torch.equal(ids, fr.tri_id), q
        assert torch.equal(dep.view(torch.int32), fr.depth.view(torch.int32)), q
        _say(f"[early-exit] view {q}: identical with every listed triangle tested")


def test_fragment_counts_agree_across_bin_tiles(gpu):
    """With every listed triangle tested, the covered (pixel, triangle) pairs
    counted by the instrumented rasterizer are a property of the frame alone:
    8x8 lists (a wave per tile) and 16x16 lists (a wave per 16x8 strip, two
    pixels per lane, each triangle tested on both) count the same number, over
    every tile of the frame; the 16x16 form executes more tests per covered
    pair, never fewer."""
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(synth.scene_1m())
    view = synth.views_1080p_sweep()[1]
    ntiles = ((view.width + 7) // 8) * ((view.height + 7) // 8)
    got = {}
    for name, flags, depth in (("tile8", 0, 256), ("tile16", vsr.VSR_BIN_TILE16, 512)):
        fr = pipeline.render(scene, view, bin_depth=depth, bin_flags=flags)
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        ids, dep = torch.empty_like(fr.tri_id), torch.empty_like(fr.depth)
        vsr.vsr_raster_stats(view, 0, fr.map, scene.setup, scene.ntri, fr.bins, depth, ids, dep, stats,
                             no_early_exit=True)
        torch.cuda.synchronize()
        assert torch.equal(ids, fr.tri_id) and torch.equal(dep.view(torch.int32), fr.depth.view(torch.int32))
        got[name] = [int(x) for x in stats[:4].cpu()]
        _say(f"[fragments] {name}: tests {got[name][0]}, covered {got[name][1]}, triangles {got[name][2]}, "
             f"tiles {got[name][3]}")
    assert got["tile8"][1] == got["tile16"][1] > 0
    assert got["tile8"][3] == got["tile16"][3] == ntiles
    assert got["tile16"][0] >= got["tile16"][1] and got["tile8"][0] >= got["tile8"][1]


def _cone_min_depth(tris):
    """FP64 smallest ray-plane depth d / (g . N_hat) over the unit directions g
    of each triangle's vertex cone: d / cos(theta), theta the angle from the
    plane's unit normal (facing away from O) to the cone (0 inside it; else
    to the nearest vertex direction or edge arc)."""
    a = tris[0:3].T.astype(np.float64)
    b = tris[3:6].T.astype(np.float64)
    c = tris[6:9].T.astype(np.float64)
    n = np.cross(a - b, c - b)
    d = np.einsum("ij,ij->i", a, n)
    u = n * np.sign(d)[:, None] / np.linalg.norm(n, axis=1, keepdims=True)
    dist = np.abs(d) / np.linalg.norm(n, axis=1)
    sig = np.sign(np.einsum("ij,ij->i", a, np.cross(b, c)))
    v = [x / np.linalg.norm(x, axis=1, keepdims=True) for x in (a, b, c)]
    cos_t = np.max([np.einsum("ij,ij->i", u, x) for x in v], axis=0)
    inside = np.ones(len(a), bool)
    for p, q in ((v[0], v[1]), (v[1], v[2]), (v[2], v[0])):
        e = np.cross(p, q) * sig[:, None]
        e /= np.linalg.norm(e, axis=1, keepdims=True)
        x = np.einsum("ij,ij->i", e, u)
        inside &= x >= 0
        w = u - e * x[:, None]
        pq = np.cross(p, q)
        within = (np.einsum("ij,ij->i", np.cross(p, w), pq) >= 0) & (np.einsum("ij,ij->i", np.cross(w, q), pq) >= 0)
        cos_t = np.where(within, np.maximum(cos_t, np.sqrt(np.maximum(0.0, 1.0 - x * x))), cos_t)
    cos_t = np.where(inside, 1.0, cos_t)
    return dist / cos_t


def test_depth_lower_bound_below_cone_minimum(gpu):
    """The FP32 depth lower bound of every live triangle (64-byte setup
    record, word 13, rank order) is at most the FP64 smallest depth over its
    vertex cone, and close to it: on shell, small, grazing and sliver
    triangles."""
    torch, pipeline, vsr = gpu
    rng = np.random.default_rng(77)
    shell = synth.scene(4000, 78)
    small = synth.small_triangles(4000, 79)
    # grazing: planes passing 1e-3..1e-1 from O relative to their size
    cen = rng.normal(size=(2000, 3)) * 5
    t1 = rng.normal(size=(2000, 3))
    t1 -= cen * (np.einsum("ij,ij->i", t1, cen) / np.einsum("ij,ij->i", cen, cen))[:, None]
    t2 = np.cross(cen, t1)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 /= np.linalg.norm(t2, axis=1, keepdims=True)
    off = cen * 10 ** rng.uniform(-3, -1, size=(2000, 1))
    ga, gb, gc = cen + off, cen + 2 * t1 + off * 0.5, cen - 2 * t1 + 3 * t2
    grazing = np.concatenate([ga.T, gb.T, gc.T]).astype(np.float32)
    # slivers: one vertex 1e-3..1e-2 off the opposite edge
    sa = rng.normal(size=(2000, 3)) * 4
    sb = sa + rng.normal(size=(2000, 3))
    sc = 0.5 * (sa + sb) + rng.normal(size=(2000, 3)) * 10 ** rng.uniform(-3, -2, size=(2000, 1))
    sliver = np.concatenate([sa.T, sb.T, sc.T]).astype(np.float32)
    tris = np.ascontiguousarray(np.concatenate([shell, small, grazing, sliver], axis=1))
    scene = pipeline.Scene(tris)
    torch.cuda.synchronize()
    n = tris.shape[1]
    rec = scene.setup[256:256 + 64 * n].cpu().numpy().view(np.float32).reshape(n, 16)
    tid = rec[:, 14].view(np.uint32)
    lb = rec[:, 13].astype(np.float64)
    live = np.isfinite(lb)
    rmin = _cone_min_depth(tris)[tid[live]]
    ratio = lb[live] / rmin
    _say(f"[depth-lb] {int(live.sum())} live of {n}: lb / cone minimum max {ratio.max():.9f}, "
         f"median {np.median(ratio):.6f}, min {ratio.min():.3e}")
    assert np.all(ratio <= 1.0)
    assert np.median(ratio) > 0.9999


@pytest.mark.parametrize("mode", [0x200, 0x400, 0xA00, 0xC00, 0x1200, 0x1A00, 1],
                         ids=["binned-blocks", "binned-supertiles", "tile16-blocks", "tile16-supertiles",
                              "persistent", "persistent-tile16", "fused"])
def test_submit_matches_single_views(gpu, mode):
    torch, pipeline, vsr = gpu
    tris = synth.scene(3000, 23)
    scene = pipeline.Scene(tris)
    views = synth.random_views(6, 99, resolutions=((96, 64), (130, 70), (64, 64)))
    _say(f"[submit] 6 mixed views vs single, mode {mode}")
    batch = pipeline.Batch([(scene, v) for v in views], mode=mode)
    outs = batch.submit()
    torch.cuda.synchronize()
    for v, (ids_t, dep_t) in zip(views, outs):
        fr = pipeline.render(scene, v)
        torch.cuda.synchronize()
        assert np.array_equal(pipeline.ids_u32(ids_t), pipeline.ids_u32(fr.tri_id))
        assert np.array_equal(dep_t.cpu().numpy().view(np.uint32), fr.depth.cpu().numpy().view(np.uint32))
    # and against the oracle for one of them
    v = views[0]
    st = compare(v, tris, pipeline.ids_u32(outs[0][0]), outs[0][1].cpu().numpy(), oracle.render(v, tris))
    assert st.ok(), st.notes


def _same_lens(view, yaw, pitch):
    return synth.View(view.width, view.height, view.k, view.l, view.s, view.omega_deg, view.aov,
                      synth.yaw_pitch_rotation(yaw, pitch))


@pytest.mark.parametrize("fmt", [0, 1], ids=["f32", "oct16"])
def test_map_is_orientation_free(gpu, fmt):
    """The map holds camera-frame directions: views that differ only in
    orientation build byte-identical maps, and a view rendered with another
    orientation's map equals rendering it with its own."""
    torch, pipeline, vsr = gpu
    tris = synth.scene(2500, 31)
    scene = pipeline.Scene(tris)
    base = synth.View(150, 90, -0.3, 0.7, 0.8, 230.0, 0)
    va, vb = _same_lens(base, 0.3, 0.2), _same_lens(base, 2.5, -0.9)
    fa = pipeline.render(scene, va, fmt=fmt)
    fb = pipeline.render(scene, vb, fmt=fmt)
    torch.cuda.synchronize()
    ntiles = ((base.width + 7) // 8) * ((base.height + 7) // 8)
    plane = ntiles * 64 * (12 if fmt == 0 else 4)
    caps = (plane + 255) // 256 * 256
    for lo, hi in ((0, plane), (caps, caps + 32 * ntiles)):  # directions, tile caps (not the padding)
        assert torch.equal(fa.map[lo:hi], fb.map[lo:hi])
    # render vb through va's map
    ids = torch.empty_like(fb.tri_id)
    dep = torch.empty_like(fb.depth)
    depth = pipeline.DEFAULT_BIN_DEPTH
    vsr.vsr_bin(vb, fmt, fa.map, scene.setup, scene.ntri, depth, 0, fa.bins)
    vsr.vsr_raster(vb, fmt, fa.map, scene.setup, scene.ntri, fa.bins, depth, ids, dep)
    torch.cuda.synchronize()
    assert torch.equal(ids, fb.tri_id)
    assert np.array_equal(dep.cpu().numpy().view(np.uint32), fb.depth.cpu().numpy().view(np.uint32))
    if fmt == 0:
        st = compare(vb, tris, pipeline.ids_u32(ids), dep.cpu().numpy(), oracle.render(vb, tris))
        _say("[map-orient] " + st.line())
        assert st.ok(), st.notes


@pytest.mark.parametrize("mode", [0x200, 0x400, 0xA00, 1], ids=["binned-blocks", "binned-supertiles", "tile16", "fused"])
def test_submit_shares_lens_maps(gpu, mode):
    """A batch whose views repeat lenses in several orientations (maps built
    once per lens) renders every view exactly as alone."""
    torch, pipeline, vsr = gpu
    tris = synth.scene(3000, 37)
    scene = pipeline.Scene(tris)
    lenses = [synth.View(120, 80, 0.6, 0.5, 1.0, 160.0, 0), synth.View(96, 96, -0.5, 0.2, 0.7, 280.0, 1)]
    views = [_same_lens(lenses[q % 2], 0.7 * q, 0.25 * (q % 3) - 0.25) for q in range(7)]
    batch = pipeline.Batch([(scene, v) for v in views], mode=mode)
    outs = batch.submit()
    torch.cuda.synchronize()
    _say(f"[submit-lens] {len(views)} views over 2 lenses, mode {mode}")
    for v, (ids_t, dep_t) in zip(views, outs):
        fr = pipeline.render(scene, v)
        torch.cuda.synchronize()
        assert np.array_equal(pipeline.ids_u32(ids_t), pipeline.ids_u32(fr.tri_id))
        assert np.array_equal(dep_t.cpu().numpy().view(np.uint32), fr.depth.cpu().numpy().view(np.uint32))


def _render_fused(gpu, tris, view, fmt=0):
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(tris)
    fr = pipeline.render_fused(scene, view, fmt=fmt)
    torch.cuda.synchronize()
    return pipeline.ids_u32(fr.tri_id), fr.depth.cpu().numpy()


FUSED_CASES = [
    ("small", synth.view_small(), lambda: synth.scene_small()),
    ("rot", synth.View(200, 150, -0.4, 0.3, 0.9, 300.0, 0, synth.yaw_pitch_rotation(1.0, 0.3)),
     lambda: synth.scene(1500, 17)),
    ("ragged", synth.View(37, 23, 0.7, 0.2, 0.95, 200.0, 3, synth.yaw_pitch_rotation(4.0, -0.8)),
     lambda: synth.scene(300, 5)),
    ("dense", synth.View(160, 96, 0.1, 0.8, 0.9, 250.0, 0, synth.yaw_pitch_rotation(0.2, 0.1)),
     lambda: synth.scene(60000, 29)),
    ("empty", synth.View(40, 30, 0.0, 1.0, 1.0, 90.0), lambda: np.zeros((9, 0), np.float32)),
]


@pytest.mark.parametrize("name,view,make", FUSED_CASES, ids=[c[0] for c in FUSED_CASES])
def test_fused_matches_plain(gpu, name, view, make):
    """vsr_render (depth-sliced, fused) gives the same bits as bin + raster."""
    tris = make()
    _say(f"[fused] {name} {view.width}x{view.height} T={tris.shape[1]}")
    a_ids, a_dep, _ = _render(gpu, tris, view, depth=2048)
    b_ids, b_dep = _render_fused(gpu, tris, view)
    assert np.array_equal(a_ids, b_ids)
    assert np.array_equal(a_dep.view(np.uint32), b_dep.view(np.uint32))
    if tris.shape[1] <= 5000:
        st = compare(view, tris, b_ids, b_dep, oracle.render(view, tris))
        assert st.ok(), st.notes


def test_oct16_tier_small(gpu):
    """Octahedral fp16 map: angular error and coverage mismatch vs FP64."""
    view, tris = synth.view_small(), synth.scene_small()
    g16, _ = _gpu_map(gpu, view, fmt=1)
    ref, ok = oracle.perspective_map(view)
    err = _angle(g16[ok], ref[ok])
    ids, dep, _ = _render(gpu, tris, view, fmt=1)
    rr = oracle.render(view, tris)
    mism = float(np.mean(ids != rr.id))
    _say(f"[oct16] angular error mean {err.mean():.2e} max {err.max():.2e}; id mismatch fraction {mism:.4f}")
    assert err.max() < 2e-3
    assert mism < 0.05


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_1080p_1m_sampled(gpu, q):
    """1920x1080 view of 1M small triangles + radius-100 icosphere on the
    stratified sample (every pixel of 64 random 16x16 tiles + 16,384 random
    pixels) against the oracle."""
    torch, pipeline, vsr = gpu
    view = synth.views_1080p_sweep()[q]
    tris = _scene_1m()
    _say(f"[1080p] k={view.k} omega={view.omega_deg}")
    ids, dep, ovf = _render(gpu, tris, view)
    pix = synth.pixel_sample(view.width, view.height, seed=100 + q)
    ref = oracle.render(view, tris, pix)
    st = compare(view, tris, ids, dep, ref, pix)
    _say(f"[1080p] k={view.k}: " + st.line() + f" overflow={ovf} " + "; ".join(st.notes))
    assert st.ok(), st.notes


_SCENE_1M = None


def _scene_1m():
    global _SCENE_1M
    if _SCENE_1M is None:
        _SCENE_1M = synth.scene_1m()
    return _SCENE_1M
