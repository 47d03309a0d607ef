"""GPU parity of the fragment-data step (section 1.1.4, vsr_resolve).

The GPU's barycentric weights and interpolated vertex data are compared with
the FP64 oracle (the paper's triple-product form) at pixels where both
agree on the winner.  The tolerance is derived per pixel: the weights of a
ray-plane point are a ratio b_A = G.(B x C) / G.N' (N' = (B-A) x (C-A)),
whose error from a direction error dG (the FP32 map: below 1e-6 rad) and
from FP32 products (about 32 ulp of the magnitudes involved) is bounded by
(1e-6 + 32 * 2^-24) * M / |G.N'| with M the largest |P| |Q - P| over the
triangle's edges; data error follows through the weights.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


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


def _dirs(view, pix):
    if getattr(view, "lens", synth.LENS_UNIVERSAL) != synth.LENS_UNIVERSAL:
        d, ok = oracle.perspective_map(view)
        return np.where(ok.reshape(-1)[pix, None], d.reshape(-1, 3)[pix], 0.0)
    out = np.zeros((len(pix), 3))
    for q, p in enumerate(pix):
        x, y = oracle.view_coord(int(p) % view.width, int(p) // view.width, view.width, view.height, view.aov)
        k, l, s, om = oracle.limits(view.k, view.l, view.s, view.omega_deg)
        g, ok = oracle.direction(x, y, k, l, s, om)
        out[q] = view.rot_matrix() @ g if ok else 0.0
    return out


def _check(gpu, view, tris, pix, seed, tag):
    torch, pipeline, vsr = gpu
    scene = pipeline.Scene(tris)
    fr = pipeline.render(scene, view)
    T = tris.shape[1]
    attr_np = synth.vertex_attributes(T, seed)
    bary, attr = pipeline.resolve(scene, view, fr, torch.from_numpy(attr_np), normalize3=True)
    torch.cuda.synchronize()
    ids = pipeline.ids_u32(fr.tri_id).reshape(-1)
    b_gpu = bary.cpu().numpy().reshape(3, -1)
    f_gpu = attr.cpu().numpy().reshape(attr_np.shape[1], -1)
    # pixels without a hit get zeros
    miss = ids == 0xFFFFFFFF
    assert not b_gpu[:, miss].any() and not f_gpu[:, miss].any()
    ref = oracle.render(view, tris, pix)
    sel = pix[(ids[pix] == ref.id) & (ref.id != 0xFFFFFFFF)]
    t = ids[sel]
    b_ref, f_ref = oracle.fragments(view, tris, attr_np, sel, t, normalize3=True)
    _, f_raw = oracle.fragments(view, tris, attr_np[:, 0:3], sel, t)   # the normal before normalising
    g = _dirs(view, sel)
    V = tris.astype(np.float64).reshape(3, 3, T)[:, :, t]                # [vertex, xyz, n]
    A, B, C = V[0].T, V[1].T, V[2].T
    Np = np.cross(B - A, C - A)
    s = np.abs(np.einsum("ij,ij->i", g, Np))
    M = np.max(np.stack([np.linalg.norm(B, axis=1) * np.linalg.norm(C - B, axis=1),
                         np.linalg.norm(C, axis=1) * np.linalg.norm(A - C, axis=1),
                         np.linalg.norm(A, axis=1) * np.linalg.norm(B - A, axis=1)]), axis=0)
    tol_b = (1e-6 + 32 * EPS32) * M / s + 1e-6
    db = np.abs(b_gpu[:, sel].T - b_ref).max(axis=1)
    a = np.abs(attr_np[:, :, t]).sum(axis=0).T                          # [n, K] sum over vertices
    tol_f = tol_b[:, None] * a + 8 * EPS32 * a
    tol_f[:, 0:3] /= np.maximum(np.linalg.norm(f_raw, axis=1), 1e-6)[:, None] / 2.0
    df = np.abs(f_gpu[:, sel].T - f_ref)
    ratio_b, ratio_f = (db / tol_b).max(), (df / tol_f).max()
    _say(f"[resolve-{tag}] {len(sel)} pixels: max |db| {db.max():.2e} (median tol {np.median(tol_b):.1e}), "
         f"max |df| {df.max():.2e}; worst error/tolerance b {ratio_b:.3f} f {ratio_f:.3f}")
    assert len(sel) > 100
    assert ratio_b <= 1.0 and ratio_f <= 1.0
    assert np.abs(b_gpu[:, sel].sum(axis=0) - 1.0).max() < 1e-5


def test_resolve_small_full_frame(gpu):
    view = synth.view_small()
    tris = synth.scene_small()
    pix = np.arange(view.width * view.height)
    _check(gpu, view, tris, pix, 11, "small")


def test_resolve_rotated_wide(gpu):
    view = synth.View(200, 150, -0.4, 0.3, 0.9, 300.0, 0, synth.yaw_pitch_rotation(1.0, 0.3))
    tris = synth.scene(1500, 19)
    pix = synth.pixel_sample(view.width, view.height, seed=12, n_tiles=8, n_pixels=4000)
    _check(gpu, view, tris, pix, 13, "rot")


def test_resolve_1080p_1m_sampled(gpu):
    view = synth.views_1080p_sweep()[1]
    tris = synth.scene_1m()
    pix = synth.pixel_sample(view.width, view.height, seed=14, n_tiles=2, n_pixels=1024)
    _check(gpu, view, tris, pix, 15, "1080p")


@pytest.mark.parametrize("nattr,normalize3", [(5, True), (4, False), (0, False), (3, True)])
def test_resolve_packed_identical(gpu, nattr, normalize3):
    """The packed copy holds the same values in one row per triangle: the
    images equal those from the arrays bit for bit (ragged view; on the
    1080p frame of the 1M-triangle scene for the five-component case)."""
    torch, pipeline, vsr = gpu
    cases = [(synth.View(77, 45, 0.3, 0.4, 0.95, 150.0, 0, synth.yaw_pitch_rotation(0.4, -0.2)),
              synth.scene(2500, 23))]
    if nattr == 5:
        cases.append((synth.views_1080p_sweep()[1], synth.scene_1m()))
    for view, tris in cases:
        scene = pipeline.Scene(tris)
        fr = pipeline.render(scene, view)
        vattr = torch.from_numpy(synth.vertex_attributes(tris.shape[1], 29)[:, :nattr].copy()) if nattr else None
        b0, a0 = pipeline.resolve(scene, view, fr, vattr, normalize3=normalize3)
        pk = pipeline.pack_resolve(scene, vattr)
        b1, a1 = pipeline.resolve(scene, view, fr, vattr, normalize3=normalize3, packed=pk)
        torch.cuda.synchronize()
        assert torch.equal(b0, b1)
        assert (a0 is None and a1 is None) or torch.equal(a0, a1)
        _say(f"[resolve-packed] {view.width}x{view.height} x {tris.shape[1]}, K={nattr}: identical")


def test_resolve_packed_widest_rows(gpu):
    """64 data components per vertex (rows of 204 floats, the largest the
    packing transposes through LDS) on a scene whose size is not a multiple
    of the packing block: the packed path equals the arrays bit for bit."""
    torch, pipeline, vsr = gpu
    view = synth.View(64, 48, 0.2, 0.5, 0.9, 140.0, 0, synth.yaw_pitch_rotation(0.2, 0.1))
    tris = synth.scene(1001, 47)
    scene = pipeline.Scene(tris)
    fr = pipeline.render(scene, view)
    rng = np.random.default_rng(48)
    vattr = torch.from_numpy(rng.standard_normal((3, 64, tris.shape[1])).astype(np.float32))
    b0, a0 = pipeline.resolve(scene, view, fr, vattr)
    b1, a1 = pipeline.resolve(scene, view, fr, vattr, packed=pipeline.pack_resolve(scene, vattr))
    torch.cuda.synchronize()
    assert torch.equal(b0, b1) and torch.equal(a0, a1)
    assert int((pipeline.ids_u32(fr.tri_id) != 0xFFFFFFFF).sum()) > 100


LENS_VIEWS = {
    "equirect": synth.View(160, 80, 0, 0, 1, 90, 0, synth.yaw_pitch_rotation(0.7, 0.3), lens=synth.LENS_EQUIRECT),
    "cube": synth.View(6 * 24, 24, 0, 0, 1, 90, 0, synth.yaw_pitch_rotation(-0.4, 0.9), lens=synth.LENS_CUBE),
    "dome": synth.View(96, 96, 0, 0, 1, 90, 0, synth.yaw_pitch_rotation(0.3, 0.4), lens=synth.LENS_DOME,
                       lens_p=(20.0, 15.0, 0.2)),
}


@pytest.mark.parametrize("name", sorted(LENS_VIEWS))
def test_resolve_lens_maps(gpu, name):
    """Fragment data on maps of other generators: the step reads only the
    map's directions, so the same parity holds on every pixel with one."""
    view = LENS_VIEWS[name]
    pix = np.arange(view.width * view.height)
    _check(gpu, view, synth.scene(1500, 41), pix, 43, name)
