"""GPU parity of the other map generators (sections 2.2.2, 2.2.4, 2.2.7-2.2.9)
and the Brown-Conrady distortion (section 2.3) against the FP64 oracle:
map directions, full rendered frames (the rule of tests/parity.py), exact
binning on 360-degree maps, aliasing-free frames across cube seams, and the
full-size sampled case."""
import sys

import numpy as np
import pytest

import oracle
import synth
from aa_parity import compare_aa, delta_plane, eps_delta
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


def _v(w, h, lens, n=1, p=(), rot=None, k=0.0, l=0.0, s=1.0, om=90.0, aov=0):
    return synth.View(w, h, k, l, s, om, aov, rot or synth.yaw_pitch_rotation(0.0, 0.0), lens=lens, lens_n=n,
                      lens_p=tuple(p))


LENS_VIEWS = [
    ("equirect", _v(256, 128, synth.LENS_EQUIRECT, rot=synth.yaw_pitch_rotation(0.7, 0.3))),
    ("equirect_ragged", _v(101, 53, synth.LENS_EQUIRECT)),
    ("cube", _v(6 * 40, 40, synth.LENS_CUBE, rot=synth.yaw_pitch_rotation(-0.4, 0.9))),
    ("cube_ragged", _v(125, 19, synth.LENS_CUBE)),
    ("screens3", _v(3 * 64, 48, synth.LENS_SCREENS, 3, (55.0,), rot=synth.yaw_pitch_rotation(1.3, -0.2))),
    ("screens5", _v(5 * 23, 37, synth.LENS_SCREENS, 5, (70.0,))),
    ("vr", _v(160, 90, synth.LENS_VR, p=(100.0, 0.42, 0.22, 0.05), rot=synth.yaw_pitch_rotation(2.0, 0.1))),
    ("vr_odd", _v(97, 61, synth.LENS_VR, p=(90.0, 0.5, 0.0, 0.0))),
    ("panorama", _v(240, 60, synth.LENS_PANORAMA, p=(250.0,), rot=synth.yaw_pitch_rotation(0.2, -0.6))),
    ("dome", _v(96, 96, synth.LENS_DOME, p=(20.0, 15.0, 0.2), rot=synth.yaw_pitch_rotation(0.3, 0.4))),
    ("dome_ragged", _v(77, 51, synth.LENS_DOME, p=(-10.0, 0.0, 0.0))),
    ("distort_diag", _v(120, 80, synth.LENS_UNIVERSAL, p=(0.12, -0.03, 0.02, -0.01, 0.01, -0.02), k=0.4,
                        l=0.6, s=0.9, om=160.0, aov=1)),
    ("distort_kneg", _v(96, 96, synth.LENS_UNIVERSAL, p=(-0.1, 0.02, 0.0, 0.0, 0.0, 0.0), k=-0.6, l=1.0,
                        s=1.0, om=170.0)),
]


def _angle(a, b):
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    d = np.einsum("...i,...i->...", a, b)
    return np.arctan2(c, d)


def _gpu_map(gpu, view):
    torch, pipeline, vsr = gpu
    buf = torch.empty(vsr.vsr_map_bytes(view.width, view.height, 0), dtype=torch.uint8, device="cuda")
    pipeline.build_map(view, 0, 0, buf)
    out = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    vsr.vsr_map_unpack(view, 0, buf, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name,view", LENS_VIEWS, ids=[n for n, _ in LENS_VIEWS])
def test_lens_map_matches_oracle(gpu, name, view):
    _say(f"[lens map] {name} {view.width}x{view.height}")
    g = _gpu_map(gpu, view)
    ref, ok = oracle.perspective_map(view)
    gok = np.any(g != 0, axis=-1)
    assert np.array_equal(gok, ok)
    err = _angle(g[ok], ref[ok])
    _say(f"[lens map] {name}: max angular error {err.max():.3e} rad")
    assert err.max() < 1e-6


@pytest.mark.parametrize("name,view", LENS_VIEWS, ids=[n for n, _ in LENS_VIEWS])
def test_lens_frame_matches_oracle(gpu, name, view):
    torch, pipeline, vsr = gpu
    tris = synth.scene(1500, 31)
    _say(f"[lens frame] {name}")
    fr = pipeline.render(pipeline.Scene(tris), view, bin_depth=1024)
    torch.cuda.synchronize()
    ref = oracle.render(view, tris)
    st = compare(view, tris, pipeline.ids_u32(fr.tri_id), fr.depth.cpu().numpy(), ref)
    # coarse pictures (a few degrees per pixel) overflow some tiles: those
    # gather their own candidates, which the parity covers
    _say(f"[lens frame] {name}: " + st.line() + f" overflowed tiles {vsr.vsr_bin_overflow(fr.bins)}")
    assert st.ok(), st.notes


@pytest.mark.parametrize("name", ["equirect", "cube", "vr", "panorama"])
def test_lens_binning_is_exact(gpu, name):
    """360-degree and segmented maps: real bins (every binner shape) give the
    same bits as listing every triangle in every tile."""
    torch, pipeline, vsr = gpu
    view = dict(LENS_VIEWS)[name]
    tris = synth.scene(5000, 8)
    scene = pipeline.Scene(tris)
    ref = pipeline.render(scene, view, bin_depth=2048, bin_flags=vsr.VSR_BIN_ALL)
    torch.cuda.synchronize()
    ref_ids, ref_dep = ref.tri_id.clone(), ref.depth.clone()
    for depth, shape in ((1024, 0), (256, vsr.VSR_BIN_BLOCKS), (256, vsr.VSR_BIN_SUPERTILES),
                         (512, vsr.VSR_BIN_TILE16 | vsr.VSR_BIN_BLOCKS), (512, vsr.VSR_BIN_TILE16 | vsr.VSR_BIN_SUPERTILES)):
        fr = pipeline.render(scene, view, bin_depth=depth, bin_flags=shape)
        torch.cuda.synchronize()
        assert torch.equal(fr.tri_id, ref_ids) and torch.equal(fr.depth, ref_dep), (name, shape)


@pytest.mark.parametrize("name", ["cube", "screens3", "vr", "equirect", "dome"])
def test_lens_aa_matches_oracle(gpu, name):
    """Aliasing-free frames on segmented maps: the delta plane takes no
    difference across cube faces, screens or eyes, on both sides."""
    torch, pipeline, vsr = gpu
    view = dict(LENS_VIEWS)[name]
    tris = synth.scene(1500, 32)
    fr = pipeline.render_aa(pipeline.Scene(tris), view)
    d = delta_plane(fr, view)
    rng = np.random.default_rng(4)
    for _ in range(300):
        i, j = int(rng.integers(0, view.width)), int(rng.integers(0, view.height))
        want = oracle.delta(view, i, j)
        assert abs(d[j, i] - want) <= eps_delta(want) * want, (name, i, j, d[j, i], want)
    compare_aa(gpu, view, tris, fr, tag=f"aa {name}")


def test_lens_argument_errors_reach_no_kernel(gpu):
    torch, pipeline, vsr = gpu
    buf = torch.empty(vsr.vsr_map_bytes(64, 32, 0), dtype=torch.uint8, device="cuda")
    for view in [_v(64, 32, 9), _v(64, 32, synth.LENS_SCREENS, 0, (60.0,)),
                 _v(64, 32, synth.LENS_SCREENS, 3, (180.0,)), _v(64, 32, synth.LENS_VR, p=(90.0, 0.5, -0.5, -0.5)),
                 _v(64, 32, synth.LENS_PANORAMA, p=(400.0,)), _v(64, 32, synth.LENS_DOME, p=(95.0, 0.0, 0.0)),
                 _v(64, 32, synth.LENS_DOME, p=(0.0, 0.0, 1.0))]:
        with pytest.raises(vsr.VsrError):
            pipeline.build_map(view, 0, 0, buf)


def test_equirect_4k_1m_sampled(gpu):
    """Full size: a 4096x2048 equirectangular view of the 1M-triangle scene,
    sampled pixels (every triangle tested per sampled pixel)."""
    torch, pipeline, vsr = gpu
    view = _v(4096, 2048, synth.LENS_EQUIRECT, rot=synth.yaw_pitch_rotation(0.3, 0.1))
    tris = synth.scene_1m()
    _say("[equirect 4K x 1M] render")
    fr = pipeline.render(pipeline.Scene(tris), view)
    torch.cuda.synchronize()
    pix = synth.pixel_sample(view.width, view.height, 5, n_tiles=8, tile=16, n_pixels=2000)
    _say(f"[equirect 4K x 1M] oracle on {len(pix)} pixels")
    ref = oracle.render(view, tris, pix)
    st = compare(view, tris, pipeline.ids_u32(fr.tri_id), fr.depth.cpu().numpy(), ref, pixels=pix)
    _say("[equirect 4K x 1M] " + st.line())
    assert st.ok(), st.notes
