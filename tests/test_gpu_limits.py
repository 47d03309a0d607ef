"""The largest view the library accepts: 32768 x 32768 pixels (the limit on
each side), 1.07e9 pixels in 16.8 million 8x8 tiles, a 12.7 GiB vector map.
Byte offsets into the map, the bin lists and the outputs pass 2^32 here, so
any 32-bit index arithmetic on the path would show.  The scene is the small
configuration's (radius-10 icosphere + 500 shell triangles, k = 0.32,
l = 0.62, s = 0.86, 270 degrees), rotated.

  * the plain path (vsr_build_map -> vsr_bin -> vsr_raster, 8x8 bin tiles)
    matches the FP64 oracle on a sample: every pixel of 16 random 16x16
    tiles, of the four corner 8x8 tiles and 8,192 random pixels, under the
    parity rule (ids bit-exact outside flagged pixels, depth within 1e-5
    relative);
  * one binned vsr_submit of the same view with 16x16 bin tiles gives the
    same ids and depth bit for bit over the whole image.
The sampled values are gathered on the device; only they travel to the host.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare

pytestmark = pytest.mark.gpu

SIDE = 32768


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class _Sampled:
    """Values at the sample's pixels standing in for a full image in
    compare(), which indexes an image only with that pixel list."""

    def __init__(self, pix, vals):
        self.pix, self.vals = pix, vals

    def reshape(self, *shape):
        return self

    def __getitem__(self, idx):
        assert idx is self.pix
        return self.vals


def _corner_tiles(w, h):
    out = []
    for x0, y0 in ((0, 0), (w - 8, 0), (0, h - 8), (w - 8, h - 8)):
        jj, ii = np.meshgrid(np.arange(y0, y0 + 8), np.arange(x0, x0 + 8), indexing="ij")
        out.append((jj * w + ii).reshape(-1))
    return np.concatenate(out).astype(np.int64)


def test_largest_view():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_10558_amd import pipeline, vsr
    oracle.build(force=False)
    view = synth.View(SIDE, SIDE, 0.32, 0.62, 0.86, 270.0, 0, synth.yaw_pitch_rotation(0.3, 0.2))
    tris = synth.scene_small()
    scene = pipeline.Scene(tris)
    _say(f"[limits] {SIDE}x{SIDE} view, {tris.shape[1]} triangles: plain path, bin depth 64")
    fr = pipeline.render(scene, view, bin_depth=64)
    torch.cuda.synchronize()
    ovf = vsr.vsr_bin_overflow(fr.bins)
    pix = np.unique(np.concatenate([synth.pixel_sample(SIDE, SIDE, seed=77, n_tiles=16, n_pixels=8192),
                                    _corner_tiles(SIDE, SIDE)]))
    pt = torch.from_numpy(pix).to("cuda")
    ids = pipeline.ids_u32(fr.tri_id.view(-1)[pt])
    dep = fr.depth.view(-1)[pt].cpu().numpy()
    del pt
    ref = oracle.render(view, tris, pix)
    st = compare(view, tris, _Sampled(pix, ids), _Sampled(pix, dep), ref, pixels=pix)
    _say(f"[limits] plain: {st.line()} overflowed tiles {ovf}")
    assert st.ok(), st.notes
    ids_p, dep_p = fr.tri_id, fr.depth
    del fr  # map and bins
    torch.cuda.empty_cache()

    _say(f"[limits] {SIDE}x{SIDE}: binned submit, 16x16 bin tiles, bin depth 128")
    b = pipeline.Batch([(scene, view)], mode=vsr.VSR_SUBMIT_BINNED | vsr.VSR_SUBMIT_BIN_TILE16, bin_depth=128)
    outs = b.submit()
    torch.cuda.synchronize()
    ids_b, dep_b = outs[0]
    n_id = int((ids_b != ids_p).sum().item())
    n_dep = int((dep_b.view(torch.int32) != dep_p.view(torch.int32)).sum().item())
    _say(f"[limits] submit vs plain: id mismatches {n_id}, depth mismatches {n_dep}, "
         f"overflowed tiles {vsr.vsr_bin_overflow(b.workspace, True)}")
    del b, outs, ids_b, dep_b, ids_p, dep_p
    torch.cuda.empty_cache()
    assert n_id == 0 and n_dep == 0
