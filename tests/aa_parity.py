"""Comparison of a GPU aliasing-free frame (coverage, depth pass, dominant
id) with the FP64 oracle.

Tolerance, per pixel, from a first-order error model of the FP32 path:
  - a direction of the FP32 map is within 1e-6 rad of the exact one, so an
    edge or miter value n.G is off by at most EPS_E = 2e-6;
  - the global delta is a difference quotient of FP32 directions: relative
    error at most EPS_D = 4e-6 * delta + 1e-5 (checked by the tests);
  - a mask m = clamp(delta x + 1/2) therefore moves by at most
    DM = delta * EPS_E + EPS_D / 2 (|delta x| <= 1/2 on the ramp);
  - coverage = min(1, sum of masks) moves by at most n * DM over the n
    fragments that take part (oracle: fragments taken + the first left out);
  - a depth r = d / (G.N) moves by r (EPS_E / cos + 4 ulp); the depth pass
    sum m_fc r by at most 2 DM sum(r) + EPS_E sum(r / cos) + 1e-6 sum(r);
    two fragments whose depths are within those errors may swap order, which
    moves the depth pass by no more than the same bound;
  - the dominant id may differ only where the oracle's largest share leads
    the second by less than 2 n DM, or two fragments' depths are within
    rounding (relative step below 4e-6 / cos).
"""
import sys

import numpy as np

import oracle

EPS_E = 2e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def delta_plane(frame, view, fmt=0):
    """The AA map's delta plane (tile-major after the plain map) as [H, W]."""
    from paper_2003_10558_amd import vsr
    W, H = view.width, view.height
    off = vsr.vsr_map_bytes(W, H, fmt)
    ntx, nty = (W + 7) // 8, (H + 7) // 8
    raw = frame.map[off:off + ntx * nty * 64 * 4].cpu().numpy().view(np.float32)
    d = raw.reshape(nty, ntx, 8, 8).transpose(0, 2, 1, 3).reshape(nty * 8, ntx * 8)
    return d[:H, :W].astype(np.float64)


def eps_delta(delta):
    return 4e-6 * delta + 1e-5


def compare_aa(gpu, view, tris, fr, pix=None, tag=""):
    """Per-pixel parity of one AA frame with the oracle (whole frame or the
    listed flat pixel indices); returns (cov err / tol, depth err / tol)."""
    torch, pipeline, vsr = gpu
    torch.cuda.synchronize()
    cov = fr.coverage.cpu().numpy().astype(np.float64).reshape(-1)
    dp = fr.depth_pass.cpu().numpy().astype(np.float64).reshape(-1)
    dom = pipeline.ids_u32(fr.dominant).reshape(-1)
    lost = int(fr.lost.cpu().item())
    assert lost == 0, (tag, lost)
    ref = oracle.aa_render(view, tris, pix)
    if pix is None:
        pix = np.arange(view.width * view.height)
        flat = lambda a: a.reshape(-1)  # noqa: E731
    else:
        flat = lambda a: a  # noqa: E731
    delta = delta_plane(fr, view).reshape(-1)[pix]
    dm = delta * EPS_E + 0.5 * eps_delta(delta)
    n_near = flat(ref.n_near)
    tol_c = n_near * dm + 1e-6
    tol_d = 2 * dm * flat(ref.sum_r) + EPS_E * flat(ref.sum_rg) + 1e-6 * flat(ref.sum_r) + 1e-6
    ec = np.abs(cov[pix] - flat(ref.cov))
    ed = np.abs(dp[pix] - flat(ref.depth))
    bad_c = np.flatnonzero(ec > tol_c)
    bad_d = np.flatnonzero(ed > tol_d)
    assert bad_c.size == 0, (tag, pix[bad_c[:5]], cov[pix][bad_c[:5]], flat(ref.cov)[bad_c[:5]], tol_c[bad_c[:5]])
    assert bad_d.size == 0, (tag, pix[bad_d[:5]], dp[pix][bad_d[:5]], flat(ref.depth)[bad_d[:5]], tol_d[bad_d[:5]])
    diff = np.flatnonzero(dom[pix] != flat(ref.dom))
    if diff.size:
        sum_r = np.maximum(flat(ref.sum_r)[diff], 1e-300)
        near_tie = flat(ref.margin)[diff] <= 2 * tol_c[diff]
        order = flat(ref.gap)[diff] <= 4e-6 * np.maximum(1.0, flat(ref.sum_rg)[diff] / sum_r)
        unexplained = diff[~(near_tie | order)]
        assert unexplained.size == 0, (tag, pix[unexplained[:5]], dom[pix][unexplained[:5]],
                                       flat(ref.dom)[unexplained[:5]], flat(ref.margin)[unexplained[:5]])
    _say(f"  {tag}: {len(pix)} px, coverage err/tol max {np.max(ec / tol_c):.3f}, depth err/tol max "
         f"{np.max(ed / tol_d):.3f}, dominant differs at {diff.size} (explained)")
    return np.max(ec / tol_c), np.max(ed / tol_d)
