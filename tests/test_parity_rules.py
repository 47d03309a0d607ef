"""The checker's own rules (tests/parity.py) on constructed cases, CPU only.

* Depth: a clean id-matching pixel passes within 1e-5 relative; a pixel
  whose winner is seen at grazing incidence (kappa = 1/|g . N_hat| above
  KAPPA_GRAZING) passes within kappa * GRAZING_PER_KAPPA and is counted as
  grazing.  The scene is one large triangle in the floor plane y = 0.05 (the
  camera's +y is down) seen through a 64 x 64 pinhole, so kappa = 1/g_y runs
  from about 1.4 at the bottom row to about 64 just below the horizon.
* Excused choices: at a pixel whose oracle winner lies within the edge band
  the GPU may show the triangle behind it; where the winner covers the pixel
  clearly, showing the one behind is an invalid choice.
"""
import numpy as np
import pytest

import synth
from parity import GRAZING_PER_KAPPA, KAPPA_GRAZING, _kappa, compare


def _floor():
    return np.array([[-100.0], [0.05], [0.01], [100.0], [0.05], [0.01], [0.0], [0.05], [200.0]], np.float32)


@pytest.fixture(scope="module")
def floor(oracle_lib):
    oracle = oracle_lib
    view = synth.View(64, 64, 1.0, 1.0, 1.0, 90.0)
    tris = _floor()
    ref = oracle.render(view, tris)
    pix = np.arange(64 * 64, dtype=np.int64)
    hit = (ref.flags.reshape(-1) == 0) & (ref.id.reshape(-1) != oracle.NO_HIT)
    kap = np.zeros(64 * 64)
    kap[hit] = _kappa(view, tris, pix[hit], ref.id.reshape(-1)[hit])
    return oracle, view, tris, ref, hit, kap


def _run(floor, scale):
    oracle, view, tris, ref, hit, kap = floor
    dep = (ref.depth.reshape(-1) * scale).astype(np.float32).reshape(64, 64)
    ids = ref.id.copy()
    return compare(view, tris, ids, dep, ref)


def test_floor_spans_both_classes(floor):
    _, _, _, _, hit, kap = floor
    assert hit.sum() > 1000
    assert (kap[hit] <= KAPPA_GRAZING).sum() > 300 and (kap[hit] > KAPPA_GRAZING).sum() > 30
    assert kap[hit].max() > 40


def test_exact_depth_passes(floor):
    st = _run(floor, 1.0)
    assert st.ok() and st.grazing == 0 and st.depth_bad == 0


def test_within_1e5_passes_everywhere(floor):
    st = _run(floor, 1.0 + 0.9e-5)
    assert st.ok() and st.grazing == 0


def test_over_1e5_fails_below_the_grazing_factor(floor):
    _, _, _, _, hit, kap = floor
    st = _run(floor, 1.0 + 1.5e-5)
    # 1.5e-5 is within kappa * GRAZING_PER_KAPPA for every kappa above the threshold
    assert 1.5e-5 < KAPPA_GRAZING * GRAZING_PER_KAPPA
    assert st.depth_bad == int((hit & (kap <= KAPPA_GRAZING)).sum())
    assert st.grazing == int((hit & (kap > KAPPA_GRAZING)).sum())
    assert not st.ok()


def test_grazing_bound_is_a_bound(floor):
    oracle, view, tris, ref, hit, kap = floor
    # every grazing pixel 1.5x beyond its own bound
    scale = np.ones(64 * 64)
    g = hit & (kap > KAPPA_GRAZING)
    scale[g] = 1.0 + 1.5 * kap[g] * GRAZING_PER_KAPPA
    dep = (ref.depth.reshape(-1) * scale).astype(np.float32).reshape(64, 64)
    st = compare(view, tris, ref.id.copy(), dep, ref)
    assert st.depth_bad == int(g.sum()) and st.grazing == 0


def _tri(a, b, c):
    return np.array([a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2]], np.float32)


def _one_pixel_case(oracle, front_eps, competitor=False):
    """1x1 pinhole (its pixel looks along +z exactly).  Front triangle at z=1
    whose edge x = front_eps passes the pixel direction at front_eps rad (the
    pixel is inside for front_eps < 0); a large back triangle at z=2."""
    view = synth.View(1, 1, 1.0, 1.0, 1.0, 90.0)
    e = front_eps
    tris = [_tri((e, -1.0, 1.0), (e, 1.0, 1.0), (1.0, 0.0, 1.0)),
            _tri((-5.0, -5.0, 2.0), (5.0, -5.0, 2.0), (0.0, 5.0, 2.0))]
    if competitor:
        # a third triangle 2e-6 behind the front one, its edge 0.5e-6 rad from the pixel
        z = 1.0 + 2e-6
        tris.append(_tri((0.5e-6 * z, -1.0, z), (0.5e-6 * z, 1.0, z), (1.0, 0.0, z)))
    tris = np.stack(tris, axis=1)
    ref = oracle.render(view, tris)
    return view, tris, ref


def test_choice_behind_a_band_winner_is_valid(oracle_lib):
    oracle = oracle_lib
    view, tris, ref = _one_pixel_case(oracle, -0.5e-6)
    assert int(ref.id[0, 0]) == 0 and ref.flags[0, 0] & oracle.FLAG_EDGE
    ids = np.array([[1]], np.uint32)  # the back triangle
    dep = np.array([[2.0]], np.float32)
    st = compare(view, tris, ids, dep, ref)
    assert st.excused_invalid_choice == 0 and st.ok()


def test_choice_behind_a_clear_winner_is_invalid(oracle_lib):
    oracle = oracle_lib
    view, tris, ref = _one_pixel_case(oracle, -1e-3, competitor=True)
    # the competitor's edge makes the pixel ambiguous, the winner covers it clearly
    assert int(ref.id[0, 0]) == 0 and ref.flags[0, 0] & oracle.FLAG_EDGE
    ids = np.array([[1]], np.uint32)
    dep = np.array([[2.0]], np.float32)
    st = compare(view, tris, ids, dep, ref)
    assert st.excused_invalid_choice == 1 and not st.ok()
