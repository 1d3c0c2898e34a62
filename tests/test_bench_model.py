"""The benchmark's algorithmic cost model (the roofline's lane-operation
count) against the count written out by hand from its stated per-unit costs:
a change of a constant or of the formula shows up here."""
import numpy as np

import bench


def _stats(cam_box, cam_leaf, cam_rays, sh_box, sh_leaf, sh_rays, shaded):
    st = np.zeros(11)
    st[:6] = [cam_box, cam_leaf, cam_rays, sh_box, sh_leaf, sh_rays]
    st[10] = shaded
    return st


def test_cost_constants_and_peak():
    # one child-box test: 6 FMA, max3 + max (tmin), min3 + min (tmax), one compare
    assert bench.C_BOX == 6 + 2 + 2 + 1
    assert bench.PEAK_LANE_OPS == 256 * 4 * 16 * 2.4e9


def test_forward_count_by_hand():
    W, H, S, L = 8, 4, 2, 3
    st = _stats(1000, 50, 64, 7000, 300, 120, 40)
    samples = W * H * S
    want = ((1000 + 7000) * bench.C_BOX + (50 + 300) * bench.C_LEAF
            + samples * (bench.C_RNG + bench.C_CAM)
            + 40 * bench.C_FRAME + 40 * L * (bench.C_RNG + bench.C_LIGHT)
            + 120 * (bench.C_SETUP + bench.C_BRDF))
    assert bench.algorithmic_ops(st, W, H, S, L) == want


def test_adjoint_counts_by_hand():
    W, H, S, L = 8, 4, 2, 3
    st = _stats(1000, 50, 64, 7000, 300, 120, 40)
    f = bench.ADJ_FACTOR
    shade = (W * H * S * (bench.C_RNG + bench.C_CAM) + 40 * bench.C_FRAME * f
             + 40 * L * (bench.C_RNG + bench.C_LIGHT * f) + 120 * (bench.C_SETUP + bench.C_BRDF * f))
    trav = (1000 + 7000) * bench.C_BOX + (50 + 300) * bench.C_LEAF
    # the adjoint that takes the forward's decisions traces nothing
    assert bench.algorithmic_ops(st, W, H, S, L, backward=True) == shade
    # the one that traces its camera and shadow rays again counts the walks too
    assert bench.algorithmic_ops(st, W, H, S, L, backward=True, traced=True) == shade + trav


def test_shading_counts_only_samples_with_a_shading_point():
    W, H, S, L = 8, 4, 2, 3
    a = bench.algorithmic_ops(_stats(0, 0, 64, 0, 0, 0, 0), W, H, S, L)
    b = bench.algorithmic_ops(_stats(0, 0, 64, 0, 0, 0, 10), W, H, S, L)
    assert b - a == 10 * (bench.C_FRAME + L * (bench.C_RNG + bench.C_LIGHT))
