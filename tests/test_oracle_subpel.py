"""Pins of the oracle's sub-pel refinement (half- and quarter-pel ME by SATD).

Interpolation follows the H.265 luma fractional-sample process for 8-bit
samples (8-tap / 7-tap filters, 14-bit intermediate, default uni-prediction
rounding).  These tests pin it by values worked by hand from the filter table
(impulse responses, ramps), by symmetries the process must have (mirror,
transposition, constant images), and the search by exact half-pel targets and
by properties that hold for any picture.  The thesis names SATD as the cost of
quarter-pel motion estimation (cost-function subsection).
"""
import numpy as np
import pytest

import oracle
import synth

F = {k: i for i, k in enumerate(oracle.NODE_FIELDS)}


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    synth.build(force=False)


# ----------------------------------------------------------------- interpolation
def test_integer_positions_return_clamped_samples():
    img = synth.white_noise(3, 24, 16)
    for (x, y) in [(0, 0), (5, 7), (23, 15), (-3, 2), (30, -4), (12, 40)]:
        cx, cy = min(max(x, 0), 23), min(max(y, 0), 15)
        assert oracle.interp_qpel(img, 4 * x, 4 * y) == img[cy, cx]


def test_constant_picture_is_preserved_at_every_phase():
    img = np.full((20, 20), 137, np.uint8)
    for fx in range(4):
        for fy in range(4):
            assert oracle.interp_qpel(img, 4 * 9 + fx, 4 * 9 + fy) == 137


@pytest.mark.parametrize("axis", ["x", "y"])
def test_ramp_values_per_phase(axis):
    # f = 2t + 10 along one axis.  Sum_i c_i (i - 3) is 15, 32 and 49 for phases 1, 2 and 3,
    # so the filtered value is 64 f + 2 * {15, 32, 49}; adding 32 and shifting by 6 gives
    # f, f + 1 and f + 2.
    t = np.arange(32)
    img = np.tile((2 * t + 10).astype(np.uint8), (32, 1))
    if axis == "y":
        img = img.T.copy()
    for pos in (8, 13, 20):
        f = 2 * pos + 10
        for ph, add in [(0, 0), (1, 0), (2, 1), (3, 2)]:
            q = 4 * pos + ph
            got = oracle.interp_qpel(img, q, 4 * 16) if axis == "x" else \
                oracle.interp_qpel(img, 4 * 16, q)
            assert got == f + add, (axis, pos, ph)


def test_one_dimensional_impulse_response():
    # Row 8 holds a single 64 at x = 8.  At phase 1 the sample at integer position xi
    # sees tap 11 - xi of [-1, 4, -10, 58, 17, -5, 1, 0], times 64; negatives clip to 0.
    img = np.zeros((16, 24), np.uint8)
    img[8, 8] = 64
    got = [oracle.interp_qpel(img, 4 * xi + 1, 4 * 8) for xi in range(5, 12)]
    assert got == [1, 0, 17, 58, 0, 4, 0]
    # Phase 3 (the mirrored filter) around the same impulse.
    got3 = [oracle.interp_qpel(img, 4 * xi + 3, 4 * 8) for xi in range(4, 11)]
    assert got3 == [0, 4, 0, 58, 17, 0, 1]


def test_two_dimensional_impulse_response():
    # A single 64 at (8, 8); at half-pel in both axes the value is
    # (c_x * c_y * 64 * 64 >> 6) = c_x c_y * 64, then (v + 32) >> 6 = floor(c_x c_y / 64 + 1/2).
    img = np.zeros((16, 16), np.uint8)
    img[8, 8] = 64
    cases = {(7, 7): 25, (8, 8): 25, (7, 5): 3, (5, 5): 0, (6, 7): 0, (10, 7): 3, (7, 10): 3}
    for (xi, yi), v in cases.items():
        assert oracle.interp_qpel(img, 4 * xi + 2, 4 * yi + 2) == v, (xi, yi)


def test_mirror_maps_phase_one_to_phase_three():
    img = synth.white_noise(5, 40, 28)
    mir = img[:, ::-1].copy()
    W = img.shape[1]
    for qx in range(30, 120, 7):
        for qy in (40, 41, 42, 43):
            assert oracle.interp_qpel(img, qx, qy) == oracle.interp_qpel(mir, 4 * (W - 1) - qx, qy)


def test_transposed_picture_swaps_the_axes():
    img = synth.white_noise(6, 30, 26)
    tr = img.T.copy()
    for qx in range(10, 100, 5):
        for qy in range(12, 90, 9):
            assert oracle.interp_qpel(img, qx, qy) == oracle.interp_qpel(tr, qy, qx)


# ------------------------------------------------------------------------ search
def _shifted(ref, sx, sy, W, H):
    """cur(x, y) = interpolated ref at (x + sx/4, y + sy/4)."""
    cur = np.zeros((H, W), np.uint8)
    for y in range(H):
        for x in range(W):
            cur[y, x] = oracle.interp_qpel(ref, 4 * x + sx, 4 * y + sy)
    return cur


@pytest.mark.parametrize("mx,my,sx,sy", [(1, 0, 6, -2), (-2, 1, -10, 2), (0, 0, 2, 2),
                                         (0, 0, 0, 0), (3, -1, 12, -4)])
def test_exact_half_pel_targets_are_found(mx, my, sx, sy):
    """A CU whose content is the reference interpolated at a half-pel offset within one step of
    4 (mx, my) is matched exactly (SATD 0) by the half-pel stage and kept by the quarter-pel
    stage."""
    sc = synth.Scene(12, 64, 48, 3, 4, 0)
    ref = sc.render(0)
    cur = _shifted(ref, sx, sy, 64, 48)
    for (x0, y0, n) in [(16, 16, 16), (24, 8, 8), (8, 16, 32)]:
        assert oracle.subpel_refine(cur, ref, x0, y0, n, mx, my, 30) == (sx, sy, 0)


def test_identical_frames_keep_zero_motion():
    f = synth.Scene(13, 96, 64, 4, 6, 0).render(0)
    out = oracle.ctu_search(f, f, 30, 6, subpel=True)
    assert np.all(out["mv"] == 0) and np.all(out["dist"] == 0)


def test_subpel_refinement_properties():
    """For every CU: the final MV lies within 3 quarter-pels of 4 x the integer MV, its SATD
    does not exceed the integer MV's, and each CTU's J does not exceed the integer search's
    (the integer MV is the first candidate of every CU)."""
    W, H, R = 128, 64, 6
    sc = synth.Scene(14, W, H, 5, 6, 2)
    ref, cur = sc.render(0), sc.render(1)
    for ctu in [(0, 0), (1, 0)]:
        full = oracle.ctu_nodes(cur, ref, 32, R, *ctu)
        sub = oracle.ctu_nodes(cur, ref, 32, R, *ctu, subpel=True)
        ins = full[:, F["kind"]] == 2
        assert np.array_equal(full[ins, F["mx"]], sub[ins, F["mx"]])
        assert np.array_equal(full[ins, F["qmx"]], 4 * full[ins, F["mx"]])
        assert np.all(np.abs(sub[ins, F["qmx"]] - 4 * sub[ins, F["mx"]]) <= 3)
        assert np.all(np.abs(sub[ins, F["qmy"]] - 4 * sub[ins, F["my"]]) <= 3)
        assert np.all(sub[ins, F["leaf_j"]] <= full[ins, F["leaf_j"]])
    a = oracle.ctu_search(cur, ref, 32, R)
    b = oracle.ctu_search(cur, ref, 32, R, subpel=True)
    assert np.all(b["cost"] <= a["cost"]) and b["cost"].sum() < a["cost"].sum()
    s = oracle.sqrt_lambda_q16(32)
    assert np.array_equal(b["cost"], b["dist"] * 65536 + s * b["bits"])


@pytest.mark.parametrize("ref_w,cur_w,m,expect", [
    (64, 128, 6, 3), (64, 128, 5, 3), (64, 128, -5, -3),   # ratio 2: m/4 * 2, halves away
    (64, 64, 6, 2), (64, 64, -2, -1), (64, 64, 4, 1),       # ratio 1: m/4
])
def test_quarter_pel_seed_maps_scale_to_integer_centres(ref_w, cur_w, m, expect):
    rm = np.zeros(((ref_w // 2 + 7) // 8, (ref_w + 7) // 8, 2), np.int16)
    rm[..., 0], rm[..., 1] = m, -m
    seed = oracle.Seed(rm, ref_w, ref_w // 2, 0, qpel=True)
    assert oracle.mv_centre(seed, cur_w, cur_w // 2, 64, 0, 0, 8) == (expect, -expect)
