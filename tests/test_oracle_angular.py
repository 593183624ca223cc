"""Pins of the oracle's angular intra prediction and of the angular mode search.

Angular prediction follows the H.265 definition (the thesis's HEVC background section names
the DC, planar and angular intra modes): intraPredAngle per mode, a reference line made of
the corner and the neighbours along the prediction's own side, the other side projected past
the corner for negative angles (invAngle), and two-tap interpolation at 1/32 sample.
Readings: no reference smoothing, no edge filters; mode bits 4 for vertical (26) and 7 for
the other angular modes (most-probable-mode list {planar, DC, vertical}).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "intra_angular_4x4.json")


def _picture_with_neighbours(case, size=16):
    """A size x size picture whose block at (x0, y0) has the given corner, top and left
    neighbours (all inside the picture, so no substitution applies)."""
    pic = np.full((size, size), 7, dtype=np.uint8)
    x0, y0, n = case["x0"], case["y0"], case["n"]
    pic[y0 - 1, x0 - 1] = case["corner"]
    pic[y0 - 1, x0:x0 + 2 * n] = case["top"]
    pic[y0:y0 + 2 * n, x0 - 1] = case["left"]
    return pic


def test_hand_worked_examples():
    cases = json.load(open(GOLDEN))["cases"]
    for case in cases:
        pic = _picture_with_neighbours(case)
        got = oracle.intra_predict(pic, case["x0"], case["y0"], case["n"], case["mode_h265"] + 1)
        assert np.array_equal(got, np.array(case["pred_rows"])), case["mode_h265"]


def _interior_block(seed, n, size=160):
    rng = np.random.default_rng(seed)
    pic = rng.integers(0, 256, size=(size, size), dtype=np.uint8)
    x0 = int(rng.integers(1, size - 2 * n)) // 4 * 4 or 4
    y0 = int(rng.integers(1, size - 2 * n)) // 4 * 4 or 4
    return pic, x0, y0


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_pure_directions(n):
    """Integer-slope modes copy neighbours: 26 the top row, 10 the left column, 34 and 2 the
    45-degree diagonals, 18 the down-right diagonal through the corner."""
    pic, x0, y0 = _interior_block(100 + n, n)
    p = pic.astype(np.int64)
    top = lambda i: p[y0 - 1, x0 + i]
    left = lambda j: p[y0 + j, x0 - 1]
    corner = p[y0 - 1, x0 - 1]
    exp = {m: np.zeros((n, n), np.int64) for m in (2, 10, 18, 26, 34)}
    for y in range(n):
        for x in range(n):
            exp[26][y, x] = top(x)
            exp[10][y, x] = left(y)
            exp[34][y, x] = top(x + y + 1)
            exp[2][y, x] = left(x + y + 1)
            exp[18][y, x] = top(x - y - 1) if x > y else (corner if x == y else left(y - x - 1))
    for m, e in exp.items():
        assert np.array_equal(oracle.intra_predict(pic, x0, y0, n, m + 1), e), m


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_transpose_symmetry(n):
    """Mode m on the transposed picture is the transpose of mode 36 - m: the horizontal
    modes mirror the vertical ones, projections and interpolation included."""
    pic, x0, y0 = _interior_block(200 + n, n, size=max(160, 2 * n + 16))
    pt = np.ascontiguousarray(pic.T)
    for m in range(2, 35):
        a = oracle.intra_predict(pt, y0, x0, n, m + 1)
        b = oracle.intra_predict(pic, x0, y0, n, 36 - m + 1)
        assert np.array_equal(a, b.T), m


def test_predictions_stay_between_neighbour_extremes():
    """Two-tap interpolation with non-negative weights summing to 32 never leaves the range
    of the reference samples it reads (substituted neighbours at picture edges included)."""
    rng = np.random.default_rng(5)
    pic = rng.integers(30, 200, size=(72, 88), dtype=np.uint8)
    for n in (4, 8, 16, 32):
        for (x0, y0) in ((0, 0), (0, 40), (56, 0), (24, 32), (88 - n, 72 - n)):
            for m in range(2, 35):
                p = oracle.intra_predict(pic, x0, y0, n, m + 1)
                assert p.min() >= 30 and p.max() < 200, (n, x0, y0, m)


def test_angular_search_never_costs_more_and_uses_the_modes():
    """More candidate modes can only lower each CTU's cost; on textured content some CUs
    pick angular modes (codes 3..35), and J = D * 65536 + s * R still holds."""
    sc = synth.Scene(synth.SEED_BASE + 9, 200, 136, 6, 8, 2)
    ref, cur = sc.render(0), sc.render(1)
    qp, R = 37, 4
    a = oracle.ctu_search(cur, ref, qp, R)
    b = oracle.ctu_search(cur, ref, qp, R, angular=True)
    assert np.all(b["cost"] <= a["cost"])
    assert b["mode"].max() <= 35 and np.any(b["mode"] >= 3)
    s = oracle.sqrt_lambda_q16(qp)
    assert np.all(b["cost"] == b["dist"] * 65536 + s * b["bits"])


def test_angular_leaf_is_the_minimum_over_all_modes():
    """Per node, the chosen leaf J is the minimum over inter, planar, DC and the 33 angular
    modes, each recomputed here from the oracle's predictions and SATD (ties keep the
    earlier mode)."""
    sc = synth.Scene(synth.SEED_BASE + 10, 64, 64, 3, 4, 1)
    ref, cur = sc.render(0), sc.render(1)
    qp, R = 35, 2
    s = oracle.sqrt_lambda_q16(qp)
    rec = oracle.ctu_nodes(cur, ref, qp, R, 0, 0, angular=True)
    f = {k: i for i, k in enumerate(oracle.NODE_FIELDS)}
    for node in (0, 1, 7, 30, 84):
        d = 0 if node == 0 else 1 if node < 5 else 2 if node < 21 else 3
        local = node - (0, 1, 5, 21)[d]
        n = 64 >> d
        x0, y0 = (local % (1 << d)) * n, (local // (1 << d)) * n
        r = rec[node]
        best = (r[f["satd_inter"]] * 65536 + s * (1 + oracle.se_bits(4 * r[f["mx"]]) +
                                                   oracle.se_bits(4 * r[f["my"]])), 0)
        cands = [(r[f["satd_planar"]] * 65536 + s * 3, 1), (r[f["satd_dc"]] * 65536 + s * 4, 2)]
        block = cur[y0:y0 + n, x0:x0 + n].astype(np.int32)
        sat_min = None
        for m in range(2, 35):
            sd = oracle.satd(block - oracle.intra_predict(cur, x0, y0, n, m + 1))
            sat_min = sd if sat_min is None else min(sat_min, sd)
            cands.append((sd * 65536 + s * (4 if m == 26 else 7), m + 1))
        for j, code in cands:
            if j < best[0]:
                best = (j, code)
        assert r[f["leaf_j"]] == best[0] and r[f["mode"]] == best[1], node
        assert r[f["satd_angular_best"]] == sat_min
