"""Pins of the oracle's seeded search (motion-vector reuse with refinement).

The seeded search takes, for every CU, the MV of the co-located unit of a
search at another resolution, scales it by the dimension ratios, clamps it and
searches the (2r+1)^2 displacements around it (x265 refine-mv option in the
analysis-refinement appendix; MV reuse across resolutions in the related-work
section).  The thesis's MV-refinement table is empty, so the mapping is a
reading; these tests pin the oracle to it by hand-worked centres, to the full
search where the two must agree, and to numpy brute force over each window.
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


def _const_map(w, h, mx, my):
    m = np.zeros(((h + 7) // 8, (w + 7) // 8, 2), np.int16)
    m[..., 0], m[..., 1] = mx, my
    return m


def _index_map(w, h):
    """MV of unit (ux, uy) = (ux, uy): the centre then names the co-located unit."""
    uh, uw = (h + 7) // 8, (w + 7) // 8
    m = np.zeros((uh, uw, 2), np.int16)
    m[..., 0] = np.arange(uw)[None, :]
    m[..., 1] = np.arange(uh)[:, None]
    return m


# ---------------------------------------------------------------- centre mapping
@pytest.mark.parametrize("ref_w,cur_w,m,expect", [
    (64, 64, 5, 5), (64, 64, -7, -7),                    # ratio 1: unchanged
    (64, 128, 3, 6), (64, 128, -5, -10),                 # ratio 2: doubled exactly
    (640, 960, 3, 5), (640, 960, -3, -5),                # 4.5 -> 5, halves away from zero
    (640, 960, 1, 2), (640, 960, -1, -2), (640, 960, 2, 3),
    (128, 64, 3, 2), (128, 64, -3, -2), (128, 64, 5, 3), (128, 64, 4, 2),  # ratio 1/2
    (40, 90, 2, 5), (40, 90, 1, 2), (40, 90, 3, 7),      # ratio 9/4: 4.5 -> 5, 2.25, 6.75
])
def test_centre_scaling_worked_examples(ref_w, cur_w, m, expect):
    # Same ratio on both axes; the MV map is constant so the co-located unit does not matter.
    rm = _const_map(ref_w, ref_w // 2, m, -m)
    seed = oracle.Seed(rm, ref_w, ref_w // 2, 0)
    assert oracle.mv_centre(seed, cur_w, cur_w // 2, 127, 0, 0, 8) == (expect, -expect)


def test_centre_clamped_to_keep_window_inside_range():
    rm = _const_map(32, 32, 5, -6)
    # Ratio 2 gives (10, -12); R = 10, r = 3 leaves centres in [-7, 7].
    assert oracle.mv_centre(oracle.Seed(rm, 32, 32, 3), 64, 64, 10, 0, 0, 16) == (7, -7)
    # r = R forces the centre to (0, 0): the window is the full search window.
    assert oracle.mv_centre(oracle.Seed(rm, 32, 32, 10), 64, 64, 10, 0, 0, 16) == (0, 0)
    # r = 0 with a large range keeps the scaled vector.
    assert oracle.mv_centre(oracle.Seed(rm, 32, 32, 0), 64, 64, 64, 0, 0, 16) == (10, -12)


def test_centre_names_the_unit_under_the_cu_centre():
    # Ratio 1: the n x n CU at (x0, y0) reads unit ((x0 + n/2) / 8, (y0 + n/2) / 8).
    rm = _index_map(256, 128)
    sd = oracle.Seed(rm, 256, 128, 0)
    assert oracle.mv_centre(sd, 256, 128, 64, 0, 0, 64) == (4, 4)
    assert oracle.mv_centre(sd, 256, 128, 64, 16, 8, 8) == (2, 1)
    assert oracle.mv_centre(sd, 256, 128, 64, 64, 64, 32) == (10, 10)
    # Ratio 2 (reference 128 x 64): CU 64 at (64, 0) has centre (96, 32) -> reference
    # sample (48, 16) -> unit (6, 2), whose MV (6, 2) doubles to (12, 4).
    sd = oracle.Seed(_index_map(128, 64), 128, 64, 0)
    assert oracle.mv_centre(sd, 256, 128, 64, 64, 0, 64) == (12, 4)
    # Unit-sized CUs map exactly like the depth bounds' units: centre 8u + 4.
    sd = oracle.Seed(_index_map(100, 68), 100, 68, 0)
    # cur 200 x 136: CU 8 at (192, 128): centre (196, 132) -> (98, 66) -> unit (12, 8);
    # MV (12, 8) scaled by 2 -> (24, 16).
    assert oracle.mv_centre(sd, 200, 136, 64, 192, 128, 8) == (24, 16)
    # Right edge: cur 204 wide, reference 102: CU 8 at x0 = 200 has centre 204 in the padded
    # picture -> 204 * 102 / 204 = 102, clamped to the last reference column 101 -> unit 12.
    sd = oracle.Seed(_index_map(102, 64), 102, 64, 0)
    assert oracle.mv_centre(sd, 204, 128, 64, 200, 0, 8) == (24, 0)


def test_invalid_seed_arguments():
    rm = _const_map(64, 64, 0, 0)
    f = np.zeros((64, 64), np.uint8)
    with pytest.raises(ValueError):
        oracle.ctu_search(f, f, 30, 4, seed=oracle.Seed(rm, 64, 64, 5))   # r > R
    with pytest.raises(ValueError):
        oracle.ctu_search(f, f, 30, 4, seed=oracle.Seed(rm, 64, 64, -1))
    with pytest.raises(ValueError):
        oracle.mv_centre(oracle.Seed(rm, 64, 64, 0), 0, 64, 4, 0, 0, 8)


# ------------------------------------------------------------- window search
def _se(v):
    """Signed Exp-Golomb length from its definition: codeNum k, length 2 floor(log2(k+1)) + 1."""
    v = int(v)
    k = 2 * v - 1 if v > 0 else -2 * v
    return 2 * (k + 1).bit_length() - 1


def _brute_window(cur, ref, x0, y0, n, cx, cy, r, s):
    """numpy brute force over the window centred at (cx, cy): clamped reference samples, first
    minimum in raster order (dy outer, dx inner)."""
    P = max(abs(cx), abs(cy)) + r + n
    pad = np.pad(ref.astype(np.int64), P, mode="edge")
    c = np.pad(cur.astype(np.int64), ((0, 7), (0, 7)), mode="edge")[y0:y0 + n, x0:x0 + n]
    best = None
    for dy in range(cy - r, cy + r + 1):
        for dx in range(cx - r, cx + r + 1):
            blk = pad[y0 + dy + P:y0 + dy + P + n, x0 + dx + P:x0 + dx + P + n]
            sad = int(np.abs(c - blk).sum())
            j = sad * 65536 + s * (_se(4 * dx) + _se(4 * dy))
            if best is None or j < best[0]:
                best = (j, dx, dy, sad)
    return best[1], best[2], best[3]


def _node_geometry(ctu_x, ctu_y):
    for d in range(4):
        n = 64 >> d
        for ly in range(1 << d):
            for lx in range(1 << d):
                yield ((0, 1, 5, 21)[d] + ly * (1 << d) + lx, ctu_x * 64 + lx * n,
                       ctu_y * 64 + ly * n, n)


@pytest.mark.parametrize("r", [0, 1, 2])
def test_seeded_me_matches_brute_force(r):
    W, H, R = 72, 40, 5
    sc = synth.Scene(31, W, H, 3, 5, 2)
    ref, cur = sc.render(0), sc.render(1)
    rng = np.random.default_rng(7 + r)
    rm = rng.integers(-4, 5, size=((H // 2 + 7) // 8, (W // 2 + 7) // 8, 2)).astype(np.int16)
    seed = oracle.Seed(rm, W // 2, H // 2, r)
    s = oracle.sqrt_lambda_q16(32)
    checked = 0
    for ctu_x, ctu_y in [(0, 0), (1, 0)]:
        rec = oracle.ctu_nodes(cur, ref, 32, R, ctu_x, ctu_y, seed=seed)
        for k, x0, y0, n in _node_geometry(ctu_x, ctu_y):
            if rec[k, F["kind"]] != 2:
                continue
            cx, cy = oracle.mv_centre(seed, W, H, R, x0, y0, n)
            assert abs(cx) <= R - r and abs(cy) <= R - r
            got = (rec[k, F["mx"]], rec[k, F["my"]], rec[k, F["sad"]])
            assert got == _brute_window(cur, ref, x0, y0, n, cx, cy, r, s), (k, x0, y0, n)
            checked += 1
    assert checked >= 10


def test_r0_takes_the_centre():
    W, H, R = 128, 64, 8
    sc = synth.Scene(41, W, H, 4, 6, 2)
    ref, cur = sc.render(0), sc.render(1)
    seed = oracle.Seed(_const_map(W // 2, H // 2, 3, -2), W // 2, H // 2, 0)  # ratio 2 -> (6, -4)
    rec = oracle.ctu_nodes(cur, ref, 30, R, 1, 0, seed=seed)
    inside = rec[:, F["kind"]] == 2
    assert inside.sum() == 85
    assert np.all(rec[inside, F["mx"]] == 6) and np.all(rec[inside, F["my"]] == -4)
    # SAD of the 64 x 64 CU at (64, 0) displaced by (6, -4), clamped reference rows.
    rows = np.clip(np.arange(0, 64) - 4, 0, H - 1)
    cols = np.clip(np.arange(64, 128) + 6, 0, W - 1)
    sad = np.abs(cur[0:64, 64:128].astype(np.int64) - ref[np.ix_(rows, cols)].astype(np.int64))
    assert rec[0, F["sad"]] == sad.sum()


@pytest.mark.parametrize("W,H,bounds", [(200, 136, False), (200, 136, True), (64, 64, False)])
def test_full_window_equals_full_search(W, H, bounds):
    R = 6
    sc = synth.Scene(51, W, H, 4, 6, 2)
    ref, cur = sc.render(0), sc.render(1)
    rng = np.random.default_rng(3)
    rm = rng.integers(-20, 21, size=((H + 7) // 8, (W + 7) // 8, 2)).astype(np.int16)
    b = None
    if bounds:
        full = oracle.ctu_search(cur, ref, 32, R)
        b = oracle.depth_bounds(full["depth"], W, H, W, H, 0, 1)
    want = oracle.ctu_search(cur, ref, 32, R, bounds=b)
    got = oracle.ctu_search(cur, ref, 32, R, bounds=b, seed=oracle.Seed(rm, W, H, R))
    for k in want:
        assert np.array_equal(want[k], got[k]), k


def test_window_holding_the_full_optimum_finds_it():
    W, H, R, r = 128, 128, 8, 2
    sc = synth.Scene(61, W, H, 5, 6, 2)
    ref, cur = sc.render(0), sc.render(1)
    rng = np.random.default_rng(11)
    rm = rng.integers(-3, 4, size=((H // 2 + 7) // 8, (W // 2 + 7) // 8, 2)).astype(np.int16)
    seed = oracle.Seed(rm, W // 2, H // 2, r)
    s = oracle.sqrt_lambda_q16(27)
    held = 0
    for ctu in [(0, 0), (1, 1)]:
        full = oracle.ctu_nodes(cur, ref, 27, R, *ctu)
        sdd = oracle.ctu_nodes(cur, ref, 27, R, *ctu, seed=seed)
        for k, x0, y0, n in _node_geometry(*ctu):
            fm, fmy = full[k, F["mx"]], full[k, F["my"]]
            cx, cy = oracle.mv_centre(seed, W, H, R, x0, y0, n)
            j_full = full[k, F["sad"]] * 65536 + s * (_se(4 * fm) + _se(4 * fmy))
            sm, smy = sdd[k, F["mx"]], sdd[k, F["my"]]
            j_seed = sdd[k, F["sad"]] * 65536 + s * (_se(4 * sm) + _se(4 * smy))
            assert j_seed >= j_full
            assert abs(sm - cx) <= r and abs(smy - cy) <= r
            if abs(fm - cx) <= r and abs(fmy - cy) <= r:
                held += 1
                assert (sm, smy, sdd[k, F["sad"]]) == (fm, fmy, full[k, F["sad"]])
    assert held >= 5


@pytest.mark.parametrize("sx,sy", [(6, -4), (-10, 8)])
def test_global_shift_found_from_scaled_seed(sx, sy):
    # cur(x, y) = ref(x + sx, y + sy); a half-resolution seed of (sx/2, sy/2) centres every
    # window on the true shift, so even r = 1 recovers it on CUs whose displaced block is
    # inside.  A zero seed with r = 1 cannot reach it and stays inside its window.
    W, H, R = 128, 96, 12
    big = synth.white_noise(78, W + 64, H + 64)
    ox = oy = 24
    ref = big[oy:oy + H, ox:ox + W]
    cur = big[oy + sy:oy + sy + H, ox + sx:ox + sx + W]
    hit = oracle.Seed(_const_map(W // 2, H // 2, sx // 2, sy // 2), W // 2, H // 2, 1)
    miss = oracle.Seed(_const_map(W // 2, H // 2, 0, 0), W // 2, H // 2, 1)
    out_hit = oracle.ctu_search(cur, ref, 27, R, seed=hit)
    out_miss = oracle.ctu_search(cur, ref, 27, R, seed=miss)
    for uy in range(H // 8):
        for ux in range(W // 8):
            x0, y0 = 8 * ux, 8 * uy
            # The unit's CU has depth d and size n; test units whose whole CU moves inside.
            n = 64 >> int(out_hit["depth"][uy, ux])
            cx0, cy0 = x0 - x0 % n, y0 - y0 % n
            if cx0 + sx >= 0 and cy0 + sy >= 0 and cx0 + n + sx <= W and cy0 + n + sy <= H:
                assert tuple(out_hit["mv"][uy, ux]) == (sx, sy)
            assert np.all(np.abs(out_miss["mv"][uy, ux]) <= 1)


# ------------------------------------------------- same resolution, several QPs
@pytest.mark.parametrize("r", [0, 1, 3, 6])
def test_same_qp_reuse_with_forced_depths_reproduces_the_master(r):
    """Ratio 1, same QP: the master's depths forced by (0, 0) bounds and its MVs as centres.
    Every CU of the forced partition is the master's CU, its centre is the master's MV (the
    full-search optimum over [-R, R]^2), and the clamped window still contains that MV, so the
    restricted arg-min is the same MV and every output equals the master's, for any r."""
    W, H, R, qp = 200, 136, 6, 30
    sc = synth.Scene(71, W, H, 5, 6, 2)
    ref, cur = sc.render(0), sc.render(1)
    master = oracle.ctu_search(cur, ref, qp, R)
    b = oracle.depth_bounds(master["depth"], W, H, W, H, 0, 0)
    dep = oracle.ctu_search(cur, ref, qp, R, bounds=b, seed=oracle.Seed(master["mv"], W, H, r))
    for k in master:
        assert np.array_equal(dep[k], master[k]), k


def test_multi_qp_dependents_stay_within_their_bounds_and_windows():
    """QPs 22, 26, 34, 38 reusing the QP-30 master (bounds (1, 1) at ratio 1, seed r = 2): every
    unit's depth lies within one of the master's, every MV within 2 of the master MV at the
    unit's CU centre, and J = D * 65536 + s * R per CTU.  (A CTU's J may fall below the full
    search's: motion is chosen by SAD cost, the leaf by SATD.)"""
    W, H, R, r = 136, 72, 8, 2
    sc = synth.Scene(72, W, H, 5, 7, 2)
    ref, cur = sc.render(0), sc.render(1)
    master = oracle.ctu_search(cur, ref, 30, R)
    b = oracle.depth_bounds(master["depth"], W, H, W, H, 1, 1)
    seed = oracle.Seed(master["mv"], W, H, r)
    for qp in (22, 26, 34, 38):
        dep = oracle.ctu_search(cur, ref, qp, R, bounds=b, seed=seed)
        full = oracle.ctu_search(cur, ref, qp, R)
        assert np.all(np.abs(dep["depth"].astype(int) - master["depth"].astype(int)) <= 1)
        for uy in range(H // 8):
            for ux in range(W // 8):
                n = 64 >> int(dep["depth"][uy, ux])
                x0, y0 = 8 * ux - (8 * ux) % n, 8 * uy - (8 * uy) % n
                cx, cy = oracle.mv_centre(seed, W, H, R, x0, y0, n)
                assert abs(int(dep["mv"][uy, ux, 0]) - cx) <= r
                assert abs(int(dep["mv"][uy, ux, 1]) - cy) <= r
        s_q = oracle.sqrt_lambda_q16(qp)
        assert np.array_equal(dep["cost"], dep["dist"] * 65536 + s_q * dep["bits"])
        assert not np.array_equal(dep["depth"], full["depth"]) or \
            not np.array_equal(dep["mv"], full["mv"]) or np.array_equal(dep["cost"], full["cost"])
