"""Pins of the CPU oracle against facts fixed by the thesis and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
hand-derived examples, a library primitive (numpy matmul), brute force on tiny
inputs, enumeration of every partition, or invariants that hold at any size.
Thesis passages: cost-function subsection (SAD and SATD equations), HEVC
background section (CU quad-tree 64..8, DC/planar intra, RDO), related-work
section (depth-bound reuse), analysis-refinement appendix (refine-intra table).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

S_QP12 = 49479  # round(sqrt(0.57) * 65536): lambda(QP 12) = 0.57 exactly


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    synth.build(force=False)


# ----------------------------------------------------------------- lambda / bits
def test_lambda_anchor_and_doubling():
    assert oracle.sqrt_lambda_q16(12) == S_QP12
    s = [oracle.sqrt_lambda_q16(q) for q in range(52)]
    # lambda doubles every 3 QP, so sqrt(lambda) doubles every 6 QP (rounding: +-1).
    for q in range(46):
        assert abs(s[q + 6] - 2 * s[q]) <= 1, q
    # ... and grows by sqrt(2) every 3 QP (two roundings: 0.5 + 0.5 * sqrt(2)).
    for q in range(49):
        assert abs(s[q + 3] - s[q] * 2 ** 0.5) <= 0.5 + 0.5 * 2 ** 0.5, q
    assert all(a < b for a, b in zip(s, s[1:]))


def _sqrt_lambda_q16_exact(qp):
    """round(sqrt(lambda) * 65536), lambda = 0.57 * 2^((QP - 12) / 3), in exact integer
    arithmetic (no libm): x = sqrt(lambda) * 2^16 satisfies x^6 = 0.57^3 * 2^(QP - 12) * 2^96,
    a rational number, so floor(2x) is an integer 6th root and round(x) = (floor(2x) + 1) // 2."""
    num, den = 64 * 57 ** 3 * 2 ** (qp + 84), 10 ** 6  # (2x)^6 = num / den
    lo, hi = 0, 1 << 30
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if mid ** 6 * den <= num:
            lo = mid
        else:
            hi = mid - 1
    return (lo + 1) // 2


# The multipliers of the QPs the workloads use (QP 12 and the ladder's 22/27/30/32/35/37).
S_TABLE = {12: 49479, 22: 157085, 27: 279893, 30: 395829, 32: 498713, 35: 705287, 37: 888606}


def test_lambda_table_exact_all_qps():
    """Every one of the 52 multipliers, in the oracle and in libmr's host code, equals the
    exact integer rounding of sqrt(0.57 * 2^((QP - 12) / 3)) * 65536, so no libm difference
    (pow vs exp2, float vs double) can shift an integer cost by one."""
    from paper_2301_12191_amd import mr
    L = mr.lib()
    exact = [_sqrt_lambda_q16_exact(q) for q in range(52)]
    for q, v in S_TABLE.items():
        assert exact[q] == v, q
    for q in range(52):
        assert oracle.sqrt_lambda_q16(q) == exact[q], q
        assert L.mr_sqrt_lambda_q16(q) == exact[q], q
    assert L.mr_sqrt_lambda_q16(-1) == -1 and L.mr_sqrt_lambda_q16(52) == -1


def _exp_golomb_lengths(limit):
    """Codeword lengths of ue(k), by enumerating the code tree: 2^L codewords of length 2L+1."""
    lengths = []
    L = 0
    while len(lengths) < limit:
        lengths += [2 * L + 1] * (2 ** L)
        L += 1
    return lengths[:limit]


def _se_order(limit):
    """Signed mapping order of se(v): codeNum 0, 1, 2, 3, 4, ... -> 0, 1, -1, 2, -2, ..."""
    vals = [0]
    m = 1
    while len(vals) < limit:
        vals += [m, -m]
        m += 1
    return vals[:limit]


def test_signed_exp_golomb_lengths():
    n = 4 * 1024 + 8
    lengths = _exp_golomb_lengths(n)
    order = _se_order(n)
    for code_num, v in enumerate(order):
        if abs(v) <= 1024:
            assert oracle.se_bits(v) == lengths[code_num], v
    for v, b in [(0, 1), (1, 3), (-1, 3), (4, 7), (-4, 7), (8, 9), (-8, 9), (64, 15),
                 (-64, 15), (512, 21), (-512, 21)]:
        assert oracle.se_bits(v) == b


# ------------------------------------------------------------------------- SATD
H4 = np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], dtype=np.int64)


def _satd_matmul(resid):
    n = resid.shape[0]
    tiles = resid.reshape(n // 4, 4, n // 4, 4).transpose(0, 2, 1, 3).astype(np.int64)
    coeff = H4 @ tiles @ H4.T
    per_tile = np.abs(coeff).sum(axis=(2, 3))
    assert np.all(per_tile % 2 == 0)  # last butterfly: |a+b| + |a-b| = 2 max(|a|, |b|)
    return int(per_tile.sum() // 2)


def test_satd_worked_example():
    d = np.array([[5, -3, 0, 2], [1, 1, -4, 0], [7, 0, 0, -1], [-2, 3, 2, 6]])
    assert np.abs(H4 @ d @ H4.T).sum() == 164
    assert oracle.satd(d) == 82


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_satd_equals_matrix_product(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(20):
        r = rng.integers(-255, 256, size=(n, n))
        assert oracle.satd(r) == _satd_matmul(r)


def test_satd_closed_forms():
    for c in (-255, -7, 0, 1, 3, 200):
        assert oracle.satd(np.full((8, 8), c)) == 4 * 8 * abs(c)  # 4 tiles x 8|c|
    for (i, j, a) in [(0, 0, 5), (1, 2, -9), (3, 3, 255)]:
        r = np.zeros((4, 4), int)
        r[i, j] = a
        assert oracle.satd(r) == 8 * abs(a)


def test_satd_pairwise_halving_matches_per_tile():
    """The thesis's C++ SATD halves once per 8x4 pair of 4x4 tiles; per-tile halving is equal."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        r = rng.integers(-255, 256, size=(4, 8))
        left = int(np.abs(H4 @ r[:, :4] @ H4.T).sum())
        right = int(np.abs(H4 @ r[:, 4:] @ H4.T).sum())
        pad = np.zeros((8, 8), int)
        pad[:4] = r
        assert oracle.satd(pad) == (left + right) >> 1


# ------------------------------------------------------------------------ intra
def test_intra_no_neighbours_is_128():
    cur = synth.white_noise(3, 64, 64)
    for mode in (1, 2):
        for n in (8, 16, 32, 64):
            assert np.all(oracle.intra_predict(cur, 0, 0, n, mode) == 128)


def test_intra_flat_neighbours():
    cur = np.full((64, 64), 77, np.uint8)
    for mode in (1, 2):
        for n in (8, 16, 32):
            assert np.all(oracle.intra_predict(cur, 32 - n if n < 32 else 32, 32, n, mode) == 77)


def _ramp_picture():
    pic = np.zeros((32, 32), np.uint8)
    for k in range(16):
        pic[7, 8 + k] = 16 + 8 * k    # top row of the CU at (8, 8)
        pic[8 + k, 7] = 16 + 8 * k    # left column
    return pic


def test_intra_worked_example_symmetric_ramp():
    pic = _ramp_picture()
    assert np.all(oracle.intra_predict(pic, 8, 8, 8, 2) == 44)
    pl = oracle.intra_predict(pic, 8, 8, 8, 1)
    assert list(pl[0]) == [24, 32, 39, 47, 54, 62, 69, 77]
    assert list(pl[7]) == [77, 77, 78, 78, 79, 79, 80, 80]


def test_intra_worked_example_asymmetric():
    """top[x] = 16 + 8x, left[y] = 200: hand-derived values catch a transposed planar."""
    pic = np.zeros((32, 32), np.uint8)
    for k in range(16):
        pic[7, 8 + k] = 16 + 8 * k
        pic[8 + k, 7] = 200
    pl = oracle.intra_predict(pic, 8, 8, 8, 1)
    assert pl[0, 0] == 112 and pl[0, 7] == 84 and pl[7, 0] == 193 and pl[7, 7] == 140
    assert np.all(oracle.intra_predict(pic, 8, 8, 8, 2) == 122)


def test_intra_substitution_right_and_bottom_edges():
    # 24x16 picture; CU (16, 8) n=8: top-right and bottom-left neighbours are outside.
    pic = np.zeros((16, 24), np.uint8)
    pic[7:16, 15] = 40      # left column incl. corner
    pic[7, 16:24] = 80      # top row
    pl = oracle.intra_predict(pic, 16, 8, 8, 1)
    assert pl[0, 0] == 60 and pl[0, 7] == 78 and pl[7, 0] == 43 and pl[7, 7] == 60
    assert np.all(oracle.intra_predict(pic, 16, 8, 8, 2) == 60)


def test_intra_substitution_from_top_row_when_left_missing():
    pic = np.zeros((16, 16), np.uint8)
    pic[7, :] = 10 + 10 * np.arange(16)
    pl = oracle.intra_predict(pic, 0, 8, 8, 1)
    assert pl[0, 0] == 15 and pl[0, 7] == 81 and pl[7, 0] == 15 and pl[7, 7] == 50
    assert np.all(oracle.intra_predict(pic, 0, 8, 8, 2) == 28)


# --------------------------------------------------------------------------- ME
def test_identical_frames_zero_motion():
    sc = synth.Scene(11, 200, 136, 4, 8, 0)
    f = sc.render(0)
    out = oracle.ctu_search(f, f, 32, 8)
    assert np.all(out["mv"] == 0)
    for (x0, y0, n) in [(0, 0, 64), (64, 64, 8), (136, 72, 16), (128, 64, 32)]:
        assert oracle.cu_motion_search(f, f, x0, y0, n, 8, 32) == (0, 0, 0)


@pytest.mark.parametrize("sx,sy", [(3, -2), (-7, 5), (0, 6), (-4, -4)])
def test_known_global_shift_recovered(sx, sy):
    W, H, R = 128, 96, 8
    big = synth.white_noise(77, W + 64, H + 64)
    ox = oy = 24
    ref = big[oy:oy + H, ox:ox + W]
    cur = big[oy + sy:oy + sy + H, ox + sx:ox + sx + W]   # cur(x, y) = ref(x + sx, y + sy)
    for n in (8, 16, 32):
        for y0 in range(0, H, n):
            for x0 in range(0, W, n):
                inside = (x0 + sx >= 0 and y0 + sy >= 0 and x0 + n + sx <= W
                          and y0 + n + sy <= H)
                if inside:
                    assert oracle.cu_motion_search(cur, ref, x0, y0, n, R, 27) == (sx, sy, 0)


def _brute_force_me(cur, ref, x0, y0, n, R, s):
    """numpy brute force: edge-padded reference, all candidates, first minimum in raster order."""
    H, W = cur.shape
    pad = np.pad(ref.astype(np.int64), R + n, mode="edge")
    c = np.pad(cur.astype(np.int64), ((0, 7), (0, 7)), mode="edge")[y0:y0 + n, x0:x0 + n]
    lengths = _exp_golomb_lengths(4 * 4 * R + 8)
    order = _se_order(4 * 4 * R + 8)
    bits = {v: lengths[order.index(v)] for v in range(-4 * R, 4 * R + 1, 4)}
    best = None
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            blk = pad[y0 + dy + R + n:y0 + dy + R + 2 * n, x0 + dx + R + n:x0 + dx + R + 2 * n]
            sad = int(np.abs(c - blk).sum())
            j = sad * 65536 + s * (bits[4 * dx] + bits[4 * dy])
            if best is None or j < best[0]:
                best = (j, dx, dy, sad)
    return best[1], best[2], best[3]


def test_me_matches_brute_force_tiny():
    sc = synth.Scene(5, 40, 24, 3, 6, 2)
    ref, cur = sc.render(0), sc.render(1)
    for qp in (12, 32, 45):
        s = oracle.sqrt_lambda_q16(qp)
        for (x0, y0, n) in [(0, 0, 8), (32, 16, 8), (16, 8, 16), (0, 0, 16)]:
            assert oracle.cu_motion_search(cur, ref, x0, y0, n, 4, qp) == \
                _brute_force_me(cur, ref, x0, y0, n, 4, s)


def test_me_tie_break_first_in_raster_order():
    # Current columns alternate 100/0 and reference columns 0/100: dx = -1 and dx = +1 both
    # give SAD 0 with equal MV bits (dx = 0 does not match); the first in raster order
    # (dx inner) is dx = -1.
    cur = np.zeros((32, 32), np.uint8)
    cur[:, 0::2] = 100
    ref = np.zeros((32, 32), np.uint8)
    ref[:, 1::2] = 100
    assert oracle.cu_motion_search(cur, ref, 8, 8, 8, 4, 30) == (-1, 0, 0)
    # Transposed pattern: dy = -1 comes before dy = +1 (dy outer).
    assert oracle.cu_motion_search(cur.T.copy(), ref.T.copy(), 8, 8, 8, 4, 30) == (0, -1, 0)


# --------------------------------------------------------------- leaf modes/ties
def test_leaf_mode_ties():
    flat = np.full((64, 64), 90, np.uint8)
    rec = oracle.ctu_nodes(flat, flat, 30, 4, 0, 0)
    f = {k: i for i, k in enumerate(oracle.NODE_FIELDS)}
    # Inter at MV (0,0) costs 1+1+1 = 3 bits, planar 3 bits, both SATD 0: inter wins the tie.
    assert np.all(rec[1:, f["mode"]] == 0)
    noisy_ref = synth.white_noise(9, 64, 64)
    rec = oracle.ctu_nodes(flat, noisy_ref, 30, 2, 0, 0)
    # Intra is exact on flat content; planar (3 bits) beats DC (4 bits) at equal SATD,
    # except the top-left CUs with no neighbours, predicted as 128 by both.
    for i in range(1, 85):
        assert rec[i, f["satd_planar"]] == rec[i, f["satd_dc"]]
        assert rec[i, f["mode"]] == 1


# ------------------------------------------------------------------- quad-tree DP
def _partitions(nodes, d, lx, ly, s):
    """Yield (J, leaves) for every admissible coding of node (d, lx, ly)."""
    off = [0, 1, 5, 21]
    idx = off[d] + ly * (1 << d) + lx
    kind = nodes[idx, 0]
    if kind == 0:
        yield 0, ()
        return
    flag = s if d < 3 else 0
    if kind == 2:
        yield int(nodes[idx, 8]) + flag, ((d, lx, ly),)
    if d < 3:
        kids = [list(_partitions(nodes, d + 1, 2 * lx + (k & 1), 2 * ly + (k >> 1), s))
                for k in range(4)]
        extra = flag if kind == 2 else 0
        for combo in itertools.product(*kids):
            yield sum(c[0] for c in combo) + extra, sum((c[1] for c in combo), ())


def test_partition_count_is_83522():
    nodes = np.zeros((85, 11), np.int64)
    nodes[:, 0] = 2
    assert sum(1 for _ in _partitions(nodes, 0, 0, 0, 1)) == 83522


def _depth_of_partition(leaves, uh, uw, cx, cy):
    dm = np.full((uh, uw), 255, np.uint8)
    for d, lx, ly in leaves:
        n8 = 8 >> d
        y0, x0 = (cy * 64 + ly * (64 >> d)) // 8, (cx * 64 + lx * (64 >> d)) // 8
        dm[y0:y0 + n8, x0:x0 + n8] = d
    return dm


@pytest.mark.parametrize("W,H,qp,seed", [(64, 64, 12, 1), (64, 64, 32, 2), (64, 64, 45, 3),
                                         (40, 48, 27, 4), (64, 24, 37, 5)])
def test_dp_equals_exhaustive_enumeration(W, H, qp, seed):
    sc = synth.Scene(seed, W, H, 3, 3, 1)
    ref, cur = sc.render(0), sc.render(1)
    R = 3
    s = oracle.sqrt_lambda_q16(qp)
    nodes = oracle.ctu_nodes(cur, ref, qp, R, 0, 0)
    best = min(_partitions(nodes, 0, 0, 0, s), key=lambda t: t[0])
    out = oracle.ctu_search(cur, ref, qp, R)
    assert out["cost"][0, 0] == best[0]
    # The oracle's partition attains the minimum.
    uh, uw = (H + 7) // 8, (W + 7) // 8
    costs = {leaves: j for j, leaves in _partitions(nodes, 0, 0, 0, s)}
    for leaves, j in costs.items():
        if np.array_equal(_depth_of_partition(leaves, uh, uw, 0, 0), out["depth"]):
            assert j == best[0]
            break
    else:
        raise AssertionError("oracle depth map is not an enumerated partition")


# -------------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def small_pair():
    sc = synth.Scene(21, 200, 136, 5, 10, 2)
    return sc.render(0), sc.render(1)


def _check_tree(out, W, H):
    depth = out["depth"]
    uh, uw = depth.shape
    for uy in range(uh):
        for ux in range(uw):
            d = depth[uy, ux]
            assert d <= 3
            n8 = 8 >> d
            y0, x0 = uy // n8 * n8, ux // n8 * n8
            blk = depth[y0:y0 + n8, x0:x0 + n8]
            assert np.all(blk == d)
            assert y0 + n8 <= uh and x0 + n8 <= uw  # leaf CU lies inside the coded picture
            assert np.all(out["mode"][y0:y0 + n8, x0:x0 + n8] == out["mode"][uy, ux])


def test_cost_identity_and_valid_tree(small_pair):
    ref, cur = small_pair
    for qp in (22, 32, 40):
        out = oracle.ctu_search(cur, ref, qp, 6)
        s = oracle.sqrt_lambda_q16(qp)
        assert np.all(out["cost"] == out["dist"] * 65536 + s * out["bits"])
        _check_tree(out, 200, 136)


def test_full_bounds_equal_full_search(small_pair):
    ref, cur = small_pair
    full = oracle.ctu_search(cur, ref, 30, 6)
    b = np.zeros(full["depth"].shape + (2,), np.uint8)
    b[..., 1] = 3
    pruned = oracle.ctu_search(cur, ref, 30, 6, bounds=b)
    for k in full:
        assert np.array_equal(full[k], pruned[k]), k


def test_pruned_cost_not_below_full(small_pair):
    ref, cur = small_pair
    full = oracle.ctu_search(cur, ref, 30, 6)
    rng = np.random.default_rng(3)
    lo = rng.integers(0, 4, size=full["depth"].shape)
    hi = np.minimum(3, lo + rng.integers(0, 2, size=lo.shape))
    b = np.stack([lo, hi], axis=-1).astype(np.uint8)
    pruned = oracle.ctu_search(cur, ref, 30, 6, bounds=b)
    assert np.all(pruned["cost"] >= full["cost"])
    _check_tree(pruned, 200, 136)


def test_force_bounds_reproduce_reference_depths(small_pair):
    ref, cur = small_pair
    full = oracle.ctu_search(cur, ref, 27, 6)
    b = oracle.depth_bounds(full["depth"], 200, 136, 200, 136, 0, 0)
    assert np.array_equal(b[..., 0], full["depth"]) and np.array_equal(b[..., 1], full["depth"])
    # Forced depths reproduce the partition whatever the QP of the dependent search.
    for qp in (22, 37):
        dep = oracle.ctu_search(cur, ref, qp, 6, bounds=b)
        assert np.array_equal(dep["depth"], full["depth"])


def test_depth_bounds_dyadic_and_non_dyadic():
    rng = np.random.default_rng(5)
    rd = rng.integers(0, 4, size=(68, 120)).astype(np.uint8)     # 960x540 reference
    b2 = oracle.depth_bounds(rd, 960, 540, 1920, 1080, 0, 0)     # x2
    uy, ux = np.mgrid[0:135, 0:240]
    assert np.array_equal(b2[..., 0], np.maximum(0, rd[uy // 2, ux // 2].astype(int) - 1))
    b4 = oracle.depth_bounds(rd, 960, 540, 3840, 2160, 0, 1)     # x4, refine n..n+1
    uy, ux = np.mgrid[0:270, 0:480]
    ds = np.maximum(0, rd[uy // 4, ux // 4].astype(int) - 2)
    assert np.array_equal(b4[..., 0], ds) and np.array_equal(b4[..., 1], np.minimum(3, ds + 1))
    # x3 (1280x720 -> 3840x2160): CU size 64>>d_r maps to 3 * (64>>d_r) pixels.
    rd3 = np.array([[0, 1, 2, 3] * 40] * 90, np.uint8)
    b3 = oracle.depth_bounds(rd3, 1280, 720, 3840, 2160, 0, 0)
    expect = {0: 0, 1: 0, 2: 1, 3: 2}
    for ux in range(0, 480, 7):
        xr = min((8 * ux + 4) * 1280 // 3840, 1279)
        assert b3[5, ux, 0] == expect[int(rd3[0, xr // 8])]
    # Bounds widen as requested and stay in [0, 3].
    bw = oracle.depth_bounds(rd, 960, 540, 1920, 1080, 3, 0)
    assert np.all(bw[..., 0] == 0) and np.array_equal(bw[..., 1], b2[..., 1])
