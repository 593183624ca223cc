"""GPU parity: libmr (HIP, through the C ABI) against the CPU oracle, element by element.

Integer outputs must match bit for bit: depth, mode, MV per 8x8 unit and the
int64 J / D / R per CTU.  Small cases run the oracle on every CTU; full-size
workloads (1080p at R 64, 2160p at R 128, the six-rung ladder) compare sampled
CTUs, which the oracle computes one by one.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("depth", "mode", "mv", "cost", "dist", "bits")


@pytest.fixture(scope="module")
def mr():
    import torch
    from paper_2301_12191_amd import mr as m
    assert torch.cuda.is_available()
    m.lib()
    oracle.build(force=False)
    synth.build(force=False)
    return m


def _gpu(mr, cur, ref, qp, R, bounds=None):
    import torch
    c = torch.from_numpy(np.ascontiguousarray(cur)).cuda()
    r = torch.from_numpy(np.ascontiguousarray(ref)).cuda()
    b = None if bounds is None else torch.from_numpy(np.ascontiguousarray(bounds)).cuda()
    out = mr.mr_ctu_search(c, r, qp, R, bounds=b)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _ctu_units(W, H, ctus):
    uh, uw = (H + 7) // 8, (W + 7) // 8
    tw = (uw * 8 + 63) // 64
    mask = np.zeros((uh, uw), bool)
    for t in ctus:
        cx, cy = (t % tw) * 8, (t // tw) * 8
        mask[cy:cy + 8, cx:cx + 8] = True
    return mask


def _compare(got, exp, W, H, ctus=None, label=""):
    if ctus is None:
        for k in FIELDS:
            if not np.array_equal(got[k], exp[k]):
                bad = np.argwhere(got[k] != exp[k])
                raise AssertionError(f"{label}: {k} differs at {bad[:5].tolist()} "
                                     f"(got {got[k][tuple(bad[0])]}, exp {exp[k][tuple(bad[0])]})")
        return
    m = _ctu_units(W, H, ctus)
    for k in ("depth", "mode", "mv"):
        g, e = got[k][m], exp[k][m]
        assert np.array_equal(g, e), f"{label}: {k} differs on sampled CTUs"
    for k in ("cost", "dist", "bits"):
        g, e = got[k].ravel()[ctus], exp[k].ravel()[ctus]
        assert np.array_equal(g, e), f"{label}: {k} differs on CTUs {ctus}: {g} vs {e}"


def _pair(seed, W, H, n_rects, mv_max, pan=0):
    sc = synth.Scene(seed, W, H, n_rects, mv_max, pan)
    return sc.render(0), sc.render(1)


@pytest.mark.parametrize("W,H,qp,R", [
    (64, 64, 32, 0), (64, 64, 32, 1), (64, 64, 22, 3), (8, 8, 30, 4), (72, 40, 27, 5),
    (200, 136, 32, 16), (203, 141, 37, 9), (130, 70, 45, 24), (96, 200, 12, 32),
    # pictures smaller than one 8x8 unit (coded picture replicated from 1 or a few samples),
    # and the QP extremes 0 and 51
    (1, 1, 30, 2), (5, 3, 0, 3), (17, 9, 51, 8), (64, 64, 51, 7), (33, 71, 0, 16),
])
def test_small_pairs_bit_exact(mr, W, H, qp, R):
    print(f"\ncase {W}x{H} qp {qp} R {R}", flush=True)
    ref, cur = _pair(1000 + W + H + R, W, H, 4, max(1, R), 2)
    _compare(_gpu(mr, cur, ref, qp, R), oracle.ctu_search(cur, ref, qp, R), W, H,
             label=f"{W}x{H} qp{qp} R{R}")


def test_pair_416x240_r16_qp32_full(mr):
    """The 416x240 pair (4 x 7 CTUs, edge CTUs clipped), R 16, QP 32: every output."""
    sc = synth.Scene(synth.SEED_BASE + 0, 416, 240, 6, 12, 0)
    ref, cur = sc.render(0), sc.render(1)
    _compare(_gpu(mr, cur, ref, 32, 16), oracle.ctu_search(cur, ref, 32, 16), 416, 240,
             label="416x240")


def test_identical_frames_zero_motion(mr):
    ref, _ = _pair(7, 256, 128, 5, 8)
    got = _gpu(mr, ref, ref, 30, 16)
    assert np.all(got["mv"] == 0)
    _compare(got, oracle.ctu_search(ref, ref, 30, 16), 256, 128, label="identical")


def test_global_shift_recovered(mr):
    W, H, R = 192, 128, 12
    big = synth.white_noise(99, W + 64, H + 64)
    sx, sy = 5, -7
    ref = big[32:32 + H, 32:32 + W]
    cur = big[32 + sy:32 + sy + H, 32 + sx:32 + sx + W]
    got = _gpu(mr, cur, ref, 27, R)
    inner = got["mv"][2:-2, 2:-2]
    assert np.all(inner[..., 0] == sx) and np.all(inner[..., 1] == sy)
    _compare(got, oracle.ctu_search(cur, ref, 27, R), W, H, label="shift")


def test_flat_and_saturated_content(mr):
    """Degenerate content: flat frames (all SADs tie) and 0/255 extremes."""
    W, H = 136, 72
    flat = np.full((H, W), 128, np.uint8)
    _compare(_gpu(mr, flat, flat, 30, 8), oracle.ctu_search(flat, flat, 30, 8), W, H,
             label="flat")
    ext = np.zeros((H, W), np.uint8)
    ext[:, ::3] = 255
    ref = np.roll(ext, 1, axis=1)
    _compare(_gpu(mr, ext, ref, 51, 6), oracle.ctu_search(ext, ref, 51, 6), W, H,
             label="extremes")
    _compare(_gpu(mr, ext, 255 - ext, 0, 4), oracle.ctu_search(ext, 255 - ext, 0, 4), W, H,
             label="qp0")


def test_deterministic_reruns(mr):
    ref, cur = _pair(3, 320, 192, 8, 16, 3)
    a = _gpu(mr, cur, ref, 32, 24)
    for _ in range(2):
        b = _gpu(mr, cur, ref, 32, 24)
        for k in FIELDS:
            assert np.array_equal(a[k], b[k])


# ------------------------------------------------------------------- bounds / depth maps
def test_bounds_full_range_equals_full_search(mr):
    ref, cur = _pair(11, 200, 136, 5, 10, 2)
    full = _gpu(mr, cur, ref, 30, 12)
    b = np.zeros(full["depth"].shape + (2,), np.uint8)
    b[..., 1] = 3
    _compare(_gpu(mr, cur, ref, 30, 12, bounds=b), full, 200, 136, label="bounds[0,3]")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_bounds_bit_exact(mr, seed):
    ref, cur = _pair(20 + seed, 216, 152, 6, 10, 2)
    uh, uw = (152 + 7) // 8, (216 + 7) // 8
    rng = np.random.default_rng(seed)
    lo = rng.integers(0, 4, size=(uh, uw))
    hi = np.minimum(3, lo + rng.integers(0, 3, size=lo.shape))
    b = np.stack([lo, hi], -1).astype(np.uint8)
    got = _gpu(mr, cur, ref, 32, 12, bounds=b)
    _compare(got, oracle.ctu_search(cur, ref, 32, 12, bounds=b), 216, 152,
             label=f"bounds seed {seed}")


@pytest.mark.parametrize("rw,rh,dw,dh,lo,hi", [
    (960, 540, 1920, 1080, 0, 1), (960, 540, 3840, 2160, 0, 0), (1280, 720, 3840, 2160, 3, 0),
    (426, 240, 640, 360, 0, 1), (640, 360, 640, 360, 0, 0), (1920, 1080, 426, 240, 1, 2),
    (8, 8, 8192, 64, 0, 3)])
def test_depth_bounds_bit_exact(mr, rw, rh, dw, dh, lo, hi):
    import torch
    rng = np.random.default_rng(rw + dw + lo)
    rd = rng.integers(0, 4, size=((rh + 7) // 8, (rw + 7) // 8)).astype(np.uint8)
    got = mr.mr_depth_bounds(torch.from_numpy(rd).cuda(), rw, rh, dw, dh, lo, hi)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.depth_bounds(rd, rw, rh, dw, dh, lo, hi))


def test_multires_chain_540p_to_1080p_pruned(mr):
    """Reference 960x540 depths bound the 1920x1080 search (box x2 of one source)."""
    import torch
    src = synth.Scene(synth.SEED_BASE + 2, 1920, 1080, 12, 24, 4)
    s0, s1 = src.render(0), src.render(1)
    r540, c540 = synth.box_downscale(s0, 2, 960, 540), synth.box_downscale(s1, 2, 960, 540)
    ref_out = _gpu(mr, c540, r540, 32, 16)
    ctus540 = [0, 14, 60, 134]
    _compare(ref_out, oracle.ctu_search(c540, r540, 32, 16, ctu_list=ctus540), 960, 540,
             ctus=ctus540, label="540p ref")
    b = mr.mr_depth_bounds(torch.from_numpy(ref_out["depth"]).cuda(), 960, 540, 1920, 1080, 0, 1)
    torch.cuda.synchronize()
    b = b.cpu().numpy()
    assert np.array_equal(b, oracle.depth_bounds(ref_out["depth"], 960, 540, 1920, 1080, 0, 1))
    got = _gpu(mr, s1, s0, 27, 24, bounds=b)
    ctus = [0, 29, 250, 509]
    _compare(got, oracle.ctu_search(s1, s0, 27, 24, bounds=b, ctu_list=ctus), 1920, 1080,
             ctus=ctus, label="1080p pruned")


# --------------------------------------------------------------- full-size sampled parity
def test_1080p_r64_sampled(mr):
    sc = synth.Scene(synth.SEED_BASE + 1, 1920, 1080, 24, 48, 4)
    ref, cur = sc.render(0), sc.render(1)
    got = _gpu(mr, cur, ref, 27, 64)
    ctus = [0, 29, 255, 480, 509]  # corners, centre, bottom edge (1080 -> 17 CTU rows)
    _compare(got, oracle.ctu_search(cur, ref, 27, 64, ctu_list=ctus), 1920, 1080, ctus=ctus,
             label="1080p R64")
    s = oracle.sqrt_lambda_q16(27)
    assert np.all(got["cost"] == got["dist"] * 65536 + s * got["bits"])


def test_2160p_r128_sampled(mr):
    sc = synth.Scene(synth.SEED_BASE + 3, 3840, 2160, 24, 96, 8)
    ref, cur = sc.render(0), sc.render(1)
    got = _gpu(mr, cur, ref, 22, 128)
    ctus = [0, 59, 1000, 2039]
    _compare(got, oracle.ctu_search(cur, ref, 22, 128, ctu_list=ctus), 3840, 2160, ctus=ctus,
             label="2160p R128")


@pytest.mark.parametrize("W,R,strip,nb", [
    (320, 16, 4, 1), (320, 24, 4, 3),   # 5 CTUs per row: strips of 4 + 1
    (448, 32, 4, 2),                    # 7: 4 + 3
    (384, 24, 4, 5),                    # 6: 4 + 2
    (320, 32, 3, 2),                    # 5: 3 + 2
    (256, 16, 3, 1),                    # 4: 3 + 1
    (192, 24, 2, 4),                    # 3: 2 + 1
    (200, 32, 1, 3),                    # 4 strips of 1
    (130, 24, 4, 1),                    # 3 CTUs, one partial strip narrower than the workgroup
])
def test_partial_strips_bit_exact(mr, W, R, strip, nb):
    """Search workgroups forced to strips of `strip` CTUs on widths that leave a partial strip
    at the right edge, whose (CTU, step) pairs are dealt over all the workgroup's wavefronts."""
    H, qp = 136, 30
    ref, cur = _pair(0x5700 + 7 * W + strip, W, H, 5, 12, 2)
    mr.mr_set_tiles4(R, 4, nb, strip, 1)  # whole CTUs per wavefront
    try:
        got = _gpu(mr, cur, ref, qp, R)
    finally:
        mr.mr_set_tiles(R, 0, 1)
    _compare(got, oracle.ctu_search(cur, ref, qp, R), W, H, label=f"W{W} R{R} strip{strip} nb{nb}")


@pytest.mark.parametrize("W,H,R,D,nb,bounded", [
    (200, 136, 16, 2, 1, False),   # 4x3 CTUs, partial bottom row
    (200, 136, 16, 5, 1, True),    # one step per CTU, bounds
    (264, 200, 24, 4, 3, False),   # three single-step bands
    (330, 130, 32, 6, 0, True),    # built-in bands, bounds
    (136, 72, 8, 8, 1, False),
    (203, 141, 64, 4, 5, True),    # the (R, R) corner left to prep, ragged
    (72, 40, 40, 5, 2, False),     # 2x1 CTUs, both partial
    (64, 64, 0, 2, 1, False),      # one candidate
])
def test_split_quadrants_bit_exact(mr, W, H, R, D, nb, bounded):
    """Split search: the four wavefronts of a workgroup take the four 32x32 quadrants of one
    CTU and sum the 64x64 SADs through LDS, on ragged pictures (edge CTUs whose 64x64 node is
    absent), with bounds (nodes that may not be leaves skip their keys and the exchange),
    and at each lane shape D."""
    qp = 31
    ref, cur = _pair(0x5A00 + W + 3 * R + D, W, H, 6, max(4, R), 2)
    b = None
    if bounded:
        rng = np.random.default_rng(W + R)
        lo = rng.integers(0, 4, size=((H + 7) // 8, (W + 7) // 8), dtype=np.uint8)
        hi = np.maximum(lo, rng.integers(0, 4, size=lo.shape, dtype=np.uint8))
        b = np.stack([lo, hi], axis=-1)
    mr.mr_set_tiles4(R, D, nb, 0, 2)
    try:
        got = _gpu(mr, cur, ref, qp, R, bounds=b)
    finally:
        mr.mr_set_tiles(R, 0, 1)
    _compare(got, oracle.ctu_search(cur, ref, qp, R, bounds=b), W, H,
             label=f"split W{W} H{H} R{R} D{D} nb{nb}")


def test_split_and_whole_jobs_in_one_batch(mr):
    """One batch mixing split jobs (R 16, 24) and whole-CTU jobs (R 40 forced whole): each
    job's outputs equal the oracle's."""
    import torch
    specs = [(200, 136, 16), (264, 136, 24), (330, 200, 40), (136, 72, 16)]
    jobs, host = [], []
    for i, (W, H, R) in enumerate(specs):
        ref, cur = _pair(0x5B00 + i, W, H, 6, R, 2)
        host.append((cur, ref, R))
        jobs.append(dict(cur=torch.from_numpy(cur).cuda(), ref=torch.from_numpy(ref).cuda(),
                         qp=30 + i, search_range=R))
    mr.mr_set_tiles4(40, 4, 0, 0, 1)
    try:
        outs = mr.mr_ctu_search_batch(jobs)
        torch.cuda.synchronize()
    finally:
        mr.mr_set_tiles(40, 0, 1)
    for i, ((cur, ref, R), o) in enumerate(zip(host, outs)):
        H, W = cur.shape
        got = {k: v.cpu().numpy() for k, v in o.items()}
        _compare(got, oracle.ctu_search(cur, ref, 30 + i, R), W, H, label=f"mixed job {i}")


@pytest.mark.parametrize("W,H,R,qp,bounded", [
    (200, 136, 64, 27, False), (136, 72, 60, 33, False), (203, 141, 64, 22, True),
])
def test_corner_candidate_left_to_prep_bit_exact(mr, W, H, R, qp, bounded):
    """Ranges whose last search task holds only (R, R) (R 60, 64: 31^2 and 33^2 tasks, one more
    than a multiple of 64): that candidate comes from the prep kernel's initial keys. Every
    output, ragged frames whose windows reach past the picture, with and without bounds."""
    ref, cur = _pair(0x6000 + W + R, W, H, 6, 40, 3)
    b = None
    if bounded:
        rng = np.random.default_rng(R)
        lo = rng.integers(0, 3, size=((H + 7) // 8, (W + 7) // 8)).astype(np.uint8)
        b = np.stack([lo, np.minimum(lo + 1, 3)], -1)
    _compare(_gpu(mr, cur, ref, qp, R, bounds=b), oracle.ctu_search(cur, ref, qp, R, bounds=b),
             W, H, label=f"{W}x{H} R{R}")


def test_padded_stride_and_unaligned_pointer(mr):
    """Frames inside larger buffers: stride > width and a base address not 4-byte aligned
    (the window staging falls back to byte loads); results equal the packed frames'."""
    import torch
    W, H = 150, 94
    ref, cur = _pair(41, W, H, 5, 9, 2)
    exp = oracle.ctu_search(cur, ref, 31, 11)
    for stride, off in ((W + 10, 0), (W + 3, 1), (W + 64, 3)):
        bufc = torch.zeros(H * stride + 64, dtype=torch.uint8)
        bufr = torch.zeros(H * stride + 64, dtype=torch.uint8)
        vc = bufc[off:off + H * stride].view(H, stride)
        vr = bufr[off:off + H * stride].view(H, stride)
        vc[:, :W] = torch.from_numpy(cur)
        vr[:, :W] = torch.from_numpy(ref)
        gc, gr = bufc.cuda(), bufr.cuda()
        fc = gc[off:off + H * stride].view(H, stride)[:, :W]
        fr = gr[off:off + H * stride].view(H, stride)[:, :W]
        o = mr.alloc_outputs(W, H)
        prm = mr.mr_search_params(31, 11)
        outs = mr.mr_search_out(*[mr._dev_ptr(o[k], t, k) for k, t in
                                  (("depth", torch.uint8), ("mode", torch.uint8),
                                   ("mv", torch.int16), ("cost", torch.int64),
                                   ("dist", torch.int64), ("bits", torch.int64))])
        import ctypes
        f1 = mr.mr_frame(ctypes.c_void_p(fc.data_ptr()), W, H, stride)
        f2 = mr.mr_frame(ctypes.c_void_p(fr.data_ptr()), W, H, stride)
        rc = mr.lib().mr_ctu_search(ctypes.byref(f1), ctypes.byref(f2), ctypes.byref(prm), None,
                                    ctypes.byref(outs), None)
        assert rc == 0
        torch.cuda.synchronize()
        _compare({k: v.cpu().numpy() for k, v in o.items()}, exp, W, H,
                 label=f"stride {stride} offset {off}")


def test_maximum_width(mr):
    """8192-wide picture (the ABI maximum), 72 rows, R 4: full parity."""
    W, H = 8192, 72
    ref, cur = _pair(43, W, H, 10, 4, 1)
    _compare(_gpu(mr, cur, ref, 34, 4), oracle.ctu_search(cur, ref, 34, 4), W, H, label="8192 wide")
