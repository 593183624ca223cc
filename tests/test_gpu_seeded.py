"""GPU parity of the seeded search (reference MV reuse with a refinement window).

libmr's mr_ctu_search_seeded (HIP, through the C ABI) against the oracle's seeded
search, element by element: depth, mode, MV per 8x8 unit and J / D / R per CTU.
Seed maps are seeded random fields (any MV map is a valid input) or the oracle's
own search of a downscaled picture.  Window widths 2r+1 cover one to five passes
of 8 candidate columns; r = R must equal the full search.  The multi-QP chain
(one resolution, a median-QP master) runs the same path at ratio 1.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from dag_spec import dag_rungs

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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _gpu(mr, cur, ref, qp, R, bounds=None, seed=None):
    b = None if bounds is None else _dev(bounds)
    sd = None
    if seed is not None:
        rm, rw, rh, r = seed
        sd = dict(ref_mv=_dev(rm), ref_w=rw, ref_h=rh, r=r)
    return _host(mr.mr_ctu_search(_dev(cur), _dev(ref), qp, R, bounds=b, seed=sd))


def _oracle(cur, ref, qp, R, bounds=None, seed=None, ctu_list=None):
    sd = None if seed is None else oracle.Seed(*seed)
    return oracle.ctu_search(cur, ref, qp, R, bounds=bounds, seed=sd, ctu_list=ctu_list)


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
        assert np.array_equal(got[k][m], exp[k][m]), f"{label}: {k} differs on sampled CTUs"
    for k in ("cost", "dist", "bits"):
        g, e = got[k].ravel()[ctus], exp[k].ravel()[ctus]
        assert np.array_equal(g, e), f"{label}: {k} differs on CTUs {ctus}: {g} vs {e}"


def _pair(seed, W, H, n_rects, mv_max, pan=0):
    sc = synth.Scene(seed, W, H, n_rects, mv_max, pan)
    return sc.render(0), sc.render(1)


def _rand_map(seed, w, h, amp):
    rng = np.random.default_rng(seed)
    return rng.integers(-amp, amp + 1, size=((h + 7) // 8, (w + 7) // 8, 2)).astype(np.int16)


@pytest.mark.parametrize("W,H,qp,R,r,rw,rh", [
    (8, 8, 30, 4, 2, 8, 8),            # one unit
    (64, 64, 32, 4, 0, 32, 32),        # r = 0: the scaled MV itself
    (64, 64, 32, 4, 4, 32, 32),        # r = R: the full search
    (72, 40, 27, 5, 1, 36, 20),        # edge CTU, ragged rows
    (200, 136, 32, 16, 2, 100, 68),    # dyadic
    (203, 141, 37, 9, 3, 135, 94),     # ratio 3/2, sizes not multiples of 8
    (130, 70, 45, 24, 7, 260, 140),    # seed from a larger picture
    (96, 200, 12, 32, 8, 48, 100),     # window of 17 candidates: passes of 9 + 8
    (416, 240, 32, 16, 15, 208, 120),  # 31 candidates: four passes, the last of 4
    (416, 240, 32, 20, 16, 208, 120),  # 33 candidates: four passes (two bands)
    (256, 128, 30, 40, 17, 128, 64),   # 35 candidates, centres clamped to +-23
    (200, 136, 30, 16, 3, 100, 68),    # 7 candidates: one pass of 9, two columns past the window
    (200, 136, 30, 16, 4, 100, 68),    # 9 candidates: exactly one pass
    (200, 136, 30, 16, 5, 100, 68),    # 11 candidates: passes of 9 + 2
    (1, 1, 30, 4, 2, 1, 1),            # one sample
    (5, 3, 0, 6, 3, 3, 2),             # smaller than one unit, QP 0
])
def test_seeded_matches_oracle(mr, W, H, qp, R, r, rw, rh):
    ref, cur = _pair(W * 7 + H, W, H, 5, min(R, 12) + 1, 2)
    seed = (_rand_map(W + 3 * r, rw, rh, R), rw, rh, r)
    _compare(_gpu(mr, cur, ref, qp, R, seed=seed), _oracle(cur, ref, qp, R, seed=seed), W, H,
             label=f"{W}x{H} R{R} r{r}")


def test_full_window_equals_full_search(mr):
    W, H, R = 200, 136, 12
    ref, cur = _pair(5, W, H, 6, 10, 2)
    seed = (_rand_map(9, W // 2, H // 2, 30), W // 2, H // 2, R)
    full = _gpu(mr, cur, ref, 30, R)
    _compare(_gpu(mr, cur, ref, 30, R, seed=seed), full, W, H, label="r = R vs full")
    _compare(full, _oracle(cur, ref, 30, R), W, H, label="full")


def test_seeded_with_depth_bounds(mr):
    W, H, R, r = 216, 152, 12, 3
    ref, cur = _pair(17, W, H, 6, 10, 2)
    rng = np.random.default_rng(4)
    lo = rng.integers(0, 4, size=((H + 7) // 8, (W + 7) // 8)).astype(np.uint8)
    hi = np.minimum(3, lo + rng.integers(0, 3, size=lo.shape)).astype(np.uint8)
    b = np.stack([lo, hi], axis=-1)
    seed = (_rand_map(8, W // 2, H // 2, 6), W // 2, H // 2, r)
    _compare(_gpu(mr, cur, ref, 32, R, bounds=b, seed=seed),
             _oracle(cur, ref, 32, R, bounds=b, seed=seed), W, H, label="seeded + bounds")


def test_chain_reference_search_seeds_dependent(mr):
    """208x120 full search -> its MVs and depths seed and bound the 416x240 search."""
    import torch
    src = synth.Scene(synth.SEED_BASE + 7, 416, 240, 6, 12, 2)
    s0, s1 = src.render(0), src.render(1)
    r0, r1 = synth.box_downscale(s0, 2, 208, 120), synth.box_downscale(s1, 2, 208, 120)
    g_ref = _gpu(mr, r1, r0, 35, 8)
    o_ref = _oracle(r1, r0, 35, 8)
    _compare(g_ref, o_ref, 208, 120, label="reference rung")
    gb = mr.mr_depth_bounds(_dev(g_ref["depth"]), 208, 120, 416, 240, 0, 1)
    torch.cuda.synchronize()
    ob = oracle.depth_bounds(o_ref["depth"], 208, 120, 416, 240, 0, 1)
    assert np.array_equal(gb.cpu().numpy(), ob)
    got = _host(mr.mr_ctu_search(_dev(s1), _dev(s0), 32, 16, bounds=gb,
                                 seed=dict(ref_mv=_dev(g_ref["mv"]), ref_w=208, ref_h=120, r=2)))
    exp = _oracle(s1, s0, 32, 16, bounds=ob, seed=(o_ref["mv"], 208, 120, 2))
    _compare(got, exp, 416, 240, label="dependent rung")


def test_1080p_seeded_from_540p_sampled(mr):
    """1920x1080 R64 seeded (r = 4) with the MVs of the oracle's 960x540 R32 search."""
    src = synth.Scene(synth.SEED_BASE + 2, 1920, 1080, 12, 24, 4)
    s0, s1 = src.render(0), src.render(1)
    r540, c540 = synth.box_downscale(s0, 2, 960, 540), synth.box_downscale(s1, 2, 960, 540)
    o540 = _oracle(c540, r540, 32, 32)
    seed = (o540["mv"], 960, 540, 4)
    got = _gpu(mr, s1, s0, 27, 64, seed=seed)
    ctus = [0, 29, 250, 509]
    _compare(got, _oracle(s1, s0, 27, 64, seed=seed, ctu_list=ctus), 1920, 1080, ctus=ctus,
             label="1080p seeded")
    s = oracle.sqrt_lambda_q16(27)
    assert np.all(got["cost"] == got["dist"] * 65536 + s * got["bits"])


def test_2160p_seeded_sampled(mr):
    """3840x2160 R128 seeded from a 1920x1080 map, r = 8 and r = 0."""
    sc = synth.Scene(synth.SEED_BASE + 3, 3840, 2160, 24, 96, 8)
    ref, cur = sc.render(0), sc.render(1)
    ctus = [0, 59, 1000, 2039]
    for r in (8, 0):
        seed = (_rand_map(21 + r, 1920, 1080, 60), 1920, 1080, r)
        _compare(_gpu(mr, cur, ref, 22, 128, seed=seed),
                 _oracle(cur, ref, 22, 128, seed=seed, ctu_list=ctus), 3840, 2160, ctus=ctus,
                 label=f"2160p r{r}")


def test_seeded_padded_stride_and_unaligned_pointer(mr):
    """The padded copy of the reference falls back to byte loads for unaligned rows."""
    import torch
    W, H, R, r = 150, 94, 11, 3
    ref, cur = _pair(41, W, H, 5, 9, 2)
    rm = _rand_map(3, 75, 47, 9)
    exp = _oracle(cur, ref, 31, R, seed=(rm, 75, 47, r))
    rm_d = _dev(rm)
    for stride, off in ((W + 10, 0), (W + 3, 1), (W + 64, 3)):
        bufc = torch.zeros(H * stride + 64, dtype=torch.uint8)
        bufr = torch.zeros(H * stride + 64, dtype=torch.uint8)
        bufc[off:off + H * stride].view(H, stride)[:, :W] = torch.from_numpy(cur)
        bufr[off:off + H * stride].view(H, stride)[:, :W] = torch.from_numpy(ref)
        gc, gr = bufc.cuda(), bufr.cuda()
        o = mr.alloc_outputs(W, H)
        f1 = mr.mr_frame(ctypes.c_void_p(gc.data_ptr() + off), W, H, stride)
        f2 = mr.mr_frame(ctypes.c_void_p(gr.data_ptr() + off), W, H, stride)
        prm = mr.mr_search_params(31, R)
        sd = mr.mr_mv_seed(ctypes.c_void_p(rm_d.data_ptr()), 75, 47, r)
        rc = mr.lib().mr_ctu_search_seeded(ctypes.byref(f1), ctypes.byref(f2), ctypes.byref(prm),
                                           None, ctypes.byref(sd), ctypes.byref(mr._out_struct(o)),
                                           None)
        assert rc == 0
        _compare(_host(o), exp, W, H, label=f"stride {stride} offset {off}")


def _job(cur, ref, qp, R, bounds=None, seed=None):
    j = dict(cur=_dev(cur), ref=_dev(ref), qp=qp, search_range=R)
    if bounds is not None:
        j["bounds"] = _dev(bounds)
    if seed is not None:
        rm, rw, rh, r = seed
        j["seed"] = dict(ref_mv=_dev(rm), ref_w=rw, ref_h=rh, r=r)
    return j


def test_mixed_batch_and_graph_replays(mr):
    """Full and seeded jobs in one batch equal per-job calls; the graph replays and
    mr_batch_set_jobs with a new seed map keep parity."""
    specs = []
    ra, ca = _pair(61, 200, 136, 5, 10, 2)
    specs.append((ca, ra, 32, 16, None, None))
    rb, cb = _pair(62, 416, 240, 6, 12, 2)
    specs.append((cb, rb, 32, 16, None, (_rand_map(1, 208, 120, 16), 208, 120, 3)))
    rc_, cc = _pair(63, 72, 40, 3, 5, 1)
    lo = np.zeros((5, 9), np.uint8)
    hi = np.full((5, 9), 2, np.uint8)
    specs.append((cc, rc_, 27, 5, np.stack([lo, hi], -1), (_rand_map(2, 36, 20, 5), 36, 20, 0)))
    rd, cd = _pair(64, 64, 64, 2, 4, 0)
    specs.append((cd, rd, 37, 4, None, None))
    exp = [_oracle(c, r, q, R, bounds=b, seed=s) for c, r, q, R, b, s in specs]
    jobs = [_job(*sp) for sp in specs]
    outs = mr.mr_ctu_search_batch(jobs)
    for i, (o, e) in enumerate(zip(outs, exp)):
        _compare(_host(o), e, specs[i][0].shape[1], specs[i][0].shape[0], label=f"batch job {i}")
    bt = mr.Batch([_job(*sp) for sp in specs])
    try:
        for rep in range(3):
            outs = bt.launch()
            for i, (o, e) in enumerate(zip(outs, exp)):
                _compare(_host(o), e, specs[i][0].shape[1], specs[i][0].shape[0],
                         label=f"replay {rep} job {i}")
        # New seed map for job 1 (same presence), replayed twice.
        s2 = (_rand_map(77, 208, 120, 16), 208, 120, 5)
        specs[1] = specs[1][:5] + (s2,)
        bt.set_jobs([_job(*sp) for sp in specs])
        e1 = _oracle(cb, rb, 32, 16, seed=s2)
        for rep in range(2):
            _compare(_host(bt.launch()[1]), e1, 416, 240, label=f"set_jobs replay {rep}")
        # Seed presence may not change.
        bad = [_job(*sp[:5]) for sp in specs]
        with pytest.raises(mr.MRError):
            bt.set_jobs(bad)
    finally:
        bt.close()


def test_batch_set_jobs_changes_refinement_width(mr):
    """A recorded batch re-targeted to seeds with a larger, then smaller, refinement
    half-width (r 1 -> 6 -> 1: one, two and one passes of candidate columns) keeps parity
    with the oracle on every replay."""
    ref, cur = _pair(65, 320, 200, 5, 10, 2)
    rm = _rand_map(5, 160, 100, 12)
    R = 16
    bt = mr.Batch([_job(cur, ref, 30, R, seed=(rm, 160, 100, 1))])
    try:
        for r in (1, 6, 1):
            bt.set_jobs([_job(cur, ref, 30, R, seed=(rm, 160, 100, r))])
            exp = _oracle(cur, ref, 30, R, seed=(rm, 160, 100, r))
            for rep in range(2):
                _compare(_host(bt.launch()[0]), exp, 320, 200, label=f"r {r} replay {rep}")
    finally:
        bt.close()


def test_multi_qp_chain_same_resolution(mr):
    """416x240 at QP 30 (master, full search) bounds (ratio 1, depths d-1..d+1) and seeds
    (r = 2) the same pair at QPs 22, 26, 34 and 38; GPU chain against the oracle's chain."""
    import torch
    W, H, R = 416, 240, 16
    ref, cur = _pair(81, W, H, 6, 12, 2)
    g_m = _gpu(mr, cur, ref, 30, R)
    o_m = _oracle(cur, ref, 30, R)
    _compare(g_m, o_m, W, H, label="QP 30 master")
    gb = mr.mr_depth_bounds(_dev(g_m["depth"]), W, H, W, H, 1, 1)
    torch.cuda.synchronize()
    ob = oracle.depth_bounds(o_m["depth"], W, H, W, H, 1, 1)
    assert np.array_equal(gb.cpu().numpy(), ob)
    gmv = _dev(g_m["mv"])
    for qp in (22, 26, 34, 38):
        got = _host(mr.mr_ctu_search(_dev(cur), _dev(ref), qp, R, bounds=gb,
                                     seed=dict(ref_mv=gmv, ref_w=W, ref_h=H, r=2)))
        exp = _oracle(cur, ref, qp, R, bounds=ob, seed=(o_m["mv"], W, H, 2))
        _compare(got, exp, W, H, label=f"QP {qp} dependent")


def test_multi_encoding_dag_against_oracle(mr):
    import torch
    sizes = [(160, 96, 8), (320, 192, 16), (640, 384, 24)]
    src = synth.Scene(synth.SEED_BASE + 9, 640, 384, 8, 16, 2)
    s0, s1 = src.render(0), src.render(1)
    frames = {}
    for (w, h, _), k in zip(sizes, (4, 2, 1)):
        frames[w] = (synth.box_downscale(s0, k, w, h), synth.box_downscale(s1, k, w, h))
    got, exp = [], []
    for (w, h, qp, R, ref, dlo, dhi, r) in dag_rungs(sizes):
        f0, f1 = frames[w]
        if ref < 0:
            g = _gpu(mr, f1, f0, qp, R)
            o = _oracle(f1, f0, qp, R)
        else:
            rw, rh = dag_rungs(sizes)[ref][:2]
            gb = mr.mr_depth_bounds(_dev(got[ref]["depth"]), rw, rh, w, h, dlo, dhi)
            g = _host(mr.mr_ctu_search(_dev(f1), _dev(f0), qp, R, bounds=gb,
                                       seed=dict(ref_mv=_dev(got[ref]["mv"]), ref_w=rw,
                                                 ref_h=rh, r=r)))
            ob = oracle.depth_bounds(exp[ref]["depth"], rw, rh, w, h, dlo, dhi)
            o = _oracle(f1, f0, qp, R, bounds=ob, seed=(exp[ref]["mv"], rw, rh, r))
        _compare(g, o, w, h, label=f"{w}x{h} QP {qp}")
        got.append(g)
        exp.append(o)
