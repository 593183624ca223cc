"""Host-side checks of libmr (no GPU): symbols, argument validation, host arithmetic."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(mr_[a-z_0-9]+)\s*\(", text,
                                flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libmr():
    from paper_2301_12191_amd import mr
    return mr.lib()


def test_library_exports_every_declared_symbol(libmr):
    names = _declared_functions()
    assert "mr_ctu_search" in names and "mr_depth_bounds" in names
    for n in names:
        assert hasattr(libmr, n), n


def test_status_strings(libmr):
    from paper_2301_12191_amd import mr
    for code in range(-8, 1):
        assert mr.mr_status_str(code).startswith("MR_")
    assert "unknown" in mr.mr_status_str(-99)


def _fake_frame(mr, w=64, h=64, stride=None, ptr=0x1000):
    return mr.mr_frame(ctypes.c_void_p(ptr), w, h, stride if stride is not None else w)


def _fake_out(mr):
    p = ctypes.c_void_p(0x2000)
    return mr.mr_search_out(p, p, p, p, p, p)


@pytest.mark.parametrize("case", ["qp_low", "qp_high", "range_neg", "range_big", "null_cur",
                                  "size_mismatch", "stride_small", "zero_width", "huge",
                                  "null_out_field", "subpel_2", "subpel_neg", "offsets_32bit",
                                  "angular_2"])
def test_search_rejects_invalid_arguments_before_launch(libmr, case):
    from paper_2301_12191_amd import mr
    cur, ref = _fake_frame(mr), _fake_frame(mr)
    prm = mr.mr_search_params(30, 16)
    out = _fake_out(mr)
    if case == "qp_low":
        prm.qp = -1
    elif case == "qp_high":
        prm.qp = 52
    elif case == "range_neg":
        prm.search_range = -1
    elif case == "range_big":
        prm.search_range = 129
    elif case == "null_cur":
        cur.luma = None
    elif case == "size_mismatch":
        ref = _fake_frame(mr, 64, 72)
    elif case == "stride_small":
        cur, ref = _fake_frame(mr, 64, 64, 32), _fake_frame(mr, 64, 64, 32)
    elif case == "zero_width":
        cur, ref = _fake_frame(mr, 0, 64), _fake_frame(mr, 0, 64)
    elif case == "huge":
        cur, ref = _fake_frame(mr, 8193, 64), _fake_frame(mr, 8193, 64)
    elif case == "null_out_field":
        out.mv = None
    elif case == "subpel_2":
        prm.subpel = 2
    elif case == "subpel_neg":
        prm.subpel = -1
    elif case == "angular_2":
        prm.angular = 2
    elif case == "offsets_32bit":  # stride * (height - 1) + width must stay below 2^31
        cur, ref = _fake_frame(mr, 64, 8192, 300000), _fake_frame(mr, 64, 8192, 300000)
    rc = libmr.mr_ctu_search(ctypes.byref(cur), ctypes.byref(ref), ctypes.byref(prm), None,
                             ctypes.byref(out), None)
    assert rc == mr.MR_EINVAL
    rc = libmr.mr_ctu_search_noalloc(ctypes.byref(cur), ctypes.byref(ref), ctypes.byref(prm),
                                     None, None, ctypes.byref(out), None)
    assert rc == mr.MR_EINVAL


@pytest.mark.parametrize("w,h,R,subpel,seeded", [
    (8192, 4320, 128, 0, False),  # 8,704 CTUs of packed current samples alone exceed the array
    (4608, 2592, 128, 1, False),  # 14.4 MB of CTU scratch fits; the padded reference of
    (4608, 2592, 64, 0, True),    # sub-pel or a seed (over 13 MB) does not
])
def test_noalloc_rejects_requests_beyond_its_scratch(libmr, w, h, R, subpel, seeded):
    """The allocation-free search refuses (MR_ESCRATCH) a request whose scratch exceeds its
    fixed array, before touching the device (the frame pointers here are never read)."""
    from paper_2301_12191_amd import mr
    cur, ref = _fake_frame(mr, w, h), _fake_frame(mr, w, h)
    prm = mr.mr_search_params(30, R, subpel)
    seed = mr.mr_mv_seed(ctypes.c_void_p(0x3000), w // 2, h // 2, 4, 0) if seeded else None
    rc = libmr.mr_ctu_search_noalloc(ctypes.byref(cur), ctypes.byref(ref), ctypes.byref(prm),
                                     None, ctypes.byref(seed) if seed else None,
                                     ctypes.byref(_fake_out(mr)), None)
    assert rc == mr.MR_ESCRATCH
    assert "scratch" in mr.mr_status_str(rc)


def test_search_rejects_null_structs(libmr):
    from paper_2301_12191_amd import mr
    cur = _fake_frame(mr)
    prm = mr.mr_search_params(30, 16)
    out = _fake_out(mr)
    assert libmr.mr_ctu_search(None, ctypes.byref(cur), ctypes.byref(prm), None,
                               ctypes.byref(out), None) == mr.MR_EINVAL
    assert libmr.mr_ctu_search(ctypes.byref(cur), ctypes.byref(cur), None, None,
                               ctypes.byref(out), None) == mr.MR_EINVAL
    assert libmr.mr_ctu_search(ctypes.byref(cur), ctypes.byref(cur), ctypes.byref(prm), None,
                               None, None) == mr.MR_EINVAL


@pytest.mark.parametrize("args", [
    (0, 64, 64, 128, 128, 0, 1), (1, 0, 64, 128, 128, 0, 1), (1, 64, 64, 0, 128, 0, 1),
    (1, 64, 64, 128, 128, -1, 1), (1, 64, 64, 128, 128, 0, 4), (1, 9000, 64, 128, 128, 0, 1)])
def test_depth_bounds_rejects_invalid_arguments(libmr, args):
    from paper_2301_12191_amd import mr
    ptr, rw, rh, dw, dh, lo, hi = args
    rc = libmr.mr_depth_bounds(ctypes.c_void_p(0x1000 if ptr else 0), rw, rh, dw, dh, lo, hi,
                               ctypes.c_void_p(0x2000), None)
    assert rc == mr.MR_EINVAL


def test_batch_rejects_invalid_jobs_before_launch(libmr):
    from paper_2301_12191_amd import mr
    assert libmr.mr_ctu_search_batch(None, 1, None) == mr.MR_EINVAL
    arr = (mr.mr_search_job * 2)()
    for i in range(2):
        arr[i] = mr.mr_search_job(_fake_frame(mr), _fake_frame(mr), mr.mr_search_params(30, 16),
                                  None, _fake_out(mr), None)
    assert libmr.mr_ctu_search_batch(arr, 0, None) == mr.MR_EINVAL
    arr[1].params.qp = 99
    assert libmr.mr_ctu_search_batch(arr, 2, None) == mr.MR_EINVAL
    h = ctypes.c_void_p()
    assert libmr.mr_batch_create(arr, 2, ctypes.byref(h)) == mr.MR_EINVAL
    assert not h.value
    assert libmr.mr_batch_create(arr, 2, None) == mr.MR_EINVAL
    assert libmr.mr_batch_launch(None, None) == mr.MR_EINVAL
    assert libmr.mr_batch_set_jobs(None, arr, 2) == mr.MR_EINVAL
    assert libmr.mr_batch_destroy(None) == mr.MR_OK


@pytest.mark.parametrize("case", ["null_map", "zero_w", "huge_h", "r_neg", "r_above_range",
                                  "qpel_2"])
def test_seeded_search_rejects_invalid_seeds_before_launch(libmr, case):
    from paper_2301_12191_amd import mr
    cur, ref = _fake_frame(mr), _fake_frame(mr)
    prm = mr.mr_search_params(30, 16)
    out = _fake_out(mr)
    sd = mr.mr_mv_seed(ctypes.c_void_p(0x3000), 32, 32, 4)
    if case == "null_map":
        sd.ref_mv = None
    elif case == "zero_w":
        sd.ref_w = 0
    elif case == "huge_h":
        sd.ref_h = 8193
    elif case == "r_neg":
        sd.refine_range = -1
    elif case == "r_above_range":
        sd.refine_range = 17
    elif case == "qpel_2":
        sd.quarter_pel = 2
    rc = libmr.mr_ctu_search_seeded(ctypes.byref(cur), ctypes.byref(ref), ctypes.byref(prm), None,
                                    ctypes.byref(sd), ctypes.byref(out), None)
    assert rc == mr.MR_EINVAL
    # The same seed inside a batch job is rejected before anything is launched.
    arr = (mr.mr_search_job * 2)()
    for i in range(2):
        arr[i] = mr.mr_search_job(_fake_frame(mr), _fake_frame(mr), mr.mr_search_params(30, 16),
                                  None, _fake_out(mr), None)
    arr[1].seed = ctypes.pointer(sd)
    assert libmr.mr_ctu_search_batch(arr, 2, None) == mr.MR_EINVAL
    h = ctypes.c_void_p()
    assert libmr.mr_batch_create(arr, 2, ctypes.byref(h)) == mr.MR_EINVAL


@pytest.mark.parametrize("reuse,r", [(2, 0), (-1, 0), (1, -1), (1, 129)])
def test_ladder_rejects_invalid_mv_reuse_config(libmr, reuse, r):
    from paper_2301_12191_amd import mr
    L = mr._ladder_lib()
    cfg = mr.mr_ladder_config()
    cfg.n_rungs = 2
    cfg.rungs[0] = mr.mr_rung(64, 64, 30, 8, -1)
    cfg.rungs[1] = mr.mr_rung(128, 128, 30, 16, 0)
    cfg.delta_lo, cfg.delta_hi = 0, 1
    cfg.hbm_budget_bytes = 1 << 30
    cfg.max_inflight, cfg.max_queue, cfg.max_batch_jobs = 8, 8, 8
    cfg.reuse_mv, cfg.refine_range = reuse, r
    h = ctypes.c_void_p()
    assert L.mr_ladder_open(ctypes.byref(cfg), ctypes.byref(h)) == mr.MR_EINVAL
    assert not h.value


@pytest.mark.parametrize("case", ["too_many_rungs", "own_policy_2", "rung_delta", "rung_refine",
                                  "cycle", "rung_subpel"])
def test_ladder_rejects_invalid_rung_policies(libmr, case):
    from paper_2301_12191_amd import mr
    L = mr._ladder_lib()
    cfg = mr.mr_ladder_config()
    cfg.n_rungs = 3
    cfg.rungs[0] = mr.mr_rung(64, 64, 30, 8, -1)
    cfg.rungs[1] = mr.mr_rung(128, 128, 30, 16, 0, own_policy=1, delta_lo=0, delta_hi=1,
                              reuse_mv=1, refine_range=4)
    cfg.rungs[2] = mr.mr_rung(128, 128, 34, 16, 1, own_policy=1, delta_lo=1, delta_hi=1,
                              reuse_mv=1, refine_range=2)
    cfg.delta_lo, cfg.delta_hi = 0, 1
    cfg.hbm_budget_bytes = 1 << 30
    cfg.max_inflight, cfg.max_queue, cfg.max_batch_jobs = 8, 8, 8
    if case == "too_many_rungs":
        cfg.n_rungs = mr.MR_MAX_RUNGS + 1
    elif case == "own_policy_2":
        cfg.rungs[1].own_policy = 2
    elif case == "rung_delta":
        cfg.rungs[2].delta_hi = 4
    elif case == "rung_refine":
        cfg.rungs[1].refine_range = 129
    elif case == "cycle":
        cfg.rungs[1].ref_rung = 2
    elif case == "rung_subpel":
        cfg.rungs[2].subpel = 2
    h = ctypes.c_void_p()
    assert L.mr_ladder_open(ctypes.byref(cfg), ctypes.byref(h)) == mr.MR_EINVAL
    assert not h.value


def test_tile_override_validation(libmr):
    from paper_2301_12191_amd import mr
    assert libmr.mr_set_tiles(200, 4, 1) == mr.MR_EINVAL
    assert libmr.mr_set_tiles(64, 3, 1) == mr.MR_EINVAL
    assert libmr.mr_set_tiles(64, 4, 0) == mr.MR_EINVAL
    assert libmr.mr_set_tiles(64, 4, 9) == mr.MR_EINVAL
    assert libmr.mr_set_tiles(64, 0, 1) == mr.MR_OK
    assert libmr.mr_set_tiles(64, 5, 1) == mr.MR_OK and libmr.mr_set_tiles(64, 6, 2) == mr.MR_OK
    assert libmr.mr_set_tiles(64, 7, 1) == mr.MR_EINVAL
    assert libmr.mr_set_tiles4(64, 4, 0, 0, 3) == mr.MR_EINVAL
    assert libmr.mr_set_tiles4(64, 4, 0, 0, -1) == mr.MR_EINVAL
    assert libmr.mr_set_tiles4(64, 4, 9, 0, 1) == mr.MR_EINVAL
    assert libmr.mr_set_tiles4(64, 4, 0, 5, 1) == mr.MR_EINVAL
    assert libmr.mr_set_tiles4(64, 4, 0, 0, 2) == mr.MR_OK
    assert libmr.mr_set_tiles(64, 0, 1) == mr.MR_OK


def test_host_lambda_and_bits_match_the_oracle():
    """libmr's host-side sqrt(lambda) table and MV bit counts equal the oracle's (all QPs)."""
    import oracle
    from paper_2301_12191_amd import mr
    L = mr.lib()
    L.mr_sqrt_lambda_q16.restype = ctypes.c_int64
    L.mr_se_bits.restype = ctypes.c_int
    for qp in range(52):
        assert L.mr_sqrt_lambda_q16(qp) == oracle.sqrt_lambda_q16(qp), qp
    for v in range(-1100, 1101):
        assert L.mr_se_bits(v) == oracle.se_bits(v), v


def test_ladder_submit_many_argument_errors(libmr):
    from paper_2301_12191_amd import mr
    L = mr._ladder_lib()
    n = ctypes.c_int32(7)
    jobs = (mr.mr_job * 1)(mr.mr_job(0, 1, 0))
    ids = (ctypes.c_uint64 * 1)()
    assert L.mr_ladder_submit_many(None, jobs, 1, ids, ctypes.byref(n)) == mr.MR_EINVAL
    assert n.value == 0  # the count is written even when the call is refused
    assert L.mr_ladder_submit_many(None, jobs, 1, ids, None) == mr.MR_EINVAL


def test_ladder_release_many_argument_errors(libmr):
    from paper_2301_12191_amd import mr
    L = mr._ladder_lib()
    n = ctypes.c_int32(7)
    ids = (ctypes.c_uint64 * 2)(1, 2)
    assert L.mr_ladder_release_many(None, ids, 2, ctypes.byref(n)) == mr.MR_EINVAL
    assert n.value == 0  # the count is written even when the call is refused
    assert L.mr_ladder_release_many(None, ids, 2, None) == mr.MR_EINVAL
