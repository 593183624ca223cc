"""Ladder server on the GPU: each job's result in the mix equals its result alone."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FIELDS = ("depth", "mode", "mv", "cost", "dist", "bits")

# Three rungs from one source: 320x180 is the reference of the two others.
RUNGS = [dict(width=320, height=180, qp=32, search_range=16, ref_rung=-1),
         dict(width=640, height=360, qp=30, search_range=24, ref_rung=0),
         dict(width=960, height=540, qp=27, search_range=32, ref_rung=0)]
FACTORS = [6, 3, 2]


@pytest.fixture(scope="module")
def mr():
    import torch
    from paper_2301_12191_amd import mr as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _frames(n_streams, n_frames):
    import torch
    fr = {}
    for s in range(n_streams):
        src = synth.Scene(synth.SEED_BASE + 4 + 1000 * s, 1920, 1080, 12, 30, 4)
        for f in range(n_frames):
            img = src.render(f)
            for r, (cfg, k) in enumerate(zip(RUNGS, FACTORS)):
                fr[(s, f, r)] = torch.from_numpy(
                    synth.box_downscale(img, k, cfg["width"], cfg["height"])).cuda()
    return fr


def _alone(mr, fr, s, f, r, ref_cache, refine=None):
    """The job run by itself through mr_ctu_search (+ mr_depth_bounds for dependents, and a
    seed of the reference job's MVs when refine is set)."""
    import torch
    cfg = RUNGS[r]
    bounds = seed = None
    if cfg["ref_rung"] >= 0:
        rr = cfg["ref_rung"]
        rcfg = RUNGS[rr]
        if (s, f) not in ref_cache:
            ref_cache[(s, f)] = mr.mr_ctu_search(fr[(s, f, rr)], fr[(s, f - 1, rr)], rcfg["qp"],
                                                 rcfg["search_range"])
        ref_out = ref_cache[(s, f)]
        bounds = mr.mr_depth_bounds(ref_out["depth"], rcfg["width"], rcfg["height"],
                                    cfg["width"], cfg["height"], 0, 1)
        if refine is not None:
            seed = dict(ref_mv=ref_out["mv"], ref_w=rcfg["width"], ref_h=rcfg["height"],
                        r=min(refine, cfg["search_range"]))
    out = mr.mr_ctu_search(fr[(s, f, r)], fr[(s, f - 1, r)], cfg["qp"], cfg["search_range"],
                           bounds=bounds, seed=seed)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _run_mix(mr, fr, jobs, many=False, **kw):
    import torch
    lad = mr.Ladder(RUNGS, **kw)
    try:
        for (s, f, r), t in fr.items():
            lad.put_frame(s, f, r, t)
        ids = {}
        if many:  # "prepared": the argument array built ahead (Ladder.prepare)
            arg = lad.prepare(jobs) if many == "prepared" else jobs
            ids = dict(zip(lad.submit_many(arg), jobs))
        else:
            for (s, f, r) in jobs:
                ids[lad.submit(s, f, r)] = (s, f, r)
        got, seen = {}, 0
        deadline = 2000
        while seen < len(ids) and deadline > 0:
            for c in lad.poll(64, 100000):
                key = (c.stream_id, c.frame_idx, c.rung)
                assert c.status == 0, (key, c.status)
                assert c.t_arrive_ns <= c.t_start_ns <= c.t_done_ns
                if c.job_id in ids:
                    seen += 1
                    torch.cuda.synchronize()
                    got[key] = {k: v.cpu().numpy() for k, v in lad.outputs(c).items()}
                lad.release(c.job_id)
            deadline -= 1
        st = lad.stats()
    finally:
        lad.close()
    assert seen == len(ids)
    return got, st


def test_mix_equals_alone(mr):
    fr = _frames(3, 3)
    rng = np.random.default_rng(0)
    jobs = [(int(s), int(f), int(r)) for s in range(3) for f in (1, 2) for r in range(3)]
    rng.shuffle(jobs)  # dependents often arrive before their reference
    got, st = _run_mix(mr, fr, jobs)
    assert st["completed"] == len(jobs) + st["implied"] and st["failed"] == 0
    cache = {}
    for key in jobs:
        exp = _alone(mr, fr, *key, cache)
        for k in FIELDS:
            assert np.array_equal(got[key][k], exp[k]), (key, k)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_angular_rungs_equal_alone(mr):
    """Rungs whose jobs score the angular intra modes (the reference rung and one
    dependent) beside a plain dependent: each job equals its angular / plain search alone."""
    import torch
    rungs = [dict(RUNGS[0], angular=True), dict(RUNGS[1], angular=True), dict(RUNGS[2])]
    fr = _frames(2, 2)
    jobs = [(s, 1, r) for s in range(2) for r in (2, 1, 0)]
    lad = mr.Ladder(rungs)
    got = {}
    try:
        for (s, f, r), t in fr.items():
            lad.put_frame(s, f, r, t)
        ids = {lad.submit(*j): j for j in jobs}
        for _ in range(2000):
            for c in lad.poll(64, 100000):
                assert c.status == 0
                if c.job_id in ids:
                    torch.cuda.synchronize()
                    got[ids[c.job_id]] = {k: v.cpu().numpy() for k, v in lad.outputs(c).items()}
                lad.release(c.job_id)
            if len(got) == len(ids):
                break
    finally:
        lad.close()
    assert len(got) == len(jobs)
    for (s, f, r) in jobs:
        ref_out = mr.mr_ctu_search(fr[(s, f, 0)], fr[(s, f - 1, 0)], RUNGS[0]["qp"],
                                   RUNGS[0]["search_range"], angular=True)
        cfg = RUNGS[r]
        if r == 0:
            exp = ref_out
        else:
            b = mr.mr_depth_bounds(ref_out["depth"], RUNGS[0]["width"], RUNGS[0]["height"],
                                   cfg["width"], cfg["height"], 0, 1)
            exp = mr.mr_ctu_search(fr[(s, f, r)], fr[(s, f - 1, r)], cfg["qp"],
                                   cfg["search_range"], bounds=b, angular=(r == 1))
        torch.cuda.synchronize()
        for k in FIELDS:
            assert np.array_equal(got[(s, f, r)][k], exp[k].cpu().numpy()), ((s, f, r), k)
        if r < 2:
            assert got[(s, f, r)]["mode"].max() >= 3


@pytest.mark.parametrize("many", [True, "prepared"])
def test_submit_many_equals_alone(mr, many):
    """The same shuffled mix as above, handed to the server in one mr_ladder_submit_many (its
    argument array built at the call, or ahead by Ladder.prepare)."""
    fr = _frames(3, 3)
    rng = np.random.default_rng(1)
    jobs = [(int(s), int(f), int(r)) for s in range(3) for f in (1, 2) for r in range(3)]
    rng.shuffle(jobs)
    got, st = _run_mix(mr, fr, jobs, many=many, max_batch_jobs=64)
    assert st["completed"] == len(jobs) + st["implied"] and st["failed"] == 0
    cache = {}
    for key in jobs:
        exp = _alone(mr, fr, *key, cache)
        for k in FIELDS:
            assert np.array_equal(got[key][k], exp[k]), (key, k)


def test_submit_many_stops_at_first_refusal(mr):
    """A rung out of range in the middle: the jobs before it stay submitted and complete, the
    rest are not submitted, and the error names how many were accepted."""
    fr = _frames(1, 2)
    lad = mr.Ladder(RUNGS)
    try:
        for (s, f, r), t in fr.items():
            lad.put_frame(s, f, r, t)
        assert lad.submit_many([]) == []
        with pytest.raises(mr.MRError) as ei:
            lad.submit_many([(0, 1, 0), (0, 1, 1), (0, 1, 7), (0, 1, 2)])
        assert ei.value.code == mr.MR_EINVAL
        accepted = ei.value.submitted
        assert len(accepted) == 2
        seen, deadline = set(), 2000
        while len(seen) < 2 and deadline > 0:
            for c in lad.poll(64, 100000):
                assert c.status == 0 and c.rung in (0, 1) and not c.implied
                seen.add(c.job_id)
                lad.release(c.job_id)
            deadline -= 1
        assert seen == set(accepted)
        assert lad.stats()["submitted"] == 2
    finally:
        lad.close()


def test_many_dependents_per_batch_equal_alone(mr):
    """Twelve streams' dependents submitted at once: a batch then carries more than 16
    dependents, whose depth bounds the server computes in chunks of 16 per launch, each
    launched behind its implied reference's running batch."""
    fr = _frames(12, 2)
    jobs = [(s, 1, r) for s in range(12) for r in (1, 2)]
    got, st = _run_mix(mr, fr, jobs, max_batch_jobs=64)
    assert st["completed"] == len(jobs) + st["implied"] and st["implied"] == 12
    assert st["failed"] == 0
    cache = {}
    for key in jobs:
        exp = _alone(mr, fr, *key, cache)
        for k in FIELDS:
            assert np.array_equal(got[key][k], exp[k]), (key, k)


def test_dependent_only_submissions_imply_reference(mr):
    fr = _frames(2, 2)
    jobs = [(0, 1, 2), (1, 1, 1), (0, 1, 1)]
    got, st = _run_mix(mr, fr, jobs)
    assert st["implied"] == 2 and st["completed"] == 5
    cache = {}
    for key in jobs:
        exp = _alone(mr, fr, *key, cache)
        for k in FIELDS:
            assert np.array_equal(got[key][k], exp[k]), (key, k)


def test_tiny_budget_admits_one_job_at_a_time(mr):
    fr = _frames(2, 2)
    jobs = [(s, 1, r) for s in range(2) for r in range(3)]
    # 1 MB holds one 960x540 job (~0.73 MB of scratch and outputs) at a time
    got, st = _run_mix(mr, fr, jobs, budget_bytes=1 << 20, max_batch_jobs=8)
    assert st["completed"] == 6 and 0 < st["peak_bytes"] <= 1 << 20
    assert st["batches"] >= 3  # the budget forces small batches
    cache = {}
    for key in jobs:
        exp = _alone(mr, fr, *key, cache)
        for k in FIELDS:
            assert np.array_equal(got[key][k], exp[k]), (key, k)


def test_ladder_errors(mr):
    import torch
    fr = _frames(1, 2)
    lad = mr.Ladder(RUNGS)
    try:
        for (s, f, r), t in fr.items():
            if r != 0:  # reference rung frames missing
                lad.put_frame(s, f, r, t)
        with pytest.raises(mr.MRError) as e:
            lad.submit(0, 1, 1)
        assert e.value.code == mr.MR_EDEPEND
        with pytest.raises(mr.MRError) as e:
            lad.submit(0, 1, 5)
        assert e.value.code == mr.MR_EINVAL
        with pytest.raises(mr.MRError) as e:
            lad.submit(3, 1, 1)  # frames of stream 3 not resident
        assert e.value.code == mr.MR_EINVAL
        assert lad.poll(4, 1000) == []
    finally:
        lad.close()
    lad = mr.Ladder(RUNGS)
    try:
        for (s, f, r), t in fr.items():
            lad.put_frame(s, f, r, t)
        with pytest.raises(mr.MRError) as e:
            lad.cancel(12345)  # unknown job
        assert e.value.code == mr.MR_EINVAL
        jid = lad.submit(0, 1, 0)
        seen = []
        for _ in range(200):
            seen += lad.poll(4, 100000)
            if seen:
                break
        assert seen and seen[0].job_id == jid and seen[0].status == mr.MR_OK
        with pytest.raises(mr.MRError) as e:
            lad.cancel(jid)  # completed: nothing to cancel
        assert e.value.code == mr.MR_ESTATE
        with pytest.raises(mr.MRError) as e:
            lad.release_many([jid, 987654321])  # the first released, the unknown id refused
        assert e.value.code == mr.MR_EINVAL and "released 1 of 2" in str(e.value)
    finally:
        lad.close()
    with pytest.raises(mr.MRError):
        mr.Ladder([dict(width=64, height=64, qp=30, search_range=8, ref_rung=0)])  # self-reference
    with pytest.raises(mr.MRError):
        mr.Ladder(RUNGS, job_timeout_us=-1)


def test_output_blocks_recycled_across_equal_rungs(mr):
    """Two root rungs of the same size (QP 30 and 35) served frame by frame: the output
    blocks of released jobs are cached and handed to the next jobs of either rung. Every
    job equals its search alone, and the caches (outputs, scratch) stay within a quarter of
    the budget each."""
    import torch
    rungs = [dict(width=320, height=180, qp=30, search_range=16, ref_rung=-1),
             dict(width=320, height=180, qp=35, search_range=16, ref_rung=-1)]
    src = synth.Scene(synth.SEED_BASE + 77, 1920, 1080, 12, 30, 4)
    imgs = [torch.from_numpy(synth.box_downscale(src.render(f), 6, 320, 180)).cuda()
            for f in range(7)]
    budget = 4 << 20
    lad = mr.Ladder(rungs, budget_bytes=budget)
    got, cached = {}, []
    try:
        for f, img in enumerate(imgs):
            lad.put_frame(0, f, 0, img)
            lad.put_frame(0, f, 1, img)
        for f in range(1, 7):
            ids = {lad.submit(0, f, r): r for r in ((0, 1) if f % 2 else (1, 0))}
            left = dict(ids)
            for _ in range(200):
                for c in lad.poll(8, 100000):
                    assert c.status == 0
                    torch.cuda.synchronize()
                    got[(f, left.pop(c.job_id))] = {k: v.cpu().numpy()
                                                    for k, v in lad.outputs(c).items()}
                    lad.release(c.job_id)
                if not left:
                    break
            assert not left
            cached.append(lad.stats()["cached_bytes"])
        st = lad.stats()
    finally:
        lad.close()
    assert st["completed"] == 12 and st["failed"] == 0
    assert max(cached) > 0 and max(cached) <= 2 * (budget // 4)
    for (f, r), g in got.items():
        exp = mr.mr_ctu_search(imgs[f], imgs[f - 1], rungs[r]["qp"], 16)
        torch.cuda.synchronize()
        for k in FIELDS:
            assert np.array_equal(g[k], exp[k].cpu().numpy()), ((f, r), k)


def test_streaming_with_dropped_frames_and_forgotten_jobs(mr):
    """A stream served frame after frame, dropping each frame once no job needs it: every job
    still equals its result alone, a dropped frame can no longer be searched, and released
    job ids are forgotten."""
    import torch
    fr = _frames(1, 5)
    lad = mr.Ladder(RUNGS)
    cache = {}
    first_ids = []
    try:
        for r in range(3):
            lad.put_frame(0, 0, r, fr[(0, 0, r)])
        for f in range(1, 5):
            for r in range(3):
                lad.put_frame(0, f, r, fr[(0, f, r)])
            ids = {lad.submit(0, f, r): r for r in (2, 1)}  # the reference is implied
            seen = 0
            for _ in range(2000):
                for c in lad.poll(16, 100000):
                    assert c.status == 0
                    if c.job_id in ids:
                        torch.cuda.synchronize()
                        got = {k: v.cpu().numpy() for k, v in lad.outputs(c).items()}
                        exp = _alone(mr, fr, 0, f, ids[c.job_id], cache)
                        for k in FIELDS:
                            assert np.array_equal(got[k], exp[k]), (f, ids[c.job_id], k)
                        seen += 1
                        if f == 1:  # not reference-rung jobs: freed on release
                            first_ids.append(c.job_id)
                    lad.release(c.job_id)
                if seen == len(ids):
                    break
            assert seen == len(ids)
            lad.drop_frames(0, f)  # frame f - 1 is no longer needed
        with pytest.raises(mr.MRError) as e:
            lad.submit(0, 2, 1)  # frame 1 was dropped
        assert e.value.code in (mr.MR_EINVAL, mr.MR_EDEPEND)
        import time
        time.sleep(0.05)  # the server loop forgets released, handed-out jobs
        assert len(first_ids) == 2
        for jid in first_ids:
            with pytest.raises(mr.MRError) as e:
                lad.release(jid)
            assert e.value.code == mr.MR_EINVAL
    finally:
        lad.close()


def test_mv_reuse_dependents_equal_seeded_alone(mr):
    """With reuse_mv, every dependent equals mr_ctu_search_seeded with its reference job's MVs
    and depth bounds; references are unchanged."""
    fr = _frames(2, 3)
    jobs = [(s, f, r) for s in range(2) for f in (1, 2) for r in (2, 1, 0)]
    got, st = _run_mix(mr, fr, jobs, refine_range=4)
    assert st["completed"] == len(jobs) + st["implied"] and st["failed"] == 0
    cache = {}
    for key in jobs:
        exp = _alone(mr, fr, *key, cache, refine=4)
        for k in FIELDS:
            assert np.array_equal(got[key][k], exp[k]), (key, k)


def test_multi_qp_ladder_with_median_master(mr):
    """One resolution at QPs 22, 26, 30, 34, 38 with the QP-30 rung as the master of the
    others (bounds d-1..d+1 at ratio 1 and MV reuse r = 2): every job equals the seeded
    search run alone with the master job's depths and MVs."""
    import torch
    qps = [22, 26, 30, 34, 38]
    rungs = [dict(width=320, height=180, qp=q, search_range=16, ref_rung=-1 if q == 30 else 2)
             for q in qps]
    fr = {}
    for s in range(2):
        src = synth.Scene(synth.SEED_BASE + 40 + 1000 * s, 1920, 1080, 12, 30, 4)
        for f in range(3):
            img = torch.from_numpy(synth.box_downscale(src.render(f), 6, 320, 180)).cuda()
            for r in range(5):
                fr[(s, f, r)] = img
    jobs = [(s, f, r) for s in range(2) for f in (1, 2) for r in (0, 4, 2, 1, 3)]
    lad = mr.Ladder(rungs, delta_lo=1, delta_hi=1, refine_range=2)
    got = {}
    try:
        for (s, f, r), t in fr.items():
            lad.put_frame(s, f, r, t)
        ids = {lad.submit(*j): j for j in jobs}
        deadline = 2000
        while len(got) < len(ids) and deadline > 0:
            for c in lad.poll(64, 100000):
                assert c.status == 0
                if c.job_id in ids:
                    torch.cuda.synchronize()
                    got[ids[c.job_id]] = {k: v.cpu().numpy() for k, v in lad.outputs(c).items()}
                lad.release(c.job_id)
            deadline -= 1
        st = lad.stats()
    finally:
        lad.close()
    assert len(got) == len(jobs) and st["failed"] == 0
    for (s, f, r) in jobs:
        master = mr.mr_ctu_search(fr[(s, f, 2)], fr[(s, f - 1, 2)], 30, 16)
        if r == 2:
            exp = master
        else:
            b = mr.mr_depth_bounds(master["depth"], 320, 180, 320, 180, 1, 1)
            exp = mr.mr_ctu_search(fr[(s, f, r)], fr[(s, f - 1, r)], qps[r], 16, bounds=b,
                                   seed=dict(ref_mv=master["mv"], ref_w=320, ref_h=180, r=2))
        torch.cuda.synchronize()
        for k in FIELDS:
            assert np.array_equal(got[(s, f, r)][k], exp[k].cpu().numpy()), ((s, f, r), k)


def test_multi_encoding_dag_through_the_ladder(mr):
    """15 rungs (3 resolutions x 5 QPs, per-rung policies): the server's results for two frames
    of two streams equal the DAG computed job by job."""
    import torch
    from dag_spec import dag_rungs
    sizes = [(160, 96, 8), (320, 192, 16), (640, 384, 24)]
    spec = dag_rungs(sizes)
    rungs = [dict(width=w, height=h, qp=q, search_range=R, ref_rung=ref, delta_lo=dlo,
                  delta_hi=dhi, refine_range=r) for (w, h, q, R, ref, dlo, dhi, r) in spec]
    fr = {}
    for s in range(2):
        src = synth.Scene(synth.SEED_BASE + 50 + 1000 * s, 640, 384, 8, 16, 2)
        for f in range(3):
            img = src.render(f)
            for i, (w, h, *_rest) in enumerate(spec):
                k = 640 // w
                fr[(s, f, i)] = torch.from_numpy(synth.box_downscale(img, k, w, h)).cuda()
    # Submit the leaves first: the server implies their masters.
    jobs = [(s, f, i) for f in (1, 2) for s in range(2) for i in reversed(range(15))]
    lad = mr.Ladder(rungs, max_batch_jobs=16)
    got = {}
    try:
        for key, t in fr.items():
            lad.put_frame(*key, t)
        ids = {}
        for j in jobs:
            ids[lad.submit(*j)] = j
        deadline = 4000
        while len(got) < len(ids) and deadline > 0:
            for c in lad.poll(64, 100000):
                assert c.status == 0
                if c.job_id in ids:
                    torch.cuda.synchronize()
                    got[ids[c.job_id]] = {k: v.cpu().numpy() for k, v in lad.outputs(c).items()}
                lad.release(c.job_id)
            deadline -= 1
        st = lad.stats()
    finally:
        lad.close()
    assert len(got) == len(jobs) and st["failed"] == 0
    for s in range(2):
        for f in (1, 2):
            alone = []
            for i, (w, h, q, R, ref, dlo, dhi, r) in enumerate(spec):
                cur, prev = fr[(s, f, i)], fr[(s, f - 1, i)]
                if ref < 0:
                    o = mr.mr_ctu_search(cur, prev, q, R)
                else:
                    rw, rh = spec[ref][:2]
                    b = mr.mr_depth_bounds(alone[ref]["depth"], rw, rh, w, h, dlo, dhi)
                    o = mr.mr_ctu_search(cur, prev, q, R, bounds=b,
                                         seed=dict(ref_mv=alone[ref]["mv"], ref_w=rw, ref_h=rh,
                                                   r=r))
                alone.append(o)
                torch.cuda.synchronize()
                for k in FIELDS:
                    assert np.array_equal(got[(s, f, i)][k], o[k].cpu().numpy()), ((s, f, i), k)
