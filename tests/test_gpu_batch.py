"""Batched and graph-replayed search: bit-exact against per-job launches and the oracle."""
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
    return m


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b, label):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), f"{label}: {k}"


def _ladder_jobs(mr, n_frames, scale_seed=0, with_bounds=False):
    """Six-rung ladder from one 3840x2160 source (box x9 crop, x6, x4, x3, x2, x1)."""
    import torch
    src = synth.Scene(synth.SEED_BASE + 3 + scale_seed, 3840, 2160, 24, 96, 8)
    frames = [src.render(t) for t in range(n_frames + 1)]
    jobs = []
    for (w, h, n, qp) in synth.LADDER:
        R = synth.search_range_for_width(w)
        rung = [torch.from_numpy(synth.box_downscale(f, n, w, h)).cuda() for f in frames]
        for k in range(1, n_frames + 1):
            jobs.append(dict(cur=rung[k], ref=rung[k - 1], qp=qp, search_range=R))
    return jobs


def test_batch_mixed_jobs_equal_single_calls(mr):
    import torch
    cases = [(200, 136, 32, 16, 1), (416, 240, 37, 16, 2), (640, 360, 30, 24, 3), (72, 40, 22, 5, 4),
             (960, 540, 27, 32, 5)]
    jobs = []
    for (W, H, qp, R, seed) in cases:
        sc = synth.Scene(seed, W, H, 5, 12, 2)
        jobs.append(dict(cur=torch.from_numpy(sc.render(1)).cuda(),
                         ref=torch.from_numpy(sc.render(0)).cuda(), qp=qp, search_range=R))
    # a bounded job in the same batch
    b = torch.randint(0, 2, (17, 25, 2), dtype=torch.uint8)
    b[..., 1] += b[..., 0] + 1
    jobs[0]["bounds"] = b.cuda()
    outs = mr.mr_ctu_search_batch(jobs)
    torch.cuda.synchronize()
    for j, o in zip(jobs, outs):
        single = mr.mr_ctu_search(j["cur"], j["ref"], j["qp"], j["search_range"], bounds=j.get("bounds"))
        torch.cuda.synchronize()
        _same(_np(o), _np(single), f"{j['cur'].shape}")
    # and against the oracle for the two small ones
    for j, o in list(zip(jobs, outs))[:2]:
        exp = oracle.ctu_search(j["cur"].cpu().numpy(), j["ref"].cpu().numpy(), j["qp"],
                                j["search_range"],
                                bounds=None if j.get("bounds") is None else j["bounds"].cpu().numpy())
        _same(_np(o), exp, "oracle")


def test_jobs_sharing_frames_equal_single_calls(mr):
    """One frame pair at several QPs and search forms in one batch: the jobs share the packed
    current CTUs and the intra SATDs, and those with equal margins the padded reference; each
    equals its own launch."""
    import torch
    sc = synth.Scene(11, 360, 200, 6, 14, 2)
    cur = torch.from_numpy(sc.render(1)).cuda()
    ref = torch.from_numpy(sc.render(0)).cuda()
    other = torch.from_numpy(sc.render(2)).cuda()
    half = synth.Scene(12, 180, 100, 6, 14, 2)
    seed_mv = mr.mr_ctu_search(torch.from_numpy(half.render(1)).cuda(),
                               torch.from_numpy(half.render(0)).cuda(), 30, 8)["mv"]
    seed = dict(ref_mv=seed_mv, ref_w=180, ref_h=100, r=2)
    b = torch.randint(0, 2, (25, 45, 2), dtype=torch.uint8)
    b[..., 1] += b[..., 0] + 1
    jobs = [dict(cur=cur, ref=ref, qp=37, search_range=16),
            dict(cur=cur, ref=ref, qp=22, search_range=16),               # shares the packed CTUs
            dict(cur=cur, ref=ref, qp=30, search_range=16, bounds=b.cuda()),
            dict(cur=cur, ref=ref, qp=27, search_range=16, seed=seed),    # pads the reference
            dict(cur=cur, ref=ref, qp=34, search_range=16, seed=seed),    # shares that copy
            dict(cur=cur, ref=ref, qp=32, search_range=16, subpel=True),  # and so does this one
            dict(cur=cur, ref=ref, qp=32, search_range=24, seed=seed),    # other margins: own copy
            dict(cur=cur, ref=other, qp=27, search_range=16, seed=seed),  # other reference
            dict(cur=other, ref=cur, qp=30, search_range=16)]             # other current frame
    # and a bounded job first: the jobs after it take its intra SATDs, also at nodes its
    # bounds exclude
    b2 = torch.zeros((25, 45, 2), dtype=torch.uint8)
    b2[..., 0] = 2
    b2[..., 1] = 3
    jobs += [dict(cur=ref, ref=other, qp=30, search_range=16, bounds=b2.cuda()),
             dict(cur=ref, ref=other, qp=22, search_range=16),
             dict(cur=ref, ref=cur, qp=35, search_range=8, seed=seed)]
    outs = mr.mr_ctu_search_batch(jobs)
    torch.cuda.synchronize()
    for k, (j, o) in enumerate(zip(jobs, outs)):
        single = mr.mr_ctu_search(j["cur"], j["ref"], j["qp"], j["search_range"],
                                  bounds=j.get("bounds"), seed=j.get("seed"),
                                  subpel=j.get("subpel", False))
        torch.cuda.synchronize()
        _same(_np(o), _np(single), f"job {k}")


def test_ladder_batch_equals_per_rung_launches(mr):
    """Six rungs x 2 frame pairs in one persistent launch == separate launches per pair."""
    import torch
    jobs = _ladder_jobs(mr, 2)
    print(f"\nladder: {len(jobs)} jobs", flush=True)
    outs = mr.mr_ctu_search_batch(jobs)
    torch.cuda.synchronize()
    got = [_np(o) for o in outs]
    for j, g in zip(jobs, got):
        single = _np(mr.mr_ctu_search(j["cur"], j["ref"], j["qp"], j["search_range"]))
        _same(g, single, f"rung {j['cur'].shape}")
    # sampled CTUs of two rungs against the oracle
    by_width = {j["cur"].shape[1]: i for i, j in enumerate(jobs)}
    for width, ctus in ((426, [0, 6, 27]), (1280, [0, 19, 239]), (1920, [0, 29, 509])):
        idx = by_width[width]
        j = jobs[idx]
        cur, ref = j["cur"].cpu().numpy(), j["ref"].cpu().numpy()
        exp = oracle.ctu_search(cur, ref, j["qp"], j["search_range"], ctu_list=ctus)
        tw = exp["cost"].shape[1]
        for t in ctus:
            cy, cx = (t // tw) * 8, (t % tw) * 8
            for k in ("depth", "mode", "mv"):
                assert np.array_equal(got[idx][k][cy:cy + 8, cx:cx + 8], exp[k][cy:cy + 8, cx:cx + 8])
            for k in ("cost", "dist", "bits"):
                assert got[idx][k].ravel()[t] == exp[k].ravel()[t]


def test_headline_batch_configuration_sampled(mr):
    """The benchmark's launch: 8 consecutive 1920x1080 pairs (R 64, QP 27) in one recorded
    batch, with the autotuner's shape installed, replayed twice; sampled CTUs of three pairs
    (corners, edges, interior, the partial strip at the right edge) against the oracle."""
    import torch
    W, H, R, QP, NP = 1920, 1080, 64, 27, 8
    scene = synth.Scene(synth.SEED_BASE + 1, W, H, 24, 48, 4)
    host = [scene.render(t) for t in range(NP + 1)]
    frames = [torch.from_numpy(f).cuda() for f in host]
    jobs = [dict(cur=frames[k + 1], ref=frames[k], qp=QP, search_range=R) for k in range(NP)]
    tune = mr.mr_autotune(jobs, reps=1)
    try:
        bt = mr.Batch(jobs)
        try:
            for _ in range(2):
                outs = bt.launch()
            got = [_np(o) for o in outs]
        finally:
            bt.close()
    finally:
        mr.mr_set_tiles(R, 0, 1)
    print(f"\nheadline batch, tiles {tune}", flush=True)
    ctus = [0, 29, 30, 58, 239, 255, 480, 509]  # 30 x 17 CTUs; strip 7 holds CTUs 28, 29
    for k in (0, 3, 7):
        exp = oracle.ctu_search(host[k + 1], host[k], QP, R, ctu_list=ctus)
        tw = exp["cost"].shape[1]
        for t in ctus:
            cy, cx = (t // tw) * 8, (t % tw) * 8
            for f in ("depth", "mode", "mv"):
                assert np.array_equal(got[k][f][cy:cy + 8, cx:cx + 8], exp[f][cy:cy + 8, cx:cx + 8]), (k, t, f)
            for f in ("cost", "dist", "bits"):
                assert got[k][f].ravel()[t] == exp[f].ravel()[t], (k, t, f)


def test_graph_replays_match_eager(mr):
    """Replay the captured graph several times with eager work and syncs in between."""
    import torch
    jobs = _ladder_jobs(mr, 1)[:5]  # five small rungs
    eager = [_np(o) for o in mr.mr_ctu_search_batch([dict(j) for j in jobs])]
    torch.cuda.synchronize()
    batch = mr.Batch(jobs)
    try:
        for rep in range(4):
            for j in jobs:
                for k in j["out"]:
                    j["out"][k].fill_(0x5A if k in ("depth", "mode") else 77)
            outs = batch.launch()
            # unrelated eager work on the same stream between replays
            x = torch.randn(256, 256, device="cuda")
            (x @ x).sum().item()
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                _same(_np(o), e, f"replay {rep}")
    finally:
        batch.close()


def test_launches_on_two_streams_are_ordered(mr):
    """Launches of one batch on two streams back to back: the second waits on the device for
    the first (they share the batch's scratch), so the outputs equal the eager search."""
    import torch
    jobs = _ladder_jobs(mr, 1)[:5]
    eager = [_np(o) for o in mr.mr_ctu_search_batch([dict(j) for j in jobs])]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    batch = mr.Batch(jobs)
    try:
        for rep in range(3):
            batch.launch(s1)
            outs = batch.launch(s2)
            batch.launch(s1)
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                _same(_np(o), e, f"two streams, round {rep}")
    finally:
        batch.close()


def test_batch_set_jobs_swaps_frames(mr):
    import torch
    sc = synth.Scene(55, 320, 192, 6, 10, 2)
    f = [torch.from_numpy(sc.render(t)).cuda() for t in range(3)]
    jobs = [dict(cur=f[1], ref=f[0], qp=30, search_range=16)]
    batch = mr.Batch(jobs)
    try:
        a = _np(batch.launch()[0])
        torch.cuda.synchronize()
        jobs2 = [dict(cur=f[2], ref=f[1], qp=30, search_range=16)]
        batch.set_jobs(jobs2)
        b = _np(batch.launch()[0])
        torch.cuda.synchronize()
        _same(a, _np(mr.mr_ctu_search(f[1], f[0], 30, 16)), "pair 1")
        _same(b, _np(mr.mr_ctu_search(f[2], f[1], 30, 16)), "pair 2")
        with pytest.raises(mr.MRError):
            batch.set_jobs([dict(cur=f[2], ref=f[1], qp=30, search_range=24)])  # other range
    finally:
        batch.close()


@pytest.mark.parametrize("R,D,nb", [(16, 2, 1), (16, 4, 3), (32, 2, 5), (32, 8, 2), (64, 4, 8),
                                    (64, 8, 1)])
def test_tile_overrides_do_not_change_results(mr, R, D, nb):
    import torch
    sc = synth.Scene(77 + R, 512, 320, 8, 20, 3)
    cur, ref = torch.from_numpy(sc.render(1)).cuda(), torch.from_numpy(sc.render(0)).cuda()
    base = _np(mr.mr_ctu_search(cur, ref, 29, R))
    mr.mr_set_tiles(R, D, nb)
    try:
        got = _np(mr.mr_ctu_search(cur, ref, 29, R))
    finally:
        mr.mr_set_tiles(R, 0, 1)
    torch.cuda.synchronize()
    _same(got, base, f"R{R} D{D} nb{nb}")


def test_autotune_installs_a_shape_and_keeps_results(mr):
    import torch
    sc = synth.Scene(91, 640, 360, 10, 16, 3)
    f = [torch.from_numpy(sc.render(t)).cuda() for t in range(3)]
    jobs = [dict(cur=f[k + 1], ref=f[k], qp=35, search_range=24) for k in range(2)]
    before = [_np(o) for o in mr.mr_ctu_search_batch([dict(j) for j in jobs])]
    try:
        res = mr.mr_autotune([dict(j) for j in jobs], reps=1)
        assert res["search_range"] == 24 and res["d"] in (2, 4, 5, 6, 8) and res["tried"] >= 4
        assert res["split"] in (1, 2)
        assert 0 < res["search_ms"] <= res["default_ms"]
        after = [_np(o) for o in mr.mr_ctu_search_batch([dict(j) for j in jobs])]
        torch.cuda.synchronize()
        for a, b in zip(before, after):
            _same(a, b, "after autotune")
    finally:
        mr.mr_set_tiles(24, 0, 1)
