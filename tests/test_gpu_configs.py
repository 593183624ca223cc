"""GPU parity at the measured workloads' own shapes, against the CPU oracle.

- Multi-resolution pruning (the thesis's inter-resolution analysis sharing): one seeded
  3840x2160 source, box-filtered to 960x540 and 1920x1080. The 960x540 reference (QP 32,
  R 32, full search) is compared in full. Its depths bound the 1920x1080 (QP 27, R 64) and
  3840x2160 (QP 22, R 128) searches at ratios 2 and 4 (depths n..n+1), and its MVs also
  seed them (refinement r = 4). The oracle side takes its own 960x540 depths and MVs, so
  the chain is checked end to end. Dependents are compared on sampled CTUs: corners, the
  partial bottom row, the left and right edges and the interior.
- The six-rung ladder (426x240 .. 3840x2160 x 16 pairs) in the launch configuration the
  benchmark times: one autotuned, graph-recorded batch, replayed; sampled CTUs of every rung
  at the first, a middle and the last pair.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("depth", "mode", "mv", "cost", "dist", "bits")
REFINE_R = 4


@pytest.fixture(scope="module")
def mr():
    import torch
    from paper_2301_12191_amd import mr as m
    assert torch.cuda.is_available()
    m.lib()
    oracle.build(force=False)
    synth.build(force=False)
    return m


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _compare(got, exp, ctus, label):
    tw = exp["cost"].shape[1]
    for t in ctus:
        cy, cx = (t // tw) * 8, (t % tw) * 8
        for k in ("depth", "mode", "mv"):
            g, e = got[k][cy:cy + 8, cx:cx + 8], exp[k][cy:cy + 8, cx:cx + 8]
            assert np.array_equal(g, e), f"{label}: {k} differs in CTU {t}"
        for k in ("cost", "dist", "bits"):
            assert got[k].ravel()[t] == exp[k].ravel()[t], \
                f"{label}: {k} of CTU {t}: {got[k].ravel()[t]} vs {exp[k].ravel()[t]}"


def _edge_samples(W, H):
    """Corners, the middle of each edge (the bottom row is partial when H % 64 != 0) and two
    interior CTUs."""
    tw, th = (W + 63) // 64, ((H + 7) // 8 * 8 + 63) // 64
    last = tw * th - 1
    mid_row = th // 2
    ctus = {0, tw - 1, last - tw + 1, last, mid_row * tw, mid_row * tw + tw - 1,
            (th - 1) * tw + tw // 2, mid_row * tw + tw // 2, (th // 3) * tw + tw // 3}
    return sorted(ctus)


def test_multires_pruning_and_reuse_at_measured_shapes(mr):
    import torch
    src = synth.Scene(synth.SEED_BASE + 2, 3840, 2160, 24, 96, 8)
    s0, s1 = src.render(0), src.render(1)
    pics = {w: (synth.box_downscale(s0, n, w, h), synth.box_downscale(s1, n, w, h))
            for (w, h, n) in ((960, 540, 4), (1920, 1080, 2), (3840, 2160, 1))}
    dev = {w: (torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()) for w, (r, c) in pics.items()}

    # 960x540 reference, full search, every CTU.
    print("\n960x540 QP 32 R 32 full search, all 135 CTUs", flush=True)
    r540, c540 = pics[960]
    g540 = mr.mr_ctu_search(dev[960][1], dev[960][0], 32, 32)
    torch.cuda.synchronize()
    e540 = oracle.ctu_search(c540, r540, 32, 32)
    got540 = _np(g540)
    for k in FIELDS:
        assert np.array_equal(got540[k], e540[k]), f"960x540 reference: {k}"

    seed_gpu = dict(ref_mv=g540["mv"], ref_w=960, ref_h=540, r=REFINE_R)
    seed_orc = oracle.Seed(e540["mv"], 960, 540, REFINE_R)
    for (w, h, qp, R) in ((1920, 1080, 27, 64), (3840, 2160, 22, 128)):
        # Depth bounds at ratio 2 and 4 from each side's own reference depths.
        bg = mr.mr_depth_bounds(g540["depth"], 960, 540, w, h, 0, 1)
        torch.cuda.synchronize()
        be = oracle.depth_bounds(e540["depth"], 960, 540, w, h, 0, 1)
        assert np.array_equal(bg.cpu().numpy(), be), f"bounds {w}x{h}"
        ref, cur = pics[w]
        ctus = _edge_samples(w, h)
        for name, use_b, use_s in (("full", False, False), ("pruned", True, False),
                                   ("reuse", True, True)):
            print(f"{w}x{h} QP {qp} R {R} {name}: CTUs {ctus}", flush=True)
            got = _np(mr.mr_ctu_search(dev[w][1], dev[w][0], qp, R, bounds=bg if use_b else None,
                                       seed=seed_gpu if use_s else None))
            torch.cuda.synchronize()
            exp = oracle.ctu_search(cur, ref, qp, R, bounds=be if use_b else None,
                                    seed=seed_orc if use_s else None, ctu_list=ctus)
            _compare(got, exp, ctus, f"{w}x{h} {name}")
            s = oracle.sqrt_lambda_q16(qp)
            assert np.all(got["cost"] == got["dist"] * 65536 + s * got["bits"])


def test_six_rung_ladder_batch_in_benchmark_configuration(mr):
    """96 jobs (6 rungs x 16 pairs) in one autotuned, recorded batch replayed twice, as the
    benchmark launches it; sampled CTUs of every rung at pairs 1, 8 and 16."""
    import torch
    nf = 16
    src = synth.Scene(synth.SEED_BASE + 3, 3840, 2160, 24, 96, 8)
    frames = [src.render(t) for t in range(nf + 1)]
    host, jobs = {}, []
    for (w, h, n, qp) in synth.LADDER:
        R = synth.search_range_for_width(w)
        rung = [synth.box_downscale(f, n, w, h) for f in frames]
        dev = [torch.from_numpy(x).cuda() for x in rung]
        for k in range(1, nf + 1):
            host[(w, k)] = (rung[k], rung[k - 1])
            jobs.append(dict(cur=dev[k], ref=dev[k - 1], qp=qp, search_range=R))
    del frames
    tune = mr.mr_autotune(jobs, reps=1)
    print(f"\nladder batch: {len(jobs)} jobs, tiles {tune}", flush=True)
    try:
        bt = mr.Batch(jobs)
        try:
            for _ in range(2):
                outs = bt.launch()
            torch.cuda.synchronize()
        finally:
            bt.close()
    finally:
        mr.mr_set_tiles(tune["search_range"], 0, 1)
    idx = 0
    for (w, h, n, qp) in synth.LADDER:
        R = synth.search_range_for_width(w)
        samples = _edge_samples(w, h)
        if w == 3840:
            samples = [0, 59, 1019, 2039]  # about 1 s of oracle time per CTU at R 128
        for k in (1, 8, 16):
            cur, ref = host[(w, k)]
            print(f"{w}x{h} pair {k}: CTUs {samples}", flush=True)
            exp = oracle.ctu_search(cur, ref, qp, R, ctu_list=samples)
            _compare(_np(outs[idx + k - 1]), exp, samples, f"{w}x{h} pair {k}")
        idx += nf
