"""Benchmark of the per-CTU coding-tree search on one MI355X.

Default workload (the headline number, `value`): the six-rung ladder, 426x240 / 640x360 /
960x540 / 1280x720 / 1920x1080 / 3840x2160 box-filtered from one seeded 3840x2160 source,
16 consecutive frame pairs per rung (frame k searched against frame k-1), QPs 37/35/32/30/
27/22, full search with R = 16/24/32/48/64/128.  One step = all 96 pairs (48,208 CTUs)
through the whole hot path (prep, motion search + arg-min, SATD / intra / quad-tree
decision) in one persistent, graph-replayed launch with the autotuned tile shape.  Frames are
resident in HBM before timing starts.

Beside it the JSON line carries:
  roofline     : the search kernel of the headline launch (dominant) as algorithmic
                 absolute differences per second against the packed-byte SAD peak, with the
                 leaf kernel of the same launch as algorithmic 16-bit SATD operations;
  single_res   : 1920x1080, 8 consecutive pairs, R 64, QP 27 (its own roofline);
  small        : the 416x240 pair (R 16, QP 32): GPU latency of one call and of a graph replay;
  small_ranges : the ladder's 426x240 / 640x360 / 960x540 rungs (R 16 / 24 / 32), 16 pairs each:
                 search time and fraction of peak per rung;
  pruned       : multi-resolution pruning on a 3840x2160 source: 960x540 reference (QP 32,
                 R 32) bounds 1920x1080 (QP 27, R 64) and 3840x2160 (QP 22, R 128), refine
                 depths n..n+1; speedup of pruned over full search and the exact RD-cost
                 increase; the same with the reference MVs reused as search centres
                 (refinement r = 4), and the refinement kernel's absdiff rate;
  subpel       : the 1080p workload with quarter-pel refinement (SATD, H.265 interpolation):
                 time, the refinement's share and operation rate, RD-cost change;
  angular      : the 1080p workload with the 33 angular intra modes: time, the leaf kernel's
                 operation rate, the share of angular CUs' units, RD-cost change;
  multi_qp     : one 1920x1080 pair at QPs 22/26/30/34/38 with the median QP as master
                 (same-resolution sharing): speedup and RD-cost increase per QP;
  dag          : the multi-encoding scheme (3 resolutions x 5 QPs, median-QP masters chained
                 540p -> 1080p -> 2160p) through the ladder server, against 15 full searches;
  serving      : 64 streams, Poisson arrivals (mean 240 jobs/s) through the ladder server:
                 p50/p99 latency overall and per rung, sustained CTUs/s;
  cpu_baseline : the CPU oracle on a stratified sample of the headline workload (every 8th
                 CTU of each rung's first pair), compared bit for bit with the GPU's outputs,
                 and the oracle on the whole first 1920x1080 pair, compared likewise.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-single]
                      [--no-small] [--no-small-ranges] [--no-pruned] [--no-subpel]
                      [--no-angular] [--no-multi-qp]
                      [--no-dag] [--no-serving] [--serve-seconds S]
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Packed-byte SAD peak: 256 CUs x 64 lanes x 2.4 GHz x 4 absolute differences per v_sad_u8.
PEAK_ABSDIFF = 256 * 64 * 2.4e9 * 4
# Packed 16-bit peak: 256 CUs x 64 lanes x 2.4 GHz x 2 operations per v_pk_* / v_dot2 lane-op.
PEAK_OPS16 = 256 * 64 * 2.4e9 * 2
# Operations of one 4x4 SATD: 16 residual subtractions, 64 additions/subtractions of the two
# butterfly passes, 16 absolute values and 15 additions of the sum.
SATD4_OPS = 16 + 64 + 16 + 15
# Refinement half-width of the seeded (MV reuse) variant.
REFINE_R = 4
# ... and of the same-resolution multi-QP dependents (exact co-located MVs).
MULTI_QP_R = 2


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def coded(n):
    return (n + 7) // 8 * 8


def search_absdiff(w, h, R):
    """Algorithmic absolute differences of a full search: (2R+1)^2 per coded sample (every
    larger CU's SAD is a sum of 8x8 SADs)."""
    return (2 * R + 1) ** 2 * coded(w) * coded(h)


def inside_tiles(w, h):
    """4x4 tiles of all quad-tree nodes (64..8) lying inside the coded picture."""
    w8, h8 = coded(w), coded(h)
    return sum((w8 // n) * (h8 // n) * (n * n // 16) for n in (64, 32, 16, 8))


def leaf_ops(w, h):
    """Algorithmic 16-bit operations of the leaf kernel on a full search: the SATDs of the
    inter, planar and DC residuals of every inside node."""
    return 3 * inside_tiles(w, h) * SATD4_OPS


def subpel_ops(w, h):
    """Algorithmic operations of the quarter-pel refinement: 16 interpolated candidates per
    inside node (8 half-pel, 8 quarter-pel), each predicted sample 8 horizontal + 8 vertical
    taps (2 operations per tap), and each candidate's 4x4 SATDs."""
    tiles = inside_tiles(w, h)
    return 16 * tiles * (16 * 16 * 2 + SATD4_OPS)


def traffic_record(name):
    """HBM bytes per launch from a committed counter record (FETCH_SIZE / WRITE_SIZE of the
    search kernel scaled by a plain copy's counters); None once any source the kernel is
    compiled from has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if rec.get("sources_sha256") == h.hexdigest():
            return rec["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def pct_of(vals, p):
    """Nearest-rank percentile of a sorted list."""
    return vals[min(len(vals) - 1, max(0, int(p * len(vals) + 0.999999) - 1))]


def timed_launches(mr, torch, fn, steps, warmup):
    """Run fn warmup times, then time `steps` calls with the library's stage events on."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    mr.mr_profile_read(reset=True)
    mr.mr_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mr.mr_profile_enable(False)
    return t1 - t0, mr.mr_profile_read(reset=True)


def stage_avg(prof):
    return {k: round(v[0] / max(1, v[1]), 4) for k, v in prof.items()}


def dag_spec(sizes, qps=(30, 22, 26, 34, 38)):
    """Rungs of the multi-encoding scheme: per resolution, the median QP (first) is the master
    of the other QPs (ratio 1: depths d-1..d+1, r = 2); masters chain across resolutions
    (ratio 2: depths d..d+1, r = 4)."""
    rungs = []
    for li, (w, h, R) in enumerate(sizes):
        for k, qp in enumerate(qps):
            if k == 0:
                rungs.append(dict(width=w, height=h, qp=qp, search_range=R,
                                  ref_rung=-1 if li == 0 else 5 * (li - 1),
                                  delta_lo=0, delta_hi=1, refine_range=REFINE_R))
            else:
                rungs.append(dict(width=w, height=h, qp=qp, search_range=R, ref_rung=5 * li,
                                  delta_lo=1, delta_hi=1, refine_range=MULTI_QP_R))
    return rungs


def run_dag(mr, synth, torch, dev, n_frames=4):
    """The 15-representation DAG served frame by frame and pipelined (all frames submitted at
    once: tiers of frame t overlap masters of frame t + 1), against 15 full searches."""
    sizes = [(960, 540, 32), (1920, 1080, 64), (3840, 2160, 128)]
    rungs = dag_spec(sizes)
    src = synth.Scene(synth.SEED_BASE + 6, 3840, 2160, 24, 96, 8)
    frames = {}
    for f in range(n_frames + 1):
        img = src.render(f)
        for (w, h, _), k in zip(sizes, (4, 2, 1)):
            frames[(f, w)] = torch.from_numpy(synth.box_downscale(img, k, w, h)).to(dev)
    n_ctus = sum(mr.ctu_shape(r["width"], r["height"])[0] * mr.ctu_shape(r["width"], r["height"])[1]
                 for r in rungs)
    # Baseline: the 15 representations of frame 1 as full searches, one batch.
    full_jobs = [dict(cur=frames[(1, r["width"])], ref=frames[(0, r["width"])], qp=r["qp"],
                      search_range=r["search_range"]) for r in rungs]
    mr.mr_ctu_search_batch(full_jobs)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    outs = mr.mr_ctu_search_batch(full_jobs)
    torch.cuda.synchronize()
    full_ms = (time.perf_counter() - ta) * 1e3
    j_full = [int(o["cost"].sum().item()) for o in outs]

    # One long-lived server: warm-up runs, then the frame-by-frame and the pipelined run,
    # each on a stream of its own (its block caches and plans warm, as in service).
    lad = mr.Ladder(rungs, max_batch_jobs=64)

    def serve(pipelined, stream):
        j_dag, lat, held, first_launch = {}, [], [], []
        st0 = lad.stats()
        for f in range(n_frames + 1):
            for i, r in enumerate(rungs):
                lad.put_frame(stream, f, i, frames[(f, r["width"])])
        # No collection of the client's garbage inside the timed region: a full collection
        # of this process's objects takes milliseconds, comparable to several frames.
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        order = [(f, i) for f in range(1, n_frames + 1) for i in range(len(rungs))]
        groups = [order] if pipelined else [[x for x in order if x[0] == f]
                                            for f in range(1, n_frames + 1)]
        group_ms = []
        # The group's jobs as the server takes them, built before the previous group ends;
        # the previous group's last completions are released after this submission.
        subs = [lad.prepare([(stream, f, i) for f, i in grp]) for grp in groups]
        pending = []
        for g, grp in enumerate(groups):
            tg = time.perf_counter()
            ids = dict(zip(lad.submit_many(subs[g]), grp))
            if pending:
                lad.release_many(pending)
                pending = []
            done, idle, starts = 0, 0, []
            while done < len(ids):
                got = lad.poll(64, 200000)
                idle = 0 if got else idle + 1
                if idle > 150:  # 30 s without a completion
                    raise RuntimeError("dag: ladder made no progress")
                rel = []
                for c in got:
                    if c.status != 0:
                        raise RuntimeError(f"dag: job failed with status {c.status}")
                    if c.job_id in ids:
                        done += 1
                        f, i = ids[c.job_id]
                        lat.append((c.t_done_ns - c.t_arrive_ns) * 1e-6)
                        starts.append((c.t_start_ns - c.t_arrive_ns) * 1e-6)
                        if f == 1:  # read after the timed region (no device sync here)
                            held.append((i, c))
                            continue
                    rel.append(c.job_id)
                if done < len(ids):
                    lad.release_many(rel)
                else:
                    pending = rel
            first_launch.append(min(starts))  # submission -> the group's first launch
            group_ms.append(round((time.perf_counter() - tg) * 1e3, 3))
        t1 = time.perf_counter()
        gc.enable()
        lad.release_many(pending)
        st = lad.stats()
        for i, c in held:
            j_dag[i] = int(lad.outputs(c)["cost"].sum().item())
        lad.release_many([c.job_id for _, c in held])
        lad.drop_frames(stream, n_frames + 1)
        nb = st["batches"] - st0["batches"]
        host = {"batches": nb,
                "host_ms_per_batch": round((st["host_launch_ms"] - st0["host_launch_ms"]) /
                                           max(1, nb), 4),
                "submit_to_first_launch_ms": round(sorted(first_launch)[len(first_launch) // 2], 4),
                "group_ms": group_ms}
        return (t1 - t0) * 1e3 / n_frames, j_dag, sorted(lat), host

    try:
        # Warm-up, one pass of each form (plans, key tables, the block caches of both forms'
        # batch sizes): a server in service has seen both.
        serve(True, 0)
        serve(False, 1)
        seq_ms, _, _, seq_host = serve(False, 2)
        pipe_ms, j_dag, lat, pipe_host = serve(True, 3)
    finally:
        lad.close()
    rd = {}
    for li, (w, h, _) in enumerate(sizes):
        jf = sum(j_full[5 * li:5 * li + 5])
        jd = sum(j_dag[i] for i in range(5 * li, 5 * li + 5))
        rd[f"{w}x{h}"] = round(100.0 * (jd - jf) / jf, 6)
    pct = lambda p: lat[min(len(lat) - 1, max(0, int(p * len(lat) + 0.999999) - 1))]
    return {
        "workload": f"{n_frames} frames of 960x540 (R32) / 1920x1080 (R64) / 3840x2160 (R128) x "
                    "QPs 30/22/26/34/38 = 15 representations per frame; per resolution the QP-30 "
                    "job masters the others (depths d-1..d+1, r = 2); QP-30 masters chain "
                    "540p -> 1080p -> 2160p (depths d..d+1, r = 4); ladder server, one stream",
        "ctus_per_frame": n_ctus,
        "full_search_frame_ms": round(full_ms, 3),
        "dag_frame_by_frame_ms": round(seq_ms, 3),
        "dag_pipelined_frame_ms": round(pipe_ms, 3),
        "speedup_pipelined_vs_full": round(full_ms / pipe_ms, 3),
        "pipelining_gain": round(seq_ms / pipe_ms, 3),
        "pipelined_ctus_per_s": round(n_ctus / (pipe_ms * 1e-3), 1),
        "job_latency_p50_ms": round(pct(0.5), 3), "job_latency_p99_ms": round(pct(0.99), 3),
        "host_frame_by_frame": seq_host, "host_pipelined": pipe_host,
        "rd_cost_increase_pct_frame1": rd}


# Encoder-time savings the thesis reports for its multi-resolution reuse: whole x265 encodes
# (preset medium) on an Intel Core i7-7500U (2 cores, 4 threads, 2.7 GHz), as
# (T_ref - T) / T_ref in percent. Quoted beside the GPU figures as context only: they time a
# whole CPU encoder, not this path. Sources: the CQP table of the inter-resolution
# analysis-sharing section (1080p from the 540p master, reuse level 10), the cVBR results of
# the inter-resolution section of the results chapter, and the proposed multi-encoding scheme's
# section.
THESIS_CONTEXT = {
    "kind": "encoder-time savings, percent; CPU x265, not comparable to kernel throughput",
    "hardware": "Intel Core i7-7500U, 2 cores / 4 threads, 2.7 GHz; x265 preset medium",
    "cqp_1080p_from_540p": {"no_refinement": 72.04, "refinement": 28.99},
    "cvbr_1080p_from_540p": {"no_refinement": 65.64, "refinement": 50.45},
    "cvbr_2160p_from_1080p": {"no_refinement": 63.96, "refinement": 52.82},
    "multi_encoding_speedup_over_prior_scheme_pct": 9,
}


def run_headline(mr, synth, torch, dev, args):
    """Six rungs x 16 pairs in one autotuned, graph-replayed batch (the headline step)."""
    nf = 16
    log(f"rendering 3840x2160 x {nf + 1} ladder source frames")
    src = synth.Scene(synth.SEED_BASE + 3, 3840, 2160, 24, 96, 8)
    srcs = [src.render(t) for t in range(nf + 1)]
    jobs, host_pair = [], {}
    for (w, h, n, qp) in synth.LADDER:
        R = synth.search_range_for_width(w)
        rung = [synth.box_downscale(f, n, w, h) for f in srcs]
        host_pair[w] = (rung[1], rung[0], qp, R)  # the first pair, for the CPU leg
        on_dev = [torch.from_numpy(x).to(dev) for x in rung]
        for k in range(1, nf + 1):
            jobs.append(dict(cur=on_dev[k], ref=on_dev[k - 1], qp=qp, search_range=R))
    del srcs
    stream = torch.cuda.current_stream()
    tune = mr.mr_autotune(jobs, reps=1)  # installs the best tile shape for R 128
    log(f"autotune: {tune}")
    batch = mr.Batch(jobs)
    elapsed, prof = timed_launches(mr, torch, lambda: batch.launch(stream), args.steps,
                                   args.warmup)
    ctus = sum(j["out"]["cost"].numel() for j in jobs)
    ms_per_step = elapsed * 1e3 / args.steps
    value = ctus * args.steps / elapsed
    log(f"headline: {ms_per_step:.3f} ms/step, {value:.0f} CTUs/s; stages {prof}")
    absdiff = sum(search_absdiff(j["cur"].shape[1], j["cur"].shape[0], j["search_range"])
                  for j in jobs)
    search_s = prof["search"][0] / 1e3 / max(1, prof["search"][1])
    leaf_s = prof["leaf"][0] / 1e3 / max(1, prof["leaf"][1])
    lops = sum(leaf_ops(j["cur"].shape[1], j["cur"].shape[0]) for j in jobs)
    roofline = {
        "bound": "alu", "achieved": round(absdiff / search_s / 1e12, 3),
        "peak": round(PEAK_ABSDIFF / 1e12, 3), "unit": "T absdiff/s",
        "frac": round(absdiff / search_s / PEAK_ABSDIFF, 4),
        "traffic": traffic_record("search_ladder_traffic.json"),
        "traffic_unit": "HBM bytes per launch",
        "kernel": "search_kernel (persistent, 96 pairs of 6 rungs per launch)",
        "avg_launch_ms": round(search_s * 1e3, 4), "absdiff_per_launch": absdiff,
        "stage_avg_ms": stage_avg(prof),
        "tiles": {"d": tune["d"], "nbands": tune["nbands"], "strip": tune["strip"],
                  "autotune_shapes": tune["tried"]},
        "leaf": {"bound": "alu", "unit": "T int16 ops/s", "ops_per_launch": lops,
                 "avg_launch_ms": round(leaf_s * 1e3, 4),
                 "achieved": round(lops / leaf_s / 1e12, 3),
                 "peak": round(PEAK_OPS16 / 1e12, 3),
                 "frac": round(lops / leaf_s / PEAK_OPS16, 4)},
    }
    outs = {}
    for i, (w, h, n, qp) in enumerate(synth.LADDER):
        o = jobs[i * nf]["out"]  # the rung's first pair
        outs[w] = {k: v.cpu().numpy() for k, v in o.items()}
    batch.close()
    mr.mr_set_tiles(tune["search_range"], 0, 1)
    config = {"workload": "6-rung ladder 426x240/640x360/960x540/1280x720/1920x1080/3840x2160 "
                          "x 16 frame pairs, QP 37/35/32/30/27/22, full search R "
                          "16/24/32/48/64/128, one persistent launch",
              "ctus_per_step": ctus, "pairs": len(jobs), "frames_per_rung": nf + 1}
    del jobs, batch
    torch.cuda.synchronize()
    return value, ms_per_step, config, roofline, outs, host_pair


def run_single_res(mr, synth, torch, dev, args):
    """1920x1080, 8 consecutive pairs, R 64, QP 27, one batch per step."""
    W, H, R, QP, NP = 1920, 1080, 64, 27, 8
    log("rendering 1920x1080 x 9 frames")
    scene = synth.Scene(synth.SEED_BASE + 1, W, H, 24, 48, 4)
    frames = [torch.from_numpy(scene.render(t)).to(dev) for t in range(NP + 1)]
    jobs = [dict(cur=frames[k + 1], ref=frames[k], qp=QP, search_range=R) for k in range(NP)]
    stream = torch.cuda.current_stream()
    tune = mr.mr_autotune(jobs, reps=2)
    batch = mr.Batch(jobs)
    elapsed, prof = timed_launches(mr, torch, lambda: batch.launch(stream), args.steps,
                                   args.warmup)
    ctus = jobs[0]["out"]["cost"].numel() * NP
    ms = elapsed * 1e3 / args.steps
    absdiff = search_absdiff(W, H, R) * NP
    search_s = prof["search"][0] / 1e3 / max(1, prof["search"][1])
    res = {
        "workload": "1920x1080 luma, 8 consecutive frame pairs, full search R64 QP27",
        "ms_per_step": round(ms, 4), "ctus_per_s": round(ctus / (ms * 1e-3), 1),
        "roofline": {"bound": "alu", "achieved": round(absdiff / search_s / 1e12, 3),
                     "peak": round(PEAK_ABSDIFF / 1e12, 3), "unit": "T absdiff/s",
                     "frac": round(absdiff / search_s / PEAK_ABSDIFF, 4),
                     "traffic": traffic_record("search_1080p_r64_traffic.json"),
                     "traffic_unit": "HBM bytes per launch",
                     "kernel": "search_kernel (persistent, 8 pairs per launch)",
                     "avg_launch_ms": round(search_s * 1e3, 4), "absdiff_per_launch": absdiff,
                     "stage_avg_ms": stage_avg(prof)},
        "tiles": {"d": tune["d"], "nbands": tune["nbands"], "strip": tune["strip"]}}
    gpu_pair0 = {k: v.cpu().numpy() for k, v in jobs[0]["out"].items()}
    host_pair0 = (frames[1].cpu().numpy(), frames[0].cpu().numpy())
    batch.close()
    mr.mr_set_tiles(R, 0, 1)
    return res, frames, jobs, gpu_pair0, host_pair0


def run_small(mr, synth, torch, dev):
    """416x240 pair, R 16, QP 32: latency of one call (eager) and of one graph replay."""
    sc = synth.Scene(synth.SEED_BASE + 0, 416, 240, 6, 12, 0)
    ref, cur = torch.from_numpy(sc.render(0)).to(dev), torch.from_numpy(sc.render(1)).to(dev)
    out = mr.alloc_outputs(416, 240, dev)
    stream = torch.cuda.current_stream()

    def lat(fn, n):
        v = []
        for _ in range(n):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            v.append((time.perf_counter() - t) * 1e3)
        return sorted(v)

    eager = lambda: mr.mr_ctu_search(cur, ref, 32, 16, out=out, stream=stream)
    for _ in range(5):
        eager()
    le = lat(eager, 200)
    batch = mr.Batch([dict(cur=cur, ref=ref, qp=32, search_range=16, out=out)])
    replay = lambda: batch.launch(stream)
    for _ in range(5):
        replay()
    lg = lat(replay, 200)
    _, prof = timed_launches(mr, torch, replay, 200, 0)
    batch.close()
    search_s = prof["search"][0] / 1e3 / max(1, prof["search"][1])
    absdiff = search_absdiff(416, 240, 16)
    return {"workload": "416x240 pair, R 16, QP 32 (28 CTUs)",
            "eager_call_ms_p50": round(pct_of(le, 0.5), 4),
            "eager_call_ms_p99": round(pct_of(le, 0.99), 4),
            "graph_replay_ms_p50": round(pct_of(lg, 0.5), 4),
            "graph_replay_ms_p99": round(pct_of(lg, 0.99), 4),
            "stage_avg_ms": stage_avg(prof),
            "search_frac_of_peak": round(absdiff / search_s / PEAK_ABSDIFF, 4)}


def run_small_ranges(mr, synth, torch, dev, args):
    """The ladder's three smallest rungs (426x240 R 16, 640x360 R 24, 960x540 R 32), 16
    consecutive pairs each from the ladder source, one batch per rung at the built-in tiles:
    search time and fraction of peak where few wavefronts carry the work."""
    nf = 16
    src = synth.Scene(synth.SEED_BASE + 3, 3840, 2160, 24, 96, 8)
    srcs = [src.render(t) for t in range(nf + 1)]
    stream = torch.cuda.current_stream()
    res = {}
    for (w, h, n, qp) in synth.LADDER[:3]:
        R = synth.search_range_for_width(w)
        rung = [torch.from_numpy(synth.box_downscale(f, n, w, h)).to(dev) for f in srcs]
        jobs = [dict(cur=rung[k], ref=rung[k - 1], qp=qp, search_range=R)
                for k in range(1, nf + 1)]
        b = mr.Batch(jobs)
        _, prof = timed_launches(mr, torch, lambda: b.launch(stream), max(5, args.steps),
                                 max(1, args.warmup))
        b.close()
        search_s = prof["search"][0] / 1e3 / max(1, prof["search"][1])
        absdiff = search_absdiff(w, h, R) * nf
        res[f"{w}x{h}"] = {"R": R, "pairs": nf, "ctus": jobs[0]["out"]["cost"].numel() * nf,
                           "search_ms": round(search_s * 1e3, 4),
                           "frac_of_peak": round(absdiff / search_s / PEAK_ABSDIFF, 4)}
    return res


def run_subpel(mr, torch, frames, jobs_int, args):
    """The 1080p workload with quarter-pel refinement; the refinement kernel is timed by its
    own stage events."""
    QP, R, NP = 27, 64, len(jobs_int)
    jobs_sp = [dict(cur=frames[k + 1], ref=frames[k], qp=QP, search_range=R, subpel=True)
               for k in range(NP)]
    stream = torch.cuda.current_stream()
    bsp = mr.Batch(jobs_sp)
    elapsed, pst = timed_launches(mr, torch, lambda: bsp.launch(stream), args.steps,
                                  max(1, args.warmup))
    j_int = sum(int(j["out"]["cost"].sum().item()) for j in jobs_int)
    j_sp = sum(int(j["out"]["cost"].sum().item()) for j in jobs_sp)
    sp_ms = elapsed * 1e3 / args.steps
    stage = stage_avg(pst)
    ref_ms = stage["subpel"]
    ops = subpel_ops(1920, 1080) * NP
    ctus = jobs_int[0]["out"]["cost"].numel() * NP
    bsp.close()
    return {
        "workload": "the 1080p 8 pairs (1920x1080, R 64, QP 27) with half- and quarter-pel "
                    "SATD refinement of every CU's MV (H.265 luma interpolation)",
        "ms_per_step": round(sp_ms, 4), "ctus_per_s": round(ctus / (sp_ms * 1e-3), 1),
        "stage_avg_ms": stage, "refinement_ms": round(ref_ms, 4),
        "refinement_roofline": {
            "bound": "alu", "unit": "T ops/s", "ops_per_launch": ops,
            "achieved": round(ops / (ref_ms * 1e-3) / 1e12, 3) if ref_ms > 0 else None,
            "peak": round(PEAK_OPS16 / 1e12, 3),
            "frac": round(ops / (ref_ms * 1e-3) / PEAK_OPS16, 4) if ref_ms > 0 else None},
        "rd_cost_change_pct": round(100.0 * (j_sp - j_int) / j_int, 6)}


def angular_ops(w, h):
    """Algorithmic operations the angular modes add to the leaf kernel: for each of the 33
    modes and every 4x4 tile of every inside node, 16 predicted samples (two products, two
    additions and a shift each) and the tile's SATD."""
    return 33 * inside_tiles(w, h) * (16 * 5 + SATD4_OPS)


def run_angular(mr, torch, frames, jobs_int, args):
    """The 1080p workload with the 33 angular intra modes scored beside planar and DC."""
    QP, R, NP = 27, 64, len(jobs_int)
    jobs_a = [dict(cur=frames[k + 1], ref=frames[k], qp=QP, search_range=R, angular=True)
              for k in range(NP)]
    stream = torch.cuda.current_stream()
    ba = mr.Batch(jobs_a)
    elapsed, pst = timed_launches(mr, torch, lambda: ba.launch(stream), args.steps,
                                  max(1, args.warmup))
    j_int = sum(int(j["out"]["cost"].sum().item()) for j in jobs_int)
    j_a = sum(int(j["out"]["cost"].sum().item()) for j in jobs_a)
    modes = torch.cat([j["out"]["mode"].flatten() for j in jobs_a])
    ang_units = int((modes >= 3).sum().item())
    ms = elapsed * 1e3 / args.steps
    stage = stage_avg(pst)
    ops = (leaf_ops(1920, 1080) + angular_ops(1920, 1080)) * NP
    ctus = jobs_int[0]["out"]["cost"].numel() * NP
    ba.close()
    return {
        "workload": "the 1080p 8 pairs (1920x1080, R 64, QP 27) with the 33 angular intra modes "
                    "(H.265 angular prediction) scored beside planar and DC",
        "ms_per_step": round(ms, 4), "ctus_per_s": round(ctus / (ms * 1e-3), 1),
        "stage_avg_ms": stage,
        "leaf_roofline": {
            "bound": "alu", "unit": "T int16 ops/s", "ops_per_launch": ops,
            "achieved": round(ops / (stage["leaf"] * 1e-3) / 1e12, 3),
            "peak": round(PEAK_OPS16 / 1e12, 3),
            "frac": round(ops / (stage["leaf"] * 1e-3) / PEAK_OPS16, 4)},
        "angular_unit_share": round(ang_units / modes.numel(), 4),
        "rd_cost_change_pct": round(100.0 * (j_a - j_int) / j_int, 6)}


def run_pruned(mr, synth, torch, dev):
    log("rendering 3840x2160 source pair")
    src = synth.Scene(synth.SEED_BASE + 2, 3840, 2160, 24, 96, 8)
    s0, s1 = src.render(0), src.render(1)
    rungs = {}
    for (w, h, n) in [(960, 540, 4), (1920, 1080, 2), (3840, 2160, 1)]:
        rungs[w] = (torch.from_numpy(synth.box_downscale(s0, n, w, h)).to(dev),
                    torch.from_numpy(synth.box_downscale(s1, n, w, h)).to(dev))
    r540, c540 = rungs[960]
    ref_out = mr.mr_ctu_search(c540, r540, 32, 32)
    deps = [(1920, 1080, 27, 64), (3840, 2160, 22, 128)]
    bounds = {w: mr.mr_depth_bounds(ref_out["depth"], 960, 540, w, h, 0, 1)
              for (w, h, _, _) in deps}
    torch.cuda.synchronize()
    seed540 = dict(ref_mv=ref_out["mv"], ref_w=960, ref_h=540, r=REFINE_R)
    variants = (("full", False, False), ("pruned", True, False), ("reuse", True, True))
    res = {f"{v}_ms": 0.0 for v, _, _ in variants}
    res.update({f"J_{v}": 0 for v, _, _ in variants})
    res["per_rung"] = {}
    reps = 3
    for (w, h, qp, rr) in deps:
        ref_t, cur_t = rungs[w]
        times, J = {}, {}
        for name, use_b, use_s in variants:
            o = mr.alloc_outputs(w, h, dev)
            kw = dict(bounds=bounds[w] if use_b else None, seed=seed540 if use_s else None,
                      out=o)
            mr.mr_ctu_search(cur_t, ref_t, qp, rr, **kw)  # warm
            torch.cuda.synchronize()
            ta = time.perf_counter()
            mr.mr_ctu_search(cur_t, ref_t, qp, rr, **kw)
            torch.cuda.synchronize()
            # enough calls for ~10 ms, so that short (seeded) calls are not timer noise
            t1 = time.perf_counter() - ta
            n = max(reps, min(100, int(0.010 / max(t1, 1e-6)) + 1))
            ta = time.perf_counter()
            for _ in range(n):
                mr.mr_ctu_search(cur_t, ref_t, qp, rr, **kw)
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - ta) * 1e3 / n
            J[name] = int(o["cost"].sum().item())
            res[f"{name}_ms"] += times[name]
            res[f"J_{name}"] += J[name]
        res["per_rung"][f"{w}x{h}"] = {
            **{f"{v}_ms": round(times[v], 3) for v, _, _ in variants},
            "speedup": round(times["full"] / times["pruned"], 4),
            "reuse_speedup": round(times["full"] / times["reuse"], 4),
            "rd_cost_increase_pct": round(100.0 * (J["pruned"] - J["full"]) / J["full"], 6),
            "reuse_rd_cost_increase_pct":
                round(100.0 * (J["reuse"] - J["full"]) / J["full"], 6)}
    pct = lambda a: round(100.0 * (res[f"J_{a}"] - res["J_full"]) / res["J_full"], 6)
    pruned = {
        "workload": "3840x2160 source; 960x540 QP32 R32 reference bounds 1920x1080 QP27 R64 "
                    "and 3840x2160 QP22 R128 (depths n..n+1); reuse adds the reference MVs "
                    f"as search centres (refinement r = {REFINE_R})",
        "speedup": round(res["full_ms"] / res["pruned_ms"], 4),
        "rd_cost_increase_pct": pct("pruned"),
        "reuse_speedup": round(res["full_ms"] / res["reuse_ms"], 4),
        "reuse_rd_cost_increase_pct": pct("reuse"),
        "full_ms": round(res["full_ms"], 3), "pruned_ms": round(res["pruned_ms"], 3),
        "reuse_ms": round(res["reuse_ms"], 3), "per_rung": res["per_rung"]}
    # The same figures as time saved, (T_full - T) / T_full in percent: the form in which
    # the thesis reports its encoder-time savings.
    pruned["time_saved_pct"] = round(100.0 * (1.0 - res["pruned_ms"] / res["full_ms"]), 3)
    pruned["reuse_time_saved_pct"] = round(100.0 * (1.0 - res["reuse_ms"] / res["full_ms"]), 3)
    log(f"pruned: {pruned}")

    # Refinement kernel throughput: 3840x2160 seeded (no bounds), every inside CU searched.
    ref_t, cur_t = rungs[3840]
    o = mr.alloc_outputs(3840, 2160, dev)
    seed = dict(ref_mv=ref_out["mv"], ref_w=960, ref_h=540, r=REFINE_R)
    mr.mr_ctu_search(cur_t, ref_t, 22, 128, seed=seed, out=o)
    torch.cuda.synchronize()
    mr.mr_profile_read(reset=True)
    mr.mr_profile_enable(True)
    for _ in range(5):
        mr.mr_ctu_search(cur_t, ref_t, 22, 128, seed=seed, out=o)
    torch.cuda.synchronize()
    stages = mr.mr_profile_read(reset=True)
    mr.mr_profile_enable(False)
    absdiff = inside_tiles(3840, 2160) * 16 * (2 * REFINE_R + 1) ** 2
    st_ms = stages["search"][0] / stages["search"][1]
    pruned["refine"] = {
        "workload": f"3840x2160 QP22 R128 seeded from 960x540 MVs, r = {REFINE_R}, no bounds",
        "stage_ms": {k: round(v[0] / v[1], 4) for k, v in stages.items()},
        "absdiff_per_launch": absdiff,
        "achieved_T_absdiff_s": round(absdiff / (st_ms * 1e-3) / 1e12, 3),
        "frac_of_peak_pad_plus_refine": round(absdiff / (st_ms * 1e-3) / PEAK_ABSDIFF, 4)}
    log(f"refine: {pruned['refine']}")
    return pruned


def run_multi_qp(mr, synth, torch, dev):
    log("multi-QP: 1920x1080 at QPs 22..38, QP 30 master")
    src = synth.Scene(synth.SEED_BASE + 5, 1920, 1080, 24, 48, 4)
    r_t = torch.from_numpy(src.render(0)).to(dev)
    c_t = torch.from_numpy(src.render(1)).to(dev)
    qps, master_qp, R = [22, 26, 30, 34, 38], 30, 64
    deps = [q for q in qps if q != master_qp]
    outs_full = {q: mr.alloc_outputs(1920, 1080, dev) for q in qps}
    outs_re = {q: mr.alloc_outputs(1920, 1080, dev) for q in qps}

    def run_full():
        mr.mr_ctu_search_batch([dict(cur=c_t, ref=r_t, qp=q, search_range=R, out=outs_full[q])
                                for q in qps])

    def run_reuse():
        m = mr.mr_ctu_search(c_t, r_t, master_qp, R, out=outs_re[master_qp])
        b = mr.mr_depth_bounds(m["depth"], 1920, 1080, 1920, 1080, 1, 1)
        seed = dict(ref_mv=m["mv"], ref_w=1920, ref_h=1080, r=MULTI_QP_R)
        mr.mr_ctu_search_batch([dict(cur=c_t, ref=r_t, qp=q, search_range=R, bounds=b,
                                     seed=seed, out=outs_re[q]) for q in deps])

    times = {}
    for name, fn in (("full", run_full), ("reuse", run_reuse)):
        fn()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        # enough calls for ~20 ms, so that the short reuse calls are not timer noise
        n = max(3, min(100, int(0.020 / max(time.perf_counter() - ta, 1e-6)) + 1))
        ta = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - ta) * 1e3 / n
    per_qp = {}
    for q in qps:
        jf = int(outs_full[q]["cost"].sum().item())
        jr = int(outs_re[q]["cost"].sum().item())
        per_qp[str(q)] = round(100.0 * (jr - jf) / jf, 6)
    return {
        "workload": "1920x1080 pair, R 64, QPs 22/26/30/34/38; full: one batch of 5 full "
                    "searches; reuse: QP 30 full search, then QPs 22/26/34/38 in one batch "
                    f"bounded by its depths (d-1..d+1) and seeded by its MVs (r = {MULTI_QP_R})",
        "full_ms": round(times["full"], 3), "reuse_ms": round(times["reuse"], 3),
        "speedup": round(times["full"] / times["reuse"], 4),
        "rd_cost_increase_pct_per_qp": per_qp}


def run_serving(mr, synth, torch, dev, seconds):
    import random
    n_streams, n_content, nfr = 64, 8, 3
    log(f"rendering serving content ({n_content} sources x {nfr} frames, 6 rungs)")
    rungs = [dict(width=w, height=h, qp=qp, search_range=synth.search_range_for_width(w),
                  ref_rung=(-1 if w == 960 else 2)) for (w, h, n, qp) in synth.LADDER]
    names = [f"{w}x{h}" for (w, h, n, qp) in synth.LADDER]
    content = {}
    for c in range(n_content):
        sc = synth.Scene(synth.SEED_BASE + 4 + 1000 * c, 3840, 2160, 24, 96, 8)
        for f in range(nfr):
            img = sc.render(f)
            for r, (w, h, n, qp) in enumerate(synth.LADDER):
                content[(c, f, r)] = torch.from_numpy(synth.box_downscale(img, n, w, h)).to(dev)

    def serve(reuse):
        """One Poisson arrival trace (same seed for both variants) through a ladder server;
        reuse adds the reference MVs as search centres (refinement r = REFINE_R)."""
        kw = dict(refine_range=REFINE_R) if reuse else {}
        lad = mr.Ladder(rungs, delta_lo=0, delta_hi=1, budget_bytes=16 << 30,
                        max_inflight=512, max_queue=1 << 16, max_batch_jobs=64, **kw)
        lat = {r: [] for r in range(len(rungs))}
        try:
            for st in range(n_streams):
                for f in range(nfr):
                    for r in range(len(rungs)):
                        lad.put_frame(st, f, r, content[(st % n_content, f, r)])
            rng = random.Random(synth.SEED_BASE + 4)
            t_next, t0s, t_log = 0.0, time.perf_counter(), 0.0
            while True:
                now = time.perf_counter() - t0s
                while t_next <= now and t_next < seconds:
                    lad.submit(rng.randrange(n_streams), rng.randrange(1, nfr),
                               rng.randrange(len(rungs)))
                    t_next += rng.expovariate(240.0)
                got = lad.poll(256, 200)
                for c in got:
                    if c.status == 0 and not c.implied:
                        lat[c.rung].append((c.t_done_ns - c.t_arrive_ns) * 1e-6)
                lad.release_many([c.job_id for c in got])
                st = lad.stats()
                if now - t_log >= 10.0:
                    t_log = now
                    log(f"serving{' (reuse)' if reuse else ''}: {now:.0f} s, "
                        f"{st['completed']} completed")
                if t_next >= seconds and st["completed"] + st["failed"] >= st["submitted"]:
                    break
                if now > seconds + 60:
                    break
            st = lad.stats()
        finally:
            lad.close()
        per_rung = {}
        for r, v in lat.items():
            v.sort()
            if v:
                per_rung[names[r]] = {"jobs": len(v), "p50_ms": round(pct_of(v, 0.5), 3),
                                      "p99_ms": round(pct_of(v, 0.99), 3)}
        return {"seconds": seconds, "jobs_submitted": st["submitted"] - st["implied"],
                "implied_reference_jobs": st["implied"], "completed": st["completed"],
                "failed": st["failed"], "batches": st["batches"],
                "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                "mean_ms": round(st["mean_ms"], 3), "max_ms": round(st["max_ms"], 3),
                "ctus_per_s": round(st["ctus_per_s"], 1), "per_rung_submitted": per_rung}

    serving = {"workload": "64 streams, 6-rung ladder frames resident, Poisson arrivals mean "
                           "240 jobs/s, rung uniform, 960x540 reference bounds the others "
                           "(depths n..n+1)",
               **serve(False)}
    serving["reuse_mv"] = {"workload": "the same arrivals; dependents also search around the "
                                       f"reference MVs (refinement r = {REFINE_R})",
                           **serve(True)}
    del content
    torch.cuda.synchronize()
    return serving


def run_cpu(synth, host_pair, gpu_outs, single=None):
    """The oracle, as it stands, on the headline workload's stratified sample (every 8th CTU
    of each rung's first pair), compared bit for bit with the GPU's outputs; and on the whole
    first 1920x1080 pair of the single-resolution workload, compared likewise."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(16, threads))  # the CPU share of one GPU on the measurement boxes

    def compare(got, exp, ctus):
        tw = exp["cost"].shape[1]
        for t in ctus:
            cy, cx = (t // tw) * 8, (t % tw) * 8
            for k in ("depth", "mode", "mv"):
                if not np.array_equal(got[k][cy:cy + 8, cx:cx + 8], exp[k][cy:cy + 8, cx:cx + 8]):
                    return False
            for k in ("cost", "dist", "bits"):
                if got[k].ravel()[t] != exp[k].ravel()[t]:
                    return False
        return True

    n_ctus, ok, t_all, per_rung = 0, True, 0.0, {}
    for (w, h, n, qp) in synth.LADDER:
        cur, ref, qp_, R = host_pair[w]
        total = gpu_outs[w]["cost"].size
        ctus = list(range(0, total, 8))
        log(f"CPU oracle: {w}x{h} R {R}, {len(ctus)} of {total} CTUs on {threads} threads")
        ta = time.perf_counter()
        exp = oracle.ctu_search(cur, ref, qp_, R, ctu_list=ctus, n_threads=threads)
        dt = time.perf_counter() - ta
        same = compare(gpu_outs[w], exp, ctus)
        ok = ok and same
        n_ctus += len(ctus)
        t_all += dt
        per_rung[f"{w}x{h}"] = {"ctus": len(ctus), "seconds": round(dt, 3), "bit_exact": same}
    cpu = {"value": round(n_ctus / t_all, 3), "unit": "CTUs/s", "cores": threads,
           "kind": "oracle",
           "sample": f"every 8th CTU (raster order) of the first pair of each of the 6 rungs "
                     f"= {n_ctus} CTUs in the headline's rung mix; {t_all:.1f} s",
           "parity": {"ctus": n_ctus, "bit_exact": ok, "against": "the headline launch's "
                      "outputs of the same pairs", "per_rung": per_rung}}
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), "")
    except OSError:
        pass
    cpu["host"] = {"cpu_model": model, "logical_cpus": os.cpu_count()}
    if single is not None:
        gpu0, (cur0, ref0) = single
        log(f"CPU oracle: whole 1920x1080 pair, R 64, on {threads} threads")
        ta = time.perf_counter()
        exp = oracle.ctu_search(cur0, ref0, 27, 64, n_threads=threads)
        dt = time.perf_counter() - ta
        same = all(np.array_equal(gpu0[k], exp[k]) for k in exp)
        cpu["full_pair_1080p"] = {"ctus": int(exp["cost"].size), "seconds": round(dt, 3),
                                  "ctus_per_s": round(exp["cost"].size / dt, 3),
                                  "bit_exact": bool(same),
                                  "against": "pair 1 of the single_res launch"}
    # The oracle on one thread over the whole small pair (416x240, R 16).
    small = synth.Scene(synth.SEED_BASE + 0, 416, 240, 6, 12, 0)
    s0, s1 = small.render(0), small.render(1)
    ta = time.perf_counter()
    out = oracle.ctu_search(s1, s0, 32, 16, n_threads=1)
    dt1 = time.perf_counter() - ta
    cpu["one_thread_small"] = {"workload": "416x240 pair, R 16, QP 32 (28 CTUs)",
                               "ctus_per_s": round(out["cost"].size / dt1, 3),
                               "seconds": round(dt1, 3)}
    return cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-small-ranges", action="store_true")
    ap.add_argument("--no-pruned", action="store_true")
    ap.add_argument("--no-multi-qp", action="store_true")
    ap.add_argument("--no-subpel", action="store_true")
    ap.add_argument("--no-angular", action="store_true")
    ap.add_argument("--no-dag", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="duration of Poisson arrivals in the serving leg (each of 2 variants)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times) and exit: "
                         "reference for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the coding-tree "
              "search runs on one GPU (sharding jobs or CTU rows over GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2301_12191_amd import mr

    assert torch.cuda.is_available(), "no GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} MiB x 3")
        return
    mr.lib()
    dev = torch.device("cuda:0")

    value, ms_per_step, config, roofline, head_outs, head_host = run_headline(
        mr, synth, torch, dev, args)

    single = subpel = angular = small = small_ranges = pruned = multi_qp = dag = None
    serving = cpu = None
    single_cpu = None
    if not args.no_single:
        single, frames, jobs, gpu0, host0 = run_single_res(mr, synth, torch, dev, args)
        single_cpu = (gpu0, host0)
        log(f"single_res: {single}")
        if not args.no_subpel:
            subpel = run_subpel(mr, torch, frames, jobs, args)
            log(f"subpel: {subpel}")
        if not args.no_angular:
            angular = run_angular(mr, torch, frames, jobs, args)
            log(f"angular: {angular}")
        del frames, jobs
    if not args.no_small:
        small = run_small(mr, synth, torch, dev)
        log(f"small: {small}")
    if not args.no_small_ranges:
        small_ranges = run_small_ranges(mr, synth, torch, dev, args)
        log(f"small_ranges: {small_ranges}")
    if not args.no_pruned:
        pruned = run_pruned(mr, synth, torch, dev)
    if not args.no_multi_qp:
        multi_qp = run_multi_qp(mr, synth, torch, dev)
        log(f"multi-QP: {multi_qp}")
    if not args.no_dag:
        dag = run_dag(mr, synth, torch, dev)
        log(f"dag: {dag}")
    if not args.no_serving:
        serving = run_serving(mr, synth, torch, dev, args.serve_seconds)
        log(f"serving: {serving}")
    if not args.no_cpu:
        cpu = run_cpu(synth, head_host, head_outs, single_cpu)
        log(f"cpu: {cpu}")

    line = {
        "metric": "CTUs/s full vs ref-pruned CU search (bit-exact); p50/p99 frame latency",
        "value": round(value, 1), "unit": "CTUs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": config, "roofline": roofline, "cpu_baseline": cpu, "single_res": single,
        "small": small, "small_ranges": small_ranges, "subpel": subpel, "angular": angular,
        "pruned": pruned,
        "multi_qp": multi_qp, "dag": dag,
        "serving": serving, "thesis_context": THESIS_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
