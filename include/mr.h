/*
 * mr.h -- C ABI of libmr: the per-CTU coding-tree search of multi-resolution
 * encoding (arxiv 2301.12191, "Multi-resolution encoding and optimization for
 * next generation video compression") on AMD Instinct MI355X (gfx950).
 *
 * What the library computes, for one frame pair (current, reference) of 8-bit
 * luma:
 *   - the picture is covered by 64x64 CTUs; each CTU is coded by a quad-tree
 *     of CUs 64, 32, 16, 8 (HEVC background section: CTB sizes and the CU
 *     quad-tree from 64x64 down to 8x8);
 *   - every CU is scored as inter (integer full-search motion estimation,
 *     SAD plus sqrt(lambda) times the MV bits; cost-function subsection, SAD
 *     equation) and as intra DC and planar (HEVC background section), each by
 *     the Hadamard SATD of its residual (cost-function subsection, SATD
 *     equation: sum |H| / 2 over 4x4 Hadamard tiles);
 *   - a bottom-up rate-distortion decision picks the partition and modes
 *     (HEVC background section: RDO over the quad-tree), optionally bounded
 *     per 8x8 unit by depths derived from a reference representation
 *     (related-work section: depth-bound reuse and arbitrary-ratio block
 *     matching; analysis-share appendix: scale factor; analysis-refinement
 *     appendix: refine-intra level 1, depth n and n+1).
 *
 * Integer arithmetic, bit-exact:
 *   s = round(sqrt(lambda) * 65536), lambda = 0.57 * 2^((QP - 12) / 3)
 *   J = D * 65536 + s * R  (int64), D = SATD, R = bits:
 *     inter: 1 + se(4 mx) + se(4 my); planar: 3; DC: 4; split flag: 1 bit
 *     for a node inside the picture with depth < 3.
 *   ME cost: SAD * 65536 + s * (se(4 dx) + se(4 dy)), candidates
 *   dx, dy in [-R, R], reference samples clamped to the picture, first strict
 *   minimum in raster order (dy outer, dx inner).
 *   Pictures whose size is not a multiple of 8 are padded by edge replication
 *   to W8 x H8; CTU nodes crossing that edge are split without a flag.
 *
 * Conventions:
 *   - every function returns an mr_status (0 = MR_OK, negative = error); no
 *     exceptions or aborts cross the ABI;
 *   - argument errors are detected on the host before any launch (MR_EINVAL)
 *     and leave outputs untouched;
 *   - compute calls are asynchronous on the caller's HIP stream (a
 *     hipStream_t passed as void*, NULL = the default stream); outputs are
 *     valid once the caller synchronises that stream;
 *   - all buffers are owned by the caller unless stated otherwise; pointers
 *     marked "device" must be device-accessible memory of the current device.
 */
#ifndef MR_H_
#define MR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MR_OK = 0,
  MR_EINVAL = -1,   /* invalid argument (checked before any launch) */
  MR_ENOMEM = -2,   /* device or host allocation failed */
  MR_EAGAIN = -3,   /* ladder: queue full or memory budget exhausted, retry later */
  MR_EDEPEND = -4,  /* ladder: reference job missing and not implied */
  MR_EHIP = -5,     /* a HIP runtime call failed */
  MR_ETIMEOUT = -6, /* ladder: poll timed out with no completion */
  MR_ESTATE = -7,   /* call not valid in the object's current state */
  MR_ESCRATCH = -8, /* mr_ctu_search_noalloc: the call needs more than its fixed scratch */
  MR_ECANCELED = -9 /* ladder: the job was cancelled before its launch */
} mr_status;

/* One 8-bit luma picture: device pointer, width x height samples, row stride
 * in bytes (stride >= width).  1 <= width, height <= 8192, and
 * stride * (height - 1) + width < 2^31 (samples are addressed with 32-bit
 * offsets); other frames are rejected with MR_EINVAL. */
typedef struct {
  const uint8_t* luma;
  int32_t width, height, stride;
} mr_frame;

/* qp: 0..51.  search_range R: 0..128 (integer-pel, candidates [-R, R]^2).
 * subpel: 0 = integer motion only; 1 = each CU's integer MV is refined to
 * quarter-pel (SATD for quarter-pel ME, cost-function subsection): H.265 8-bit
 * luma fractional interpolation (8-tap / 7-tap filters, 14-bit intermediate,
 * default uni-prediction rounding, reference coordinates clamped), a half-pel
 * stage then a quarter-pel stage, each over the current best and its 8
 * neighbours at the stage's step, J = SATD * 65536 + s * (se(qx) + se(qy))
 * with (qx, qy) in quarter-pel units, the centre keeping ties, then raster
 * order (dy outer).  The leaf's inter candidate is then that MV and SATD, and
 * out.mv holds quarter-pel units.
 * angular: 0 = intra DC and planar only; 1 = also the 33 angular intra modes
 * (HEVC background section: DC, planar and angular modes), H.265 angular
 * prediction from the same substituted neighbours, no reference smoothing and
 * no edge filters, each scored by its SATD with 4 mode bits for vertical
 * (mode 26) and 7 for the others (most-probable-mode list of a block with
 * unavailable neighbours: planar, DC, vertical); ties in the order inter <
 * planar < DC < angular by mode number; out.mode then holds 1 + the H.265
 * mode (3..35) for angular CUs. */
typedef struct {
  int32_t qp;
  int32_t search_range;
  int32_t subpel;
  int32_t angular;
} mr_search_params;

/* Outputs (device, caller-allocated).  With U = ceil(H/8) rows and
 * V = ceil(W/8) columns of 8x8 units, and T = ceil(H/64) x ceil(W/64) CTUs in
 * raster order:
 *   depth[U][V]   u8: depth 0..3 of the CU covering the unit (CU size 64 >> d)
 *   mode[U][V]    u8: 0 inter, 1 planar, 2 DC, 3..35 angular (1 + H.265 mode)
 *   mv[U][V][2]  i16: (mx, my) best integer MV of that CU (also for intra CUs)
 *   ctu_cost[T], ctu_dist[T], ctu_bits[T] i64: J, D and R of each CTU, with
 *     J == D * 65536 + s * R. */
typedef struct {
  uint8_t* depth;
  uint8_t* mode;
  int16_t* mv;
  int64_t* ctu_cost;
  int64_t* ctu_dist;
  int64_t* ctu_bits;
} mr_search_out;

/* Coding-tree search of one frame pair.  cur and ref must have equal width
 * and height.  bounds: NULL for full search, else device [U][V][2] u8
 * {lo, hi} with 0 <= lo <= 3, 0 <= hi <= 3 (as written by mr_depth_bounds):
 * a node at depth d covering units S may stop (be a leaf) iff
 * d >= min_S lo or it may not split, and may split iff d < 3 and
 * d < max_S hi.  Scratch memory is allocated stream-ordered on hip_stream.
 * Errors: MR_EINVAL (null pointers, sizes, qp, R, subpel, angular), MR_ENOMEM,
 * MR_EHIP. */
int mr_ctu_search(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                  const uint8_t* bounds, mr_search_out* out, void* hip_stream);

/* Reference motion vectors for a seeded search (motion-vector reuse with
 * refinement: the x265 refine-mv option of the analysis-refinement appendix,
 * and the reuse of a reference representation's motion vectors at scaled
 * resolutions in the related-work section).
 *   ref_mv: device [ceil(ref_h/8)][ceil(ref_w/8)][2] i16, the mv output of a
 *     search of the same content at ref_w x ref_h (1..8192 each);
 *   refine_range: r, 0 <= r <= search_range.
 * Every CU (n x n at (x0, y0) of a W x H picture) takes the MV (mx, my) of
 * the reference unit co-located with its centre sample:
 *   xr = min(((x0 + n/2) * ref_w) / W, ref_w - 1), yr likewise with heights;
 * scales it to cx = mx * W / ref_w, cy = my * H / ref_h rounded to nearest
 * with halves away from zero, clamps both to [-(R - r), R - r], and searches
 * dx in [cx - r, cx + r], dy in [cy - r, cy + r] with the full search's ME
 * cost and tie order (first minimum in raster order).  MV bits keep the
 * (0, 0) predictor.  r = R is the full search.  The thesis leaves the
 * refinement table empty; this is the library's definition. */
typedef struct {
  const int16_t* ref_mv;
  int32_t ref_w, ref_h;
  int32_t refine_range;
  int32_t quarter_pel; /* 1: ref_mv is in quarter-pel units (written by a search
                          with subpel = 1); the scaled centre divides by 4 more,
                          cx = mx * W / (4 ref_w) rounded as above */
} mr_mv_seed;

/* mr_ctu_search with a seed: NULL seed = mr_ctu_search.  The seed's map is
 * read on the device during the call (stream-ordered).  Scratch of a seeded or
 * sub-pel search includes an edge-padded copy of the reference,
 * (H8 + 2R + 16) x (W8 + 2P) bytes with P = R + 24 rounded up to a multiple
 * of 4.
 * Errors: MR_EINVAL (as mr_ctu_search, plus a null ref_mv, seed sizes,
 * r outside [0, R] or quarter_pel not 0 / 1), MR_ENOMEM, MR_EHIP. */
int mr_ctu_search_seeded(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                         const uint8_t* bounds, const mr_mv_seed* seed, mr_search_out* out,
                         void* hip_stream);

/* Allocation-free variant of mr_ctu_search_seeded, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid allocation): same arguments, checks, results and stream
 * semantics, but every kernel's scratch (job descriptor, queue counters,
 * arg-min key tables, packed CTUs, keys, eligibility, and for seeded or
 * sub-pel searches the padded reference) lives in one file-scope device array
 * of MR_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; the key
 * tables are built on the device in each call.  No hipMalloc, hipFree,
 * stream-ordered allocation or host-to-device copy is made, and stage
 * profiling (mr_profile_enable) does not apply.  The caller still owns the
 * frames, bounds, seed map and outputs.
 * Every call on one GPU shares that GPU's array: calls on one stream run in
 * order, but calls that overlap on one GPU (different streams or host
 * threads without ordering) race and corrupt each other's results.  The
 * array keeps the last call's contents; what must start at zero is cleared
 * by the call's own kernels.
 * Size: under 1 KiB of descriptor and counters; the key tables of a full or
 * bounded search (at most 1.4 MiB, at R 128); per 64x64 CTU about 4.8 KiB
 * (+ 680 bytes with sub-pel); and (H8 + 2R + 16) x (W8 + 2P) bytes for a
 * seeded or sub-pel search (P as for mr_ctu_search_seeded).  A 3840x2160
 * search at R 128 fits with or without sub-pel or seed (23 MB at most);
 * larger requests are refused.
 * Errors: those of mr_ctu_search_seeded (without MR_ENOMEM), and MR_ESCRATCH
 * (before any launch) when the request does not fit the array. */
#define MR_NOALLOC_SCRATCH_BYTES ((uint64_t)24 << 20)
int mr_ctu_search_noalloc(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                          const uint8_t* bounds, const mr_mv_seed* seed, mr_search_out* out,
                          void* hip_stream);

/* One frame pair of a batch (same meaning as the mr_ctu_search_seeded
 * arguments; seed points to host memory and NULL means full search). */
typedef struct {
  mr_frame cur, ref;
  mr_search_params params;
  const uint8_t* bounds; /* device [U][V][2] or NULL */
  mr_search_out out;
  const mr_mv_seed* seed; /* host pointer or NULL */
} mr_search_job;

/* Batched coding-tree search: the CTUs of all jobs (frames of any sizes,
 * ranges and QPs) go through one persistent work-queue search launch fed by a
 * flattened item list ordered longest-first, between one prep and one leaf
 * launch over the flattened CTUs; seeded jobs go through one refinement
 * launch over their CTUs instead of the full search.  Results are identical to calling
 * mr_ctu_search per job.  Host-blocking while it uploads the job list, then
 * asynchronous on hip_stream.  Errors: MR_EINVAL (n_jobs < 1 or any job
 * invalid; nothing is launched), MR_ENOMEM, MR_EHIP. */
int mr_ctu_search_batch(const mr_search_job* jobs, int32_t n_jobs, void* hip_stream);

/* A reusable batch: plans tiles, tables and work items once, owns its device
 * scratch, and records prep -> search -> leaf as a HIP graph that
 * mr_batch_launch replays.  Caller-owned frames, bounds and outputs must stay
 * valid while launches that use them are in flight.
 *   mr_batch_create : plan + allocate + capture (host-blocking).
 *   mr_batch_set_jobs: swap in new frame / bounds / seed / output pointers
 *     for jobs of the same count, sizes, QPs, ranges, bounds presence and
 *     seed presence (else MR_EINVAL); waits for this batch's previous launch
 *     to finish.  Seeds may change their refinement half-width; a new
 *     largest half-width re-records the graph (host-blocking).
 *   mr_batch_launch : replay on hip_stream (with stage profiling enabled, the
 *     three kernels are launched directly between timing events instead).
 *     Launches of one batch share its scratch, so each launch waits on the
 *     device for the batch's previous one, whatever stream either is on.
 *   mr_batch_destroy: waits for the last launch, frees everything (NULL ok).
 * Errors: MR_EINVAL, MR_ENOMEM, MR_EHIP. */
typedef struct mr_batch mr_batch;
int mr_batch_create(const mr_search_job* jobs, int32_t n_jobs, mr_batch** out);
int mr_batch_set_jobs(mr_batch* b, const mr_search_job* jobs, int32_t n_jobs);
int mr_batch_launch(mr_batch* b, void* hip_stream);
int mr_batch_destroy(mr_batch* b);

/* ---------------------------------------------------------------- serving
 * A ladder server: frame-pair jobs of the rungs of an ABR ladder arrive over
 * time (the thesis's multi-encoding schemes: one master representation,
 * dependent tiers bounded by its analysis; concurrent tiers are its future
 * work).  Frames stay resident in device memory (registered with
 * mr_ladder_put_frame, caller-owned).  A job (stream, frame, rung) searches
 * frame `frame` against `frame - 1` of that stream and rung.  A rung with
 * ref_rung >= 0 is a dependent: its depth search is bounded by
 * mr_depth_bounds(delta_lo, delta_hi) of the depth map of the job of the
 * reference rung for the same (stream, frame).  It is launched once that job
 * has been launched, in a later batch that waits for it on the device; if the
 * reference job fails, the dependent fails with MR_EDEPEND.  Submitting
 * a dependent whose reference job does not exist creates it (an implied job)
 * if the reference rung's frames are resident, else fails with MR_EDEPEND.
 * A request loop (one host thread, two device streams of default priority;
 * for 300 us after any activity it polls without sleeping, so it occupies a
 * CPU core while jobs flow and sleeps once they stop) admits ready jobs in arrival order while their device footprint (scratch +
 * outputs + bounds) fits hbm_budget_bytes and fewer than max_inflight jobs
 * run, batches up to max_batch_jobs of them into one persistent search launch,
 * keeps up to four batches in flight, and releases dependents as references
 * are launched (continuous batching).  Done reference jobs stay resident for later
 * dependents until their memory is needed.  The output blocks of finished jobs
 * are kept for reuse by later jobs of the same size, and finished batches'
 * scratch for later batches, outside the admission budget but each capped at
 * a quarter of it (at most 512 MiB; mr_ladder_stats reports them), until
 * mr_ladder_close; a device allocation that fails first
 * empties that cache and retries.  Device memory comes from the server's own
 * stream-ordered pool, which keeps up to hbm_budget_bytes mapped when blocks
 * are freed (destroyed by mr_ladder_close).  With reuse_mv, a dependent's search is
 * also seeded with its reference job's MV map.  Each rung may carry
 * its own policy (own_policy), so that one configuration holds both
 * cross-resolution and same-resolution (multi-QP) edges, e.g. the
 * multi-encoding scheme whose per-resolution median-QP masters chain
 * 540p -> 1080p -> 2160p (proposed multi-encoding section).  Jobs of
 * different frames overlap freely (a dependent of frame t runs beside its
 * master's frame t + 1: frame-delay overlap of tiers, future-work section).
 * Results equal mr_ctu_search_seeded on the same frames (with the same bounds
 * and seed). */
typedef struct {
  int32_t width, height, qp, search_range;
  int32_t ref_rung;   /* index of the rung whose job bounds (and seeds) this one, -1 = none */
  int32_t subpel;     /* quarter-pel refinement of this rung's MVs (mr_search_params) */
  int32_t own_policy; /* 0: the config's delta_lo/delta_hi/reuse_mv/refine_range apply;
                         1: this rung's four fields below (same ranges) */
  int32_t delta_lo, delta_hi;
  int32_t reuse_mv, refine_range;
  int32_t angular;    /* this rung's jobs also score the angular intra modes (mr_search_params) */
} mr_rung;

#define MR_MAX_RUNGS 16

typedef struct {
  int32_t n_rungs;       /* 1..MR_MAX_RUNGS */
  mr_rung rungs[MR_MAX_RUNGS];
  int32_t delta_lo, delta_hi;  /* bound policy of dependents (0..3 each) */
  uint64_t hbm_budget_bytes;   /* admission budget, > 0 */
  int32_t max_inflight;        /* 1..65536 admitted, unfinished jobs */
  int32_t max_queue;           /* 1..1<<20 submitted, unfinished jobs (else MR_EAGAIN) */
  int32_t max_batch_jobs;      /* 1..4096 jobs per device launch */
  int32_t reuse_mv;            /* 0: dependents run the (bounded) full search;
                                  1: dependents are also seeded (mr_mv_seed) with
                                  their reference job's MVs */
  int32_t refine_range;        /* r of seeded dependents, 0..128 (capped at each
                                  rung's search_range); ignored when reuse_mv = 0 */
  int32_t job_timeout_us;      /* >= 0; a job still waiting for its launch this long
                                  after its submission (for its reference, for memory
                                  or for a batch slot) completes with MR_ETIMEOUT and
                                  its dependents with MR_EDEPEND; 0 = no limit.  A
                                  launched job runs to completion (device work is not
                                  interrupted). */
} mr_ladder_config;

typedef struct {
  int32_t stream_id; /* >= 0 */
  int32_t frame_idx; /* >= 1 */
  int32_t rung;
} mr_job;

typedef struct {
  uint64_t job_id;
  int32_t status;    /* MR_OK, or the failure (MR_EDEPEND if its reference failed) */
  int32_t stream_id, frame_idx, rung;
  int32_t implied;   /* 1: created by the server as a reference */
  int32_t n_ctus;
  int64_t t_arrive_ns, t_start_ns, t_done_ns;  /* steady clock */
  mr_search_out out; /* device, owned by the ladder until mr_ladder_release */
} mr_completion;

typedef struct {
  int64_t submitted, implied, completed, failed, rejected, batches, ctus_done;
  double p50_ms, p99_ms, mean_ms, max_ms; /* arrival -> completion of completed jobs */
  double ctus_per_s;                      /* ctus_done / (last done - first start) */
  uint64_t bytes_in_use, peak_bytes;      /* footprint of admitted jobs (the budget's) */
  int64_t cancelled, timed_out;           /* of the failed ones */
  uint64_t cached_bytes;                  /* retired output and scratch blocks kept */
  double host_launch_ms;                  /* server thread's time in batch launches
                                             (plan, allocation, upload, kernel launches) */
  int64_t device_allocs;                  /* device allocations made by the server
                                             (outputs and batch scratch not served from
                                             its caches) */
} mr_ladder_stats;

typedef struct mr_ladder mr_ladder;

/* Errors: MR_EINVAL (config), MR_ENOMEM, MR_EHIP. */
int mr_ladder_open(const mr_ladder_config* cfg, mr_ladder** out);
/* Register a resident frame (device luma of the rung's size, stride >= width).
 * Errors: MR_EINVAL (null, rung or ids out of range). Re-registering replaces. */
int mr_ladder_put_frame(mr_ladder* l, int32_t stream_id, int32_t frame_idx, int32_t rung,
                        const uint8_t* luma, int32_t stride);
/* Forget every registered frame of stream_id with frame_idx < before_frame
 * (all rungs), so that a long-running server's frame table holds the frames
 * still in use; the caller may then reuse or free that memory once the jobs
 * that read those frames have completed.  A job submitted earlier whose frames
 * are dropped before it starts completes with MR_EDEPEND.  Done reference jobs
 * of the stream's frames up to before_frame, which no later dependent can use,
 * stop staying resident: once released their output blocks are freed.
 * Errors: MR_EINVAL (null ladder, negative stream id). */
int mr_ladder_drop_frames(mr_ladder* l, int32_t stream_id, int32_t before_frame);
/* Errors: MR_EINVAL (ids, frames not resident), MR_EDEPEND, MR_EAGAIN (queue
 * full, or the job alone exceeds the budget), MR_ESTATE (closed). */
int mr_ladder_submit(mr_ladder* l, const mr_job* job, uint64_t* job_id);
/* Submits jobs[0..n) in order under one hold of the server's lock, so the
 * scheduler sees them together (a frame's whole ladder, say) rather than as
 * they trickle in one call at a time.  job_ids[i] receives job i's id.  Stops
 * at the first job that mr_ladder_submit would refuse and returns that error;
 * *n_submitted (always written when non-null) counts the jobs accepted before
 * it, which stay submitted.  n = 0 is MR_OK.
 * Errors: MR_EINVAL (null ladder or n_submitted, n < 0, null arrays with
 * n > 0), else those of mr_ladder_submit. */
int mr_ladder_submit_many(mr_ladder* l, const mr_job* jobs, int32_t n, uint64_t* job_ids,
                          int32_t* n_submitted);
/* Up to max completions, waiting up to timeout_us for the first one
 * (0 = do not wait; the first 300 us of a wait spin, the rest sleep).
 * MR_ETIMEOUT if none arrived. */
int mr_ladder_poll(mr_ladder* l, mr_completion* out, int32_t max, int32_t timeout_us,
                   int32_t* n_out);
/* Cancel a job that has not been launched yet (waiting for its reference,
 * for memory or for a batch slot): it completes with MR_ECANCELED, and its
 * dependents fail with MR_EDEPEND.  Errors: MR_EINVAL (null ladder, unknown
 * id), MR_ESTATE (already launched or completed: device work runs to its end). */
int mr_ladder_cancel(mr_ladder* l, uint64_t job_id);
/* Give a completed job's outputs back (MR_ESTATE if not completed yet).  Once
 * a job is released, handed out by mr_ladder_poll and needed by no dependent,
 * the server forgets it (its id then gives MR_EINVAL). */
int mr_ladder_release(mr_ladder* l, uint64_t job_id);
/* mr_ladder_release of ids[0 .. n - 1] under one lock (a client that handles
 * a poll's completions together saves a call per job).  Stops at the first id
 * that fails and returns its status; *n_released = the ids released before it
 * (n_released may be NULL).  Errors: MR_EINVAL (null ids with n > 0, n < 0),
 * then those of mr_ladder_release. */
int mr_ladder_release_many(mr_ladder* l, const uint64_t* ids, int32_t n, int32_t* n_released);
int mr_ladder_get_stats(mr_ladder* l, mr_ladder_stats* out);
/* Waits for in-flight work, frees everything the ladder owns (NULL ok). */
int mr_ladder_close(mr_ladder* l);

/* Depth bounds of a dependent representation (dep_w x dep_h) from the depth
 * map of its reference representation (ref_w x ref_h, as written by
 * mr_ctu_search), for multi-resolution reuse.  For dependent unit (ux, uy):
 *   xr = min(((8 ux + 4) * ref_w) / dep_w, ref_w - 1), yr likewise;
 *   d_r = ref_depth[yr / 8][xr / 8];
 *   d_s = smallest d in 0..3 with (64 >> d) * ref_w <= (64 >> d_r) * dep_w
 *         (3 if none): the co-located CU size scaled to the dependent;
 *   bounds_out[uy][ux] = {max(0, d_s - delta_lo), min(3, d_s + delta_hi)}.
 * delta_lo = 0, delta_hi = 1 evaluates depths n and n+1 (refine-intra level 1
 * of the analysis-refinement appendix); (0, 0) forces the scaled depth;
 * (3, 0) searches only depths <= the co-located one (related-work section).
 * ref_depth: device [ceil(ref_h/8)][ceil(ref_w/8)] u8 (values 0..3);
 * bounds_out: device [ceil(dep_h/8)][ceil(dep_w/8)][2] u8.
 * Errors: MR_EINVAL (null pointers, sizes <= 0 or > 8192, deltas outside 0..3). */
int mr_depth_bounds(const uint8_t* ref_depth, int32_t ref_w, int32_t ref_h, int32_t dep_w,
                    int32_t dep_h, int32_t delta_lo, int32_t delta_hi, uint8_t* bounds_out,
                    void* hip_stream);

/* Tile override for one search range R (an autotuner knob): the search
 * kernel gives each lane 4 horizontal x d vertical candidate shifts (d = 2, 4,
 * 5, 6 or 8) and splits the search window into nbands dy bands (1..8), one
 * workgroup per (CTU, band).  d = 0 removes the override (built-in choice).
 * Results are identical for every setting; only speed changes.
 * Errors: MR_EINVAL (R outside 0..128, d not 0/2/4/5/6/8, nbands outside
 * 1..8). */
int mr_set_tiles(int32_t search_range, int32_t d, int32_t nbands);
/* Same with the strip width (CTUs per workgroup, 1..4; 0 = built-in). */
int mr_set_tiles3(int32_t search_range, int32_t d, int32_t nbands, int32_t strip);
/* Same with the work split: split = 1 gives each wavefront a whole CTU (a
 * workgroup searches a strip of CTUs), split = 2 gives the four wavefronts of
 * a workgroup the four 32x32 quadrants of one CTU (the 64x64 SAD is summed
 * across them in LDS), which spreads small search ranges over four times as
 * many wavefronts; 0 = built-in (split for R <= 64).  nbands 0 = built-in.
 * A batch with split jobs runs strips of 4 for its other jobs.
 * Errors: MR_EINVAL (as mr_set_tiles3, nbands 0..8, split outside 0..2). */
int mr_set_tiles4(int32_t search_range, int32_t d, int32_t nbands, int32_t strip, int32_t split);

/* Autotuner.  Times tile shapes of the search kernel on the given batch (the
 * jobs a later mr_batch_create / mr_ctu_search_batch will run) and installs
 * the fastest as the tile override of the batch's dominant search range (the
 * job with the most candidate work).  Coarse-to-fine: d in {2, 4, 5, 6, 8} x split
 * in {1, 2} (mr_set_tiles4) at the built-in band count, then nbands 1..8 for
 * the best pair, then, for split = 1, strip (CTUs per workgroup) in
 * {1, 2, 3, 4}.  Each shape is run once to warm up and then `reps`
 * times (1..20) with HIP events around the search kernel; the minimum counts.
 * Blocking; overwrites the jobs' outputs.  *out receives the choice.
 * Errors: MR_EINVAL, MR_ENOMEM, MR_EHIP. */
typedef struct {
  int32_t search_range, d, nbands, strip;
  double search_ms;  /* best measured search-kernel time */
  double default_ms; /* time of the built-in choice */
  int32_t tried;     /* shapes measured */
  int32_t split;     /* 1 whole CTU, 2 quadrant per wavefront (mr_set_tiles4) */
} mr_tune_result;
int mr_autotune(const mr_search_job* jobs, int32_t n_jobs, int32_t reps, mr_tune_result* out);

/* Stage timing, a profiling aid for benchmarks.  While enabled, every
 * mr_ctu_search call records HIP events on its stream around its four
 * stages: 0 prep (pack current CTUs, reset keys), 1 search (padded
 * reference, motion search or refinement, arg-min), 2 subpel (quarter-pel
 * refinement; about 0 ms when no job of the call has it), 3 leaf (SATD,
 * intra, quad-tree decision).  mr_profile_read waits for the recorded events,
 * adds their elapsed times (milliseconds) and counts per stage into *out and,
 * if reset != 0, forgets them.
 * Errors: MR_EINVAL (out NULL), MR_EHIP. */
typedef struct {
  double ms[4];
  int64_t launches[4];
} mr_profile;

int mr_profile_enable(int on);
int mr_profile_read(mr_profile* out, int reset);

/* Host helpers (no device work): s = round(sqrt(lambda) * 65536) for qp 0..51
 * (-1 outside), and the length in bits of the signed Exp-Golomb code se(v)
 * (v maps to codeNum 2v-1 for v > 0, -2v otherwise; ue(k) has
 * 2 floor(log2(k+1)) + 1 bits), as used by every cost above. */
int64_t mr_sqrt_lambda_q16(int32_t qp);
int32_t mr_se_bits(int32_t v);

/* Human-readable name of a status code (static string, never NULL). */
const char* mr_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* MR_H_ */
