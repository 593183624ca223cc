// Host-side runtime of libmr: search layouts, key tables, plans of job batches.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mr.h"
#include "mr_internal.h"

namespace mr {

// sqrt(lambda) in Q16 with lambda = 0.57 * 2^((qp - 12) / 3).
int64_t sqrt_lambda_q16(int qp);
// Bits of the signed Exp-Golomb code of v.
int se_bits(int v);

// Tile choice of the search kernel.
struct TileConfig {
  int D;       // vertical shifts per lane (2, 4 or 8)
  int nbands;  // dy bands the window is split into (1..kMaxBands); 0 = derive
  int strip;   // CTUs per workgroup (1..kMaxStrip); 0 = derive
  int split;   // 0 = derive, 1 = a wavefront searches a whole CTU, 2 = its quadrant
};
// Tile override for one search range (autotuner / user knob); D == 0 clears it.
int set_tile_override(int R, const TileConfig& tc);
bool get_tile_override(int R, TileConfig* tc);

SearchLayout make_layout(int R, int D, int nbands);
// Bands for a job: smallest count whose window fits the LDS budget, raised until
// the job alone has at least min_items items (when min_items > 0).
int choose_bands(int R, int D, int strip, int ctus_w, int ctus_h, size_t lds_budget,
                 int min_items, int min_steps_per_band = 2);
// Whether full-search jobs of range R run split (a CTU's quadrants on four
// wavefronts) when nothing overrides it.
bool default_split(int R);
// Vertical shifts per lane when nothing overrides them, for a batch whose
// dominant range is R with `ctus` CTUs of full search.
int default_D(int R, int64_t ctus);
size_t window_bytes(const SearchLayout& L, int strip);

// Device tables of the rank-ordered arg-min keys for (qp, layout); cached per device.
struct KeyTables {
  const uint32_t* qtab;
  const uint64_t* dtab;
};
int get_key_tables(int qp, const SearchLayout& L, KeyTables* out);

int validate_job(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                 const mr_search_out* out);
int validate_seed(const mr_mv_seed* seed, const mr_search_params* p);

// A planned batch: job descriptors (scratch pointers relative to a base until
// bound), the search items in longest-first order, and launch geometry.
struct Plan {
  int D = 4, strip = 4;
  int n_jobs = 0, n_ctus = 0, n_items = 0, n_wg = 0;
  size_t lds_bytes = 0;
  std::vector<JobDesc> jobs;
  std::vector<uint2> items;           // empty when implicit (single job)
  std::vector<size_t> job_off;        // per-job scratch offset
  // Per job, the earlier job of the batch whose packed current CTUs (cur_owner)
  // or padded reference (pad_owner) it shares: same frame, size and stride (and
  // margins), or -1 for its own copy.
  std::vector<int> cur_owner, pad_owner;
  // Per job, the earlier job whose intra SATDs it takes (same current frame,
  // neither angular), or -1; any_shared_intra: some job takes them.
  std::vector<int> intra_owner;
  std::vector<char> intra_owned;  // 1: some job takes this job's intra SATDs
  bool any_shared_intra = false;
  // With shared intra SATDs, the leaf runs twice: over the jobs that take none
  // (llist[0 .. n_ljobs0), n_lctus0 CTUs), then over those that do (the rest of
  // llist, n_lctus1 CTUs); lctu_start numbers each job's CTUs in its launch.
  std::vector<int> llist;
  int n_ljobs0 = 0, n_lctus0 = 0, n_lctus1 = 0;
  size_t scratch_bytes = 0;           // per-job scratch total (curpack, keys, elig, refpad)
  // Seeded jobs (refinement) in rctu_start order, sub-pel jobs in sctu_start
  // order, jobs with a padded reference (seeded or sub-pel).
  std::vector<int> rlist, slist, plist;
  int n_rjobs = 0, n_rctus = 0, max_r = 0;
  int n_sjobs = 0, n_sctus = 0;
  int pad_rows_total = 0;  // rows of all padded references the batch copies
  bool any_angular = false;  // some job scores the angular intra modes
  QueueOffsets qoff{};   // search items of each per-XCD queue
  // Input to make_plan: true leaves the jobs' key tables (qtab, dtab) null
  // for the caller to place and fill, instead of the cached device copies.
  bool defer_tables = false;
};

// Build a plan.  seeds: null, or per job a seed (null entry = full search);
// materialize_items: false only for a single job (the kernel derives items
// from the job).
int make_plan(const mr_frame* const* cur, const mr_frame* const* ref,
              const mr_search_params* const* p, const uint8_t* const* bounds,
              const mr_search_out* const* out, const mr_mv_seed* const* seeds, int n_jobs,
              bool materialize_items, Plan* P);
// Copy a seed's fields into a job descriptor (seed null: full search).
void set_job_seed(JobDesc& jb, const mr_mv_seed* seed);
// Device copies of a plan's job lists (all null for a single job).
struct PlanLists {
  const int* rlist;
  const int* slist;
  const int* plist;
  const int* llist;
};
// Device layout of a planned batch (job array, items, job lists, counter,
// scratch), its upload, and the device job lists inside it.
struct BatchLayout {
  size_t jobs, items, rlist, slist, plist, llist, counter, scratch, total;
};
BatchLayout batch_layout(const Plan& P);
// The host image of [0, bytes) of the layout (bytes at least the end of the
// last list, at most L.counter): descriptors, items, lists, zeros between them.
void batch_image(const Plan& P, const BatchLayout& L, uint8_t* img, size_t bytes);
hipError_t batch_upload(const Plan& P, uint8_t* mem, const BatchLayout& L, hipStream_t st);
PlanLists batch_lists(uint8_t* mem, const BatchLayout& L);
// prep -> [pad] -> [search] -> [refine] -> [subpel] -> leaf for a bound plan.
hipError_t launch_plan(const Plan& P, JobDesc* jobs_d, const uint2* items_d, const PlanLists& L,
                       uint32_t* counter, hipStream_t st, struct StageEvents* ev);
// Point each job's scratch fields into `base` (device memory of P.scratch_bytes).
void bind_scratch(Plan& P, uint8_t* base);

int device_cu_count();
size_t device_lds_max();

// Kernel launches (defined with the kernels).
hipError_t launch_store_job(const JobDesc& jb, JobDesc* dst, hipStream_t st);
hipError_t launch_prep(const JobDesc* jobs, int n_jobs, int n_ctus, uint32_t* counter,
                       hipStream_t st);
hipError_t launch_search(const JobDesc* jobs, const uint2* items, const QueueOffsets& qoff,
                         int D, int strip, int n_wg, size_t lds_bytes, uint32_t* counter,
                         hipStream_t st);
// Leaf over all jobs (llist null), or, with shared intra SATDs, its two launches.
hipError_t launch_leaf(const JobDesc* jobs, int n_jobs, int n_ctus, bool angular,
                       const int* llist, int n_ljobs0, int n_lctus0, int n_lctus1,
                       hipStream_t st);
hipError_t launch_pad(const JobDesc* jobs, const int* plist, int n_pjobs, int total_rows,
                      hipStream_t st);
hipError_t launch_subpel(const JobDesc* jobs, const int* slist, int n_sjobs, int n_sctus,
                         hipStream_t st);
hipError_t launch_refine(const JobDesc* jobs, const int* rlist, int n_rjobs, int n_rctus,
                         int max_r, hipStream_t st);
hipError_t launch_depth_bounds(const uint8_t* ref_depth, int ref_w, int ref_h, int dep_w,
                               int dep_h, int dlo, int dhi, uint8_t* out, hipStream_t st);
// Copy of a host image of at most kUploadMaxBytes (a multiple of 4) to `dst`
// by a kernel that takes it as its argument.
hipError_t launch_upload(const uint8_t* img, size_t bytes, uint8_t* dst, hipStream_t st);
// Depth bounds of several dependents (one launch per kMaxBoundsJobs of them).
hipError_t launch_depth_bounds_batch(const BoundsJob* jobs, int n, hipStream_t st);
int search_occupancy(int D, int strip, size_t lds_bytes);

// Stage profiling (mr_profile_*).
bool profile_on();
struct StageEvents {
  hipEvent_t e[5];  // start, after prep, after search, after sub-pel, after leaf
};
int profile_begin(StageEvents* ev, hipStream_t st);
void profile_mark(StageEvents* ev, int k, hipStream_t st);
void profile_push(const StageEvents& ev);

}  // namespace mr
