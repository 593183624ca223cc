// Autotuner of the search kernel's tile shape (vertical shifts per lane D,
// dy bands per CTU, CTUs per workgroup), measured on the caller's batch.
#include <algorithm>
#include <cfloat>
#include <vector>

#include "mr_runtime.h"

using namespace mr;

namespace {

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Search-kernel time (ms, minimum over reps) of the current override for a batch.
int time_search(const mr_search_job* jobs, int n, int reps, double* ms_out) {
  std::vector<const mr_frame*> cur(n), ref(n);
  std::vector<const mr_search_params*> p(n);
  std::vector<const uint8_t*> b(n);
  std::vector<const mr_search_out*> o(n);
  for (int j = 0; j < n; ++j)
    cur[j] = &jobs[j].cur, ref[j] = &jobs[j].ref, p[j] = &jobs[j].params,
    b[j] = jobs[j].bounds, o[j] = &jobs[j].out;
  Plan P;
  int rc = make_plan(cur.data(), ref.data(), p.data(), b.data(), o.data(), nullptr, n, true, &P);
  if (rc != MR_OK) return rc;
  const size_t off_items = up256(sizeof(JobDesc) * n);
  const size_t off_ctr = off_items + up256(sizeof(uint2) * P.items.size());
  const size_t off_scr = off_ctr + 256;
  uint8_t* mem = nullptr;
  if (hipMalloc((void**)&mem, off_scr + P.scratch_bytes) != hipSuccess) return MR_ENOMEM;
  bind_scratch(P, mem + off_scr);
  JobDesc* jobs_d = (JobDesc*)mem;
  const uint2* items_d = (const uint2*)(mem + off_items);
  uint32_t* ctr = (uint32_t*)(mem + off_ctr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = MR_OK;
  if (hipMemcpy(jobs_d, P.jobs.data(), sizeof(JobDesc) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy((void*)items_d, P.items.data(), sizeof(uint2) * P.items.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = MR_EHIP;
  double best = DBL_MAX;
  for (int r = 0; rc == MR_OK && r <= reps; ++r) {
    hipError_t e = launch_prep(jobs_d, n, P.n_ctus, ctr, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess)
      e = launch_search(jobs_d, items_d, P.qoff, P.D, P.strip, P.n_wg, P.lds_bytes, ctr,
                        nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = MR_EHIP;
    if (r > 0) best = std::min(best, (double)ms);  // r == 0 warms up
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(mem);
  *ms_out = best;
  return rc;
}

}  // namespace

extern "C" int mr_autotune(const mr_search_job* jobs, int32_t n_jobs, int32_t reps,
                           mr_tune_result* out) {
  if (!jobs || n_jobs < 1 || !out || reps < 1 || reps > 20) return MR_EINVAL;
  for (int j = 0; j < n_jobs; ++j) {
    const int rc = validate_job(&jobs[j].cur, &jobs[j].ref, &jobs[j].params, &jobs[j].out);
    if (rc != MR_OK) return rc;
  }
  int heavy = 0;
  double hw = -1;
  for (int j = 0; j < n_jobs; ++j) {
    const double r = 2.0 * jobs[j].params.search_range + 1;
    const double w = r * r * (double)jobs[j].cur.width * jobs[j].cur.height;
    if (w > hw) hw = w, heavy = j;
  }
  const int R = jobs[heavy].params.search_range;
  int64_t ctus = 0;
  for (int j = 0; j < n_jobs; ++j)
    if (!jobs[j].seed)
      ctus += (int64_t)(((jobs[j].cur.width + 7) / 8 * 8 + 63) / 64) *
              (((jobs[j].cur.height + 7) / 8 * 8 + 63) / 64);
  const int builtin_D = default_D(R, ctus);
  TileConfig saved{0, 0, 0, 0};
  const bool had = get_tile_override(R, &saved);
  out->search_range = R;
  out->tried = 0;
  // A shape whose window does not fit LDS is skipped (make_plan reports MR_EINVAL).
  auto measure = [&](TileConfig tc, double* ms) {
    int rc = set_tile_override(R, tc);
    if (rc == MR_OK) rc = time_search(jobs, n_jobs, reps, ms);
    if (rc == MR_EINVAL) *ms = DBL_MAX, rc = MR_OK;
    else ++out->tried;
    return rc;
  };
  // Built-in choice first (no override).
  int rc = set_tile_override(R, TileConfig{0, 0, 0, 0});
  double def_ms = DBL_MAX;
  if (rc == MR_OK) rc = time_search(jobs, n_jobs, reps, &def_ms);
  ++out->tried;
  TileConfig best{0, 0, 0, 0};
  double best_ms = def_ms;
  // 1. D x split (whole CTU or quadrant per wavefront) at the built-in bands
  //    (nbands 0 = derive) and strip.
  for (int sp : {1, 2})
    for (int D : {2, 4, 5, 6, 8}) {
      if (rc != MR_OK) break;
      double ms;
      rc = measure(TileConfig{D, 0, 0, sp}, &ms);
      if (rc == MR_OK && ms < best_ms) best_ms = ms, best = TileConfig{D, 0, 0, sp};
    }
  const int bestD = best.D ? best.D : builtin_D;
  const int bestSp = best.D ? best.split : (default_split(R) ? 2 : 1);
  // 2. bands, 3. strip (CTUs per workgroup, whole-CTU wavefronts only).
  for (int nb = 1; rc == MR_OK && nb <= kMaxBands; ++nb) {
    double ms;
    rc = measure(TileConfig{bestD, nb, 0, bestSp}, &ms);
    if (rc == MR_OK && ms < best_ms) best_ms = ms, best = TileConfig{bestD, nb, 0, bestSp};
  }
  for (int sw : {1, 2, 3, 4}) {
    if (rc != MR_OK || !best.D || best.split == 2) break;
    double ms;
    TileConfig tc = best;
    tc.strip = sw;
    rc = measure(tc, &ms);
    if (rc == MR_OK && ms < best_ms) best_ms = ms, best = tc;
  }
  if (rc != MR_OK) {
    (void)set_tile_override(R, had ? saved : TileConfig{0, 0, 0, 0});
    return rc;
  }
  (void)set_tile_override(R, best);
  out->d = best.D ? best.D : builtin_D;
  out->nbands = best.nbands;
  out->strip = best.strip;
  out->split = best.D ? best.split : (default_split(R) ? 2 : 1);
  out->search_ms = best_ms;
  out->default_ms = def_ms;
  return MR_OK;
}
