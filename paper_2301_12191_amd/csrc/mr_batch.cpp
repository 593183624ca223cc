// Batched coding-tree search: one persistent work-queue search launch over the
// flattened (job, strip, band) items of many frame pairs, and a reusable batch
// object that replays prep -> search -> leaf as a captured HIP graph.
#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#include "mr_runtime.h"

using namespace mr;

struct mr_batch {
  int device = 0;
  Plan plan;
  uint8_t* mem = nullptr;      // device: jobs | items | job lists | counter | scratch
  JobDesc* jobs_d = nullptr;
  uint2* items_d = nullptr;
  PlanLists lists{nullptr, nullptr, nullptr};
  uint32_t* counter_d = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t last = nullptr;   // end of the latest launch
  bool launched = false;
};

namespace {

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Unpacked {
  std::vector<const mr_frame*> cur, ref;
  std::vector<const mr_search_params*> p;
  std::vector<const uint8_t*> bounds;
  std::vector<const mr_search_out*> out;
  std::vector<const mr_mv_seed*> seed;
};

int unpack(const mr_search_job* jobs, int n, Unpacked* u) {
  if (!jobs || n < 1) return MR_EINVAL;
  u->cur.resize(n), u->ref.resize(n), u->p.resize(n), u->bounds.resize(n), u->out.resize(n);
  u->seed.resize(n);
  for (int j = 0; j < n; ++j) {
    u->cur[j] = &jobs[j].cur;
    u->ref[j] = &jobs[j].ref;
    u->p[j] = &jobs[j].params;
    u->bounds[j] = jobs[j].bounds;
    u->out[j] = &jobs[j].out;
    u->seed[j] = jobs[j].seed;
  }
  return MR_OK;
}

}  // namespace

namespace mr {

// Device layout of a planned batch: job array, items, the seeded / sub-pel /
// padded job lists, queue counter, then per-job scratch.
BatchLayout batch_layout(const Plan& P) {
  // Packed at 16 bytes so that the head of most batches fits one upload
  // kernel's arguments; the counters start a 256-byte line.
  auto up16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
  BatchLayout L;
  L.jobs = 0;
  L.items = up16(sizeof(JobDesc) * P.n_jobs);
  L.rlist = L.items + up16(sizeof(uint2) * P.items.size());
  L.slist = L.rlist + up16(sizeof(int) * P.rlist.size());
  L.plist = L.slist + up16(sizeof(int) * P.slist.size());
  L.llist = L.plist + up16(sizeof(int) * P.plist.size());
  L.counter = up256(L.llist + up16(sizeof(int) * P.llist.size()));
  L.scratch = L.counter + kCounterBytes;
  L.total = L.scratch + P.scratch_bytes;
  return L;
}

PlanLists batch_lists(uint8_t* mem, const BatchLayout& L) {
  return PlanLists{(const int*)(mem + L.rlist), (const int*)(mem + L.slist),
                   (const int*)(mem + L.plist), (const int*)(mem + L.llist)};
}

// Upload the job array, items and job lists of a bound plan: one copy of a
// host image of the head of the layout (they are contiguous, from offset 0 to
// the counter).  A copy from pageable memory reads its source before it
// returns, so the image may go out of scope.
void batch_image(const Plan& P, const BatchLayout& L, uint8_t* img, size_t bytes) {
  std::memset(img, 0, bytes);
  std::memcpy(img + L.jobs, P.jobs.data(), sizeof(JobDesc) * P.n_jobs);
  if (!P.items.empty())
    std::memcpy(img + L.items, P.items.data(), sizeof(uint2) * P.items.size());
  const std::pair<const std::vector<int>*, size_t> lists[4] = {
      {&P.rlist, L.rlist}, {&P.slist, L.slist}, {&P.plist, L.plist}, {&P.llist, L.llist}};
  for (const auto& pl : lists)
    if (!pl.first->empty())
      std::memcpy(img + pl.second, pl.first->data(), sizeof(int) * pl.first->size());
}

hipError_t batch_upload(const Plan& P, uint8_t* mem, const BatchLayout& L, hipStream_t st) {
  // The image ends at the counters; of it only [0, end of the last list) is
  // needed (the rest is alignment).
  const size_t used = (L.llist + sizeof(int) * P.llist.size() + 3) & ~(size_t)3;
  if (used <= kUploadMaxBytes) {
    uint8_t img[kUploadMaxBytes];
    batch_image(P, L, img, used);
    return launch_upload(img, used, mem, st);
  }
  std::vector<uint8_t> img(L.counter);
  batch_image(P, L, img.data(), L.counter);
  return hipMemcpyAsync(mem, img.data(), img.size(), hipMemcpyHostToDevice, st);
}

}  // namespace mr

extern "C" {

int mr_ctu_search_batch(const mr_search_job* jobs, int32_t n_jobs, void* hip_stream) {
  Unpacked u;
  int rc = unpack(jobs, n_jobs, &u);
  if (rc != MR_OK) return rc;
  Plan P;
  rc = make_plan(u.cur.data(), u.ref.data(), u.p.data(), u.bounds.data(), u.out.data(),
                 u.seed.data(), n_jobs, true, &P);
  if (rc != MR_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  const BatchLayout L = batch_layout(P);
  uint8_t* mem = nullptr;
  if (hipMallocAsync((void**)&mem, L.total, st) != hipSuccess) return MR_ENOMEM;
  bind_scratch(P, mem + L.scratch);
  hipError_t e = batch_upload(P, mem, L, st);
  StageEvents ev{};
  const bool prof = e == hipSuccess && profile_on() && profile_begin(&ev, st) == MR_OK;
  if (e == hipSuccess)
    e = launch_plan(P, (JobDesc*)(mem + L.jobs), (const uint2*)(mem + L.items),
                    batch_lists(mem, L), (uint32_t*)(mem + L.counter), st,
                    prof ? &ev : nullptr);
  if (prof) profile_push(ev);
  const hipError_t ef = hipFreeAsync(mem, st);
  return (e == hipSuccess && ef == hipSuccess) ? MR_OK : MR_EHIP;
}

// Capture prep -> [pad] -> [search] -> [refine] -> [sub-pel] -> leaf of the
// batch's plan (replacing an earlier graph).  The work-queue head is reset by
// the prep kernel itself, so the graph holds kernel nodes only.
static hipError_t capture(mr_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec), b->exec = nullptr;
  if (b->graph) (void)hipGraphDestroy(b->graph), b->graph = nullptr;
  hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t el = launch_plan(b->plan, b->jobs_d, b->items_d, b->lists, b->counter_d,
                                      b->cap_stream, nullptr);
    e = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (el != hipSuccess) e = el;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  return e;
}

int mr_batch_destroy(mr_batch* b) {
  if (!b) return MR_OK;
  int rc = MR_OK;
  if (b->last && b->launched && hipEventSynchronize(b->last) != hipSuccess) rc = MR_EHIP;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->last) (void)hipEventDestroy(b->last);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
  return rc;
}

int mr_batch_create(const mr_search_job* jobs, int32_t n_jobs, mr_batch** out) {
  if (!out) return MR_EINVAL;
  *out = nullptr;
  Unpacked u;
  int rc = unpack(jobs, n_jobs, &u);
  if (rc != MR_OK) return rc;
  mr_batch* b = new mr_batch();
  (void)hipGetDevice(&b->device);
  rc = make_plan(u.cur.data(), u.ref.data(), u.p.data(), u.bounds.data(), u.out.data(),
                 u.seed.data(), n_jobs, true, &b->plan);
  if (rc != MR_OK) {
    delete b;
    return rc;
  }
  const BatchLayout L = batch_layout(b->plan);
  if (hipMalloc((void**)&b->mem, L.total) != hipSuccess) {
    mr_batch_destroy(b);
    return MR_ENOMEM;
  }
  b->jobs_d = (JobDesc*)(b->mem + L.jobs);
  b->items_d = (uint2*)(b->mem + L.items);
  b->lists = batch_lists(b->mem, L);
  b->counter_d = (uint32_t*)(b->mem + L.counter);
  bind_scratch(b->plan, b->mem + L.scratch);
  if (batch_upload(b->plan, b->mem, L, nullptr) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess ||
      hipEventCreateWithFlags(&b->last, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    mr_batch_destroy(b);
    return MR_EHIP;
  }
  if (capture(b) != hipSuccess) {
    mr_batch_destroy(b);
    return MR_EHIP;
  }
  *out = b;
  return MR_OK;
}

int mr_batch_set_jobs(mr_batch* b, const mr_search_job* jobs, int32_t n_jobs) {
  if (!b || !jobs || n_jobs != b->plan.n_jobs) return MR_EINVAL;
  for (int j = 0; j < n_jobs; ++j) {
    const JobDesc& jd = b->plan.jobs[j];
    const mr_search_job& q = jobs[j];
    int rc = validate_job(&q.cur, &q.ref, &q.params, &q.out);
    if (rc == MR_OK) rc = validate_seed(q.seed, &q.params);
    if (rc != MR_OK) return rc;
    if (q.cur.width != jd.w || q.cur.height != jd.h || q.params.search_range != jd.R ||
        sqrt_lambda_q16(q.params.qp) != jd.s || (q.bounds != nullptr) != (jd.bounds != nullptr) ||
        (q.seed != nullptr) != (jd.seed_mv != nullptr) || q.params.subpel != jd.subpel ||
        q.params.angular != jd.angular)
      return MR_EINVAL;
  }
  if (b->launched && hipEventSynchronize(b->last) != hipSuccess) return MR_EHIP;
  for (int j = 0; j < n_jobs; ++j) {
    JobDesc& jd = b->plan.jobs[j];
    const mr_search_job& q = jobs[j];
    jd.cur = q.cur.luma;
    jd.ref = q.ref.luma;
    jd.stride = q.cur.stride;
    jd.bounds = q.bounds;
    jd.depth = q.out.depth;
    jd.mode = q.out.mode;
    jd.mv = q.out.mv;
    jd.ctu_cost = q.out.ctu_cost;
    jd.ctu_dist = q.out.ctu_dist;
    jd.ctu_bits = q.out.ctu_bits;
    set_job_seed(jd, q.seed);
  }
  if (hipMemcpy(b->jobs_d, b->plan.jobs.data(), sizeof(JobDesc) * n_jobs,
                hipMemcpyHostToDevice) != hipSuccess)
    return MR_EHIP;
  // The refinement grid follows the largest refinement half-width: a new one
  // needs a new graph.
  int max_r = 0;
  for (int j = 0; j < n_jobs; ++j)
    if (jobs[j].seed) max_r = std::max(max_r, jobs[j].seed->refine_range);
  if (max_r != b->plan.max_r) {
    b->plan.max_r = max_r;
    if (capture(b) != hipSuccess) return MR_EHIP;
  }
  return MR_OK;
}

int mr_batch_launch(mr_batch* b, void* hip_stream) {
  if (!b) return MR_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e;
  // Every launch of a batch uses the batch's one scratch (packed CTUs, keys,
  // queue counters): a launch on another stream than the previous one waits
  // for it on the device instead of overlapping it.
  if (b->launched && hipStreamWaitEvent(st, b->last, 0) != hipSuccess) return MR_EHIP;
  if (profile_on()) {
    StageEvents ev{};
    if (profile_begin(&ev, st) != MR_OK) return MR_EHIP;
    e = launch_plan(b->plan, b->jobs_d, b->items_d, b->lists, b->counter_d, st, &ev);
    profile_push(ev);
  } else {
    e = hipGraphLaunch(b->exec, st);
  }
  if (e == hipSuccess) e = hipEventRecord(b->last, st);
  if (e != hipSuccess) return MR_EHIP;
  b->launched = true;
  return MR_OK;
}

}  // extern "C"
