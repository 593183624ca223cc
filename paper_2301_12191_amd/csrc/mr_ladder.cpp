// Ladder server (mr_ladder_*): the GPU executor of the serving scheduler and
// its request-loop thread.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <sys/prctl.h>
#include <thread>
#include <tuple>
#include <vector>

#include "mr_runtime.h"
#include "mr_sched.h"

using namespace mr;

namespace {

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct FrameRef {
  const uint8_t* luma;
  int stride;
};

// A batch's completion event, shared by the batch and its jobs' outputs.  A
// later batch may wait for it on the device (its jobs' references); it is
// destroyed with the last of them, after the reference outputs are freed, so
// after every dependent batch, and so every wait on it, has completed.
// The event goes back to its executor's pool (it has completed by then)
// instead of being destroyed: creating one costs tens of microseconds.
struct SharedEvent {
  hipEvent_t ev = nullptr;
  int refs = 0;
  std::vector<hipEvent_t>* pool = nullptr;
};
static void unref(SharedEvent* e) {
  if (e && --e->refs == 0) {
    if (e->pool) e->pool->push_back(e->ev);
    else (void)hipEventDestroy(e->ev);
    delete e;
  }
}

struct JobOut {
  uint8_t* mem = nullptr;  // one allocation: outputs then bounds
  size_t bytes = 0;
  mr_search_out out{};
  uint8_t* bounds = nullptr;
  hipStream_t stream = nullptr;   // stream that wrote it
  SharedEvent* batch = nullptr;   // its batch's completion event
  bool batch_running = false;     // that batch not yet retired
};

struct BatchState {
  SharedEvent* done = nullptr;
  hipStream_t stream = nullptr;
  uint8_t* scratch = nullptr;  // the batch's device scratch (back to the cache when done)
  size_t scratch_bytes = 0;
};

class GpuExecutor : public Executor {
 public:
  explicit GpuExecutor(const SchedConfig& cfg)
      : cfg_(cfg), pool_max_(std::min<size_t>(kPoolMaxBytes, cfg.budget_bytes / 4)) {}

  int init() {
    if (hipGetDevice(&device_) != hipSuccess) return MR_EHIP;
    for (auto& s : streams_)
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return MR_EHIP;
    // The server's own stream-ordered pool, which keeps the memory it has
    // mapped (up to the budget) when blocks are freed.  The device's default
    // pool returns freed memory at every synchronisation, and mapping a large
    // block anew takes ~150 us, inside a launch on the serving path.
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device_;
    if (hipMemPoolCreate(&mp_, &props) != hipSuccess) {
      mp_ = nullptr;
      return MR_EHIP;
    }
    uint64_t keep = cfg_.budget_bytes;
    if (hipMemPoolSetAttribute(mp_, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess)
      return MR_EHIP;
    return MR_OK;
  }

  ~GpuExecutor() override {
    // Cached blocks came from the stream-ordered allocator: free them the same way.
    if (streams_[0]) {
      for (auto& kv : pool_) (void)hipFreeAsync(kv.second, streams_[0]);
      for (auto& kv : scratch_free_) (void)hipFreeAsync(kv.second, streams_[0]);
    }
    for (auto& s : streams_)
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    for (hipEvent_t ev : events_) (void)hipEventDestroy(ev);
    // Every block has been freed and its stream synchronised (the ladder frees
    // the jobs' outputs before it deletes the executor).
    if (mp_) (void)hipMemPoolDestroy(mp_);
  }

  int device() const { return device_; }

  int64_t now_ns() override {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
  }

  void put_frame(int stream, int frame, int rung, const uint8_t* luma, int stride) {
    std::lock_guard<std::mutex> lk(mu_);
    frames_[std::make_tuple(stream, frame, rung)] = FrameRef{luma, stride};
  }

  // Forget the frames of `stream` before `before_frame` (every rung).
  void drop_frames(int stream, int before_frame) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = frames_.lower_bound(std::make_tuple(stream, 0, 0));
    while (it != frames_.end() && std::get<0>(it->first) == stream &&
           std::get<1>(it->first) < before_frame)
      it = frames_.erase(it);
  }

  bool frames_resident(int stream, int frame, int rung) override {
    std::lock_guard<std::mutex> lk(mu_);
    return frames_.count(std::make_tuple(stream, frame, rung)) &&
           frames_.count(std::make_tuple(stream, frame - 1, rung));
  }

  static size_t out_bytes(const RungCfg& r, bool bounded, size_t* off) {
    const size_t U = (r.height + 7) / 8, V = (r.width + 7) / 8;
    const size_t T = ((U * 8 + 63) / 64) * ((V * 8 + 63) / 64);
    size_t o = 0;
    off[0] = o, o += up256(U * V);          // depth
    off[1] = o, o += up256(U * V);          // mode
    off[2] = o, o += up256(U * V * 4);      // mv
    off[3] = o, o += up256(T * 8);          // cost
    off[4] = o, o += up256(T * 8);          // dist
    off[5] = o, o += up256(T * 8);          // bits
    off[6] = o, o += bounded ? up256(U * V * 2) : 0;
    return o;
  }

  // Refinement half-width of a rung's jobs, -1 for the full search.
  static int refine_of(const RungCfg& r) {
    return (r.refine >= 0 && r.ref_rung >= 0) ? std::min(r.refine, r.search_range) : -1;
  }

  size_t footprint(const SchedJob& j) override {
    const RungCfg& r = cfg_.rungs[j.rung];
    size_t off[7];
    const size_t w8 = (r.width + 7) / 8 * 8, h8 = (r.height + 7) / 8 * 8;
    const size_t T = ((h8 + 63) / 64) * ((w8 + 63) / 64);
    size_t pad = 0;  // padded reference of a seeded or sub-pel search, sub-pel results
    if (refine_of(r) >= 0 || r.subpel)
      pad = (h8 + 2 * (size_t)refine_pad_y(r.search_range)) *
                (w8 + 2 * (size_t)refine_pad_x(r.search_range)) + 256;
    if (r.subpel) pad += T * kNodes * 8 + 256;
    return out_bytes(r, r.ref_rung >= 0, off) + T * (4096 + 85 * 9) + pad + 4096;
  }

  int launch(const std::vector<SchedJob*>& jobs, void** handle) override {
    const int n = (int)jobs.size();
    // References whose batches still run (chain_on_launch): this batch goes on
    // the stream of the first of them, where the order is given; it waits for
    // the others on the device.  A batch without running references takes the
    // streams in turn.  (A wait between streams adds about 10 us between the
    // reference's last kernel and the dependent's first.)
    hipStream_t st = nullptr;
    {
      std::vector<const JobOut*> running;
      for (SchedJob* j : jobs) {
        if (!j->ref_job) continue;
        const JobOut* ro = (const JobOut*)ref_state_(j->ref_job);
        if (!ro) return MR_EDEPEND;
        if (ro->batch && ro->batch_running) running.push_back(ro);
      }
      st = running.empty() ? streams_[next_++ & 1] : running.front()->stream;
      std::vector<hipEvent_t> waits;
      for (const JobOut* ro : running)
        if (ro->stream != st && std::find(waits.begin(), waits.end(), ro->batch->ev) == waits.end())
          waits.push_back(ro->batch->ev);
      for (hipEvent_t ev : waits)
        if (hipStreamWaitEvent(st, ev, 0) != hipSuccess) return MR_EHIP;
    }
    std::vector<mr_frame> cur(n), ref(n);
    std::vector<mr_search_params> prm(n);
    std::vector<const uint8_t*> bnd(n, nullptr);
    std::vector<mr_search_out> outs(n);
    std::vector<mr_mv_seed> seeds(n);
    std::vector<const mr_mv_seed*> ps(n, nullptr);
    std::vector<BoundsJob> bjobs;  // the dependents' depth bounds, one launch
    for (int i = 0; i < n; ++i) {
      SchedJob& j = *jobs[i];
      const RungCfg& r = cfg_.rungs[j.rung];
      FrameRef fc, fr;
      {
        // The scheduler admits only jobs whose frames are resident; a frame
        // dropped since then fails the batch instead of being read.
        std::lock_guard<std::mutex> lk(mu_);
        auto ic = frames_.find(std::make_tuple(j.stream, j.frame, j.rung));
        auto ir = frames_.find(std::make_tuple(j.stream, j.frame - 1, j.rung));
        if (ic == frames_.end() || ir == frames_.end()) return MR_EDEPEND;
        fc = ic->second, fr = ir->second;
      }
      cur[i] = mr_frame{fc.luma, r.width, r.height, fc.stride};
      ref[i] = mr_frame{fr.luma, r.width, r.height, fr.stride};
      prm[i] = mr_search_params{r.qp, r.search_range, r.subpel, r.angular};
      JobOut* o = new JobOut();
      size_t off[7];
      const size_t bytes = out_bytes(r, j.ref_job != 0, off);
      o->mem = take_block(bytes);
      if (!o->mem && !alloc(&o->mem, bytes, st)) {
        delete o;
        return MR_ENOMEM;
      }
      o->bytes = bytes;
      o->stream = st;
      o->out = mr_search_out{o->mem + off[0], o->mem + off[1], (int16_t*)(o->mem + off[2]),
                             (int64_t*)(o->mem + off[3]), (int64_t*)(o->mem + off[4]),
                             (int64_t*)(o->mem + off[5])};
      j.exec_state = o;
      const int U = (r.height + 7) / 8, V = (r.width + 7) / 8;
      j.n_ctus = ((U * 8 + 63) / 64) * ((V * 8 + 63) / 64);
      if (j.ref_job) {
        o->bounds = o->mem + off[6];
        const RungCfg& rr = cfg_.rungs[r.ref_rung];
        const JobOut* ro = (const JobOut*)ref_state_(j.ref_job);
        if (!ro) return MR_EDEPEND;
        bjobs.push_back(BoundsJob{ro->out.depth, o->bounds, rr.width, rr.height, r.width,
                                  r.height, r.dlo, r.dhi});
        bnd[i] = o->bounds;
        const int rr_refine = refine_of(r);
        if (rr_refine >= 0) {
          seeds[i] = mr_mv_seed{ro->out.mv, rr.width, rr.height, rr_refine, rr.subpel};
          ps[i] = &seeds[i];
        }
      }
      outs[i] = o->out;
    }
    if (!bjobs.empty() &&
        launch_depth_bounds_batch(bjobs.data(), (int)bjobs.size(), st) != hipSuccess)
      return MR_EHIP;
    std::vector<const mr_frame*> pc(n), pr(n);
    std::vector<const mr_search_params*> pp(n);
    std::vector<const mr_search_out*> po(n);
    for (int i = 0; i < n; ++i) pc[i] = &cur[i], pr[i] = &ref[i], pp[i] = &prm[i], po[i] = &outs[i];
    // A batch of one job leaves its search items implicit (the kernel derives
    // them from the job): less to plan and a smaller upload.
    Plan P;
    int rc = make_plan(pc.data(), pr.data(), pp.data(), bnd.data(), po.data(), ps.data(), n, n > 1,
                       &P);
    if (rc != MR_OK) return rc;
    const BatchLayout L = batch_layout(P);
    size_t mem_bytes = 0;
    uint8_t* mem = take_scratch(L.total, &mem_bytes);
    if (!mem) {
      // Sizes rounded up to 1 MiB so that later batches of similar size reuse it.
      mem_bytes = (L.total + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
      if (!alloc(&mem, mem_bytes, st)) return MR_ENOMEM;
    }
    bind_scratch(P, mem + L.scratch);
    hipError_t e = batch_upload(P, mem, L, st);
    if (e == hipSuccess)
      e = launch_plan(P, (JobDesc*)(mem + L.jobs),
                      P.items.empty() ? nullptr : (const uint2*)(mem + L.items),
                      batch_lists(mem, L), (uint32_t*)(mem + L.counter), st, nullptr);
    hipEvent_t ev = nullptr;
    if (!events_.empty()) {
      ev = events_.back();
      events_.pop_back();
    } else if (e == hipSuccess) {
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e != hipSuccess) {
      if (ev) (void)hipEventDestroy(ev);
      (void)hipFreeAsync(mem, st);
      return MR_EHIP;
    }
    BatchState* b = new BatchState();
    b->stream = st;
    b->scratch = mem;
    b->scratch_bytes = mem_bytes;
    b->done = new SharedEvent{ev, 1 + n, &events_};
    for (SchedJob* j : jobs) {
      JobOut* o = (JobOut*)j->exec_state;
      o->batch = b->done;
      o->batch_running = true;
    }
    *handle = b;
    return MR_OK;
  }

  int query(void* handle) override {
    const hipError_t e = hipEventQuery(((BatchState*)handle)->done->ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return -1;
  }

  void finish(void* handle, const std::vector<SchedJob*>& jobs) override {
    BatchState* b = (BatchState*)handle;
    for (SchedJob* j : jobs)
      if (j->exec_state) ((JobOut*)j->exec_state)->batch_running = false;
    // The batch has finished on the device: its scratch may serve the next one.
    if (scratch_free_bytes_ + b->scratch_bytes <= pool_max_) {
      scratch_free_.emplace(b->scratch_bytes, b->scratch);
      scratch_free_bytes_ += b->scratch_bytes;
    } else {
      (void)hipFreeAsync(b->scratch, b->stream);
    }
    unref(b->done);
    delete b;
    for (SchedJob* j : jobs) j->status = MR_OK;
  }

  // A job that succeeded and whose batch has retired is freed only once every
  // dependent has completed, so no work in flight reads its block: the block
  // goes to a per-size cache for later jobs (a serving loop allocates the same
  // few sizes over and over) instead of back to the allocator.  Other blocks
  // are freed in the order of the stream that wrote them.
  void free_job(SchedJob& j) override {
    JobOut* o = (JobOut*)j.exec_state;
    if (!o) return;
    if (j.state == kDone && !o->batch_running &&
        pool_bytes_ + o->bytes <= pool_max_) {
      pool_.emplace(o->bytes, o->mem);
      pool_bytes_ += o->bytes;
    } else {
      (void)hipFreeAsync(o->mem, o->stream);
    }
    unref(o->batch);
    delete o;
  }

  // Lookup of a job's executor state through the scheduler (set by the ladder).
  std::function<void*(uint64_t)> ref_state_;

  void sync() {
    for (auto& s : streams_) (void)hipStreamSynchronize(s);
  }

  size_t cached_bytes() const { return pool_bytes_ + scratch_free_bytes_; }
  int64_t device_allocs() const { return allocs_; }

 private:
  SchedConfig cfg_;
  // Stream-ordered allocation; when it fails, the cached output blocks go back
  // to the allocator (in the order of `st`, so a retry on `st` may reuse them)
  // and it is tried once more.
  bool alloc(uint8_t** p, size_t bytes, hipStream_t st) {
    ++allocs_;
    if (hipMallocFromPoolAsync((void**)p, bytes, mp_, st) == hipSuccess) return true;
    (void)hipGetLastError();
    if (pool_.empty() && scratch_free_.empty()) return false;
    for (auto& kv : pool_) (void)hipFreeAsync(kv.second, st);
    for (auto& kv : scratch_free_) (void)hipFreeAsync(kv.second, st);
    pool_.clear();
    scratch_free_.clear();
    pool_bytes_ = scratch_free_bytes_ = 0;
    return hipMallocFromPoolAsync((void**)p, bytes, mp_, st) == hipSuccess;
  }
  // A cached scratch block of at least `bytes` (and at most twice that), or null.
  uint8_t* take_scratch(size_t bytes, size_t* got) {
    auto it = scratch_free_.lower_bound(bytes);
    if (it == scratch_free_.end() || it->first > 2 * bytes + ((size_t)1 << 20)) return nullptr;
    uint8_t* m = it->second;
    *got = it->first;
    scratch_free_bytes_ -= it->first;
    scratch_free_.erase(it);
    return m;
  }
  // A cached block of exactly `bytes`, or null.
  uint8_t* take_block(size_t bytes) {
    auto it = pool_.find(bytes);
    if (it == pool_.end()) return nullptr;
    uint8_t* m = it->second;
    pool_.erase(it);
    pool_bytes_ -= bytes;
    return m;
  }

  hipMemPool_t mp_ = nullptr;
  static constexpr size_t kPoolMaxBytes = size_t(512) << 20;
  std::multimap<size_t, uint8_t*> pool_;  // retired output blocks by size
  // Cap of each cache (outputs, scratch): a quarter of the budget, <= 512 MiB.
  // Separate caps, so that a pipelined run's large batch scratch does not
  // crowd the outputs of its many jobs out of theirs.
  size_t pool_max_ = 0;
  size_t pool_bytes_ = 0;
  std::multimap<size_t, uint8_t*> scratch_free_;  // scratch of finished batches by size
  size_t scratch_free_bytes_ = 0;
  std::vector<hipEvent_t> events_;                // completed batch events for reuse
  int64_t allocs_ = 0;                            // calls of alloc()
  int device_ = 0;
  hipStream_t streams_[2] = {nullptr, nullptr};
  unsigned next_ = 0;
  std::mutex mu_;
  std::map<std::tuple<int, int, int>, FrameRef> frames_;
};

}  // namespace

struct mr_ladder {
  SchedConfig cfg;
  std::unique_ptr<GpuExecutor> ex;
  std::unique_ptr<Scheduler> sched;
  std::mutex mu;                 // guards sched
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  std::atomic<bool> stop{false};
  bool closed = false;
  // Raised (under mu) by every call that may give the loop work (submissions,
  // cancels, releases) and by the loop when it publishes completions: the
  // spinning loop and pollers watch them without the lock.
  std::atomic<uint64_t> work_seq{0}, done_seq{0};
};

// After any activity (a launch, a completion, a call that may give work) the
// loop polls without sleeping for this long, and a poll call spins this long
// for a completion before it blocks: a sleeping thread takes 10-20 us to wake,
// which at a frame boundary (client sees the last completion, submits the next
// frame, the loop launches it) is paid twice with the device idle.  Beyond the
// window the loop sleeps in 5 us steps while batches run, 5 ms when idle.
constexpr auto kSpinWindow = std::chrono::microseconds(300);

static void ladder_loop(mr_ladder* l) {
  (void)hipSetDevice(l->ex->device());
  // With Linux's default 50 us timer slack each 5 us wait would last ten times
  // that; 1 us of slack for this thread.
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  using clock = std::chrono::steady_clock;
  std::unique_lock<std::mutex> lk(l->mu);
  clock::time_point last_active = clock::now();
  while (!l->stop.load()) {
    const uint64_t seen = l->work_seq.load(std::memory_order_acquire);
    const int before = l->sched->batches_in_flight();
    const int done = l->sched->step();
    if (done) {
      l->done_seq.fetch_add(1, std::memory_order_release);
      l->cv_done.notify_all();
    }
    const bool idle = l->sched->idle();
    if (done || l->sched->batches_in_flight() != before) last_active = clock::now();
    if (clock::now() - last_active < kSpinWindow) {
      // Poll without sleeping, the lock released: until new work arrives, and
      // while batches run for at most 2 us before the next step.
      lk.unlock();
      const clock::time_point until = clock::now() + std::chrono::microseconds(2);
      while (!l->stop.load(std::memory_order_relaxed) &&
             l->work_seq.load(std::memory_order_acquire) == seen) {
        const clock::time_point t = clock::now();
        if ((!idle && t >= until) || t - last_active >= kSpinWindow) break;
        std::this_thread::yield();
      }
      lk.lock();
    } else {
      l->cv_work.wait_for(lk, idle ? std::chrono::microseconds(5000) : std::chrono::microseconds(5),
                          [&] { return l->stop.load() || l->work_seq.load() != seen; });
    }
    if (l->work_seq.load(std::memory_order_acquire) != seen) last_active = clock::now();
  }
  // Drain: wait for batches in flight so their outputs are complete.
  while (l->sched->batches_in_flight() > 0) {
    l->sched->step();
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::microseconds(50));
    lk.lock();
  }
  l->cv_done.notify_all();
}

extern "C" {

int mr_ladder_open(const mr_ladder_config* cfg, mr_ladder** out) {
  if (!out) return MR_EINVAL;
  *out = nullptr;
  auto policy_ok = [](int dlo, int dhi, int reuse, int refine) {
    return dlo >= 0 && dlo <= 3 && dhi >= 0 && dhi <= 3 && reuse >= 0 && reuse <= 1 &&
           (!reuse || (refine >= 0 && refine <= 128));
  };
  if (!cfg || cfg->n_rungs < 1 || cfg->n_rungs > MR_MAX_RUNGS ||
      !policy_ok(cfg->delta_lo, cfg->delta_hi, cfg->reuse_mv, cfg->refine_range) ||
      cfg->hbm_budget_bytes == 0 ||
      cfg->max_inflight < 1 || cfg->max_inflight > 65536 || cfg->max_queue < 1 ||
      cfg->max_queue > (1 << 20) || cfg->max_batch_jobs < 1 || cfg->max_batch_jobs > 4096 ||
      cfg->job_timeout_us < 0)
    return MR_EINVAL;
  SchedConfig sc;
  for (int r = 0; r < cfg->n_rungs; ++r) {
    const mr_rung& g = cfg->rungs[r];
    if (g.width < 1 || g.height < 1 || g.width > 8192 || g.height > 8192 || g.qp < 0 ||
        g.qp > 51 || g.search_range < 0 || g.search_range > 128 || g.ref_rung < -1 ||
        g.ref_rung >= cfg->n_rungs || g.ref_rung == r || g.own_policy < 0 || g.own_policy > 1 ||
        (g.own_policy && !policy_ok(g.delta_lo, g.delta_hi, g.reuse_mv, g.refine_range)))
      return MR_EINVAL;
    if (g.subpel < 0 || g.subpel > 1 || g.angular < 0 || g.angular > 1) return MR_EINVAL;
    RungCfg rc{g.width, g.height, g.qp, g.search_range, g.ref_rung};
    rc.subpel = g.subpel;
    rc.angular = g.angular;
    const bool own = g.own_policy != 0;
    rc.dlo = own ? g.delta_lo : cfg->delta_lo;
    rc.dhi = own ? g.delta_hi : cfg->delta_hi;
    const int reuse = own ? g.reuse_mv : cfg->reuse_mv;
    rc.refine = reuse ? (own ? g.refine_range : cfg->refine_range) : -1;
    sc.rungs.push_back(rc);
  }
  // Reference chains must end (no cycles).
  for (int r = 0; r < cfg->n_rungs; ++r) {
    int x = r, hops = 0;
    while (x >= 0 && hops <= cfg->n_rungs) x = sc.rungs[x].ref_rung, ++hops;
    if (x >= 0) return MR_EINVAL;
  }
  sc.budget_bytes = cfg->hbm_budget_bytes;
  sc.max_inflight = cfg->max_inflight;
  sc.max_queue = cfg->max_queue;
  sc.max_batch_jobs = cfg->max_batch_jobs;
  sc.job_timeout_ns = (int64_t)cfg->job_timeout_us * 1000;
  sc.chain_on_launch = true;  // dependents wait for their references on the device
  sc.max_batches_in_flight = 4;  // a reference chain of up to 4 levels in flight
  mr_ladder* l = new mr_ladder();
  l->cfg = sc;
  l->ex.reset(new GpuExecutor(sc));
  if (l->ex->init() != MR_OK) {
    delete l;
    return MR_EHIP;
  }
  l->sched.reset(new Scheduler(sc, l->ex.get()));
  Scheduler* s = l->sched.get();
  l->ex->ref_state_ = [s](uint64_t id) -> void* {
    const SchedJob* j = s->job(id);
    return j ? j->exec_state : nullptr;
  };
  l->worker = std::thread(ladder_loop, l);
  *out = l;
  return MR_OK;
}

int mr_ladder_put_frame(mr_ladder* l, int32_t stream_id, int32_t frame_idx, int32_t rung,
                        const uint8_t* luma, int32_t stride) {
  if (!l || !luma || stream_id < 0 || frame_idx < 0 || rung < 0 ||
      rung >= (int)l->cfg.rungs.size() || stride < l->cfg.rungs[rung].width)
    return MR_EINVAL;
  l->ex->put_frame(stream_id, frame_idx, rung, luma, stride);
  return MR_OK;
}

int mr_ladder_drop_frames(mr_ladder* l, int32_t stream_id, int32_t before_frame) {
  if (!l || stream_id < 0) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);  // not between the scheduler's check and a launch
  l->ex->drop_frames(stream_id, before_frame);
  l->sched->frames_dropped(stream_id, before_frame);  // their resident references are freed
  l->work_seq.fetch_add(1, std::memory_order_release);
  return MR_OK;
}

int mr_ladder_submit(mr_ladder* l, const mr_job* job, uint64_t* job_id) {
  if (!l || !job) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);
  if (l->closed) return MR_ESTATE;
  const int rc = l->sched->submit(job->stream_id, job->frame_idx, job->rung, job_id);
  if (rc == MR_OK) {
    l->work_seq.fetch_add(1, std::memory_order_release);
    l->cv_work.notify_all();
  }
  return rc;
}

int mr_ladder_submit_many(mr_ladder* l, const mr_job* jobs, int32_t n, uint64_t* job_ids,
                          int32_t* n_submitted) {
  if (n_submitted) *n_submitted = 0;
  if (!l || n < 0 || !n_submitted || (n > 0 && (!jobs || !job_ids))) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);
  if (l->closed) return MR_ESTATE;
  int rc = MR_OK;
  for (int32_t i = 0; i < n && rc == MR_OK; ++i) {
    rc = l->sched->submit(jobs[i].stream_id, jobs[i].frame_idx, jobs[i].rung, &job_ids[i]);
    if (rc == MR_OK) ++*n_submitted;
  }
  if (*n_submitted > 0) {
    l->work_seq.fetch_add(1, std::memory_order_release);
    l->cv_work.notify_all();
  }
  return rc;
}

int mr_ladder_poll(mr_ladder* l, mr_completion* out, int32_t max, int32_t timeout_us,
                   int32_t* n_out) {
  if (!l || !out || max < 1 || timeout_us < 0 || !n_out) return MR_EINVAL;
  *n_out = 0;
  std::unique_lock<std::mutex> lk(l->mu);
  std::vector<uint64_t> ids = l->sched->take_completions(max);
  if (ids.empty() && timeout_us > 0) {
    using clock = std::chrono::steady_clock;
    const clock::time_point until = clock::now() + std::chrono::microseconds(timeout_us);
    // Spin first, the lock released, for a completion published within the
    // spin window (done_seq is read under the lock, after the empty take).
    const clock::time_point spin_until = std::min(until, clock::now() + kSpinWindow);
    while (ids.empty() && clock::now() < spin_until) {
      const uint64_t seen = l->done_seq.load(std::memory_order_acquire);
      lk.unlock();
      while (l->done_seq.load(std::memory_order_acquire) == seen && clock::now() < spin_until)
        std::this_thread::yield();
      lk.lock();
      ids = l->sched->take_completions(max);
    }
    while (ids.empty() && clock::now() < until) {
      l->cv_done.wait_until(lk, until);
      ids = l->sched->take_completions(max);
    }
  }
  if (ids.empty()) return MR_ETIMEOUT;
  for (size_t i = 0; i < ids.size(); ++i) {
    const SchedJob* j = l->sched->job(ids[i]);
    mr_completion& c = out[i];
    std::memset(&c, 0, sizeof(c));
    c.job_id = j->id;
    c.status = j->status;
    c.stream_id = j->stream, c.frame_idx = j->frame, c.rung = j->rung;
    c.implied = j->implied ? 1 : 0;
    c.n_ctus = j->n_ctus;
    c.t_arrive_ns = j->t_arrive, c.t_start_ns = j->t_start, c.t_done_ns = j->t_done;
    if (j->exec_state) c.out = ((JobOut*)j->exec_state)->out;
  }
  *n_out = (int32_t)ids.size();
  return MR_OK;
}

int mr_ladder_cancel(mr_ladder* l, uint64_t job_id) {
  if (!l) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);
  const int rc = l->sched->cancel(job_id);
  if (rc == MR_OK) {
    l->done_seq.fetch_add(1, std::memory_order_release);
    l->work_seq.fetch_add(1, std::memory_order_release);  // its budget may admit others
    l->cv_done.notify_all();
  }
  return rc;
}

int mr_ladder_release(mr_ladder* l, uint64_t job_id) {
  if (!l) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);
  const int rc = l->sched->release(job_id);
  if (rc == MR_OK) l->work_seq.fetch_add(1, std::memory_order_release);  // freed budget
  return rc;
}

int mr_ladder_release_many(mr_ladder* l, const uint64_t* ids, int32_t n, int32_t* n_released) {
  if (n_released) *n_released = 0;
  if (!l || n < 0 || (n > 0 && !ids)) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);
  int rc = MR_OK;
  int32_t i = 0;
  for (; i < n && rc == MR_OK; ++i) {
    rc = l->sched->release(ids[i]);
    if (rc == MR_OK && n_released) *n_released = i + 1;
  }
  if (n > 0) l->work_seq.fetch_add(1, std::memory_order_release);  // freed budget
  return rc;
}

int mr_ladder_get_stats(mr_ladder* l, mr_ladder_stats* out) {
  if (!l || !out) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(l->mu);
  const SchedStats s = l->sched->stats();
  std::memset(out, 0, sizeof(*out));
  out->submitted = s.submitted, out->implied = s.implied, out->completed = s.completed;
  out->failed = s.failed, out->rejected = s.rejected, out->batches = s.batches;
  out->ctus_done = s.ctus_done;
  out->p50_ms = s.p50_ms, out->p99_ms = s.p99_ms, out->mean_ms = s.mean_ms, out->max_ms = s.max_ms;
  const double span = (s.last_done_ns - s.first_start_ns) * 1e-9;
  out->ctus_per_s = span > 0 ? s.ctus_done / span : 0.0;
  out->bytes_in_use = s.bytes_in_use, out->peak_bytes = s.peak_bytes;
  out->cancelled = s.cancelled, out->timed_out = s.timed_out;
  out->cached_bytes = l->ex->cached_bytes();
  out->device_allocs = l->ex->device_allocs();
  out->host_launch_ms = s.host_launch_ns * 1e-6;
  return MR_OK;
}

int mr_ladder_close(mr_ladder* l) {
  if (!l) return MR_OK;
  {
    std::lock_guard<std::mutex> lk(l->mu);
    l->closed = true;
  }
  l->stop.store(true);
  l->cv_work.notify_all();
  if (l->worker.joinable()) l->worker.join();
  l->ex->sync();
  // Free every job's outputs still held.
  {
    std::lock_guard<std::mutex> lk(l->mu);
    l->sched->free_all();
  }
  l->ex->sync();
  delete l;
  return MR_OK;
}

}  // extern "C"
