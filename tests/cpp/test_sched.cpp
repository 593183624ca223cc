// CPU test of the serving scheduler's state machine with a fake executor:
// dependencies and implied references, footprint admission, queue limits,
// failure propagation, resident references and eviction, continuous batching,
// latency statistics.  Exit code 0 = all checks passed.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "mr.h"
#include "mr_sched.h"

using namespace mr;

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

struct FakeBatch {
  int64_t done_at;
  bool fail;
};

struct FakeExec : Executor {
  int64_t t = 0;                       // fake clock (ns), advanced by the test
  int64_t batch_ns = 1000000;          // every batch takes 1 ms
  std::vector<int64_t> next_ns;        // durations of the next launches (then batch_ns)
  std::set<std::tuple<int, int, int>> frames;
  std::map<int, size_t> fp;            // per-rung footprint
  std::vector<std::vector<uint64_t>> launched;
  int freed = 0;
  bool fail_next = false;
  std::set<FakeBatch*> live;
  ~FakeExec() override {
    for (FakeBatch* b : live) delete b;
  }
  int64_t now_ns() override { return t; }
  size_t footprint(const SchedJob& j) override { return fp[j.rung]; }
  bool frames_resident(int s, int f, int r) override {
    return frames.count(std::make_tuple(s, f, r)) && frames.count(std::make_tuple(s, f - 1, r));
  }
  int launch(const std::vector<SchedJob*>& jobs, void** h) override {
    std::vector<uint64_t> ids;
    for (SchedJob* j : jobs) {
      ids.push_back(j->id);
      j->exec_state = (void*)1;
      j->n_ctus = 10;
    }
    launched.push_back(ids);
    int64_t ns = batch_ns;
    if (!next_ns.empty()) ns = next_ns.front(), next_ns.erase(next_ns.begin());
    FakeBatch* fb = new FakeBatch{t + ns, fail_next};
    live.insert(fb);
    *h = fb;
    fail_next = false;
    return MR_OK;
  }
  int query(void* h) override {
    FakeBatch* b = (FakeBatch*)h;
    if (t < b->done_at) return 0;
    return b->fail ? -1 : 1;
  }
  void finish(void* h, const std::vector<SchedJob*>& jobs) override {
    live.erase((FakeBatch*)h);
    delete (FakeBatch*)h;
    for (SchedJob* j : jobs) j->status = MR_OK;
  }
  void free_job(SchedJob& j) override {
    ++freed;
    j.exec_state = nullptr;
  }
};

static SchedConfig ladder_cfg(uint64_t budget) {
  SchedConfig c;
  // rung 0: 960x540 root; rungs 1, 2 depend on it
  c.rungs = {{960, 540, 32, 32, -1}, {1920, 1080, 27, 64, 0}, {3840, 2160, 22, 128, 0}};
  c.budget_bytes = budget;
  c.max_inflight = 64;
  c.max_queue = 16;
  c.max_batch_jobs = 8;
  return c;
}

static void add_frames(FakeExec& ex, int stream, int nframes, int rungs) {
  for (int f = 0; f < nframes; ++f)
    for (int r = 0; r < rungs; ++r) ex.frames.insert(std::make_tuple(stream, f, r));
}

static void run_until_idle(Scheduler& s, FakeExec& ex, int max_steps = 1000) {
  for (int i = 0; i < max_steps && !s.idle(); ++i) {
    s.step();
    ex.t += 100000;  // 0.1 ms per loop iteration
  }
}

static void test_dependency_and_implied_reference() {
  FakeExec ex;
  ex.fp = {{0, 100}, {1, 400}, {2, 1600}};
  add_frames(ex, 0, 3, 3);
  Scheduler s(ladder_cfg(1 << 20), &ex);
  uint64_t d = 0;
  CHECK(s.submit(0, 1, 1, &d) == MR_OK);  // dependent first: implies rung-0 job
  CHECK(s.stats().implied == 1 && s.stats().submitted == 2);
  const SchedJob* dj = s.job(d);
  CHECK(dj && dj->ref_job != 0 && dj->state == kQueued);
  const SchedJob* rj = s.job(dj->ref_job);
  CHECK(rj && rj->implied && rj->rung == 0 && rj->state == kReady);
  s.step();
  CHECK(ex.launched.size() == 1 && ex.launched[0].size() == 1 && ex.launched[0][0] == rj->id);
  ex.t += 2000000;
  s.step();  // reference completes; dependent becomes ready and launches
  CHECK(rj->state == kDone);
  CHECK(ex.launched.size() == 2 && ex.launched[1][0] == d);
  run_until_idle(s, ex);
  CHECK(dj->state == kDone && dj->t_start >= rj->t_done);
  // a second dependent of the same (stream, frame) reuses the resident reference
  uint64_t d2 = 0;
  CHECK(s.submit(0, 1, 2, &d2) == MR_OK);
  CHECK(s.job(d2)->ref_job == rj->id && s.job(d2)->state == kReady);
  CHECK(s.stats().implied == 1);
}

static void test_missing_reference_frames() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  ex.frames = {{0, 0, 1}, {0, 1, 1}};  // only rung-1 frames
  Scheduler s(ladder_cfg(1000), &ex);
  uint64_t id = 7;
  CHECK(s.submit(0, 1, 1, &id) == MR_EDEPEND && id == 0);
  CHECK(s.submit(0, 5, 1, &id) == MR_EINVAL);   // frames not resident
  CHECK(s.submit(-1, 1, 0, &id) == MR_EINVAL);
  CHECK(s.submit(0, 0, 0, &id) == MR_EINVAL);   // frame 0 has no predecessor
  CHECK(s.submit(0, 1, 3, &id) == MR_EINVAL);
}

static void test_budget_admission_and_rejection() {
  FakeExec ex;
  ex.fp = {{0, 600}, {1, 400}, {2, 5000}};
  add_frames(ex, 0, 4, 3);
  add_frames(ex, 1, 4, 3);
  Scheduler s(ladder_cfg(1000), &ex);
  uint64_t a, b, c;
  CHECK(s.submit(0, 1, 0, &a) == MR_OK);
  CHECK(s.submit(1, 1, 0, &b) == MR_OK);
  CHECK(s.submit(0, 2, 2, &c) == MR_EAGAIN);  // 5000 bytes can never fit 1000
  CHECK(s.stats().rejected == 1);
  s.step();
  // only one 600-byte job fits at a time
  CHECK(ex.launched.size() == 1 && ex.launched[0].size() == 1 && ex.launched[0][0] == a);
  CHECK(s.stats().bytes_in_use == 600);
  ex.t += 2000000;
  s.step();
  // a is done but not released: b still cannot fit (600 + 600 > 1000)
  CHECK(ex.launched.size() == 1);
  CHECK(s.release(a) == MR_OK);
  // a is a reference rung with no pending dependents: it stays resident until
  // b needs the memory, then it is evicted
  s.step();
  CHECK(ex.launched.size() == 2 && ex.launched[1][0] == b);
  CHECK(ex.freed == 1 && s.stats().bytes_in_use == 600);
  CHECK(s.release(b + 100) == MR_EINVAL);
  CHECK(s.release(b) == MR_ESTATE);  // still running
}

static void test_queue_limit() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  SchedConfig cfg = ladder_cfg(1 << 20);
  cfg.max_queue = 3;
  for (int st = 0; st < 5; ++st) add_frames(ex, st, 2, 3);
  Scheduler s(cfg, &ex);
  uint64_t id;
  for (int st = 0; st < 3; ++st) CHECK(s.submit(st, 1, 0, &id) == MR_OK);
  CHECK(s.submit(4, 1, 0, &id) == MR_EAGAIN);
  run_until_idle(s, ex);
  CHECK(s.submit(4, 1, 0, &id) == MR_OK);  // room again once jobs completed
}

static void test_reference_failure_fails_dependents() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 2, 3);
  Scheduler s(ladder_cfg(1 << 20), &ex);
  uint64_t d1, d2;
  CHECK(s.submit(0, 1, 1, &d1) == MR_OK);
  CHECK(s.submit(0, 1, 2, &d2) == MR_OK);
  CHECK(s.stats().implied == 1);  // both dependents share the one implied reference
  ex.fail_next = true;  // the reference batch fails
  run_until_idle(s, ex);
  const SchedJob* r = s.job(s.job(d1)->ref_job);
  CHECK(r->state == kFailed && r->status == MR_EHIP);
  CHECK(s.job(d1)->state == kFailed && s.job(d1)->status == MR_EDEPEND);
  CHECK(s.job(d2)->state == kFailed && s.job(d2)->status == MR_EDEPEND);
  if (!(s.stats().failed == 3 && s.stats().completed == 0))
    std::fprintf(stderr, "failed=%lld completed=%lld\n", (long long)s.stats().failed,
                 (long long)s.stats().completed);
  CHECK(s.stats().failed == 3 && s.stats().completed == 0);
  CHECK(ex.launched.size() == 1);
}

static void test_continuous_batching_and_latency() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  for (int st = 0; st < 8; ++st) add_frames(ex, st, 2, 3);
  SchedConfig cfg = ladder_cfg(1 << 20);
  cfg.max_batch_jobs = 4;
  cfg.max_batches_in_flight = 2;
  cfg.max_queue = 64;
  Scheduler s(cfg, &ex);
  uint64_t id;
  for (int st = 0; st < 3; ++st) CHECK(s.submit(st, 1, 0, &id) == MR_OK);
  s.step();  // batch 1 (3 jobs) on the device
  for (int st = 3; st < 8; ++st) CHECK(s.submit(st, 1, 0, &id) == MR_OK);
  s.step();  // arrivals during batch 1 form batch 2 while batch 1 runs
  CHECK(ex.launched.size() == 2 && ex.launched[0].size() == 3 && ex.launched[1].size() == 4);
  CHECK(s.batches_in_flight() == 2);
  CHECK(s.submit(0, 1, 1, &id) == MR_OK);  // dependent of stream 0's reference
  s.step();
  CHECK(ex.launched.size() == 2);  // at most 2 batches in flight
  run_until_idle(s, ex);
  // after batch 1: stream 7's job and the (now ready) dependent share batch 3
  CHECK(ex.launched.size() == 3 && ex.launched[2].size() == 2);
  const SchedStats st = s.stats();
  CHECK(st.completed == 9 && st.ctus_done == 90 && st.batches == 3);
  CHECK(st.p50_ms > 0.9 && st.p99_ms >= st.p50_ms && st.max_ms >= st.p99_ms);
  std::vector<uint64_t> c = s.take_completions(100);
  CHECK(c.size() == 9);
  CHECK(s.take_completions(100).empty());
}

static void test_finished_jobs_are_forgotten() {
  // A long run: jobs are submitted, completed, handed out and released over and
  // over; the scheduler's tables must hold only live jobs (no growth with time).
  // Released reference jobs stay resident (for later dependents) until
  // admission needs their memory: a budget of 10 jobs bounds them.
  FakeExec ex;
  ex.fp = {{0, 100}, {1, 100}, {2, 100}};
  SchedConfig cfg = ladder_cfg(1000);
  cfg.max_queue = 64;
  Scheduler s(cfg, &ex);
  size_t most = 0;
  for (int f = 1; f <= 200; ++f) {
    add_frames(ex, 0, f + 1, 3);
    uint64_t a, b;
    CHECK(s.submit(0, f, 1, &a) == MR_OK);  // implies the rung-0 reference
    CHECK(s.submit(0, f, 2, &b) == MR_OK);
    run_until_idle(s, ex);
    for (uint64_t id : s.take_completions(100)) CHECK(s.release(id) == MR_OK);
    s.step();
    most = std::max(most, s.jobs_known());
  }
  // at most the resident references the budget holds, plus the frame in flight
  CHECK(most <= 12);
  CHECK(s.stats().bytes_in_use <= 1000);
  CHECK(s.stats().completed == 600 && s.stats().implied == 200);
  // a forgotten job's id is unknown
  CHECK(s.job(1) == nullptr && s.release(1) == MR_EINVAL);
  // the references still resident are freed by free_all
  const int before = ex.freed;
  s.free_all();
  CHECK(ex.freed > before);
}

// A released reference of a stream's frame is freed once a job of its rung
// kKeepFrames frames later is done, without budget pressure; a dependent of
// that frame submitted afterwards gets a new (implied) reference, one of the
// last kKeepFrames frames still finds its reference.
static void test_superseded_references_freed() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 6, 3);
  Scheduler s(ladder_cfg(1 << 20), &ex);
  for (int f = 1; f <= 5; ++f) {
    uint64_t a = 0;
    CHECK(s.submit(0, f, 0, &a) == MR_OK);
    run_until_idle(s, ex);
    for (uint64_t id : s.take_completions(100)) CHECK(s.release(id) == MR_OK);
    s.step();
    // the references of the last kKeepFrames frames stay resident, earlier ones are freed
    CHECK(ex.freed == std::max(0, f - kKeepFrames));
    CHECK((int)s.jobs_known() == std::min(f, kKeepFrames));
  }
  uint64_t d = 0;
  CHECK(s.submit(0, 2, 1, &d) == MR_OK);  // frame 2's reference is gone: implied again
  CHECK(s.stats().implied == 1 && s.job(s.job(d)->ref_job)->implied);
  run_until_idle(s, ex);
  CHECK(s.job(d)->state == kDone && s.job(d)->status == MR_OK);
  // the frame-4 and frame-5 references are still resident: their dependents reuse them
  uint64_t d4 = 0, d5 = 0;
  CHECK(s.submit(0, 4, 2, &d4) == MR_OK);
  CHECK(s.submit(0, 5, 2, &d5) == MR_OK);
  CHECK(s.stats().implied == 1 && !s.job(s.job(d4)->ref_job)->implied &&
        !s.job(s.job(d5)->ref_job)->implied);
}

static void test_dropped_frames_fail_alone() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 3, 3);
  add_frames(ex, 1, 3, 3);
  Scheduler s(ladder_cfg(1 << 20), &ex);
  uint64_t a, b;
  CHECK(s.submit(0, 2, 0, &a) == MR_OK);
  CHECK(s.submit(1, 2, 0, &b) == MR_OK);
  // stream 0's frames go away before the jobs are admitted
  for (int r = 0; r < 3; ++r) ex.frames.erase(std::make_tuple(0, 1, r));
  run_until_idle(s, ex);
  CHECK(s.job(a)->state == kFailed && s.job(a)->status == MR_EDEPEND);
  CHECK(s.job(b)->state == kDone);
  CHECK(ex.launched.size() == 1 && ex.launched[0].size() == 1 && ex.launched[0][0] == b);
  CHECK(s.submit(0, 2, 0, &a) == MR_EINVAL);  // not resident any more
}

// Dropping a stream's frames frees its resident references that no later
// dependent can use (frames up to the drop point), and only those.
static void test_dropped_frames_free_references() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 5, 3);
  Scheduler s(ladder_cfg(1 << 20), &ex);
  for (int f = 3; f <= 4; ++f) {
    uint64_t a = 0;
    CHECK(s.submit(0, f, 0, &a) == MR_OK);
    run_until_idle(s, ex);
    for (uint64_t id : s.take_completions(100)) CHECK(s.release(id) == MR_OK);
    s.step();
  }
  CHECK(ex.freed == 0 && s.jobs_known() == 2);  // both references resident
  s.frames_dropped(0, 3);  // frames 0..2 go: frame 3's reference can serve nobody
  s.step();
  CHECK(ex.freed == 1 && s.jobs_known() == 1);
  uint64_t d = 0;
  CHECK(s.submit(0, 4, 1, &d) == MR_OK);  // frame 4's reference still serves
  CHECK(s.stats().implied == 0);
  run_until_idle(s, ex);
  CHECK(s.job(d)->state == kDone && s.job(d)->status == MR_OK);
}

// chain_on_launch: a dependent launches in the batch after its reference's,
// in the same step, while that batch still runs; a reference that then fails
// takes the already-launched dependent with it.
static void test_chain_on_launch() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 3, 3);
  SchedConfig cfg = ladder_cfg(1 << 20);
  cfg.chain_on_launch = true;
  {
    Scheduler s(cfg, &ex);
    uint64_t d = 0;
    CHECK(s.submit(0, 1, 1, &d) == MR_OK);  // implies the rung-0 reference
    const SchedJob* dj = s.job(d);
    const SchedJob* rj = s.job(dj->ref_job);
    s.step();  // the reference launches, and the dependent behind it in its own batch
    CHECK(ex.launched.size() == 2 && ex.launched[0][0] == rj->id && rj->state == kRunning);
    CHECK(ex.launched[1].size() == 1 && ex.launched[1][0] == d);
    CHECK(rj->state == kRunning && dj->state == kRunning);
    run_until_idle(s, ex);
    CHECK(rj->state == kDone && dj->state == kDone && dj->status == MR_OK);
    CHECK(s.stats().completed == 2 && s.stats().failed == 0);
  }
  {
    ex.launched.clear();
    Scheduler s(cfg, &ex);
    uint64_t d = 0;
    CHECK(s.submit(0, 2, 1, &d) == MR_OK);
    const SchedJob* dj = s.job(d);
    const SchedJob* rj = s.job(dj->ref_job);
    ex.fail_next = true;  // the reference batch fails when it completes
    s.step();
    ex.t += 100000;
    s.step();
    CHECK(ex.launched.size() == 2 && dj->state == kRunning);
    run_until_idle(s, ex);
    CHECK(rj->state == kFailed && rj->status == MR_EHIP);
    CHECK(dj->state == kFailed && dj->status == MR_EDEPEND);
    CHECK(s.stats().failed == 2 && s.stats().completed == 0);
  }
  {
    // A dependent made ready by its running reference but not yet admitted
    // (no batch slot) fails without a launch when the reference fails.
    ex.launched.clear();
    SchedConfig c1 = cfg;
    c1.max_batches_in_flight = 1;
    Scheduler s(c1, &ex);
    uint64_t d = 0;
    CHECK(s.submit(0, 2, 2, &d) == MR_OK);
    const SchedJob* dj = s.job(d);
    ex.fail_next = true;
    s.step();  // reference launches and takes the only batch slot
    ex.t += 100000;
    s.step();
    CHECK(ex.launched.size() == 1 && dj->state == kReady);
    run_until_idle(s, ex);
    CHECK(dj->state == kFailed && dj->status == MR_EDEPEND && ex.launched.size() == 1);
  }
}

// A dependent's batch that finishes before its reference's batch is not
// retired first: the reference's failure still reaches it.
static void test_dependent_batch_done_first() {
  FakeExec ex;
  ex.fp = {{0, 1}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 3, 3);
  SchedConfig cfg = ladder_cfg(1 << 20);
  cfg.chain_on_launch = true;
  Scheduler s(cfg, &ex);
  uint64_t d = 0;
  CHECK(s.submit(0, 1, 1, &d) == MR_OK);
  const SchedJob* dj = s.job(d);
  const SchedJob* rj = s.job(dj->ref_job);
  ex.next_ns = {3000000, 500000};  // reference batch 3 ms, dependent batch 0.5 ms
  ex.fail_next = true;             // and the reference batch fails
  s.step();                        // reference launches
  ex.t += 100000;
  s.step();                        // dependent launches behind it
  CHECK(ex.launched.size() == 2 && dj->state == kRunning);
  ex.t += 1000000;                 // the dependent's batch reports done, the reference's not
  s.step();
  CHECK(dj->state == kRunning && rj->state == kRunning);
  CHECK(s.stats().completed == 0 && s.stats().failed == 0);
  run_until_idle(s, ex);
  CHECK(rj->state == kFailed && rj->status == MR_EHIP);
  CHECK(dj->state == kFailed && dj->status == MR_EDEPEND);
  // An independent batch that finishes early is not held back.
  ex.launched.clear();
  Scheduler s2(cfg, &ex);
  uint64_t a = 0, b = 0;
  add_frames(ex, 1, 3, 3);
  ex.next_ns = {3000000, 500000};
  CHECK(s2.submit(0, 1, 0, &a) == MR_OK);
  s2.step();
  ex.t += 100000;
  CHECK(s2.submit(1, 1, 0, &b) == MR_OK);
  s2.step();
  ex.t += 1000000;
  s2.step();
  CHECK(s2.job(b)->state == kDone && s2.job(a)->state == kRunning);
  run_until_idle(s2, ex);
}

static void test_cancel() {
  FakeExec ex;
  ex.fp = {{0, 600}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 3, 3);
  add_frames(ex, 1, 3, 3);
  Scheduler s(ladder_cfg(1000), &ex);
  uint64_t a = 0, b = 0, d = 0;
  CHECK(s.submit(0, 1, 0, &a) == MR_OK);
  CHECK(s.submit(1, 1, 0, &b) == MR_OK);   // waits: 600 + 600 > 1000
  CHECK(s.submit(1, 1, 1, &d) == MR_OK);   // dependent of b
  s.step();
  CHECK(ex.launched.size() == 1 && ex.launched[0][0] == a);
  CHECK(s.cancel(a) == MR_ESTATE);         // launched: runs to its end
  CHECK(s.cancel(b) == MR_OK);             // waiting for memory
  CHECK(s.job(b)->state == kFailed && s.job(b)->status == MR_ECANCELED);
  CHECK(s.cancel(b) == MR_ESTATE && s.cancel(999) == MR_EINVAL);
  run_until_idle(s, ex);
  CHECK(s.job(d)->state == kFailed && s.job(d)->status == MR_EDEPEND);
  CHECK(s.job(a)->state == kDone);
  CHECK(ex.launched.size() == 1);          // neither b nor its dependent ran
  const SchedStats st = s.stats();
  CHECK(st.cancelled == 1 && st.failed == 2 && st.completed == 1);
  std::vector<uint64_t> c = s.take_completions(10);
  CHECK(c.size() == 3);
  for (uint64_t id : c) CHECK(s.release(id) == MR_OK);
  s.step();
}

static void test_timeout() {
  FakeExec ex;
  ex.fp = {{0, 600}, {1, 1}, {2, 1}};
  add_frames(ex, 0, 3, 3);
  add_frames(ex, 1, 3, 3);
  SchedConfig cfg = ladder_cfg(1000);
  cfg.job_timeout_ns = 2000000;  // 2 ms
  Scheduler s(cfg, &ex);
  ex.batch_ns = 5000000;         // the running job holds the memory for 5 ms
  uint64_t a = 0, b = 0, d = 0;
  CHECK(s.submit(0, 1, 0, &a) == MR_OK);
  CHECK(s.submit(1, 1, 0, &b) == MR_OK);
  s.step();                       // a launches; b cannot fit
  ex.t += 1000000;
  CHECK(s.submit(1, 1, 2, &d) == MR_OK);  // a dependent of b, 1 ms later
  s.step();
  CHECK(s.job(b)->state == kReady && s.job(d)->state == kQueued);
  ex.t += 1500000;                // 2.5 ms after arrival
  s.step();
  CHECK(s.job(b)->state == kFailed && s.job(b)->status == MR_ETIMEOUT);
  CHECK(s.job(a)->state == kRunning);  // launched jobs are not timed out
  run_until_idle(s, ex);
  CHECK(s.job(a)->state == kDone && s.job(a)->status == MR_OK);
  CHECK(s.job(d)->state == kFailed && s.job(d)->status == MR_EDEPEND);
  CHECK(s.stats().timed_out == 1 && s.stats().failed == 2);
  CHECK(ex.launched.size() == 1);
}

int main() {
  test_dependent_batch_done_first();
  test_cancel();
  test_timeout();
  test_chain_on_launch();
  test_dependency_and_implied_reference();
  test_missing_reference_frames();
  test_budget_admission_and_rejection();
  test_queue_limit();
  test_reference_failure_fails_dependents();
  test_continuous_batching_and_latency();
  test_finished_jobs_are_forgotten();
  test_dropped_frames_fail_alone();
  test_superseded_references_freed();
  test_dropped_frames_free_references();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("scheduler: all checks passed\n");
  return 0;
}
