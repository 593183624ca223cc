// Serving scheduler of the ladder server: job state machine, reference-depth
// dependencies, memory-footprint admission, continuous batching and latency
// statistics.  Pure host C++ (no HIP): the device work goes through an
// Executor, so the state machine is testable on the CPU with a fake one.
#pragma once
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

namespace mr {

enum JobState { kQueued = 0, kReady = 1, kRunning = 2, kDone = 3, kFailed = 4 };

// A done reference job is kept for later dependents of its frame until a job
// of its stream and rung this many frames later is done (or admission needs
// its memory).
constexpr int kKeepFrames = 2;

struct RungCfg {
  int width, height, qp, search_range, ref_rung;  // ref_rung -1: a root (no dependency)
  int dlo = 0, dhi = 1;  // depth-bound policy of this rung as a dependent
  int refine = -1;       // refinement half-width of its seed, -1: not seeded
  int subpel = 0;        // quarter-pel refinement of its MVs
  int angular = 0;       // angular intra modes
};

struct SchedConfig {
  std::vector<RungCfg> rungs;
  uint64_t budget_bytes = 0;  // footprint of admitted, not yet released jobs
  int max_inflight = 64;      // jobs admitted (running or done-unreleased excluded)
  int max_queue = 4096;       // submitted, not yet completed
  int max_batch_jobs = 64;    // jobs per device launch
  int max_batches_in_flight = 2;
  // A dependent may launch once its reference's batch has been launched, not
  // only once it is done: the executor orders the two batches on the device.
  // A dependent whose reference then fails fails with it.
  bool chain_on_launch = false;
  // A job not launched within this time of its arrival completes with
  // MR_ETIMEOUT (0: no limit).  Launched jobs run to completion: device work
  // is not interrupted.
  int64_t job_timeout_ns = 0;
};

struct SchedJob {
  uint64_t id = 0;
  int stream = 0, frame = 0, rung = 0;
  JobState state = kQueued;
  int status = 0;
  bool implied = false;            // created by the server for a dependent
  bool stale = false;              // its frames were dropped: serves no later dependent
  bool released = false;           // caller released the outputs
  bool handed_out = false;         // completion taken by take_completions
  uint64_t ref_job = 0;            // job whose depth map bounds this one (0 none)
  int pending_dependents = 0;      // dependents that still need this job's depth map
  bool depth_ready = false;        // reference depth map available (job done)
  size_t footprint = 0;            // device bytes while admitted
  bool admitted = false;
  int64_t t_arrive = 0, t_start = 0, t_done = 0;
  int64_t cost_sum = 0;
  int n_ctus = 0;
  void* exec_state = nullptr;      // executor-owned per-job data (outputs)
};

// Device side of the server.  All calls come from the scheduler's thread.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual int64_t now_ns() = 0;
  // Bytes a job occupies on the device while admitted (scratch + outputs + bounds).
  virtual size_t footprint(const SchedJob& j) = 0;
  // Are both frames (frame and frame-1) of (stream, rung) resident?
  virtual bool frames_resident(int stream, int frame, int rung) = 0;
  // Launch a batch; jobs' references (ref_job) are done, or with chain_on_launch
  // launched in an earlier batch.  Returns 0 or an mr_status.
  virtual int launch(const std::vector<SchedJob*>& jobs, void** handle) = 0;
  // 1 done, 0 still running, < 0 failed.
  virtual int query(void* handle) = 0;
  // After query() != 0: fill per-job results (cost_sum, status) and free batch resources.
  virtual void finish(void* handle, const std::vector<SchedJob*>& jobs) = 0;
  // Free a job's outputs (released and no longer needed by dependents).
  virtual void free_job(SchedJob& j) = 0;
};

struct SchedStats {
  int64_t submitted = 0, implied = 0, completed = 0, failed = 0, rejected = 0;
  int64_t batches = 0, ctus_done = 0;
  int64_t cancelled = 0, timed_out = 0;
  int64_t first_start_ns = 0, last_done_ns = 0;
  int64_t host_launch_ns = 0;  // host time spent in Executor::launch
  double p50_ms = 0, p99_ms = 0, mean_ms = 0, max_ms = 0;
  uint64_t bytes_in_use = 0, peak_bytes = 0;
};

class Scheduler {
 public:
  Scheduler(const SchedConfig& cfg, Executor* ex);
  // Validate and enqueue; may create the implied reference job.  Returns an mr_status.
  int submit(int stream, int frame, int rung, uint64_t* id);
  // One loop iteration: retire finished batches, release dependents, admit and
  // launch.  Returns the number of jobs completed in this call.
  int step();
  // Completed jobs not yet handed out (ids in completion order).
  std::vector<uint64_t> take_completions(int max);
  // A job stays known (job(id) != null) until it is finished, handed out,
  // released, its outputs are freed and no dependent needs it; step() then
  // forgets it, so the tables hold live jobs only.
  const SchedJob* job(uint64_t id) const;
  int release(uint64_t id);
  // Cancel a job that has not been launched: it completes with MR_ECANCELED
  // (its dependents then fail with MR_EDEPEND).  MR_ESTATE once launched or
  // finished, MR_EINVAL for an unknown id.
  int cancel(uint64_t id);
  bool idle() const;  // nothing queued or running
  SchedStats stats() const;
  int batches_in_flight() const { return (int)running_.size(); }
  size_t jobs_known() const { return jobs_.size(); }
  // Free the outputs of every job still holding them (server shutdown).
  void free_all();
  // The client dropped the frames of `stream` before `before_frame`: done
  // reference jobs of frames up to `before_frame` can serve no later
  // dependent (one needs its frame and the previous one) and stop staying
  // resident.
  void frames_dropped(int stream, int before_frame);

 private:
  struct Batch {
    void* handle;
    std::vector<SchedJob*> jobs;
  };
  SchedJob* find_ref(int stream, int frame, int ref_rung);
  bool superseded(const SchedJob& j) const;
  void maybe_free(SchedJob& j);
  void complete(SchedJob& j, int status, int64_t t);
  void retire_finished();
  // Phases 2 and 3 of step(): dependents become ready (or fail), timeouts,
  // then one batch is admitted and launched.  1 if a batch was launched.
  int launch_ready(int64_t now, int& done);
  SchedConfig cfg_;
  Executor* ex_;
  uint64_t next_id_ = 1;
  std::map<uint64_t, std::unique_ptr<SchedJob>> jobs_;
  std::map<std::tuple<int, int, int>, uint64_t> latest_;  // (stream, frame, rung) -> job
  std::deque<uint64_t> queue_;                           // submitted, not launched (FIFO)
  std::vector<Batch> running_;
  std::deque<uint64_t> completions_;
  std::vector<double> latencies_ms_;
  std::deque<uint64_t> retire_check_;  // jobs whose retirement conditions may now hold
  SchedStats st_;
  int inflight_ = 0;
  int open_ = 0;  // submitted, not yet completed
};

}  // namespace mr
