// Serving scheduler (see mr_sched.h).
#include "mr_sched.h"

#include <algorithm>

#include "mr.h"

namespace mr {

Scheduler::Scheduler(const SchedConfig& cfg, Executor* ex) : cfg_(cfg), ex_(ex) {}

static bool is_reference_rung(const SchedConfig& cfg, int rung) {
  for (const RungCfg& r : cfg.rungs)
    if (r.ref_rung == rung) return true;
  return false;
}

SchedJob* Scheduler::find_ref(int stream, int frame, int ref_rung) {
  auto it = latest_.find(std::make_tuple(stream, frame, ref_rung));
  if (it == latest_.end()) return nullptr;
  auto jt = jobs_.find(it->second);
  if (jt == jobs_.end()) return nullptr;
  SchedJob* r = jt->second.get();
  if (r->state == kFailed) return nullptr;
  if (r->state == kDone && !r->exec_state) return nullptr;  // outputs already freed
  return r;
}

int Scheduler::submit(int stream, int frame, int rung, uint64_t* id) {
  if (id) *id = 0;
  if (stream < 0 || frame < 1 || rung < 0 || rung >= (int)cfg_.rungs.size()) return MR_EINVAL;
  if (!ex_->frames_resident(stream, frame, rung)) return MR_EINVAL;
  if (open_ >= cfg_.max_queue) {
    ++st_.rejected;
    return MR_EAGAIN;
  }
  SchedJob* ref = nullptr;
  const int rr = cfg_.rungs[rung].ref_rung;
  if (rr >= 0) {
    ref = find_ref(stream, frame, rr);
    if (!ref) {
      if (!ex_->frames_resident(stream, frame, rr)) return MR_EDEPEND;
      uint64_t rid = 0;
      const int rc = submit(stream, frame, rr, &rid);  // the implied reference job
      if (rc != MR_OK) return rc == MR_EINVAL ? MR_EDEPEND : rc;
      ref = jobs_[rid].get();
      ref->implied = true;
      ++st_.implied;
    }
  }
  auto j = std::make_unique<SchedJob>();
  j->id = next_id_++;
  j->stream = stream, j->frame = frame, j->rung = rung;
  j->t_arrive = ex_->now_ns();
  j->footprint = ex_->footprint(*j);
  if (j->footprint > cfg_.budget_bytes) {
    ++st_.rejected;
    return MR_EAGAIN;  // can never be admitted under this budget
  }
  if (ref) {
    j->ref_job = ref->id;
    ref->pending_dependents++;
    j->state = ref->depth_ready ? kReady : kQueued;
  } else {
    j->state = kReady;
  }
  const uint64_t jid = j->id;
  latest_[std::make_tuple(stream, frame, rung)] = jid;
  jobs_[jid] = std::move(j);
  queue_.push_back(jid);
  ++open_;
  ++st_.submitted;
  if (id) *id = jid;
  return MR_OK;
}

// A done job of the same stream and rung kKeepFrames or more frames later?
bool Scheduler::superseded(const SchedJob& j) const {
  for (auto it = latest_.lower_bound(std::make_tuple(j.stream, j.frame + kKeepFrames, 0));
       it != latest_.end() && std::get<0>(it->first) == j.stream; ++it) {
    if (std::get<2>(it->first) != j.rung) continue;
    auto jt = jobs_.find(it->second);
    if (jt != jobs_.end() && jt->second->state == kDone) return true;
  }
  return false;
}

void Scheduler::maybe_free(SchedJob& j) {
  if (!j.exec_state) return;
  if (j.state != kDone && j.state != kFailed) return;
  if (!j.released || j.pending_dependents > 0) return;
  // A done reference job stays resident (its depth map serves later
  // dependents of its frame) until admission needs its memory (see step()) or
  // a job of its stream and rung kKeepFrames frames later is done: a
  // dependent submitted for its frame after that gets a new reference job.  So
  // a stream that moves forward keeps the references of its last frames only,
  // and the older ones' blocks serve the next frames' jobs; clients that
  // revisit the last frames still find theirs.
  if (j.state == kDone && is_reference_rung(cfg_, j.rung) && !j.stale && !superseded(j)) return;
  ex_->free_job(j);
  j.exec_state = nullptr;
  if (j.admitted) st_.bytes_in_use -= j.footprint, j.admitted = false;
  retire_check_.push_back(j.id);
}

// Forget jobs that are finished, handed out, released and freed, and that no
// dependent still needs.
void Scheduler::retire_finished() {
  while (!retire_check_.empty()) {
    const uint64_t id = retire_check_.front();
    retire_check_.pop_front();
    auto it = jobs_.find(id);
    if (it == jobs_.end()) continue;
    const SchedJob& j = *it->second;
    if ((j.state != kDone && j.state != kFailed) || !j.handed_out || !j.released ||
        j.exec_state || j.pending_dependents > 0)
      continue;
    auto lt = latest_.find(std::make_tuple(j.stream, j.frame, j.rung));
    if (lt != latest_.end() && lt->second == id) latest_.erase(lt);
    jobs_.erase(it);
  }
}

void Scheduler::frames_dropped(int stream, int before_frame) {
  std::vector<SchedJob*> old;
  for (auto it = latest_.lower_bound(std::make_tuple(stream, 0, 0));
       it != latest_.end() && std::get<0>(it->first) == stream &&
       std::get<1>(it->first) <= before_frame;
       ++it) {
    auto jt = jobs_.find(it->second);
    if (jt != jobs_.end()) old.push_back(jt->second.get());
  }
  for (SchedJob* r : old) {
    r->stale = true;
    maybe_free(*r);
  }
}

void Scheduler::free_all() {
  for (auto& kv : jobs_) {
    SchedJob& j = *kv.second;
    if (!j.exec_state) continue;
    ex_->free_job(j);
    j.exec_state = nullptr;
    if (j.admitted) st_.bytes_in_use -= j.footprint, j.admitted = false;
  }
}

void Scheduler::complete(SchedJob& j, int status, int64_t t) {
  j.t_done = t;
  j.status = status;
  j.state = status == MR_OK ? kDone : kFailed;
  j.depth_ready = status == MR_OK;
  --inflight_;
  --open_;
  if (status == MR_OK) {
    ++st_.completed;
    st_.ctus_done += j.n_ctus;
    st_.last_done_ns = std::max(st_.last_done_ns, t);
    latencies_ms_.push_back((t - j.t_arrive) * 1e-6);
  } else {
    ++st_.failed;
  }
  completions_.push_back(j.id);
  if (j.ref_job) {
    auto it = jobs_.find(j.ref_job);
    if (it != jobs_.end()) {
      it->second->pending_dependents--;
      maybe_free(*it->second);
      retire_check_.push_back(j.ref_job);
    }
  }
  // References of this stream and rung kKeepFrames or more frames earlier are
  // superseded.
  if (status == MR_OK && is_reference_rung(cfg_, j.rung)) {
    std::vector<SchedJob*> older;
    for (auto it = latest_.lower_bound(std::make_tuple(j.stream, 0, 0));
         it != latest_.end() && std::get<0>(it->first) == j.stream &&
         std::get<1>(it->first) <= j.frame - kKeepFrames;
         ++it) {
      if (std::get<2>(it->first) != j.rung) continue;
      auto jt = jobs_.find(it->second);
      if (jt != jobs_.end()) older.push_back(jt->second.get());
    }
    for (SchedJob* r : older) maybe_free(*r);
  }
}

int Scheduler::step() {
  int done = 0;
  retire_finished();
  const int64_t now = ex_->now_ns();
  // 1. Retire finished batches.  A batch holding a dependent whose reference's
  //    batch has not been retired yet waits for it (chain_on_launch): the
  //    reference's outcome decides the dependent's.
  for (size_t b = 0; b < running_.size();) {
    bool ref_running = false;
    for (const SchedJob* j : running_[b].jobs) {
      if (!j->ref_job) continue;
      auto it = jobs_.find(j->ref_job);
      if (it != jobs_.end() && it->second->state == kRunning) ref_running = true;
    }
    const int q = ref_running ? 0 : ex_->query(running_[b].handle);
    if (q == 0) {
      ++b;
      continue;
    }
    ex_->finish(running_[b].handle, running_[b].jobs);
    const int64_t t = ex_->now_ns();
    for (SchedJob* j : running_[b].jobs) {
      int status = q < 0 ? MR_EHIP : j->status;
      if (status == MR_OK && j->ref_job) {
        // Launched behind a reference that has failed since (its batch was
        // retired first, see above).
        auto it = jobs_.find(j->ref_job);
        if (it != jobs_.end() && it->second->state == kFailed) status = MR_EDEPEND;
      }
      complete(*j, status, t);
      ++done;
    }
    running_.erase(running_.begin() + b);
  }
  // 2, 3: with chain_on_launch a launch makes its dependents ready at once, so
  // the next batch of a reference chain goes out in the same step.
  while (launch_ready(now, done)) {
  }
  return done;
}

int Scheduler::launch_ready(int64_t now, int& done) {
  // 2. Dependents of finished (with chain_on_launch: of launched) references
  //    become ready, or fail with them.
  for (uint64_t id : queue_) {
    SchedJob& j = *jobs_[id];
    if ((j.state != kQueued && j.state != kReady) || !j.ref_job) continue;
    const SchedJob& r = *jobs_[j.ref_job];
    if (j.state == kQueued &&
        (r.state == kDone || (cfg_.chain_on_launch && r.state == kRunning)))
      j.state = kReady;
    if (r.state == kFailed) {
      j.state = kRunning;  // transient; completed below
      ++inflight_;
      complete(j, MR_EDEPEND, now);
      ++done;
    }
  }
  // Jobs that waited longer than the timeout without a launch give up.
  if (cfg_.job_timeout_ns > 0) {
    for (uint64_t id : queue_) {
      SchedJob& j = *jobs_[id];
      if ((j.state == kQueued || j.state == kReady) && now - j.t_arrive > cfg_.job_timeout_ns) {
        j.state = kRunning;  // transient; completed below
        ++inflight_;
        complete(j, MR_ETIMEOUT, now);
        ++st_.timed_out;
        ++done;
      }
    }
  }
  queue_.erase(std::remove_if(queue_.begin(), queue_.end(),
                              [&](uint64_t id) { return jobs_[id]->state == kFailed; }),
               queue_.end());
  // 3. Admit ready jobs in arrival order (head of line blocks: no starvation of
  //    large jobs) and launch them as one batch.
  if ((int)running_.size() >= cfg_.max_batches_in_flight) return 0;
  std::vector<SchedJob*> batch;
  for (uint64_t id : queue_) {
    SchedJob& j = *jobs_[id];
    if (j.state == kQueued) continue;  // waiting for its reference
    if (!ex_->frames_resident(j.stream, j.frame, j.rung)) {
      // Its frames were dropped after submission: it fails alone.
      j.state = kRunning;  // transient; completed below
      ++inflight_;
      complete(j, MR_EDEPEND, now);
      ++done;
      continue;
    }
    if ((int)batch.size() >= cfg_.max_batch_jobs || inflight_ >= cfg_.max_inflight) break;
    if (st_.bytes_in_use + j.footprint > cfg_.budget_bytes) {
      // Evict resident reference jobs nobody needs any more (oldest first).
      for (auto& kv : jobs_) {
        SchedJob& r = *kv.second;
        if (st_.bytes_in_use + j.footprint <= cfg_.budget_bytes) break;
        if (r.exec_state && r.state == kDone && r.released && r.pending_dependents == 0) {
          ex_->free_job(r);
          r.exec_state = nullptr;
          if (r.admitted) st_.bytes_in_use -= r.footprint, r.admitted = false;
          retire_check_.push_back(r.id);
        }
      }
      if (st_.bytes_in_use + j.footprint > cfg_.budget_bytes) break;
    }
    j.admitted = true;
    st_.bytes_in_use += j.footprint;
    st_.peak_bytes = std::max(st_.peak_bytes, st_.bytes_in_use);
    ++inflight_;
    batch.push_back(&j);
  }
  queue_.erase(std::remove_if(queue_.begin(), queue_.end(),
                              [&](uint64_t id) { return jobs_[id]->state == kFailed; }),
               queue_.end());
  if (batch.empty()) return 0;
  for (SchedJob* j : batch) j->state = kRunning;
  queue_.erase(std::remove_if(queue_.begin(), queue_.end(),
                              [&](uint64_t id) { return jobs_[id]->state == kRunning; }),
               queue_.end());
  void* handle = nullptr;
  const int64_t t0 = ex_->now_ns();
  const int rc = ex_->launch(batch, &handle);
  const int64_t t = ex_->now_ns();
  st_.host_launch_ns += t - t0;
  if (rc != MR_OK) {
    for (SchedJob* j : batch) {
      complete(*j, rc, t);
      ++done;
    }
    return 0;
  }
  for (SchedJob* j : batch) j->t_start = t;
  if (!st_.first_start_ns) st_.first_start_ns = t;
  ++st_.batches;
  running_.push_back(Batch{handle, batch});
    return 1;
}

std::vector<uint64_t> Scheduler::take_completions(int max) {
  std::vector<uint64_t> out;
  while (!completions_.empty() && (int)out.size() < max) {
    const uint64_t id = completions_.front();
    completions_.pop_front();
    auto it = jobs_.find(id);
    if (it != jobs_.end()) it->second->handed_out = true;
    retire_check_.push_back(id);  // retired at the next step(), after the caller read it
    out.push_back(id);
  }
  return out;
}

const SchedJob* Scheduler::job(uint64_t id) const {
  auto it = jobs_.find(id);
  return it == jobs_.end() ? nullptr : it->second.get();
}

int Scheduler::release(uint64_t id) {
  auto it = jobs_.find(id);
  if (it == jobs_.end()) return MR_EINVAL;
  SchedJob& j = *it->second;
  if (j.state != kDone && j.state != kFailed) return MR_ESTATE;
  j.released = true;
  maybe_free(j);
  retire_check_.push_back(id);
  return MR_OK;
}

int Scheduler::cancel(uint64_t id) {
  auto it = jobs_.find(id);
  if (it == jobs_.end()) return MR_EINVAL;
  SchedJob& j = *it->second;
  if (j.state != kQueued && j.state != kReady) return MR_ESTATE;
  j.state = kRunning;  // transient, as for the other failures before a launch
  ++inflight_;
  complete(j, MR_ECANCELED, ex_->now_ns());
  ++st_.cancelled;
  queue_.erase(std::remove(queue_.begin(), queue_.end(), id), queue_.end());
  return MR_OK;
}

bool Scheduler::idle() const { return queue_.empty() && running_.empty(); }

SchedStats Scheduler::stats() const {
  SchedStats s = st_;
  if (!latencies_ms_.empty()) {
    std::vector<double> v = latencies_ms_;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const size_t k = (size_t)std::min<double>(v.size() - 1, std::max(0.0, p * v.size() - 1e-9));
      return v[k];
    };
    s.p50_ms = pct(0.50);
    s.p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    s.mean_ms = sum / v.size();
    s.max_ms = v.back();
  }
  return s;
}

}  // namespace mr
