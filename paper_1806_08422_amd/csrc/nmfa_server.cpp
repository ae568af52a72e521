// Continuous-batching annealing server (nmfa_server_* in include/nmfa.h).
//
// A scheduler thread owns three HIP streams (with the null stream, which the uploads use, that is
// HIP's default of four hardware queues per process); an admission thread takes requests from a
// FIFO queue
// by device memory budget and a cap on concurrently admitted requests, and does their host-side
// set-up and upload beside the running rounds. Admitted requests advance in rounds of
// chunk_iters iterations of Algorithm 1:
//   * all admitted requests on the persistent small-N path share ONE launch per round
//     (anneal_small_batched over every request's replica blocks; each workgroup reads its own
//     request's arguments), on the third stream;
//   * larger requests advance by the same chunk on their own kernels in the same round, over the
//     three streams, so that their kernels run side by side with the batched launch and with
//     each other. The workgroups of one persistent XCD-group launch wait for each other, so
//     group launches run side by side only where all of them fit on the chip at once: each of
//     the three streams has a workgroup budget (half, a quarter and a quarter of the CUs, in
//     multiples of the XCD count), each group launch on a stream is capped at that stream's
//     budget (a request that needs more takes several launches in turn), and a stream runs one
//     launch at a time, so the resident group workgroups never exceed the CUs. Requests go to the
//     stream that would finish them first (largest first). A round with a single group request
//     gives it the whole chip; such a launch waits for the other streams' group launches, and
//     theirs for it. The sparse and per-iteration kernels never wait for other workgroups, so
//     they take the second and third streams and at worst delay a group launch's start;
//   * two rounds are in flight: round k+1 is enqueued before the host waits for round k, so the
//     device has work queued while finished requests are read back. A request's consecutive
//     chunks are ordered by its stream, or by its event when the stream changes. The spin state
//     stays on the device between chunks (resuming is bit-exact). Finished requests' device
//     memory is freed in batches, since freeing waits for the device.
// Every request's arithmetic depends only on that request (counter-based noise keyed by its own
// seed, replica and iteration), so its result is identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nmfa_ctx.h"

using namespace nmfa;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t round_up_sz(size_t v, size_t m) { return (v + m - 1) / m * m; }

struct Job {
  uint64_t id = 0;
  int n = 0, R = 0, t_f = 0;
  uint64_t seed = 0;
  std::vector<double> J, h;  // host copies until the request is admitted
  size_t bytes = 0;          // device memory charged to the budget
  int status = NMFA_JOB_QUEUED;  // or a negative error code once failed / cancelled
  bool cancel = false;
  bool failed = false;       // a chunk could not be enqueued: ends as a device error
  nmfa_ctx* ctx = nullptr;
  int t_done = 0;            // iterations complete on the device
  int t_sched = 0;           // iterations enqueued (up to two chunks ahead of t_done)
  int lane = -2;             // stream of the last enqueued chunk: -1 batched stream, 0.. lanes
  hipEvent_t ev = nullptr;   // recorded after the last enqueued chunk
  uint64_t last_round = 0;   // round of the last enqueued chunk
  std::vector<double> E;
  std::vector<int64_t> Eint;
  std::vector<int8_t> spins;
  double t_submit = 0, t_finish = 0;
  std::string msg;
};

// Upper bound of the device memory one request needs on any kernel path (J operand copy, exact
// energy copy, normalisers, schedule, state, spins, energies and the spin operand buffers).
size_t job_bytes(int n, int R, int t_f, bool j_integral) {
  const size_t Kp = std::max<size_t>(512, round_up_sz(n, 256)), Mp = round_up_sz(n, 128);  // either XCD layout
  const size_t Rp = round_up_sz(R, 128);
  size_t b = Mp * Kp * 2;                          // J operand (BF16 or smaller)
  b += (size_t)n * n * (j_integral ? 1 : 8);       // J for exact energies
  b += 2 * Mp * 4 + (size_t)t_f * 4 + (size_t)n * 8;
  b += (size_t)R * n * 4 + (size_t)R * n + (size_t)R * 16;
  b += 2 * Rp * Kp * 2;                            // spin operand double buffer
  b += 96 * 1024;                                  // control block and alignment slack
  return b;
}

}  // namespace

constexpr int SERVER_LANES = 3;  // kernel streams (with the null stream: 4 hardware queues in all)

// One round of the pipeline: the chunk of every request advanced in it, and what the host keeps
// until the round's work is complete (the batched launch's staging).
struct Round {
  bool inflight = false;
  uint64_t id = 0;
  std::vector<Job*> ran;
  std::vector<int> t_end;      // parallel to ran
  std::vector<char> last;      // parallel to ran: the request's final chunk (energies enqueued)
  hipEvent_t ev[1 + SERVER_LANES] = {};  // end of the round on every stream
  std::vector<AnnealArgs> h_args;
  std::vector<int2> h_tasks;
  AnnealArgs* d_jobs = nullptr;
  int cap_jobs = 0;
  int2* d_tasks = nullptr;
  int cap_tasks = 0;
};

// A finished request's device state, kept until it can be freed without stalling the pipeline
// (freeing device memory waits for the device).
struct Retired {
  nmfa_ctx* ctx;
  hipEvent_t ev;
  size_t bytes;
};

struct nmfa_server {
  nmfa_server_params p{};
  int device = 0;
  hipStream_t stream = nullptr;            // the batched small-N launch: the last lane
  hipStream_t lanes[SERVER_LANES] = {};    // group kernels on all three; sparse, per-iteration on [1..]
  int cus = 256;                           // compute units of the device
  std::mutex mu;
  std::condition_variable cv_work, cv_admit, cv_done;  // scheduler, admission thread, clients
  std::deque<Job*> queue;
  std::vector<Job*> active;  // touched by the scheduler thread only (plus stats under mu)
  std::unordered_map<uint64_t, Job*> jobs;
  size_t used_bytes = 0, peak_bytes = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker, admitter;
  int admitting = 0;                       // requests whose set-up is under way
  bool want_free = false;                  // admission waits for memory held by retired requests
  Round rounds[2];
  uint64_t next_round = 1, completed_round = 0;
  std::vector<Retired> retired;            // scheduler thread only
  size_t retired_bytes = 0;
  hipEvent_t ev_group[SERVER_LANES] = {};  // after the last group launch on each lane
  bool group_rec[SERVER_LANES] = {};
  hipEvent_t ev_wide = nullptr;            // after the last whole-chip group launch
  bool wide_rec = false;
  nmfa_server_stats st{};
};

extern "C" void nmfa_server_params_default(nmfa_server_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(nmfa_server_params);
  p->precision = NMFA_BF16;
  p->hbm_budget_bytes = 8ull << 30;
  p->max_active = 256;
  p->chunk_iters = 250;
}

namespace {

// Finish a request (under the lock, with none of its work in flight): record the outcome and
// retire its device state; its memory stays charged to the budget until free_retired.
void finish_job(nmfa_server* s, Job* j, int status) {
  if (j->ctx) {
    s->retired.push_back(Retired{j->ctx, j->ev, j->bytes});
    s->retired_bytes += j->bytes;
    j->ctx = nullptr;
    j->ev = nullptr;
  } else {
    s->used_bytes -= std::min(s->used_bytes, j->bytes);
  }
  j->status = status;
  j->t_finish = now_s();
  if (status == NMFA_JOB_DONE) ++s->st.completed;
  else if (status == NMFA_ECANCELED) ++s->st.cancelled;
  else ++s->st.failed;
}

// Stream and per-launch workgroup cap of each of the round's XCD-group requests (lane -1 for the
// others). Budgets: lane 0 half of the CUs, lanes 1 and 2 a quarter each, rounded down to a
// multiple of the 8 XCDs so that the round-robin placement of a launch's workgroups over the XCDs
// also fits. A request goes to the lane on which, after the work already given to it, it would
// finish first, with per-launch time taken as proportional to Mp (the k length) and the number
// of launches as its groups over the groups that fit the budget.
void plan_group_lanes(const nmfa_server* s, const std::vector<Job*>& jobs, const std::vector<int>& t_end,
                      std::vector<int>* lane, std::vector<int>* cap) {
  lane->assign(jobs.size(), -1);
  cap->assign(jobs.size(), 0);
  std::vector<int> idx, P(jobs.size()), G(jobs.size());
  for (size_t k = 0; k < jobs.size(); ++k)
    if (jobs[k]->ctx && ctx_group_shape(jobs[k]->ctx, jobs[k]->R, &P[k], &G[k])) idx.push_back((int)k);
  for (int k : idx) (*lane)[k] = 0;  // default: one stream, whole chip
  const int budget[SERVER_LANES] = {s->cus / 2 / 8 * 8, s->cus / 4 / 8 * 8, s->cus / 4 / 8 * 8};
  if (idx.size() < 2 || budget[1] < 8) return;
  for (int k : idx)
    if (P[k] > budget[0]) return;
  auto iters = [&](int k) { return (double)(t_end[k] - jobs[k]->t_sched); };
  std::sort(idx.begin(), idx.end(), [&](int x, int y) {
    return (double)G[x] * P[x] * jobs[x]->ctx->Mp * iters(x) > (double)G[y] * P[y] * jobs[y]->ctx->Mp * iters(y);
  });
  double load[SERVER_LANES] = {0, 0, 0};
  for (int k : idx) {
    int best = -1;
    double best_end = 0, best_t = 0;
    for (int L = 0; L < SERVER_LANES; ++L) {
      if (P[k] > budget[L]) continue;
      const int per = budget[L] / P[k];
      const double t = (double)((G[k] + per - 1) / per) * jobs[k]->ctx->Mp * iters(k);
      if (best < 0 || load[L] + t < best_end) {
        best = L;
        best_end = load[L] + t;
        best_t = t;
      }
    }
    load[best] += best_t;
    (*lane)[k] = best;
    (*cap)[k] = budget[best];
  }
}

int ensure_staging(Round& r, int n_jobs, int n_tasks) {
  if (n_jobs > r.cap_jobs) {
    (void)hipFree(r.d_jobs);
    r.d_jobs = nullptr;
    const int cap = std::max(n_jobs, 2 * r.cap_jobs);
    if (hipMalloc(&r.d_jobs, sizeof(AnnealArgs) * cap) != hipSuccess) return NMFA_ENOMEM;
    r.cap_jobs = cap;
  }
  if (n_tasks > r.cap_tasks) {
    (void)hipFree(r.d_tasks);
    r.d_tasks = nullptr;
    const int cap = std::max(n_tasks, 2 * r.cap_tasks);
    if (hipMalloc(&r.d_tasks, sizeof(int2) * cap) != hipSuccess) return NMFA_ENOMEM;
    r.cap_tasks = cap;
  }
  return NMFA_OK;
}

// Free the retired requests' device state and release their budget. Waits for the work in
// flight (freeing device memory does), so it runs when the pipeline is empty or memory is needed.
void free_retired(nmfa_server* s) {
  std::vector<Retired> rs;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rs.swap(s->retired);
  }
  size_t freed = 0;
  for (const Retired& r : rs) {
    nmfa_destroy(r.ctx);
    if (r.ev) (void)hipEventDestroy(r.ev);
    freed += r.bytes;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->used_bytes -= std::min(s->used_bytes, freed);
    s->retired_bytes -= std::min(s->retired_bytes, freed);
    s->want_free = false;
  }
  s->cv_admit.notify_one();
}

// Whether the head of the queue can be admitted now (or rejected outright); under the lock.
bool admissible(const nmfa_server* s) {
  if (s->queue.empty() || (int)s->active.size() + s->admitting >= s->p.max_active) return false;
  const Job* j = s->queue.front();
  return j->bytes > s->p.hbm_budget_bytes || s->used_bytes + j->bytes <= s->p.hbm_budget_bytes;
}

// Admission thread. Admits queued requests (FIFO by device memory budget and slots; the head of
// the queue is never overtaken) and does their host-side set-up and upload (nmfa_create) beside
// the scheduler's rounds instead of between them: the server's streams do not synchronise with
// the null stream that the uploads use. When the head waits for memory that retired requests
// still hold, it asks the scheduler to free them.
void admitter(nmfa_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<Job*> admitted;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_admit.wait(lk, [&] {
        if (s->stop || admissible(s)) return true;
        if (!s->queue.empty() && s->retired_bytes > 0 && !s->want_free &&
            (int)s->active.size() + s->admitting < s->p.max_active) {
          s->want_free = true;
          s->cv_work.notify_one();
        }
        return false;
      });
      if (s->stop) break;
      while (admissible(s)) {
        Job* j = s->queue.front();
        s->queue.pop_front();
        if (j->bytes > s->p.hbm_budget_bytes) {
          j->msg = "request needs more device memory than the whole budget";
          j->bytes = 0;  // never charged to the budget
          finish_job(s, j, NMFA_ENOMEM);
          s->cv_done.notify_all();
          continue;
        }
        s->used_bytes += j->bytes;
        s->peak_bytes = std::max(s->peak_bytes, s->used_bytes);
        ++s->admitting;
        admitted.push_back(j);
      }
    }
    for (Job* j : admitted) {  // outside the lock
      nmfa_params prm;
      nmfa_params_default(&prm);
      prm.precision = s->p.precision;
      nmfa_ctx* c = nullptr;
      int rc = nmfa_create(j->n, j->J.data(), j->h.empty() ? nullptr : j->h.data(), &prm, &c);
      if (rc == NMFA_OK && hipEventCreateWithFlags(&j->ev, hipEventDisableTiming) != hipSuccess) {
        nmfa_destroy(c);
        c = nullptr;
        j->ev = nullptr;
        rc = nmfa_fail(NMFA_EDEVICE, "server: event creation failed");
      }
      std::lock_guard<std::mutex> lk(s->mu);
      --s->admitting;
      if (rc != NMFA_OK) {
        j->msg = nmfa_last_error();
        finish_job(s, j, rc);
        s->cv_done.notify_all();
        continue;
      }
      j->ctx = c;
      std::vector<double>().swap(j->J);
      std::vector<double>().swap(j->h);
      if (s->stop) {
        finish_job(s, j, NMFA_ECANCELED);
        s->cv_done.notify_all();
        continue;
      }
      j->status = NMFA_JOB_RUNNING;
      s->active.push_back(j);
      s->cv_work.notify_one();
    }
  }
}

// Enqueue the next chunk of every running request into round r (nothing if none has iterations
// left to enqueue). A request's chunks follow each other on one stream or, when its stream
// changes, through its event.
void enqueue_round(nmfa_server* s, Round& r) {
  r.ran.clear();
  r.t_end.clear();
  r.last.clear();
  r.h_args.clear();
  r.h_tasks.clear();
  std::vector<Job*> jobs;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<Job*> keep;
    for (Job* j : s->active) {
      if (j->cancel && j->last_round <= s->completed_round) {  // nothing of it in flight
        finish_job(s, j, j->failed ? NMFA_EDEVICE : NMFA_ECANCELED);
        s->cv_done.notify_all();
        continue;
      }
      keep.push_back(j);
      if (!j->cancel && j->t_sched < j->t_f) jobs.push_back(j);
    }
    s->active.swap(keep);
  }
  if (jobs.empty()) return;
  r.id = s->next_round++;
  std::vector<int> te(jobs.size());
  for (size_t k = 0; k < jobs.size(); ++k) te[k] = std::min(jobs[k]->t_sched + s->p.chunk_iters, jobs[k]->t_f);
  std::vector<Job*> failed;
  auto fail_job = [&](Job* j) {
    j->msg = nmfa_last_error();
    failed.push_back(j);
  };
  auto ran = [&](Job* j, int t_end, int lane, hipStream_t st) {
    j->t_sched = t_end;
    j->lane = lane;
    j->last_round = r.id;
    j->ctx->state_valid = true;  // the next chunk, enqueued behind this one, resumes from its state
    bool last = t_end == j->t_f;
    if (last && ctx_finish_run(j->ctx, st) != NMFA_OK) {
      last = false;
      fail_job(j);
    }
    (void)hipEventRecord(j->ev, st);
    r.ran.push_back(j);
    r.t_end.push_back(t_end);
    r.last.push_back(last ? 1 : 0);
  };

  // requests on the persistent small-N path: one batched launch
  int max_Mp = 0;
  size_t lds = 0;
  std::vector<std::pair<Job*, int>> batched;
  for (size_t k = 0; k < jobs.size(); ++k) {
    Job* j = jobs[k];
    if (j->ctx->path != 0) continue;
    AnnealArgs a{};
    if (ctx_prepare_run(j->ctx, j->R, j->t_f, j->t_sched + 1, te[k], j->seed, s->stream, &a) != NMFA_OK) {
      fail_job(j);
      continue;
    }
    const int job_index = (int)r.h_args.size();
    r.h_args.push_back(a);
    for (int b = 0; b < (j->R + 15) / 16; ++b) r.h_tasks.push_back(make_int2(job_index, b));
    max_Mp = std::max(max_Mp, j->ctx->Mp);
    lds = std::max(lds, small_lds_bytes(j->ctx->prec, j->ctx->Mp, j->ctx->lds_stride));
    batched.emplace_back(j, te[k]);
  }
  if (!batched.empty()) {
    const bool ok =
        ensure_staging(r, (int)r.h_args.size(), (int)r.h_tasks.size()) == NMFA_OK &&
        hipMemcpyAsync(r.d_jobs, r.h_args.data(), sizeof(AnnealArgs) * r.h_args.size(), hipMemcpyHostToDevice,
                       s->stream) == hipSuccess &&
        hipMemcpyAsync(r.d_tasks, r.h_tasks.data(), sizeof(int2) * r.h_tasks.size(), hipMemcpyHostToDevice,
                       s->stream) == hipSuccess &&
        launch_anneal_small_batched(s->p.precision, r.d_jobs, r.d_tasks, (int)r.h_tasks.size(), max_Mp, lds,
                                    s->stream) == hipSuccess;
    if (ok) {
      ++s->st.batched_launches;
      for (auto& jt : batched) ran(jt.first, jt.second, -1, s->stream);
    } else {
      (void)nmfa_fail(NMFA_EDEVICE, "server: batched launch failed");
      for (auto& jt : batched) fail_job(jt.first);
    }
  }

  // the others on their own kernels, over the lanes
  std::vector<int> group_lane, group_cap;
  plan_group_lanes(s, jobs, te, &group_lane, &group_cap);
  for (size_t k = 0; k < jobs.size(); ++k) {
    Job* j = jobs[k];
    if (j->ctx->path == 0) continue;
    const bool group = group_lane[k] >= 0;
    const int lane = group ? group_lane[k] : 1 + (int)(j->id % (SERVER_LANES - 1));
    hipStream_t st = s->lanes[lane];
    if (j->lane != lane && j->lane != -2) (void)hipStreamWaitEvent(st, j->ev, 0);
    if (group) {
      // group launches side by side must fit on the chip together: a whole-chip launch waits for
      // the other lanes' group launches, and later group launches on them wait for it
      if (group_cap[k] == 0) {
        for (int L = 0; L < SERVER_LANES; ++L)
          if (L != lane && s->group_rec[L]) (void)hipStreamWaitEvent(st, s->ev_group[L], 0);
      } else if (s->wide_rec) {
        (void)hipStreamWaitEvent(st, s->ev_wide, 0);
      }
    }
    if (ctx_launch_run(j->ctx, j->R, j->t_f, j->t_sched + 1, te[k], j->seed, st, false, group_cap[k]) != NMFA_OK) {
      fail_job(j);
      continue;
    }
    if (group) {
      (void)hipEventRecord(s->ev_group[lane], st);
      s->group_rec[lane] = true;
      if (group_cap[k] == 0) {
        (void)hipEventRecord(s->ev_wide, st);
        s->wide_rec = true;
      }
    }
    ran(j, te[k], lane, st);
  }
  (void)hipEventRecord(r.ev[0], s->stream);
  for (int L = 0; L < SERVER_LANES; ++L) (void)hipEventRecord(r.ev[1 + L], s->lanes[L]);
  r.inflight = true;
  if (!failed.empty()) {
    // a request whose chunk could not be enqueued fails once nothing of it is in flight
    std::lock_guard<std::mutex> lk(s->mu);
    for (Job* j : failed) {
      j->cancel = true;
      j->failed = true;
    }
  }
}

// Wait for round r and hand over its results: requests whose final chunk it held return their
// energies and spins; cancelled or failed requests with nothing left in flight are retired.
// Returns false on a device error.
bool complete_round(nmfa_server* s, Round& r) {
  hipError_t se = hipSuccess;
  for (hipEvent_t e : r.ev) {
    const hipError_t x = hipEventSynchronize(e);
    if (se == hipSuccess) se = x;
  }
  r.inflight = false;
  std::vector<char> ok(r.ran.size(), 0), read(r.ran.size(), 0);
  {
    std::lock_guard<std::mutex> lk(s->mu);  // cancel flags are set by clients
    for (size_t k = 0; k < r.ran.size(); ++k) read[k] = r.last[k] && !r.ran[k]->cancel;
  }
  for (size_t k = 0; k < r.ran.size(); ++k) {
    Job* j = r.ran[k];
    j->t_done = r.t_end[k];
    if (read[k] && se == hipSuccess) {
      j->E.resize(j->R);
      j->Eint.resize(j->R);
      j->spins.resize((size_t)j->R * j->n);
      const int r3 = ctx_read_results(j->ctx, j->E.data(), j->Eint.data(), j->spins.data());
      ok[k] = r3 == NMFA_OK ? 1 : 0;
      if (r3 != NMFA_OK) j->msg = nmfa_last_error();
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  ++s->st.rounds;
  s->completed_round = r.id;
  bool notify = false;
  for (size_t k = 0; k < r.ran.size(); ++k) {
    Job* j = r.ran[k];
    if (j->last_round != r.id) continue;  // a later chunk is in flight
    if (se != hipSuccess) {
      j->msg = hipGetErrorString(se);
      finish_job(s, j, NMFA_EDEVICE);
    } else if (j->cancel) {
      finish_job(s, j, j->failed ? NMFA_EDEVICE : NMFA_ECANCELED);
    } else if (r.last[k]) {
      finish_job(s, j, ok[k] ? NMFA_JOB_DONE : NMFA_EDEVICE);
    } else {
      continue;
    }
    notify = true;
  }
  std::vector<Job*> keep;
  for (Job* j : s->active)
    if (j->ctx) keep.push_back(j);
  s->active.swap(keep);
  if (notify) {
    s->cv_done.notify_all();
    s->cv_admit.notify_one();
  }
  return se == hipSuccess;
}

void scheduler(nmfa_server* s) {
  (void)hipSetDevice(s->device);
  constexpr size_t kRetireBatch = 64;
  for (;;) {
    const bool busy = s->rounds[0].inflight || s->rounds[1].inflight;
    if (!busy) free_retired(s);  // nothing in flight: freeing stalls nothing
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (!busy) s->cv_work.wait(lk, [&] { return s->stop || !s->active.empty() || s->want_free; });
      if (s->stop && s->queue.empty() && s->active.empty() && !busy) break;  // the admission thread retires what it still sets up
    }
    // round k+1 is enqueued before round k is waited for, so that the device has the next round
    // queued while the host collects results
    Round& r = s->rounds[s->rounds[0].inflight ? 1 : 0];
    Round& other = s->rounds[&r == &s->rounds[0] ? 1 : 0];
    enqueue_round(s, r);
    Round* wait = nullptr;
    if (r.inflight && other.inflight) wait = other.id < r.id ? &other : &r;
    else if (!r.inflight && other.inflight) wait = &other;
    if (wait && !complete_round(s, *wait)) {
      // after a device error, drain the other round too; its requests fail with it
      Round& o = wait == &r ? other : r;
      if (o.inflight) {
        {
          std::lock_guard<std::mutex> lk(s->mu);
          for (Job* j : o.ran) {
            j->cancel = true;
            j->failed = true;
            if (j->msg.empty()) j->msg = "device error in the previous round";
          }
        }
        (void)complete_round(s, o);
      }
    }
    bool free_now;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      free_now = s->want_free || s->retired.size() >= kRetireBatch;
    }
    if (free_now) free_retired(s);
  }
  free_retired(s);
}

}  // namespace

// Streams, events and staging of a server whose scheduler thread has ended (or never started).
static void destroy_server_resources(nmfa_server* s) {
  for (Round& r : s->rounds) {
    (void)hipFree(r.d_jobs);
    (void)hipFree(r.d_tasks);
    for (hipEvent_t e : r.ev)
      if (e) (void)hipEventDestroy(e);
  }
  for (hipEvent_t e : s->ev_group)
    if (e) (void)hipEventDestroy(e);
  if (s->ev_wide) (void)hipEventDestroy(s->ev_wide);
  for (hipStream_t ls : s->lanes)
    if (ls) (void)hipStreamDestroy(ls);
  delete s;
}

extern "C" int nmfa_server_create(const nmfa_server_params* p, nmfa_server** out) {
  if (!out) return nmfa_fail(NMFA_EINVAL, "nmfa_server_create: out is NULL");
  *out = nullptr;
  nmfa_server_params dp;
  nmfa_server_params_default(&dp);
  if (!p) p = &dp;
  if (p->struct_size != sizeof(nmfa_server_params))
    return nmfa_fail(NMFA_EINVAL, "nmfa_server_create: params.struct_size mismatch");
  if (p->precision > NMFA_FP8J_FP8S || p->max_active < 1 || p->chunk_iters < 1 || p->hbm_budget_bytes == 0)
    return nmfa_fail(NMFA_EINVAL, "nmfa_server_create: invalid parameters");
  nmfa_server* s = new nmfa_server();
  s->p = *p;
  // Non-blocking streams, so that uploads of newly admitted requests (null stream) overlap the
  // running rounds. Three of them: with the null stream that is HIP's default of four hardware
  // queues per process, so that no copy waits behind a kernel that merely shares its queue. The
  // batched small-N launch shares the last lane.
  bool ok = hipGetDevice(&s->device) == hipSuccess;
  for (hipStream_t& ls : s->lanes) ok = ok && hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) == hipSuccess;
  s->stream = s->lanes[SERVER_LANES - 1];
  if (!ok) {
    destroy_server_resources(s);
    return nmfa_fail(NMFA_EDEVICE, "nmfa_server_create: no HIP device / stream");
  }
  if (hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess || s->cus < 8)
    s->cus = 8;
  bool ev_ok = hipEventCreateWithFlags(&s->ev_wide, hipEventDisableTiming) == hipSuccess;
  for (hipEvent_t& e : s->ev_group) ev_ok = ev_ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  for (Round& r : s->rounds)
    for (hipEvent_t& e : r.ev) ev_ok = ev_ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ev_ok) {
    destroy_server_resources(s);
    return nmfa_fail(NMFA_EDEVICE, "nmfa_server_create: event creation failed");
  }
  s->worker = std::thread(scheduler, s);
  s->admitter = std::thread(admitter, s);
  *out = s;
  return NMFA_OK;
}

extern "C" int nmfa_server_submit(nmfa_server* s, int32_t n, const double* J, const double* h, int32_t R,
                                  int32_t t_f, uint64_t seed, uint64_t* ticket) {
  if (!s || !J || !ticket) return nmfa_fail(NMFA_EINVAL, "nmfa_server_submit: NULL argument");
  if (n < 1 || n > 16384 || R < 1 || R > (1 << 24) || t_f < 1)
    return nmfa_fail(NMFA_EINVAL, "nmfa_server_submit: n, R or t_f out of range");
  Job* j = new Job();
  j->n = n;
  j->R = R;
  j->t_f = t_f;
  j->seed = seed;
  j->J.assign(J, J + (size_t)n * n);
  if (h) j->h.assign(h, h + n);
  bool integral = true;
  for (double v : j->J)
    if (!(std::isfinite(v) && v == std::floor(v) && std::fabs(v) <= 127)) {
      integral = false;
      break;
    }
  j->bytes = job_bytes(n, R, t_f, integral);
  j->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete j;
      return nmfa_fail(NMFA_ESTATE, "nmfa_server_submit: server is stopping");
    }
    j->id = s->next_id++;
    s->jobs[j->id] = j;
    s->queue.push_back(j);
    ++s->st.submitted;
    *ticket = j->id;
  }
  s->cv_admit.notify_one();
  return NMFA_OK;
}

static Job* find_job(nmfa_server* s, uint64_t ticket) {
  auto it = s->jobs.find(ticket);
  return it == s->jobs.end() ? nullptr : it->second;
}

static bool finished(const Job* j) { return j->status == NMFA_JOB_DONE || j->status < 0; }

extern "C" int nmfa_server_poll(nmfa_server* s, uint64_t ticket, int32_t* status) {
  if (!s || !status) return nmfa_fail(NMFA_EINVAL, "nmfa_server_poll: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return nmfa_fail(NMFA_EINVAL, "nmfa_server_poll: unknown ticket");
  *status = j->status;
  return NMFA_OK;
}

extern "C" int nmfa_server_wait(nmfa_server* s, uint64_t ticket, int32_t timeout_ms) {
  if (!s) return nmfa_fail(NMFA_EINVAL, "nmfa_server_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return nmfa_fail(NMFA_EINVAL, "nmfa_server_wait: unknown ticket");
  auto pred = [&] { return finished(j); };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, pred);
    return NMFA_OK;
  }
  if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
    return nmfa_fail(NMFA_ESTATE, "nmfa_server_wait: timed out");
  return NMFA_OK;
}

extern "C" int nmfa_server_result(nmfa_server* s, uint64_t ticket, double* E, int64_t* E_int, int8_t* spins,
                                  double* latency_ms) {
  if (!s) return nmfa_fail(NMFA_EINVAL, "nmfa_server_result: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return nmfa_fail(NMFA_EINVAL, "nmfa_server_result: unknown ticket");
  if (j->status < 0) return nmfa_fail(j->status, "request failed: %s", j->msg.c_str());
  if (j->status != NMFA_JOB_DONE) return nmfa_fail(NMFA_ESTATE, "nmfa_server_result: request not finished");
  if (E) std::copy(j->E.begin(), j->E.end(), E);
  if (E_int) std::copy(j->Eint.begin(), j->Eint.end(), E_int);
  if (spins) std::copy(j->spins.begin(), j->spins.end(), spins);
  if (latency_ms) *latency_ms = (j->t_finish - j->t_submit) * 1e3;
  return NMFA_OK;
}

extern "C" int nmfa_server_release(nmfa_server* s, uint64_t ticket) {
  if (!s) return nmfa_fail(NMFA_EINVAL, "nmfa_server_release: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return nmfa_fail(NMFA_EINVAL, "nmfa_server_release: unknown ticket");
  if (!finished(j)) return nmfa_fail(NMFA_ESTATE, "nmfa_server_release: request not finished");
  s->jobs.erase(ticket);
  delete j;
  return NMFA_OK;
}

extern "C" int nmfa_server_cancel(nmfa_server* s, uint64_t ticket) {
  if (!s) return nmfa_fail(NMFA_EINVAL, "nmfa_server_cancel: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return nmfa_fail(NMFA_EINVAL, "nmfa_server_cancel: unknown ticket");
  if (finished(j)) return nmfa_fail(NMFA_ESTATE, "nmfa_server_cancel: request already finished");
  auto it = std::find(s->queue.begin(), s->queue.end(), j);
  if (it != s->queue.end()) {
    s->queue.erase(it);
    j->status = NMFA_ECANCELED;
    j->t_finish = now_s();
    ++s->st.cancelled;
    s->cv_done.notify_all();
  } else {
    j->cancel = true;
  }
  return NMFA_OK;
}

extern "C" int nmfa_server_stats_get(nmfa_server* s, nmfa_server_stats* out) {
  if (!s || !out) return nmfa_fail(NMFA_EINVAL, "nmfa_server_stats_get: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = s->queue.size();
  out->active = s->active.size();
  out->bytes_in_use = s->used_bytes;
  out->peak_bytes = s->peak_bytes;
  return NMFA_OK;
}

extern "C" void nmfa_server_destroy(nmfa_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Job* j : s->queue) {
      j->status = NMFA_ECANCELED;
      ++s->st.cancelled;
    }
    s->queue.clear();
    for (Job* j : s->active) j->cancel = true;
  }
  s->cv_work.notify_all();
  s->cv_admit.notify_all();
  if (s->admitter.joinable()) s->admitter.join();
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  free_retired(s);  // set-ups that ended after the scheduler
  for (auto& kv : s->jobs) {
    if (kv.second->ctx) nmfa_destroy(kv.second->ctx);
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    delete kv.second;
  }
  destroy_server_resources(s);
}
