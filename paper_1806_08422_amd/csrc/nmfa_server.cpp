// Continuous-batching annealing server (nmfa_server_* in include/nmfa.h).
//
// One scheduler thread owns four HIP streams. Requests wait in a FIFO queue; admission is by
// device memory budget and a cap on concurrently admitted requests. Admitted requests are
// advanced in rounds of chunk_iters iterations of Algorithm 1:
//   * all admitted requests on the persistent small-N path share ONE launch per round
//     (anneal_small_batched over every request's replica blocks; each workgroup reads its own
//     request's arguments), so newly admitted work overlaps with running work on the device;
//   * larger requests advance by the same chunk on their own kernels in the same round, on the
//     other three streams, so that their kernels run side by side with the batched launch and
//     with each other. The workgroups of one persistent XCD-group launch wait for each other, so
//     group launches run side by side only where all of them fit on the chip at once: each of
//     the three streams has a workgroup budget (half, a quarter and a quarter of the CUs, in
//     multiples of the XCD count), each group launch on a stream is capped at that stream's
//     budget (a request that needs more takes several launches in turn), and a stream runs one
//     launch at a time, so the resident group workgroups never exceed the CUs. Requests go to the
//     stream that would finish them first (largest first). A round with a single group request
//     gives it the whole chip. The sparse and per-iteration kernels never wait for other
//     workgroups, so they spread over the second and third streams and at worst delay a group
//     launch's start;
//   * between rounds the spin state stays on the device (resuming is bit-exact), finished
//     requests return their energies/spins and release their memory, and queued requests are
//     admitted.
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
  nmfa_ctx* ctx = nullptr;
  int t_done = 0;
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

constexpr int SERVER_LANES = 3;  // streams besides the batched launch's (4 hardware queues in all)

struct nmfa_server {
  nmfa_server_params p{};
  int device = 0;
  hipStream_t stream = nullptr;            // the batched small-N launch
  hipStream_t lanes[SERVER_LANES] = {};    // group kernels on all three; sparse, per-iteration on [1..]
  int cus = 256;                           // compute units of the device
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::vector<Job*> active;  // touched by the scheduler thread only (plus stats under mu)
  std::unordered_map<uint64_t, Job*> jobs;
  size_t used_bytes = 0, peak_bytes = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  AnnealArgs* d_jobs = nullptr;
  int cap_jobs = 0;
  int2* d_tasks = nullptr;
  int cap_tasks = 0;
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

// Finish a request (under the lock): record the outcome, free its device memory and budget.
void finish_job(nmfa_server* s, Job* j, int status) {
  if (j->ctx) {
    nmfa_destroy(j->ctx);
    j->ctx = nullptr;
  }
  j->status = status;
  j->t_finish = now_s();
  s->used_bytes -= std::min(s->used_bytes, j->bytes);
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
  auto iters = [&](int k) { return (double)(t_end[k] - jobs[k]->t_done); };
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

int ensure_staging(nmfa_server* s, int n_jobs, int n_tasks) {
  if (n_jobs > s->cap_jobs) {
    (void)hipFree(s->d_jobs);
    s->d_jobs = nullptr;
    const int cap = std::max(n_jobs, 2 * s->cap_jobs);
    if (hipMalloc(&s->d_jobs, sizeof(AnnealArgs) * cap) != hipSuccess) return NMFA_ENOMEM;
    s->cap_jobs = cap;
  }
  if (n_tasks > s->cap_tasks) {
    (void)hipFree(s->d_tasks);
    s->d_tasks = nullptr;
    const int cap = std::max(n_tasks, 2 * s->cap_tasks);
    if (hipMalloc(&s->d_tasks, sizeof(int2) * cap) != hipSuccess) return NMFA_ENOMEM;
    s->cap_tasks = cap;
  }
  return NMFA_OK;
}

// Admit queued requests (FIFO by device memory budget and slots; the head of the queue is never
// overtaken) and upload their instances. Runs while the previous round's kernels execute: the
// server's streams do not synchronise with the null stream that the uploads use.
void admit_queued(nmfa_server* s) {
  std::vector<Job*> admitted;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->queue.empty() && (int)(s->active.size() + admitted.size()) < s->p.max_active) {
      Job* j = s->queue.front();
      if (j->bytes > s->p.hbm_budget_bytes) {
        s->queue.pop_front();
        j->msg = "request needs more device memory than the whole budget";
        j->bytes = 0;  // never charged to the budget
        finish_job(s, j, NMFA_ENOMEM);
        s->cv_done.notify_all();
        continue;
      }
      if (s->used_bytes + j->bytes > s->p.hbm_budget_bytes) break;
      s->queue.pop_front();
      s->used_bytes += j->bytes;
      s->peak_bytes = std::max(s->peak_bytes, s->used_bytes);
      admitted.push_back(j);
    }
  }
  for (Job* j : admitted) {  // outside the lock
    nmfa_params prm;
    nmfa_params_default(&prm);
    prm.precision = s->p.precision;
    nmfa_ctx* c = nullptr;
    const int rc = nmfa_create(j->n, j->J.data(), j->h.empty() ? nullptr : j->h.data(), &prm, &c);
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc != NMFA_OK) {
      j->msg = nmfa_last_error();
      finish_job(s, j, rc);
      s->cv_done.notify_all();
      continue;
    }
    j->ctx = c;
    std::vector<double>().swap(j->J);
    std::vector<double>().swap(j->h);
    j->status = NMFA_JOB_RUNNING;
    s->active.push_back(j);
  }
}

void scheduler(nmfa_server* s) {
  (void)hipSetDevice(s->device);
  std::vector<AnnealArgs> h_args;
  std::vector<int2> h_tasks;
  for (;;) {
    bool idle;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
      if (s->stop && s->queue.empty() && s->active.empty()) break;
      idle = s->active.empty();
    }
    if (idle) admit_queued(s);  // nothing runs yet to overlap the uploads with

    // ---- one round ---------------------------------------------------------------------
    std::vector<Job*> round_jobs;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      std::vector<Job*> keep;
      for (Job* j : s->active) {
        if (j->cancel) {
          finish_job(s, j, NMFA_ECANCELED);
          s->cv_done.notify_all();
        } else {
          keep.push_back(j);
        }
      }
      s->active.swap(keep);
      round_jobs = s->active;
    }
    if (round_jobs.empty()) continue;

    int rc = NMFA_OK;
    std::vector<Job*> ran;
    std::vector<int> t_end_of(round_jobs.size());
    h_args.clear();
    h_tasks.clear();
    int max_Mp = 0;
    size_t lds = 0;
    int prec = s->p.precision;
    std::vector<Job*> batched;
    for (size_t k = 0; k < round_jobs.size(); ++k) {
      Job* j = round_jobs[k];
      const int tb = j->t_done + 1;
      const int te = std::min(j->t_done + s->p.chunk_iters, j->t_f);
      t_end_of[k] = te;
      if (j->ctx->path == 0) {
        AnnealArgs a{};
        int r2 = ctx_prepare_run(j->ctx, j->R, j->t_f, tb, te, j->seed, s->stream, &a);
        if (r2 != NMFA_OK) {
          std::lock_guard<std::mutex> lk(s->mu);
          j->msg = nmfa_last_error();
          finish_job(s, j, r2);
          s->cv_done.notify_all();
          continue;
        }
        const int job_index = (int)h_args.size();
        h_args.push_back(a);
        for (int b = 0; b < (j->R + 15) / 16; ++b) h_tasks.push_back(make_int2(job_index, b));
        max_Mp = std::max(max_Mp, j->ctx->Mp);
        lds = std::max(lds, small_lds_bytes(j->ctx->prec, j->ctx->Mp, j->ctx->lds_stride));
        batched.push_back(j);
      }
    }
    if (!batched.empty()) {
      rc = ensure_staging(s, (int)h_args.size(), (int)h_tasks.size());
      if (rc == NMFA_OK &&
          (hipMemcpyAsync(s->d_jobs, h_args.data(), sizeof(AnnealArgs) * h_args.size(), hipMemcpyHostToDevice,
                          s->stream) != hipSuccess ||
           hipMemcpyAsync(s->d_tasks, h_tasks.data(), sizeof(int2) * h_tasks.size(), hipMemcpyHostToDevice,
                          s->stream) != hipSuccess ||
           launch_anneal_small_batched(prec, s->d_jobs, s->d_tasks, (int)h_tasks.size(), max_Mp, lds, s->stream) !=
               hipSuccess))
        rc = NMFA_EDEVICE;
      if (rc == NMFA_OK) {
        ++s->st.batched_launches;
        for (Job* j : batched) ran.push_back(j);
      }
    }
    int spread = 0;
    std::vector<hipStream_t> stream_of(round_jobs.size(), s->stream);
    std::vector<int> group_lane, group_cap;
    plan_group_lanes(s, round_jobs, t_end_of, &group_lane, &group_cap);
    for (size_t k = 0; k < round_jobs.size() && rc == NMFA_OK; ++k) {
      Job* j = round_jobs[k];
      if (!j->ctx || j->ctx->path == 0) continue;
      const int te = t_end_of[k];
      stream_of[k] = group_lane[k] >= 0 ? s->lanes[group_lane[k]] : s->lanes[1 + (spread++ % (SERVER_LANES - 1))];
      int r2 = ctx_launch_run(j->ctx, j->R, j->t_f, j->t_done + 1, te, j->seed, stream_of[k], false, group_cap[k]);
      if (r2 != NMFA_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        j->msg = nmfa_last_error();
        finish_job(s, j, r2);
        s->cv_done.notify_all();
        continue;
      }
      ran.push_back(j);
    }
    // energies of the requests that complete in this round
    std::vector<Job*> done;
    for (Job* j : ran) {
      const size_t k = std::find(round_jobs.begin(), round_jobs.end(), j) - round_jobs.begin();
      if (t_end_of[k] == j->t_f) {
        if (ctx_finish_run(j->ctx, stream_of[k]) != NMFA_OK) rc = NMFA_EDEVICE;
        done.push_back(j);
      }
    }
    // requests admitted now upload while the round runs and join the next one
    if (rc == NMFA_OK) admit_queued(s);
    hipError_t se = hipStreamSynchronize(s->stream);
    for (hipStream_t ls : s->lanes) {
      const hipError_t e = hipStreamSynchronize(ls);
      if (se == hipSuccess) se = e;
    }
    ++s->st.rounds;
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc != NMFA_OK || se != hipSuccess) {
      // a device failure ends every request of the round
      for (Job* j : ran) {
        j->msg = se != hipSuccess ? hipGetErrorString(se) : "launch failed in the scheduler";
        finish_job(s, j, NMFA_EDEVICE);
      }
      std::vector<Job*> keep;
      for (Job* j : s->active)
        if (j->ctx) keep.push_back(j);
      s->active.swap(keep);
      s->cv_done.notify_all();
      continue;
    }
    for (Job* j : ran) {
      const size_t k = std::find(round_jobs.begin(), round_jobs.end(), j) - round_jobs.begin();
      j->t_done = t_end_of[k];
      j->ctx->state_valid = true;  // the next round resumes from this state
    }
    for (Job* j : done) {
      j->E.resize(j->R);
      j->Eint.resize(j->R);
      j->spins.resize((size_t)j->R * j->n);
      int r3 = nmfa_energies(j->ctx, j->E.data(), j->Eint.data());
      if (r3 == NMFA_OK) r3 = nmfa_spins(j->ctx, j->spins.data(), 0);
      if (r3 != NMFA_OK) j->msg = nmfa_last_error();
      finish_job(s, j, r3 == NMFA_OK ? NMFA_JOB_DONE : r3);
    }
    std::vector<Job*> keep;
    for (Job* j : s->active)
      if (j->ctx) keep.push_back(j);
    s->active.swap(keep);
    if (!done.empty()) s->cv_done.notify_all();
  }
}

}  // namespace

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
  // non-blocking streams: uploads of newly admitted requests (null stream) overlap the running round
  bool ok = hipGetDevice(&s->device) == hipSuccess &&
            hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
  for (hipStream_t& ls : s->lanes) ok = ok && hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    for (hipStream_t ls : s->lanes)
      if (ls) (void)hipStreamDestroy(ls);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return nmfa_fail(NMFA_EDEVICE, "nmfa_server_create: no HIP device / stream");
  }
  if (hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess || s->cus < 8)
    s->cus = 8;
  s->worker = std::thread(scheduler, s);
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
  s->cv_work.notify_one();
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
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->jobs) {
    if (kv.second->ctx) nmfa_destroy(kv.second->ctx);
    delete kv.second;
  }
  (void)hipFree(s->d_jobs);
  (void)hipFree(s->d_tasks);
  (void)hipStreamDestroy(s->stream);
  for (hipStream_t ls : s->lanes) (void)hipStreamDestroy(ls);
  delete s;
}
