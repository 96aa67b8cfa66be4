// Serving loop for leverage-score jobs (host code).
//
// A server owns a fixed number of slots. Each slot has a library context
// (with its own device workspace), a HIP stream of default priority and a
// worker thread. Jobs arrive at any time through slso_server_submit and wait
// in a queue. A worker takes the next job when it is idle and the job fits
// the server's HBM budget. Jobs on different slots run concurrently on their
// own streams, so their sketch, QR, scoring and ordering kernels overlap on
// the device.
//
// The budget counts the workspace each slot holds; inputs and outputs belong
// to the caller and are already resident. A slot's capacity only grows while
// it is in use. When the job at the head of the queue does not fit because
// idle slots still hold memory, those slots release their workspaces.
// Admission is first-in first-out, with backfilling: a later job that fits
// may start while the head waits for memory. The head may be bypassed at most
// 2 * slots times before backfilling stops.
//
// Each job's result equals the result of the same slso_leverage (+ slso_order)
// call made alone: every kernel sums in a fixed order, so the result does not
// depend on what else runs on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "slso.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  int64_t ticket = 0;
  slso_job desc{};
  size_t need = 0;  // workspace the job's context allocates
  double submit_ms = 0, start_ms = 0, end_ms = 0;
  int status = 0;
  int slot = -1;
  slso_info info{};
  bool done = false;
};

struct Slot {
  slso_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  size_t cap = 0;  // workspace bytes this slot's context may hold
  Job* cur = nullptr;
  std::thread th;
};

}  // namespace

struct slso_server {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::unordered_map<int64_t, std::unique_ptr<Job>> jobs;
  std::vector<Slot> slots;
  int64_t next_ticket = 1;
  int64_t head_bypass = 0;
  bool stop = false;
  size_t allocated = 0;
  int running = 0;
  int max_running = 0;
  int64_t completed = 0;
  Clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
  bool fits(const Slot& s, const Job* j) const {
    const size_t after = allocated - s.cap + std::max(s.cap, j->need);
    return after <= budget;
  }
  size_t busy_cap() const {
    size_t b = 0;
    for (const Slot& s : slots)
      if (s.cur) b += s.cap;
    return b;
  }
};

namespace {

// Next job for idle slot i, or nullptr; called with the lock held.
Job* pick(slso_server* S, int i) {
  Slot& sl = S->slots[i];
  if (S->queue.empty()) return nullptr;
  Job* head = S->queue.front();
  if (!S->fits(sl, head) && sl.cap > 0 &&
      S->busy_cap() + head->need <= S->budget) {
    // the head waits only for memory held by idle slots: release this one
    (void)slso::ctx_release_workspace(sl.ctx);
    S->allocated -= sl.cap;
    sl.cap = 0;
  }
  if (S->fits(sl, head)) {
    S->queue.pop_front();
    S->head_bypass = 0;
    return head;
  }
  if (S->head_bypass >= 2 * static_cast<int64_t>(S->slots.size()))
    return nullptr;
  for (auto it = S->queue.begin() + 1; it != S->queue.end(); ++it) {
    if (S->fits(sl, *it)) {
      Job* j = *it;
      S->queue.erase(it);
      ++S->head_bypass;
      return j;
    }
  }
  return nullptr;
}

void worker(slso_server* S, int i) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    Job* j = pick(S, i);
    if (!j) {
      if (S->stop && S->queue.empty()) break;
      S->cv_work.wait(lk);
      continue;
    }
    Slot& sl = S->slots[i];
    size_t grow = 0;
    if (j->need > sl.cap) {
      // reserve before the context grows, with headroom (up to twice the
      // job's need, within the slot's share of the budget and the budget
      // left) so that later jobs rarely make it grow again: a workspace
      // that grows frees its old buffer, which waits for the whole device
      size_t want = j->need;
      const size_t share = S->budget / S->slots.size();
      // (whole 2 MiB units: the granularity the context allocates in)
      const size_t head = std::min(2 * j->need, share) >> 21 << 21;
      if (head > want && S->allocated - sl.cap + head <= S->budget) want = head;
      S->allocated += want - sl.cap;
      sl.cap = want;
      grow = want;
    }
    sl.cur = j;
    j->slot = i;
    j->start_ms = S->now_ms();
    S->running++;
    S->max_running = std::max(S->max_running, S->running);
    lk.unlock();

    const slso_job& d = j->desc;
    int st = grow ? slso::ctx_reserve_workspace(sl.ctx, grow) : SLSO_OK;
    // the job as one enqueue (no host wait between its stages) when its
    // options allow; the rare cases the device path leaves to the host are
    // rerun by slso_leverage_finish
    slso_options o = d.opt;
    const bool ns = o.refine == 0 &&
                    (o.flags & (SLSO_OPT_EPS_HAT | SLSO_OPT_SVD_RANK)) == 0;
    if (ns) o.flags |= SLSO_OPT_NO_SYNC;
    if (st >= 0)
      st = slso_leverage(sl.ctx, &d.X, d.seed, d.r, d.k, &o, d.scores, &j->info,
                         sl.stream);
    const bool pending = ns && st >= 0;
    if (st >= 0 && d.perm) {
      const int so = slso_order(sl.ctx, d.scores, d.X.n, d.perm, sl.stream);
      if (so < 0) st = so;
    }
    if (hipStreamSynchronize(sl.stream) != hipSuccess && st >= 0)
      st = SLSO_EDEVICE;
    if (pending) {
      const int fs = slso_leverage_finish(sl.ctx, &j->info);
      if (st >= 0) st = fs;
      if (st >= 0 && (j->info.flags & SLSO_INFO_RERUN) && d.perm) {
        const int so = slso_order(sl.ctx, d.scores, d.X.n, d.perm, sl.stream);
        if (so < 0) st = so;
        if (hipStreamSynchronize(sl.stream) != hipSuccess && st >= 0)
          st = SLSO_EDEVICE;
      }
    }

    lk.lock();
    j->status = st;
    j->end_ms = S->now_ms();
    j->done = true;
    sl.cur = nullptr;
    S->running--;
    S->completed++;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

void fill_result(const Job* j, slso_job_result* res) {
  if (!res) return;
  res->status = j->status;
  res->slot = j->slot;
  res->info = j->info;
  res->submit_ms = j->submit_ms;
  res->start_ms = j->start_ms;
  res->end_ms = j->end_ms;
}

}  // namespace

extern "C" {

int slso_server_create(slso_server** out, int device, int slots,
                       size_t hbm_budget) {
  if (!out || slots < 1 || slots > 64 || hbm_budget == 0) return SLSO_EINVAL;
  *out = nullptr;
  auto* S = new slso_server();
  S->device = device;
  S->budget = hbm_budget;
  S->t0 = Clock::now();
  S->slots.resize(static_cast<size_t>(slots));
  int st = SLSO_OK;
  for (Slot& sl : S->slots) {
    st = slso_create(&sl.ctx, device, 0);
    if (st) break;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
      st = SLSO_EDEVICE;
      break;
    }
  }
  if (st) {
    for (Slot& sl : S->slots) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.ctx) (void)slso_destroy(sl.ctx);
    }
    delete S;
    return st;
  }
  for (int i = 0; i < slots; ++i)
    S->slots[static_cast<size_t>(i)].th = std::thread(worker, S, i);
  *out = S;
  return SLSO_OK;
}

int slso_server_submit(slso_server* S, const slso_job* job, int64_t* ticket) {
  if (!S || !job || !ticket) return SLSO_EINVAL;
  if (!job->scores) return SLSO_EINVAL;
  size_t need = 0;
  const int st = slso_workspace_size(&job->X, job->r, job->k, &job->opt, &need);
  if (st) return st;
  if (need > S->budget) return SLSO_ENOMEM;
  auto j = std::make_unique<Job>();
  j->desc = *job;
  j->need = need;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return SLSO_EINVAL;
  j->ticket = S->next_ticket++;
  j->submit_ms = S->now_ms();
  *ticket = j->ticket;
  S->queue.push_back(j.get());
  S->jobs.emplace(j->ticket, std::move(j));
  S->cv_work.notify_all();
  return SLSO_OK;
}

int slso_server_poll(slso_server* S, int64_t ticket, slso_job_result* res) {
  if (!S) return SLSO_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return SLSO_EINVAL;
  if (!it->second->done) return 0;
  fill_result(it->second.get(), res);
  S->jobs.erase(it);
  return 1;
}

int slso_server_wait(slso_server* S, int64_t ticket, slso_job_result* res) {
  if (!S) return SLSO_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return SLSO_EINVAL;
  Job* j = it->second.get();
  S->cv_done.wait(lk, [j] { return j->done; });
  fill_result(j, res);
  S->jobs.erase(ticket);
  return SLSO_OK;
}

int slso_server_stats(slso_server* S, slso_server_counters* out) {
  if (!S || !out) return SLSO_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  out->queued = static_cast<int64_t>(S->queue.size());
  out->running = S->running;
  out->max_running = S->max_running;
  out->completed = S->completed;
  out->allocated_bytes = S->allocated;
  out->budget_bytes = S->budget;
  return SLSO_OK;
}

int slso_server_destroy(slso_server* S) {
  if (!S) return SLSO_EINVAL;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  for (Slot& sl : S->slots)
    if (sl.th.joinable()) sl.th.join();
  for (Slot& sl : S->slots) {
    (void)slso_destroy(sl.ctx);
    (void)hipStreamDestroy(sl.stream);
  }
  delete S;
  return SLSO_OK;
}

}  // extern "C"
