// Continuous-batching server for MMFD solves.
//
// A scheduler thread owns the GPU work.  Each quantum it
//   1. enqueues one batched run that advances every active slot by
//      min(quantum, remaining steps) on the server stream (asynchronous),
//   2. while that runs, admits queued requests in arrival order as long as a
//      slot is free and the HBM budget holds the new request's device bytes
//      (solver creation and the host-to-device copy use a separate stream),
//   3. waits for the run, then retires finished slots: copies each result to
//      the caller's buffer, stamps its completion time and frees its memory.
// Requests that arrive while others are on the GPU therefore join at the next
// quantum and their steps run in the same launches as the older requests.
// The first quantum that holds a kind the blocked batch kernel takes runs the
// batch autotuner once for that kind.
// Latency is measured from submission to the moment the result is in the
// caller's buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mfd.h"
#include "batch.h"
#include "solver.h"

namespace mfd {

namespace {
using Clock = std::chrono::steady_clock;
double secs(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}
}  // namespace

struct Ticket {
  mfd_request req;
  Clock::time_point t_submit, t_admit, t_done;
  int state = 0;  // 0 queued, 1 running, 2 done, < 0 failed
  int error = 0;
  mfd_solver *solver = nullptr;
  int64_t remaining = 0;
  int64_t bytes = 0;
  int64_t lups = 0;
};

struct Server {
  int64_t budget = 0, used = 0;
  int max_slots = 0;
  int64_t quantum = 0;
  hipStream_t run_stream = nullptr, admit_stream = nullptr;
  mfd_batch *batch = nullptr;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<int64_t> pending;
  std::map<int64_t, Ticket> tickets;
  std::vector<Ticket *> active;  // touched by the scheduler thread only
  int64_t next_id = 1;
  bool stop = false;
  std::thread th;
  std::vector<double> latencies;
  int64_t completed = 0, failed = 0, lups_done = 0;
  Clock::time_point t_first{}, t_last{};
  bool have_first = false;

  static int64_t request_bytes(const mfd_request &r, int64_t *state_bytes) {
    const int dim = 2;
    const int64_t N = r.n[0] * r.n[1];
    const int nf = r.eq == MFD_NSE ? 1 + dim : 1;
    const int64_t es = r.precision == MFD_FP64 ? 8 : 4;
    *state_bytes = nf * N * es;
    // level ring of three moment buffers + reduction scratch
    return 3 * nf * N * es + (64 << 10);
  }

  int admit(Ticket &t) {
    const mfd_request &r = t.req;
    mfd_grid g{};
    g.dim = 2;
    g.precision = r.precision;
    g.form = MFD_MMFD;
    g.n[0] = r.n[0];
    g.n[1] = r.n[1];
    g.n[2] = 1;
    g.dx = r.dx;
    mfd_solver *s = nullptr;
    int rc = mfd_create(&s, &g);
    if (rc < 0) return rc;
    rc = mfd_set_lattice(s, r.lattice, r.d0);
    if (rc >= 0) rc = mfd_set_equation(s, r.eq, &r.ep);
    if (rc >= 0)
      rc = mfd_set_scheme(s, r.kind, r.a, r.kind == MFD_THREE_LEVEL ? r.ah : nullptr, nullptr,
                          nullptr, 1.0, 0, r.dt);
    if (rc >= 0) rc = mfd_set_stream(s, admit_stream);
    int64_t sb = 0;
    request_bytes(r, &sb);
    if (rc >= 0) rc = mfd_set_state(s, 0, r.state0, sb, 0, 0);
    if (rc >= 0 && r.prev0 && r.kind == MFD_THREE_LEVEL) rc = mfd_set_state(s, 1, r.prev0, sb, 0, 0);
    if (rc < 0) {
      mfd_destroy(s);
      return rc;
    }
    mfd_set_stream(s, run_stream);
    t.solver = s;
    return MFD_OK;
  }

  void retire(Ticket &t) {
    int64_t sb = 0;
    request_bytes(t.req, &sb);
    int rc = MFD_OK;
    if (t.req.result_out) {
      if (t.req.result_bytes != sb) rc = MFD_E_ARG;
      else rc = mfd_get_state(t.solver, 0, t.req.result_out, sb, 0, 0);
    }
    mfd_destroy(t.solver);
    t.solver = nullptr;
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(mu);
    used -= t.bytes;
    t.t_done = now;
    if (rc < 0) {
      t.state = -1;
      t.error = rc;
      ++failed;
    } else {
      t.state = 2;
      ++completed;
      lups_done += t.lups;
      if (!t.req.exclude_from_stats) latencies.push_back(secs(t.t_submit, now));
      if (!have_first) {
        t_first = t.t_submit;
        have_first = true;
      }
      t_last = now;
    }
    cv_done.notify_all();
  }

  void loop() {
    while (true) {
      // ---- enqueue a quantum for the active slots
      bool ran = false;
      std::vector<std::pair<Ticket *, int64_t>> advanced;  // (slot, steps)
      if (!active.empty()) {
        mfd_batch_clear(batch);
        Batch *bp = reinterpret_cast<Batch *>(batch);
        bool untuned = false;
        for (Ticket *t : active) {
          const int64_t k = std::min(quantum, t->remaining);
          mfd_batch_add(batch, t->solver, k, nullptr);
          advanced.push_back({t, k});
          const BatchKey key = batch_key_of(reinterpret_cast<Solver *>(t->solver));
          if (batch_blockable(key) && !bp->tuned.count(key)) untuned = true;
        }
        // the first quantum holding a blockable kind picks its launch plan
        if (untuned) mfd_batch_autotune(batch);
        if (mfd_batch_run(batch) == MFD_OK) ran = true;
      }
      // ---- admit while the quantum runs
      std::vector<Ticket *> to_admit;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (!ran && active.empty()) {
          cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return stop || !pending.empty(); });
        }
        if (stop && pending.empty() && active.empty()) return;
        while (!pending.empty() && (int)(active.size() + to_admit.size()) < max_slots) {
          Ticket &t = tickets[pending.front()];
          if (used + t.bytes > budget) {
            if (t.bytes > budget) {  // can never fit
              t.state = -1;
              t.error = MFD_E_BUDGET;
              ++failed;
              pending.pop_front();
              cv_done.notify_all();
              continue;
            }
            break;
          }
          used += t.bytes;
          to_admit.push_back(&t);
          pending.pop_front();
        }
      }
      std::vector<Ticket *> admitted;
      for (Ticket *tp : to_admit) {
        const int rc = admit(*tp);
        std::lock_guard<std::mutex> lk(mu);
        if (rc < 0) {
          tp->state = -1;
          tp->error = rc;
          used -= tp->bytes;
          ++failed;
          cv_done.notify_all();
        } else {
          tp->state = 1;
          tp->t_admit = Clock::now();
          admitted.push_back(tp);
        }
      }
      // ---- finish the quantum and retire finished slots
      if (ran) mfd_batch_wait(batch);
      std::vector<Ticket *> still;
      for (auto &ak : advanced) {
        Ticket *t = ak.first;
        t->remaining -= ak.second;
        if (t->remaining <= 0) retire(*t);
        else still.push_back(t);
      }
      for (Ticket *t : admitted) {
        if (t->remaining <= 0) retire(*t);
        else still.push_back(t);
      }
      active.swap(still);
    }
  }
};

}  // namespace mfd

using namespace mfd;

extern "C" int mfd_server_create(mfd_server **out, int64_t hbm_budget_bytes, int32_t max_slots,
                                 int64_t quantum_steps) {
  if (!out || hbm_budget_bytes <= 0 || max_slots <= 0 || quantum_steps <= 0) return MFD_E_ARG;
  Server *s = new (std::nothrow) Server();
  if (!s) return MFD_E_OOM;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->quantum = quantum_steps;
  if (hipStreamCreate(&s->run_stream) != hipSuccess || hipStreamCreate(&s->admit_stream) != hipSuccess ||
      mfd_batch_create(&s->batch) != MFD_OK) {
    delete s;
    return MFD_E_HIP;
  }
  mfd_batch_set_stream(s->batch, s->run_stream);
  mfd_batch_set_graph(s->batch, 0);  // membership changes every quantum
  s->th = std::thread([s] { s->loop(); });
  *out = reinterpret_cast<mfd_server *>(s);
  return MFD_OK;
}

extern "C" int mfd_server_submit(mfd_server *h, const mfd_request *r, int64_t *ticket) {
  if (!h || !r || !ticket) return MFD_E_ARG;
  Server *s = reinterpret_cast<Server *>(h);
  if (r->n[0] < 3 || r->n[1] < 3 || r->nsteps < 0 || !r->state0 || !(r->dx > 0) || !(r->dt > 0))
    return MFD_E_ARG;
  if (r->eq != MFD_LCDE && r->eq != MFD_BURGERS && r->eq != MFD_NSE) return MFD_E_ARG;
  if (r->lattice != MFD_D2Q9 && r->lattice != MFD_D2Q5) return MFD_E_UNSUPPORTED;
  Ticket t;
  t.req = *r;
  t.t_submit = Clock::now();
  int64_t sb = 0;
  t.bytes = Server::request_bytes(*r, &sb);
  t.remaining = r->nsteps;
  t.lups = r->n[0] * r->n[1] * r->nsteps;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return MFD_E_ORDER;
  const int64_t id = s->next_id++;
  s->tickets[id] = t;
  s->pending.push_back(id);
  *ticket = id;
  s->cv.notify_all();
  return MFD_OK;
}

extern "C" int mfd_server_poll(mfd_server *h, int64_t ticket, int32_t *state, double *latency_s) {
  if (!h || !state) return MFD_E_ARG;
  Server *s = reinterpret_cast<Server *>(h);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return MFD_E_ARG;
  *state = it->second.state;
  if (latency_s)
    *latency_s = it->second.state == 2 ? secs(it->second.t_submit, it->second.t_done) : -1.0;
  return it->second.state < 0 ? it->second.error : MFD_OK;
}

extern "C" int mfd_server_drain(mfd_server *h, double timeout_s) {
  if (!h) return MFD_E_ARG;
  Server *s = reinterpret_cast<Server *>(h);
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                      [&] { return s->completed + s->failed == s->next_id - 1; });
  return ok ? MFD_OK : MFD_E_ORDER;
}

extern "C" int mfd_server_stats(mfd_server *h, double *p50_s, double *p99_s, double *req_per_s,
                                int64_t *completed, double *glups) {
  if (!h) return MFD_E_ARG;
  Server *s = reinterpret_cast<Server *>(h);
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->latencies;
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    const double pos = p * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
  };
  const double span = s->have_first ? secs(s->t_first, s->t_last) : 0.0;
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (completed) *completed = s->completed;
  if (req_per_s) *req_per_s = span > 0 ? s->completed / span : 0.0;
  if (glups) *glups = span > 0 ? s->lups_done / span / 1e9 : 0.0;
  return MFD_OK;
}

extern "C" int mfd_server_destroy(mfd_server *h) {
  if (!h) return MFD_OK;
  Server *s = reinterpret_cast<Server *>(h);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->pending.clear();
    s->cv.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (auto &kv : s->tickets)
    if (kv.second.solver) mfd_destroy(kv.second.solver);
  mfd_batch_destroy(s->batch);
  (void)hipStreamDestroy(s->run_stream);
  (void)hipStreamDestroy(s->admit_stream);
  delete s;
  return MFD_OK;
}
