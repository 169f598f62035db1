// Continuous-batching server for MMFD solves.
//
// A scheduler thread owns the GPU work.  Each quantum it
//   1. drops requests that were cancelled or ran past their timeout,
//   2. enqueues one batched run that advances every active slot by
//      min(quantum, remaining steps) on the server stream (asynchronous),
//   3. while that runs, admits queued requests in arrival order as long as a
//      slot is free and the HBM budget holds the new request's device bytes
//      (solver creation and the host-to-device copy use a separate stream),
//   4. waits for the run, then retires finished slots: checks that the final
//      level is finite (FP64 sums), copies it to the caller's buffer, stamps
//      the completion time and frees the slot's memory.
// Requests that arrive while others are on the GPU therefore join at the next
// quantum and their steps run in the same launches as the older requests.
// A request that fails (its batch entry is refused, its result is not finite,
// it is cancelled or times out) frees its slot and budget alone; a failed
// batch run fails the requests it held and the batch object is replaced.
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
  bool cancel = false;  // set by mfd_server_cancel while running
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

  // state bytes of one level, and the device bytes a request holds while
  // admitted: the solver's own buffers (level ring, fourth level of blocked
  // three-level steps, reduction scratch), one more level for the batch
  // autotuner's copy of the spare level, and the batch's per-instance tables
  static int64_t state_bytes(const mfd_request &r) {
    const int64_t N = r.n[0] * r.n[1];
    const int nf = r.eq == MFD_NSE ? 3 : 1;
    return nf * N * (r.precision == MFD_FP64 ? 8 : 4);
  }
  static int64_t request_bytes(const mfd_request &r, int64_t solver_bytes) {
    const int64_t tiles = (r.n[0] / 8 + 2) * (r.n[1] / 8 + 2);
    return solver_bytes + state_bytes(r) + tiles * (int64_t)sizeof(int) + (64 << 10);
  }

  // configure a solver for a request (no device memory is allocated until
  // its state is set)
  static int configure(const mfd_request &r, mfd_solver **out) {
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
    if (rc < 0) {
      mfd_destroy(s);
      return rc;
    }
    *out = s;
    return MFD_OK;
  }

  int admit(Ticket &t) {
    const mfd_request &r = t.req;
    mfd_solver *s = nullptr;
    int rc = configure(r, &s);
    if (rc < 0) return rc;
    rc = mfd_set_stream(s, admit_stream);
    const int64_t sb = state_bytes(r);
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

  // end a ticket: free its solver and budget, record the outcome
  void finish(Ticket &t, int rc) {
    if (t.solver) mfd_destroy(t.solver);
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

  // a batch that failed may hold a sticky HIP error: replace it
  void reset_batch() {
    mfd_batch_destroy(batch);
    batch = nullptr;
    if (mfd_batch_create(&batch) == MFD_OK) {
      mfd_batch_set_stream(batch, run_stream);
      mfd_batch_set_graph(batch, 0);
    }
  }

  void retire(Ticket &t) {
    // the final level must be finite (FP64 sums and residual)
    double sums[4], res = 0.0;
    int rc = mfd_reduce(t.solver, sums, &res);
    if (rc >= 0 && t.req.result_out) {
      const int64_t sb = state_bytes(t.req);
      if (t.req.result_bytes != sb) rc = MFD_E_ARG;
      else rc = mfd_get_state(t.solver, 0, t.req.result_out, sb, 0, 0);
    }
    finish(t, rc < 0 ? rc : MFD_OK);
  }

  // requests to drop at this quantum boundary: cancelled or past their timeout
  int drop_code(const Ticket &t, Clock::time_point now) {
    if (t.cancel) return MFD_E_CANCELLED;
    if (t.req.timeout_s > 0 && secs(t.t_submit, now) > t.req.timeout_s) return MFD_E_TIMEOUT;
    return MFD_OK;
  }

  void loop() {
    while (true) {
      // ---- drop cancelled / timed-out requests, queued or running
      {
        const auto now = Clock::now();
        std::vector<std::pair<Ticket *, int>> drop;
        std::vector<Ticket *> keep;
        {
          std::lock_guard<std::mutex> lk(mu);
          for (auto it = pending.begin(); it != pending.end();) {
            Ticket &t = tickets[*it];
            const int c = drop_code(t, now);
            if (c < 0) {
              t.state = -1;
              t.error = c;
              t.t_done = now;
              ++failed;
              it = pending.erase(it);
              cv_done.notify_all();
            } else {
              ++it;
            }
          }
          for (Ticket *t : active) {
            const int c = drop_code(*t, now);
            if (c < 0) drop.push_back({t, c});
            else keep.push_back(t);
          }
        }
        for (auto &d : drop) finish(*d.first, d.second);
        if (!drop.empty()) active.swap(keep);
      }
      // ---- enqueue a quantum for the active slots
      bool ran = false;
      std::vector<std::pair<Ticket *, int64_t>> advanced;  // (slot, steps)
      if (!active.empty() && batch) {
        mfd_batch_clear(batch);
        Batch *bp = reinterpret_cast<Batch *>(batch);
        bool untuned = false;
        std::vector<Ticket *> kept;
        for (Ticket *t : active) {
          const int64_t k = std::min(quantum, t->remaining);
          const int rc = mfd_batch_add(batch, t->solver, k, nullptr);
          if (rc < 0) {  // this request alone cannot be batched
            finish(*t, rc);
            continue;
          }
          kept.push_back(t);
          advanced.push_back({t, k});
          const BatchKey key = batch_key_of(reinterpret_cast<Solver *>(t->solver));
          if (batch_blockable(key) && !bp->tuned.count(key)) untuned = true;
        }
        active.swap(kept);
        // the first quantum holding a blockable kind picks its launch plan
        int rc = MFD_OK;
        if (!advanced.empty()) {
          if (untuned) rc = mfd_batch_autotune(batch);
          if (rc >= 0) rc = mfd_batch_run(batch);
          if (rc < 0) {
            // the run (or the tuning, which moves the spare levels) failed:
            // the states of its requests are not known to be right
            for (auto &ak : advanced) finish(*ak.first, rc);
            advanced.clear();
            active.clear();
            reset_batch();
          } else {
            ran = true;
          }
        }
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
        if (rc < 0) {
          finish(*tp, rc);
        } else {
          std::lock_guard<std::mutex> lk(mu);
          tp->state = 1;
          tp->t_admit = Clock::now();
          admitted.push_back(tp);
        }
      }
      // ---- finish the quantum and retire finished slots
      if (ran) {
        const int rc = mfd_batch_wait(batch);
        if (rc < 0) {
          for (auto &ak : advanced) finish(*ak.first, rc);
          std::vector<Ticket *> rest;
          for (Ticket *t : active)
            if (t->solver) rest.push_back(t);
          active.swap(rest);
          advanced.clear();
          reset_batch();
        }
      }
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
  if (r->n[0] < 3 || r->n[1] < 3 || r->nsteps < 0 || !r->state0 || !(r->dx > 0) || !(r->dt > 0) ||
      !(r->timeout_s >= 0))
    return MFD_E_ARG;
  if (r->eq != MFD_LCDE && r->eq != MFD_BURGERS && r->eq != MFD_NSE) return MFD_E_ARG;
  if (r->precision != MFD_FP32 && r->precision != MFD_FP64) return MFD_E_ARG;
  if (r->lattice != MFD_D2Q9 && r->lattice != MFD_D2Q5) return MFD_E_UNSUPPORTED;
  if (r->kind != MFD_TWO_LEVEL && r->kind != MFD_THREE_LEVEL) return MFD_E_UNSUPPORTED;
  // the configuration must be valid, and its device bytes set the admission
  // budget (host-side only: no device memory is allocated here)
  mfd_solver *probe = nullptr;
  int rc = Server::configure(*r, &probe);
  if (rc < 0) return rc;
  int64_t dev_bytes = 0;
  rc = mfd_state_size(probe, nullptr, nullptr, &dev_bytes);
  mfd_destroy(probe);
  if (rc < 0) return rc;
  if (r->result_out && r->result_bytes != Server::state_bytes(*r)) return MFD_E_ARG;
  Ticket t;
  t.req = *r;
  t.t_submit = Clock::now();
  t.bytes = Server::request_bytes(*r, dev_bytes);
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

extern "C" int mfd_server_request_bytes(const mfd_request *r, int64_t *bytes) {
  if (!r || !bytes) return MFD_E_ARG;
  if (r->kind != MFD_TWO_LEVEL && r->kind != MFD_THREE_LEVEL) return MFD_E_UNSUPPORTED;
  mfd_solver *probe = nullptr;
  int rc = Server::configure(*r, &probe);
  if (rc < 0) return rc;
  int64_t dev_bytes = 0;
  rc = mfd_state_size(probe, nullptr, nullptr, &dev_bytes);
  mfd_destroy(probe);
  if (rc < 0) return rc;
  *bytes = Server::request_bytes(*r, dev_bytes);
  return MFD_OK;
}

extern "C" int mfd_server_cancel(mfd_server *h, int64_t ticket) {
  if (!h) return MFD_E_ARG;
  Server *s = reinterpret_cast<Server *>(h);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return MFD_E_ARG;
  Ticket &t = it->second;
  if (t.state == 0) {
    for (auto p = s->pending.begin(); p != s->pending.end(); ++p)
      if (*p == ticket) {
        s->pending.erase(p);
        break;
      }
    t.state = -1;
    t.error = MFD_E_CANCELLED;
    t.t_done = Clock::now();
    ++s->failed;
    s->cv_done.notify_all();
    return MFD_OK;
  }
  if (t.state == 1) {
    t.cancel = true;  // dropped by the scheduler at the next quantum boundary
    return MFD_OK;
  }
  return MFD_E_ORDER;  // already done or failed
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
  if (s->batch) mfd_batch_destroy(s->batch);
  (void)hipStreamDestroy(s->run_stream);
  (void)hipStreamDestroy(s->admit_stream);
  delete s;
  return MFD_OK;
}
