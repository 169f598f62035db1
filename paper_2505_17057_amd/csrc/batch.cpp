// Batched stepping of many solvers: groups, tile tables, the step sequence
// captured once into a hipGraph and replayed, and the level-ring hand-back
// to each solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/mfd.h"
#include "batch.h"
#include "batch_kernels.h"
#include "mfd_internal.h"
#include "solver.h"

namespace mfd {

int Batch::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
  return code;
}

int Batch::hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return MFD_OK;
  sticky = true;
  return fail(MFD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void Batch::free_graph() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
}

void Batch::free_groups() {
  for (auto &g : groups) {
    if (g.d_inst) dev_free(g.d_inst);
    if (g.d_tile_inst) dev_free(g.d_tile_inst);
    if (g.d_lane) dev_free(g.d_lane);
  }
  groups.clear();
  for (auto &r : res)
    if (r.d) dev_free(r.d);
  res.clear();
}

BatchKey batch_key_of(const Solver *s) {
  return BatchKey{s->consts.lattice, s->consts.eq, s->consts.three, s->consts.three_stencil,
                  s->grid.precision, s->consts.eq == kBurgers && s->consts.beta_one ? 1 : 0};
}

bool batch_blockable(const BatchKey &k) {
  if (k.lattice != MFD_D2Q5 && k.lattice != MFD_D2Q9) return false;
  if (k.eq == kNSE) return !k.three_st;
  return !k.three && (k.eq == kLCDE || k.eq == kBurgers);
}

static int elem_of(const BatchKey &k) { return k.precision == MFD_FP64 ? 8 : 4; }

// a blocked plan the group's kernel can run: 64-column windows (the general
// batched kernels), or 128-column ones (the lane-shared kernel)
static bool group_plan_valid(const BatchKey &k, const TbPlan &p) {
  if (p.w == 128)
    return lane_batch_applies(k) && tb_plan_valid(p, 1, 4) && lane_tb_window_fits(p);
  if (p.w != 64) return false;
  if (k.eq == kNSE) return nse_tb_plan_valid(p, k.lattice == MFD_D2Q9 ? 4 : 2, elem_of(k));
  return tb_plan_valid(p, 2, elem_of(k));
}

static int tile_ty(int eq) { return eq == kNSE ? kBatchTYNse : kBatchTY; }

// tile shape of a group under its plan
static void tile_shape(const Group &g, int *tx, int *ty) {
  if (g.plan.tb > 1) {
    *tx = g.plan.w - 2 * g.plan.tb;
    *ty = g.plan.h - 2 * g.plan.tb;
  } else {
    *tx = kBatchTX;
    *ty = tile_ty(g.key.eq);
  }
}

// tile table of a group for its current plan (host and device)
int Batch::make_tables(Group &g) {
  int TX, TY;
  tile_shape(g, &TX, &TY);
  std::vector<int> tile_inst;
  g.tile0.clear();
  g.tiles_x.clear();
  for (int slot = 0; slot < (int)g.order.size(); ++slot) {
    const Solver *s = entries[g.order[slot]].s;
    const int tx = (int)((s->G.n[0] + TX - 1) / TX);
    const int tyc = (int)((s->G.n[1] + TY - 1) / TY);
    g.tile0.push_back((int)tile_inst.size());
    g.tiles_x.push_back(tx);
    for (int k = 0; k < tx * tyc; ++k) tile_inst.push_back(slot);
  }
  g.ntiles = (int)tile_inst.size();
  if (g.ntiles > g.tile_cap) {
    if (g.d_tile_inst) dev_free(g.d_tile_inst);
    g.d_tile_inst = nullptr;
    g.tile_cap = 0;
    int rc = hip(dev_malloc((void **)&g.d_tile_inst, sizeof(int) * (size_t)g.ntiles), "hipMalloc (tiles)");
    if (rc) return rc;
    g.tile_cap = g.ntiles;
  }
  if (g.ntiles)
    return hip(hipMemcpyAsync(g.d_tile_inst, tile_inst.data(), sizeof(int) * g.ntiles,
                              hipMemcpyHostToDevice, stream),
               "hipMemcpyAsync (tiles)");
  return MFD_OK;
}

int Batch::build() {
  free_graph();
  free_groups();
  if (!stream) {
    int rc = hip(hipStreamCreate(&own_stream), "hipStreamCreate");
    if (rc) return rc;
    stream = own_stream;
  }
  std::map<BatchKey, std::vector<int>> by_key, res_key;
  for (int i = 0; i < (int)entries.size(); ++i) {
    const Solver *s = entries[i].s;
    const BatchKey k = batch_key_of(s);
    if (entries[i].nsteps > 0 && s->G.N <= resident_max && resident_applies(k, s->G.n[0], s->G.n[1]))
      res_key[k].push_back(i);
    else
      by_key[k].push_back(i);
  }
  max_steps = 0;
  lups_per_run = 0;
  for (auto &kv : res_key) {
    res.emplace_back();
    ResGroup &r = res.back();
    r.key = kv.first;
    r.order = kv.second;
    r.h.resize(r.order.size());
    for (int i : r.order) {
      max_steps = std::max(max_steps, entries[i].nsteps);
      lups_per_run += entries[i].s->G.N * entries[i].nsteps;
    }
    int rc = hip(dev_malloc((void **)&r.d, sizeof(ResInst) * r.order.size()),
                 "hipMalloc (resident instances)");
    if (rc) return rc;
  }
  if (!res.empty() && !side) {
    // default-priority stream and events of the resident branch
    int rc = hip(hipStreamCreateWithFlags(&side, hipStreamNonBlocking), "hipStreamCreate (side)");
    if (!rc) rc = hip(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming), "hipEventCreate");
    if (!rc) rc = hip(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming), "hipEventCreate");
    if (rc) return rc;
  }
  for (auto &kv : by_key) {
    groups.emplace_back();
    Group &g = groups.back();
    g.key = kv.first;
    g.order = kv.second;
    std::stable_sort(g.order.begin(), g.order.end(),
                     [&](int a, int b) { return entries[a].nsteps > entries[b].nsteps; });
    g.tb_ok = batch_blockable(g.key);
    if (g.tb_ok) {
      auto it = tuned.find(g.key);
      if (req.tb > 0) g.plan = req;
      else if (it != tuned.end()) g.plan = it->second;
      if (g.plan.tb > 1 && g.plan.w == 128) {
        // the lane-shared kernel needs every instance's constants to suit it;
        // else the same plan in 64-column windows
        bool ok = group_plan_valid(g.key, g.plan);
        for (int i : g.order) ok = ok && lane_shared_fp32(entries[i].s->consts);
        if (!ok) g.plan.w = 64;
      }
      if (g.plan.tb > 1 && !group_plan_valid(g.key, g.plan)) g.plan = TbPlan{1, 0};
    }
    for (int slot = 0; slot < (int)g.order.size(); ++slot) {
      const BatchEntry &e = entries[g.order[slot]];
      g.steps.push_back(e.nsteps);
      max_steps = std::max(max_steps, e.nsteps);
      lups_per_run += e.s->G.N * e.nsteps;
    }
    const size_t isz = g.key.precision == MFD_FP64 ? sizeof(BatchInst<double>) : sizeof(BatchInst<float>);
    g.inst_bytes = isz * g.order.size();
    int rc = hip(dev_malloc(&g.d_inst, g.inst_bytes), "hipMalloc (instances)");
    if (!rc && lane_batch_applies(g.key)) {
      g.lane_bytes = lane_inst_bytes(g.key) * g.order.size();
      rc = hip(dev_malloc(&g.d_lane, g.lane_bytes), "hipMalloc (lane instances)");
      g.h_lane.resize(g.lane_bytes);
    }
    if (!rc) rc = make_tables(g);
    if (rc) return rc;
    g.h_inst.resize(g.inst_bytes);
  }
  return hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
}

// active tiles of a group at step s: instances are sorted by decreasing step
// count, so those with steps > s are a prefix
static int active_tiles(const Group &g, int64_t s) {
  int m = 0;
  while (m < (int)g.steps.size() && g.steps[m] > s) ++m;
  if (m == (int)g.steps.size()) return g.ntiles;
  return g.tile0[m];
}

// one blocked launch of a group (its `l`-th) over the first nt tiles
static hipError_t launch_group_tb_impl(const Group &g, int nt, int64_t l, const TbPlan &p,
                                       hipStream_t stream) {
  if (p.w == 128) return launch_batch_lane_tb(g.key, g.d_lane, g.d_tile_inst, nt, l, p, stream);
  if (g.key.precision == MFD_FP64) {
    const BatchInst<double> *in = (const BatchInst<double> *)g.d_inst;
    return g.key.eq == kNSE ? launch_batch_nse_tb<double>(g.key, in, g.d_tile_inst, nt, l, p, stream)
                            : launch_batch_tb<double>(g.key, in, g.d_tile_inst, nt, l, p, stream);
  }
  const BatchInst<float> *in = (const BatchInst<float> *)g.d_inst;
  return g.key.eq == kNSE ? launch_batch_nse_tb<float>(g.key, in, g.d_tile_inst, nt, l, p, stream)
                          : launch_batch_tb<float>(g.key, in, g.d_tile_inst, nt, l, p, stream);
}

hipError_t Batch::launch_group_tb(const Group &g, int nt, int64_t l) {
  return launch_group_tb_impl(g, nt, l, g.plan, stream);
}

int Batch::enqueue_steps() {
  launches_per_run = 0;
  // the LDS-resident instances on a branch of their own, joined at the end
  if (!res.empty()) {
    int rc = hip(hipEventRecord(ev_fork, stream), "hipEventRecord (fork)");
    if (!rc) rc = hip(hipStreamWaitEvent(side, ev_fork, 0), "hipStreamWaitEvent (fork)");
    for (auto &r : res) {
      if (rc) break;
      int64_t nmax = 0;
      for (int i : r.order) nmax = std::max(nmax, entries[i].s->G.N);
      rc = hip(launch_batch_resident(r.key, r.d, (int)r.order.size(), (int)nmax, side),
               "resident batch launch");
      ++launches_per_run;
    }
    if (!rc) rc = hip(hipEventRecord(ev_join, side), "hipEventRecord (join)");
    if (rc) return rc;
  }
  int rc = enqueue_group_steps();
  if (!res.empty()) {
    const int rj = hip(hipStreamWaitEvent(stream, ev_join, 0), "hipStreamWaitEvent (join)");
    if (!rc) rc = rj;
  }
  return rc;
}

int Batch::enqueue_group_steps() {
  for (auto &g : groups) {
    const int64_t gmax = g.steps.empty() ? 0 : g.steps[0];
    if (g.plan.tb > 1) {
      const int64_t nl = (gmax + g.plan.tb - 1) / g.plan.tb;
      for (int64_t l = 0; l < nl; ++l) {
        const int nt = active_tiles(g, l * g.plan.tb);
        if (nt == 0) continue;
        const hipError_t e = launch_group_tb(g, nt, l);
        if (e != hipSuccess) return hip(e, "blocked batch launch");
        ++launches_per_run;
      }
      continue;
    }
    for (int64_t s = 0; s < gmax; ++s) {
      const int nt = active_tiles(g, s);
      if (nt == 0) continue;
      hipError_t e;
      if (g.key.precision == MFD_FP64)
        e = launch_batch_step<double>(g.key, (const BatchInst<double> *)g.d_inst, g.d_tile_inst,
                                      nt, s, stream);
      else
        e = launch_batch_step<float>(g.key, (const BatchInst<float> *)g.d_inst, g.d_tile_inst,
                                     nt, s, stream);
      if (e != hipSuccess) return hip(e, "batch step launch");
      ++launches_per_run;
    }
  }
  return MFD_OK;
}

template <typename T>
static void fill_inst(const Group &g, const std::vector<BatchEntry> &entries,
                      std::vector<unsigned char> &h) {
  BatchInst<T> *bi = reinterpret_cast<BatchInst<T> *>(h.data());
  for (int slot = 0; slot < (int)g.order.size(); ++slot) {
    const Solver *s = entries[g.order[slot]].s;
    BatchInst<T> b;
    std::memset(&b, 0, sizeof(b));
    if (s->consts.three && g.plan.tb > 1) {
      // blocked three-level: launches move between the pairs (t, t - dt)
      b.ring[0] = (T *)s->buf[s->ic];
      b.ring[1] = (T *)s->buf[s->ip];
      b.ring[2] = (T *)s->buf[s->io];
      b.ring[3] = (T *)s->buf[s->ix];
      b.ring_len = 4;
    } else if (s->consts.three) {
      b.ring[0] = (T *)s->buf[s->ic];
      b.ring[1] = (T *)s->buf[s->io];
      b.ring[2] = (T *)s->buf[s->ip];
      b.ring_len = 3;
    } else {
      b.ring[0] = (T *)s->buf[s->ic];
      b.ring[1] = (T *)s->buf[s->ip];
      b.ring_len = 2;
    }
    b.nx = (int)s->G.n[0];
    b.ny = (int)s->G.n[1];
    b.c0 = 0;
    b.tiles_x = g.tiles_x[slot];
    b.tile0 = g.tile0[slot];
    b.nsteps = g.steps[slot];
    b.kc = make_kc<T>(s->consts);
    bi[slot] = b;
  }
}

int Batch::upload_instances() {
  for (auto &r : res) {
    for (int k = 0; k < (int)r.order.size(); ++k) {
      const BatchEntry &e = entries[r.order[k]];
      const Solver *s = e.s;
      ResInst ri;
      std::memset(&ri, 0, sizeof(ri));
      ri.lv[0] = (float *)s->buf[s->ic];
      ri.lv[1] = (float *)s->buf[s->ip];
      ri.nx = (int)s->G.n[0];
      ri.ny = (int)s->G.n[1];
      ri.nsteps = e.nsteps;
      ri.kc = make_kc<float>(s->consts);
      r.h[k] = ri;
    }
    int rc = hip(hipMemcpyAsync(r.d, r.h.data(), sizeof(ResInst) * r.h.size(), hipMemcpyHostToDevice,
                                stream),
                 "hipMemcpyAsync (resident instances)");
    if (rc) return rc;
  }
  for (auto &g : groups) {
    if (g.key.precision == MFD_FP64) fill_inst<double>(g, entries, g.h_inst);
    else fill_inst<float>(g, entries, g.h_inst);
    int rc = hip(hipMemcpyAsync(g.d_inst, g.h_inst.data(), g.inst_bytes, hipMemcpyHostToDevice, stream),
                 "hipMemcpyAsync (instances)");
    if (rc) return rc;
    if (g.plan.tb > 1 && g.plan.w == 128) {
      const size_t isz = lane_inst_bytes(g.key);
      for (int slot = 0; slot < (int)g.order.size(); ++slot) {
        Solver *s = entries[g.order[slot]].s;
        if (!lane_inst_fill(g.key, s->consts, (float *)s->buf[s->ic], (float *)s->buf[s->ip],
                            (int)s->G.n[0], (int)s->G.n[1], g.tiles_x[slot], g.tile0[slot],
                            g.steps[slot], g.h_lane.data() + isz * slot))
          return fail(MFD_E_UNSUPPORTED, "a batched solver does not suit 128-column windows");
      }
      rc = hip(hipMemcpyAsync(g.d_lane, g.h_lane.data(), g.lane_bytes, hipMemcpyHostToDevice, stream),
               "hipMemcpyAsync (lane instances)");
      if (rc) return rc;
    }
  }
  return MFD_OK;
}

static int check_ready(Batch &b) {
  for (auto &e : b.entries) {
    Solver *s = e.s;
    if (s->sticky || !s->state_set || !s->configured)
      return b.fail(MFD_E_ORDER, "a batched solver is not ready (configure it and set its state)");
  }
  return MFD_OK;
}

int Batch::run() {
  if (sticky) return fail(MFD_E_HIP, "batch is in a failed HIP state");
  if (entries.empty()) return MFD_OK;
  int rc = check_ready(*this);
  if (rc) return rc;
  if (dirty) {
    rc = build();
    if (rc) return rc;
  }
  // instance tables from the solvers' current level roles
  rc = upload_instances();
  if (rc) return rc;
  if (use_graph) {
    if (dirty || !exec) {
      free_graph();
      rc = hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      if (rc) return rc;
      rc = enqueue_steps();
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(stream, &gr);
      if (rc) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      rc = hip(e, "hipStreamEndCapture");
      if (rc) return rc;
      graph = gr;
      rc = hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
      if (rc) return rc;
    }
    rc = hip(hipGraphLaunch(exec, stream), "hipGraphLaunch");
    if (rc) return rc;
  } else {
    rc = enqueue_steps();
    if (rc) return rc;
  }
  dirty = false;
  for (auto &g : groups)
    for (int i : g.order) entries[i].tb = g.plan.tb;
  for (auto &r : res)
    for (int i : r.order) entries[i].tb = 1;  // the roles of a run of single steps
  // hand the rotated level roles back to the solvers
  for (auto &e : entries) {
    Solver *s = e.s;
    const int64_t n = e.nsteps;
    if (n == 0) continue;
    if (s->consts.three && e.tb > 1) {
      // each blocked launch moves to the other (t, t - dt) pair
      const int64_t nl = (n + e.tb - 1) / e.tb;
      if (nl & 1) {
        const int oc = s->ic, op = s->ip;
        s->ic = s->io;
        s->ip = s->ix;
        s->io = oc;
        s->ix = op;
      }
      s->prev_gap = 1;
    } else if (s->consts.three) {
      const int ring[3] = {s->ic, s->io, s->ip};
      s->ic = ring[n % 3];
      s->io = ring[(n + 1) % 3];
      s->ip = ring[(n + 2) % 3];
      s->prev_gap = 1;
    } else if (e.tb > 1) {
      // one ping-pong swap per blocked launch; the last launch advanced the
      // remainder, so the held previous level is that many steps old
      const int64_t nl = (n + e.tb - 1) / e.tb;
      const int ring[2] = {s->ic, s->ip};
      s->ic = ring[nl % 2];
      s->ip = ring[(nl + 1) % 2];
      s->prev_gap = (int)(n - (nl - 1) * e.tb);
    } else {
      const int ring[2] = {s->ic, s->ip};
      s->ic = ring[n % 2];
      s->ip = ring[(n + 1) % 2];
      s->prev_gap = 1;
    }
    s->steps_done += n;
  }
  return MFD_OK;
}

// Batch autotuner: for every group that can use the blocked kernel, time one
// launch of each candidate plan over all its instances (the first launch of a
// run: it reads each instance's level t and overwrites only its spare level,
// so repeating it is harmless), keep the fastest per node update, and restore
// the spare levels afterwards.
int Batch::autotune() {
  if (sticky) return fail(MFD_E_HIP, "batch is in a failed HIP state");
  if (entries.empty()) return MFD_OK;
  int rc = check_ready(*this);
  if (rc) return rc;
  const TbPlan saved_req = req;
  req = TbPlan{0, 0};
  rc = build();
  if (rc) {
    req = saved_req;
    return rc;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = hip(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = hip(hipEventCreate(&e1), "hipEventCreate");
  for (auto &g : groups) {
    if (rc) break;
    if (!g.tb_ok) continue;
    const int es = elem_of(g.key);
    // save the spare level of every instance
    int64_t total = 0;
    for (int i : g.order) total += entries[i].s->mom_elems();
    void *save = nullptr;
    rc = hip(dev_malloc(&save, (size_t)total * es), "hipMalloc (autotune copy)");
    if (rc) break;
    int64_t off = 0;
    for (int i : g.order) {
      Solver *s = entries[i].s;
      const size_t b = (size_t)s->mom_elems() * es;
      if (!rc) rc = hip(hipMemcpyAsync((char *)save + off, s->buf[s->ip], b, hipMemcpyDeviceToDevice, stream),
                        "hipMemcpyAsync (save)");
      off += (int64_t)b;
    }
    std::vector<TbPlan> cands{TbPlan{1, 0}};
    bool lane_ok = lane_batch_applies(g.key);
    for (int i : g.order) lane_ok = lane_ok && lane_shared_fp32(entries[i].s->consts);
    for (int d : {2, 3, 4, 6, 8})
      for (int h : {32, 48, 64, 96, 128})
        if (group_plan_valid(g.key, TbPlan{d, h})) cands.push_back(TbPlan{d, h});
    if (lane_ok)
      for (int d : {4, 6, 8, 10, 12})
        for (int h : {48, 64, 80, 96, 112, 128})
          if (group_plan_valid(g.key, TbPlan{d, h, 128})) cands.push_back(TbPlan{d, h, 128});
    float best = 1e30f;
    TbPlan best_p{1, 0};
    for (const TbPlan &p : cands) {
      if (rc) break;
      g.plan = p;
      rc = make_tables(g);
      if (!rc) rc = upload_instances();
      if (rc) break;
      double lups = 0;
      for (int slot = 0; slot < (int)g.order.size(); ++slot) {
        const int64_t n = std::min<int64_t>(g.steps[slot], p.tb);
        lups += (double)entries[g.order[slot]].s->G.N * (double)n;
      }
      const int nt = active_tiles(g, 0);
      if (nt == 0 || lups == 0) continue;
      auto launch = [&]() -> hipError_t {
        if (p.tb > 1) return launch_group_tb(g, nt, 0);
        return g.key.precision == MFD_FP64
                   ? launch_batch_step<double>(g.key, (const BatchInst<double> *)g.d_inst,
                                               g.d_tile_inst, nt, 0, stream)
                   : launch_batch_step<float>(g.key, (const BatchInst<float> *)g.d_inst,
                                              g.d_tile_inst, nt, 0, stream);
      };
      rc = hip(launch(), "autotune launch");
      if (!rc) rc = hip(hipEventRecord(e0, stream), "hipEventRecord");
      for (int k = 0; k < 3 && !rc; ++k) rc = hip(launch(), "autotune launch");
      if (!rc) rc = hip(hipEventRecord(e1, stream), "hipEventRecord");
      if (!rc) rc = hip(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      if (!rc) rc = hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      const float per = (float)(ms / (3.0 * lups));
      if (!rc && per < best) {
        best = per;
        best_p = p;
      }
    }
    // restore the spare levels
    off = 0;
    for (int i : g.order) {
      Solver *s = entries[i].s;
      const size_t b = (size_t)s->mom_elems() * es;
      if (!rc) rc = hip(hipMemcpyAsync(s->buf[s->ip], (char *)save + off, b, hipMemcpyDeviceToDevice, stream),
                        "hipMemcpyAsync (restore)");
      off += (int64_t)b;
    }
    if (!rc) rc = hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    dev_free(save);
    if (!rc) tuned[g.key] = best_p;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  req = saved_req;
  dirty = true;
  return rc;
}

}  // namespace mfd

using namespace mfd;

extern "C" int mfd_batch_create(mfd_batch **out) {
  if (!out) return MFD_E_ARG;
  Batch *b = new (std::nothrow) Batch();
  if (!b) return MFD_E_OOM;
  *out = reinterpret_cast<mfd_batch *>(b);
  return MFD_OK;
}

extern "C" int mfd_batch_destroy(mfd_batch *h) {
  if (!h) return MFD_OK;
  Batch *b = reinterpret_cast<Batch *>(h);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);
  b->free_graph();
  b->free_groups();
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  delete b;
  return MFD_OK;
}

extern "C" const char *mfd_batch_last_error(const mfd_batch *h) {
  if (!h) return "null batch";
  return reinterpret_cast<const Batch *>(h)->err.c_str();
}

extern "C" int mfd_batch_set_stream(mfd_batch *h, void *stream) {
  if (!h) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  if (!stream) return b->fail(MFD_E_ARG, "a batch needs a non-null stream (graph capture)");
  b->stream = (hipStream_t)stream;
  b->dirty = true;
  return MFD_OK;
}

extern "C" int mfd_batch_set_graph(mfd_batch *h, int use_graph) {
  if (!h) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  b->use_graph = use_graph != 0;
  b->dirty = true;
  return MFD_OK;
}

extern "C" int mfd_batch_add(mfd_batch *h, mfd_solver *sh, int64_t nsteps, int32_t *slot) {
  if (!h || !sh) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  Solver *s = reinterpret_cast<Solver *>(sh);
  if (nsteps < 0) return b->fail(MFD_E_ARG, "nsteps < 0");
  if (!s->configured || !s->state_set)
    return b->fail(MFD_E_ORDER, "configure the solver and set its state before batching it");
  if (s->grid.form != MFD_MMFD || s->grid.dim != 2 || s->cfg.kind == MFD_THETA ||
      (s->consts.lattice != MFD_D2Q9 && s->consts.lattice != MFD_D2Q5))
    return b->fail(MFD_E_UNSUPPORTED, "batches hold 2D explicit MMFD solvers (D2Q5 / D2Q9)");
  if (s->src_on) return b->fail(MFD_E_UNSUPPORTED, "batches hold solvers without a source term");
  if (s->dirichlet) return b->fail(MFD_E_UNSUPPORTED, "batches hold periodic solvers");
  for (auto &e : b->entries)
    if (e.s == s) return b->fail(MFD_E_ARG, "solver already in the batch");
  if (slot) *slot = (int32_t)b->entries.size();
  b->entries.push_back(BatchEntry{s, nsteps});
  b->dirty = true;
  return MFD_OK;
}

extern "C" int mfd_batch_clear(mfd_batch *h) {
  if (!h) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  b->entries.clear();
  b->dirty = true;
  return MFD_OK;
}

extern "C" int mfd_batch_run(mfd_batch *h) {
  if (!h) return MFD_E_ARG;
  return reinterpret_cast<Batch *>(h)->run();
}

extern "C" int mfd_batch_wait(mfd_batch *h) {
  if (!h) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  if (!b->stream) return MFD_OK;
  return b->hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
}

extern "C" int mfd_batch_set_plan(mfd_batch *h, int32_t tb_depth, int32_t window_rows,
                                  int32_t window_cols) {
  if (!h) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  if (tb_depth < 0) return b->fail(MFD_E_ARG, "negative depth");
  if (window_cols == 0) window_cols = 64;
  if (window_cols != 64 && window_cols != 128)
    return b->fail(MFD_E_ARG, "window columns must be 64 or 128");
  const TbPlan p{tb_depth, window_rows, window_cols};
  if (tb_depth > 1 &&
      (window_cols == 128 ? !(tb_plan_valid(p, 1, 4) && lane_tb_window_fits(p))
                          : !tb_plan_valid(p, 2, 8) && !tb_plan_valid(p, 2, 4)))
    return b->fail(MFD_E_ARG, "plan (%d, %d, %d) exceeds the blocked kernels' limits", tb_depth,
                   window_rows, window_cols);
  b->req = tb_depth > 1 ? p : TbPlan{tb_depth, 0};
  b->dirty = true;
  return MFD_OK;
}

extern "C" int mfd_batch_autotune(mfd_batch *h) {
  if (!h) return MFD_E_ARG;
  return reinterpret_cast<Batch *>(h)->autotune();
}

extern "C" int mfd_batch_plan(const mfd_batch *h, int32_t group, int32_t *tb_depth,
                              int32_t *window_rows, int32_t *window_cols) {
  if (!h) return MFD_E_ARG;
  const Batch *b = reinterpret_cast<const Batch *>(h);
  if (group < 0 || group >= (int32_t)b->groups.size()) return MFD_E_ARG;
  const TbPlan &p = b->groups[group].plan;
  if (tb_depth) *tb_depth = p.tb;
  if (window_rows) *window_rows = p.tb > 1 ? p.h : 0;
  if (window_cols) *window_cols = p.tb > 1 ? p.w : 0;
  return MFD_OK;
}

extern "C" int mfd_batch_set_resident(mfd_batch *h, int32_t max_nodes) {
  if (!h) return MFD_E_ARG;
  Batch *b = reinterpret_cast<Batch *>(h);
  if (max_nodes < 0) return b->fail(MFD_E_ARG, "max_nodes < 0");
  b->resident_max = max_nodes;
  b->dirty = true;
  return MFD_OK;
}

extern "C" int mfd_batch_resident(const mfd_batch *h, int32_t *count) {
  if (!h || !count) return MFD_E_ARG;
  const Batch *b = reinterpret_cast<const Batch *>(h);
  int32_t c = 0;
  for (auto &r : b->res) c += (int32_t)r.order.size();
  *count = c;
  return MFD_OK;
}

extern "C" int mfd_batch_stats(const mfd_batch *h, int64_t *launches, int64_t *lups,
                               int64_t *tiles) {
  if (!h) return MFD_E_ARG;
  const Batch *b = reinterpret_cast<const Batch *>(h);
  if (launches) *launches = b->launches_per_run;
  if (lups) *lups = b->lups_per_run;
  if (tiles) {
    int64_t t = 0;
    for (auto &g : b->groups) t += g.ntiles;
    *tiles = t;
  }
  return MFD_OK;
}
