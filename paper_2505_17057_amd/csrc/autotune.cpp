// Launch-plan autotuner: picks the temporal-blocking plan (steps per launch,
// window height) of a solver's configuration by timing every supported
// candidate on the solver's own state (saved before and restored after), and
// caches the choice for the process under a key of (lattice, equation, form,
// precision, levels, grid).
#include <hip/hip_runtime.h>

#include <map>
#include <algorithm>
#include <mutex>
#include <vector>
#include <tuple>

#include "../../include/mfd.h"
#include "mfd_internal.h"
#include "solver.h"

namespace mfd {

namespace {

using Key = std::tuple<int, int, int, int, int, int, int64_t, int64_t, int64_t, int, int>;
std::mutex g_mu;
std::map<Key, TbPlan> g_cache;

Key key_of(const Solver &s) {
  return Key(s.consts.lattice, s.consts.eq, s.grid.form, s.grid.precision, s.consts.three,
             s.consts.three_stencil, s.G.n[0], s.G.n[1], s.G.n[2], s.dirichlet ? 1 : 0,
             s.src_on ? 1 : 0);
}

bool tunable(const Solver &s) {
  if (s.cfg.kind == MFD_THETA) return false;
  // with a source term: the blocked MMFD source step (2D linear CDE)
  if (s.src_on) return s.grid.form == MFD_MMFD && s.consts.dim == 2 && tb_equation_supported(s.consts);
  if (s.grid.form == MFD_MESOFD)
    return s.consts.dim == 2 && !s.consts.three && (s.consts.eq == kLCDE || s.consts.eq == kBurgers);
  return tb_equation_supported(s.consts);
}

// default window height for a requested depth: the tallest window whose
// levels leave room for three workgroups per CU (NSE: the 32-row window)
int default_h(const Solver &s, int tb) {
  if (s.consts.eq == kNSE) {
    const TbPlan p{tb, 32};
    return s.plan_supported(p) ? 32 : 0;
  }
  static const int hs[] = {96, 80, 64, 48, 32};
  for (int h : hs) {
    const TbPlan p{tb, h};
    if (tb_lds_bytes(s.consts, p, (int)s.elem()) * 3 <= 160 * 1024 && s.plan_supported(p)) return h;
  }
  return 0;
}

}  // namespace

bool Solver::plan_supported(const TbPlan &p) const {
  if (cfg.kind == MFD_THETA) return false;
  if (src_on) return grid.form == MFD_MMFD && source_tb_supported(consts, G, p, (int)elem());
  // Dirichlet nodes are set by the 64-column windows (the in-place 128-column
  // window of the linear CDE has no boundary handling)
  if (dirichlet && (p.w != 64 || p.tb > kMaxBcSteps)) return false;
  if (grid.form == MFD_MESOFD) return mesofd_tb_supported(consts, G, p, (int)elem());
  return tb_supported(consts, G, p, (int)elem());
}

TbPlan Solver::effective_plan() const {
  if (!tunable(*this)) return TbPlan{1, 0};
  if (tb == 1) return TbPlan{1, 0};
  // a plan chosen before a source term was set may not suit the source step
  // (128-column windows): then the default window of the same depth
  if (tb > 1) {
    if (tuned.tb == tb && plan_supported(tuned)) return tuned;
    const int h = default_h(*this, tb);
    return h ? TbPlan{tb, h} : TbPlan{1, 0};
  }
  if (tuned.tb > 0 && plan_supported(tuned)) return tuned;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key_of(*this));
    if (it != g_cache.end() && plan_supported(it->second)) return it->second;
  }
  const int h = default_h(*this, 4);
  return h ? TbPlan{4, h} : TbPlan{1, 0};
}

int Solver::autotune(int32_t *chosen) {
  if (sticky) return fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!tunable(*this) || !state_set) {
    if (chosen) *chosen = effective_plan().tb;
    return MFD_OK;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key_of(*this));
    if (it != g_cache.end()) {
      tuned = it->second;
      if (chosen) *chosen = effective_plan().tb;
      return MFD_OK;
    }
  }
  // save the live levels (MesoFD: and the current populations)
  const bool meso = grid.form == MFD_MESOFD;
  const size_t bytes = (size_t)(mom_elems() * elem());
  const size_t pbytes = meso ? (size_t)(pop_elems() * elem()) : 0;
  void *save[3] = {nullptr, nullptr, nullptr};
  for (int k = 0; k < (meso ? 3 : 2); ++k) {
    hipError_t e = dev_malloc(&save[k], k == 2 ? pbytes : bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      for (int j = 0; j < k; ++j) dev_free(save[j]);
      return fail(MFD_E_OOM, "autotune: no memory for the state copy");
    }
  }
  int rc = hip(hipMemcpyAsync(save[0], buf[ic], bytes, hipMemcpyDeviceToDevice, stream), "copy");
  if (!rc) rc = hip(hipMemcpyAsync(save[1], buf[ip], bytes, hipMemcpyDeviceToDevice, stream), "copy");
  if (!rc && meso)
    rc = hip(hipMemcpyAsync(save[2], buf[pc], pbytes, hipMemcpyDeviceToDevice, stream), "copy");
  const int saved_tb = tb;
  const TbPlan saved_tuned = tuned;
  const int64_t saved_steps = steps_done;
  const int saved_gap = prev_gap;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) rc = hip(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = hip(hipEventCreate(&e1), "hipEventCreate");
  // trial length: ~2^29 node updates, in whole blocks of each depth; the
  // candidates are compared by time per step
  int64_t trial0 = ((int64_t)1 << 29) / G.N;
  trial0 = trial0 < 96 ? 96 : (trial0 > 480 ? 480 : trial0);
  const int depths[] = {1, 2, 4, 6, 8, 10, 12, 14, 16};
  int heights[49];
  for (int i = 0; i < 49; ++i) heights[i] = 32 + 2 * i;  // 32 .. 128
  const int widths[] = {64, 128};
  // time per step of plan p over about `steps` steps (whole blocks of its depth)
  auto time_plan = [&](const TbPlan &p, int64_t steps, float *ms) {
    tb = p.tb;
    tuned = p;
    const int64_t trial = p.tb * ((steps + p.tb - 1) / p.tb);
    int r = step(trial);  // warm-up
    if (!r) r = hip(hipEventRecord(e0, stream), "hipEventRecord");
    if (!r) r = step(trial);
    if (!r) r = hip(hipEventRecord(e1, stream), "hipEventRecord");
    if (!r) r = hip(hipEventSynchronize(e1), "hipEventSynchronize");
    if (!r) r = hip(hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime");
    *ms /= (float)trial;
    return r;
  };
  // scan every plan, then time the four fastest again over four times the
  // steps (the scan's short trials rank close plans by noise)
  std::vector<std::pair<float, TbPlan>> timed;
  for (int d : depths) {
    for (int w : widths)
    for (int h : heights) {
      if (rc) break;
      TbPlan p{d, d == 1 ? 0 : h, w};
      if (d == 1 && (h != heights[0] || w != widths[0])) continue;
      if (d > 1 && !plan_supported(p)) continue;
      float ms = 0.f;
      rc = time_plan(p, trial0, &ms);
      if (!rc) timed.emplace_back(ms, p);
    }
  }
  std::stable_sort(timed.begin(), timed.end(),
                   [](const std::pair<float, TbPlan> &a, const std::pair<float, TbPlan> &b) {
                     return a.first < b.first;
                   });
  // the finalists are timed in three interleaved rounds and each keeps its
  // fastest round, so a drift of the clocks during the refinement does not
  // decide between plans a few per cent apart
  const size_t nfin = std::min<size_t>(timed.size(), 4);
  std::vector<float> fin_ms(nfin, 1e30f);
  for (int round = 0; round < 3 && !rc; ++round) {
    for (size_t i = 0; i < nfin && !rc; ++i) {
      float ms = 0.f;
      rc = time_plan(timed[i].second, 4 * trial0, &ms);
      if (!rc) fin_ms[i] = std::min(fin_ms[i], ms);
    }
  }
  float best_ms = 1e30f;
  TbPlan best{1, 0};
  for (size_t i = 0; i < nfin; ++i) {
    if (fin_ms[i] < best_ms) {
      best_ms = fin_ms[i];
      best = timed[i].second;
    }
  }
  tb = saved_tb;
  tuned = saved_tuned;
  if (!rc) {
    rc = hip(hipMemcpyAsync(buf[ic], save[0], bytes, hipMemcpyDeviceToDevice, stream), "copy");
    if (!rc) rc = hip(hipMemcpyAsync(buf[ip], save[1], bytes, hipMemcpyDeviceToDevice, stream), "copy");
    if (!rc && meso)
      rc = hip(hipMemcpyAsync(buf[pc], save[2], pbytes, hipMemcpyDeviceToDevice, stream), "copy");
    if (!rc) rc = hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
  }
  steps_done = saved_steps;
  prev_gap = saved_gap;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void *p : save)
    if (p) dev_free(p);
  if (rc) return rc;
  tuned = best;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key_of(*this)] = best;
  }
  if (chosen) *chosen = effective_plan().tb;
  return MFD_OK;
}

}  // namespace mfd
