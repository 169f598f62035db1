// Launch-plan autotuner: picks the temporal-blocking depth of a solver's
// configuration by timing every supported candidate on the solver's own
// state (saved before and restored after), and caches the choice for the
// process under a key of (lattice, equation, form, precision, levels, grid).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/mfd.h"
#include "mfd_internal.h"
#include "solver.h"

namespace mfd {

namespace {

using Key = std::tuple<int, int, int, int, int, int, int64_t, int64_t, int64_t>;
std::mutex g_mu;
std::map<Key, int> g_cache;

Key key_of(const Solver &s) {
  return Key(s.consts.lattice, s.consts.eq, s.grid.form, s.grid.precision, s.consts.three,
             s.consts.three_stencil, s.G.n[0], s.G.n[1], s.G.n[2]);
}

bool tunable(const Solver &s) {
  return s.grid.form == MFD_MMFD && s.cfg.kind != MFD_THETA && s.consts.eq == kLCDE &&
         s.consts.dim == 2 && (s.consts.lattice == MFD_D2Q5 || s.consts.lattice == MFD_D2Q9);
}

}  // namespace

int Solver::effective_tb() const {
  if (tb > 0) return tb;
  if (tb_tuned > 0) return tb_tuned;
  if (!tunable(*this)) return 1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(key_of(*this));
  if (it != g_cache.end()) return it->second;
  return 4;  // default depth before tuning
}

int Solver::autotune(int32_t *chosen) {
  if (sticky) return fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!tunable(*this) || !state_set) {
    if (chosen) *chosen = effective_tb();
    return MFD_OK;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key_of(*this));
    if (it != g_cache.end()) {
      tb_tuned = it->second;
      if (chosen) *chosen = tb > 0 ? tb : tb_tuned;
      return MFD_OK;
    }
  }
  // save the live levels
  const size_t bytes = (size_t)(mom_elems() * elem());
  void *save[2] = {nullptr, nullptr};
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipMalloc(&save[k], bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (save[0]) (void)hipFree(save[0]);
      return fail(MFD_E_OOM, "autotune: no memory for the state copy");
    }
  }
  int rc = hip(hipMemcpyAsync(save[0], buf[ic], bytes, hipMemcpyDeviceToDevice, stream), "copy");
  if (!rc) rc = hip(hipMemcpyAsync(save[1], buf[ip], bytes, hipMemcpyDeviceToDevice, stream), "copy");
  const int saved_tb = tb;
  const int64_t saved_steps = steps_done;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) rc = hip(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = hip(hipEventCreate(&e1), "hipEventCreate");
  const int cands[5] = {1, 2, 4, 6, 8};
  // enough steps per trial that every candidate runs whole blocks
  const int64_t trial = G.N >= (1 << 20) ? 241 : 481;
  float best_ms = 1e30f;
  int best = 1;
  for (int ci = 0; ci < 5 && !rc; ++ci) {
    const int d = cands[ci];
    if (d > 1 && !lcde_tb_supported(consts, G, d)) continue;
    tb = d;
    rc = step(trial);  // warm-up (also instantiates code objects)
    if (rc) break;
    rc = hip(hipEventRecord(e0, stream), "hipEventRecord");
    if (!rc) rc = step(trial);
    if (!rc) rc = hip(hipEventRecord(e1, stream), "hipEventRecord");
    if (!rc) rc = hip(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    if (!rc) rc = hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (!rc && ms < best_ms) {
      best_ms = ms;
      best = d;
    }
  }
  tb = saved_tb;
  if (!rc) {
    // restore the levels into the current roles
    rc = hip(hipMemcpyAsync(buf[ic], save[0], bytes, hipMemcpyDeviceToDevice, stream), "copy");
    if (!rc) rc = hip(hipMemcpyAsync(buf[ip], save[1], bytes, hipMemcpyDeviceToDevice, stream), "copy");
    if (!rc) rc = hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
  }
  steps_done = saved_steps;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(save[0]);
  (void)hipFree(save[1]);
  if (rc) return rc;
  tb_tuned = best;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key_of(*this)] = best;
  }
  if (chosen) *chosen = tb > 0 ? tb : best;
  return MFD_OK;
}

}  // namespace mfd
