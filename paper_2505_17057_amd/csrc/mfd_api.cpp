// C ABI of the single-grid solver: configuration, state ownership and I/O,
// the step loop (level ring rotation), reductions and the linear stability
// report.  See include/mfd.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mfd.h"
#include "mfd_internal.h"
#include "scheme.h"
#include "solver.h"
#include "mg.h"

using namespace mfd;

namespace mfd {

// Work levels of mfd_step_noalloc: a fixed device array per GPU, held until
// the process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a host-side stand-in); it uses the device address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// device address of `scratch` on the current device (looked up once per
// device, with that device current)
hipError_t noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

namespace {
std::mutex g_alloc_mu;
std::unordered_map<void *, size_t> g_alloc;
int64_t g_alloc_now = 0, g_alloc_peak = 0;
}  // namespace

hipError_t dev_malloc(void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc[*p] = bytes;
  g_alloc_now += (int64_t)bytes;
  if (g_alloc_now > g_alloc_peak) g_alloc_peak = g_alloc_now;
  return e;
}

void dev_free(void *p) {
  if (!p) return;
  (void)hipFree(p);
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  auto it = g_alloc.find(p);
  if (it == g_alloc.end()) return;
  g_alloc_now -= (int64_t)it->second;
  g_alloc.erase(it);
}

int Solver::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
  return code;
}

int Solver::hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return MFD_OK;
  sticky = true;
  return fail(MFD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t Solver::nf() const { return cfg.eq == kNSE ? 1 + grid.dim : 1; }
int64_t Solver::q() const { return consts.q; }

int64_t Solver::mom_elems() const { return nf() * G.N; }
int64_t Solver::pop_elems() const { return grid.form == MFD_MESOFD ? q() * G.N : 0; }

int64_t Solver::device_bytes_needed() const {
  if (!configured) return 0;
  const int64_t es = elem();
  int64_t b = 3 * mom_elems() * es;  // level ring (MMFD) / moment ping-pong + scratch (MesoFD)
  if (grid.form == MFD_MESOFD) b += 2 * pop_elems() * es;
  if (cfg.kind == MFD_THETA) b += 2 * mom_elems() * es + theta_buf_bytes();
  if (grid.form == MFD_MMFD && consts.three && tb_equation_supported(consts))
    b += mom_elems() * es;
  b += (kReduceBlocks * 8 + 8) * (int64_t)sizeof(double);
  b += mg_bytes();
  return b;
}

// three arrays (iterate, right-hand side, scratch) of each coarser level (the
// fine level works in the theta buffers)
int64_t Solver::mg_bytes() const {
  if (cfg.kind != MFD_THETA || mg_levels < 2) return 0;
  int64_t e = 0;
  int64_t nx = G.n[0], ny = G.n[1];
  for (int l = 1; l < mg_levels; ++l) {
    nx /= 2;
    ny /= 2;
    e += 3 * nx * ny;
  }
  return e * elem();
}

// control block and two binary64 partials per tile of the largest chunk
// tiling (tiles hold at least 8 x 8 interior nodes)
int64_t Solver::theta_buf_bytes() const {
  if (cfg.kind != MFD_THETA) return 0;
  const int64_t tiles = (G.n[0] / 8 + 2) * (G.n[1] / 8 + 2);
  return kThetaCtlBytes + 2 * 8 * tiles;
}

void Solver::release() {
  for (auto &p : buf) {
    if (p) dev_free(p);
    p = nullptr;
  }
  allocated_bytes = 0;
}

int Solver::ensure_buffers() {
  if (!configured) return fail(MFD_E_ORDER, "lattice, equation and scheme must be set first");
  const int64_t need = device_bytes_needed();
  if (buf[0] && need == allocated_bytes) return MFD_OK;
  release();
  const int64_t es = elem(), me = mom_elems() * es, pe = pop_elems() * es;
  int64_t sizes[kNumBuf] = {me, me, me, pe, pe, me, me, (kReduceBlocks * 8 + 8) * 8, me,
                            theta_buf_bytes(), mg_bytes()};
  if (cfg.kind != MFD_THETA) sizes[5] = sizes[6] = 0;
  if (!(grid.form == MFD_MMFD && consts.three && tb_equation_supported(consts))) sizes[8] = 0;
  for (int i = 0; i < kNumBuf; ++i) {
    if (sizes[i] == 0) continue;
    hipError_t e = dev_malloc(&buf[i], (size_t)sizes[i]);
    if (e != hipSuccess) {
      release();
      (void)hipGetLastError();
      return fail(MFD_E_OOM, "hipMalloc of %lld bytes failed", (long long)sizes[i]);
    }
    e = hipMemsetAsync(buf[i], 0, (size_t)sizes[i], stream);
    if (e != hipSuccess) return hip(e, "hipMemsetAsync");
  }
  allocated_bytes = need;
  ic = 0; ip = 1; io = 2; pc = 3; pn = 4; ix = 8;
  steps_done = 0;
  return hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
}

int Solver::copy_in(void *dst, const void *src, int64_t bytes, int on_device) {
  hipError_t e = hipMemcpyAsync(dst, src, (size_t)bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip(e, "hipMemcpyAsync (in)");
  return hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
}

int Solver::copy_out(void *dst, const void *src, int64_t bytes, int on_device) {
  hipError_t e = hipMemcpyAsync(dst, src, (size_t)bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip(e, "hipMemcpyAsync (out)");
  return hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
}

template <typename T>
int Solver::step_t(int64_t nsteps) {
  T *B[kNumBuf];
  for (int i = 0; i < kNumBuf; ++i) B[i] = (T *)buf[i];
  if (src_on) {
    // with a source term: one launch per step (3D: the step, then the source)
    if (!source_supported())
      return fail(MFD_E_UNSUPPORTED, "the source term needs the linear CDE with an explicit "
                                     "scheme (MesoFD form: 1D / 2D)");
    src.dt = cfg.dt;
    src.dx = grid.dx;
    if (grid.form == MFD_MESOFD) {
      for (int64_t s = 0; s < nsteps; ++s) {
        const bool final_step = s + 1 == nsteps;
        hipError_t e = launch_mesofd_source_step<T>(consts, G, src, steps_done, B[ic], B[ip],
                                                    final_step ? B[pn] : nullptr, B[io],
                                                    (const T *)d_src, stream);
        if (e != hipSuccess) return hip(e, "mesofd source step launch");
        if (final_step) std::swap(pc, pn);
        const int t = ip;
        ip = ic;
        ic = io;
        io = t;
        ++steps_done;
      }
      prev_gap = 1;
      return MFD_OK;
    }
    // 2D: blocks of d steps in the blocked window (G staged once per launch),
    // then single steps for the remainder
    const TbPlan pl = effective_plan();
    if (pl.tb > 1 && source_tb_supported(consts, G, pl, (int)sizeof(T))) {
      const int d = pl.tb;
      const int64_t nblk = nsteps / d;
      for (int64_t b = 0; b < nblk; ++b) {
        hipError_t e;
        if (!consts.three) {
          e = launch_mmfd_source_tb<T>(consts, G, src, steps_done, pl, B[ic], nullptr, B[ip],
                                       nullptr, (const T *)d_src, stream);
          if (e != hipSuccess) return hip(e, "blocked source launch");
          std::swap(ic, ip);
        } else {
          e = launch_mmfd_source_tb<T>(consts, G, src, steps_done, pl, B[ic], B[ip], B[io], B[ix],
                                       (const T *)d_src, stream);
          if (e != hipSuccess) return hip(e, "blocked source launch");
          const int oc = ic, op = ip;
          ic = io;
          ip = ix;
          io = oc;
          ix = op;
        }
        steps_done += d;
      }
      nsteps -= nblk * d;
      if (nblk > 0) prev_gap = consts.three ? 1 : d;
    }
    for (int64_t s = 0; s < nsteps; ++s) {
      T *out = consts.three ? B[io] : B[ip];
      hipError_t e = launch_mmfd_source_step<T>(consts, G, src, steps_done, B[ic], B[ip], out,
                                                (const T *)d_src, stream);
      if (e != hipSuccess) return hip(e, "source step launch");
      if (!consts.three) {
        std::swap(ic, ip);
      } else {
        const int t = ip;
        ip = ic;
        ic = io;
        io = t;
      }
      ++steps_done;
    }
    if (nsteps > 0) prev_gap = 1;
    return MFD_OK;
  }
  if (cfg.kind != MFD_THETA && wave1d_applies(consts, G) && nsteps > 1) {
    // the whole run in one wavefront's registers; levels stay in place
    const bool meso = grid.form == MFD_MESOFD;
    hipError_t e = launch_1d_wave<T>(consts, G, meso, B[ic], B[ip], meso ? B[pc] : nullptr,
                                     nsteps, stream);
    if (e != hipSuccess) return hip(e, "1d wavefront launch");
    steps_done += nsteps;
    prev_gap = 1;
    return MFD_OK;
  }
  if (grid.form == MFD_MMFD && cfg.kind != MFD_THETA && mmfd_1d_resident_fits(consts, G, sizeof(T)) &&
      nsteps > 1) {
    // ga = level t, gb = level t - dt; afterwards the same roles
    hipError_t e = launch_mmfd_1d_resident<T>(consts, G, B[ic], B[ip], B[io], nsteps, stream);
    if (e != hipSuccess) return hip(e, "mmfd 1d resident launch");
    steps_done += nsteps;
    return MFD_OK;
  }
  if (grid.form == MFD_MESOFD && mesofd_1d_resident_fits(consts, G, sizeof(T)) && nsteps > 1) {
    // levels stay in place: B[ic] / B[ip] in and out, final populations in pop[pc]
    hipError_t e = launch_mesofd_1d_resident<T>(consts, G, B[ic], B[ip], B[pc], nsteps, stream);
    if (e != hipSuccess) return hip(e, "mesofd 1d resident launch");
    steps_done += nsteps;
    prev_gap = 1;
    return MFD_OK;
  }
  if (cfg.kind == MFD_THETA && mg_levels >= 2 && consts.eq == kLCDE && grid.dim == 2)
    return theta_mg_steps<T>(nsteps);
  if (cfg.kind == MFD_THETA && (consts.eq == kBurgers || consts.eq == kNSE))
    return theta_picard_steps<T>(nsteps);
  if (cfg.kind == MFD_THETA && theta_tol > 0.0) return theta_solve_steps<T>(nsteps);
  const TbPlan pl = effective_plan();
  const int d = pl.tb;
  if (grid.form == MFD_MMFD && cfg.kind != MFD_THETA && d > 1 &&
      tb_supported(consts, G, pl, (int)sizeof(T))) {
    // blocks of d steps, then single steps for the remainder.  A two-level
    // block returns only its last level, so after it the held previous level
    // is d steps old (prev_gap = d), which the residual accounts for.
    const int64_t nblk = nsteps / d;
    for (int64_t b = 0; b < nblk; ++b) {
      hipError_t e;
      const DirBC bc = dir_bc(steps_done + b * d, d);
      if (!consts.three) {
        e = launch_mmfd_tb<T>(consts, G, pl, B[ic], nullptr, B[ip], nullptr, stream, &bc);
        if (e != hipSuccess) return hip(e, "blocked step launch");
        std::swap(ic, ip);
      } else {
        e = launch_mmfd_tb<T>(consts, G, pl, B[ic], B[ip], B[io], B[ix], stream, &bc);
        if (e != hipSuccess) return hip(e, "blocked step launch");
        const int oc = ic, op = ip;
        ic = io;
        ip = ix;
        io = oc;
        ix = op;
      }
    }
    nsteps -= nblk * d;
    steps_done += nblk * d;
    if (nblk > 0) prev_gap = consts.three ? 1 : d;
  }
  if (nsteps > 0) prev_gap = 1;
  for (int64_t s = 0; s < nsteps; ++s) {
    hipError_t e;
    if (grid.form == MFD_MMFD) {
      if (cfg.kind == MFD_THETA && theta_fused_rows(consts, G, cfg.theta_iters, (int)sizeof(T))) {
        e = launch_theta_fused<T>(consts, G, cfg.theta_iters, B[ic], B[io], stream);
        if (e != hipSuccess) return hip(e, "fused theta launch");
        std::swap(ic, io);
        ip = io;
      } else if (cfg.kind == MFD_THETA) {
        // rhs -> buf 5, sweeps alternate io / buf 6, final in io
        e = launch_theta_rhs<T>(consts, G, B[ic], B[5], stream);
        if (e != hipSuccess) return hip(e, "theta rhs launch");
        const T *src = B[ic];
        const int it = cfg.theta_iters;
        for (int k = 0; k < it; ++k) {
          T *dst = ((it - k) % 2 == 1) ? B[io] : B[6];
          e = launch_theta_sweep<T>(consts, G, src, B[5], dst, stream);
          if (e != hipSuccess) return hip(e, "theta sweep launch");
          src = dst;
        }
        if (it == 0) {
          e = hipMemcpyAsync(B[io], B[ic], mom_elems() * sizeof(T), hipMemcpyDeviceToDevice, stream);
          if (e != hipSuccess) return hip(e, "theta copy");
        }
        std::swap(ic, io);  // two-level: old current becomes prev
        ip = io;
      } else if (!consts.three) {
        const DirBC bc = dir_bc(steps_done + s, 1);
        e = launch_mmfd_step<T>(consts, G, B[ic], B[ip], B[ip], tb, stream, &bc);
        if (e != hipSuccess) return hip(e, "mmfd step launch");
        std::swap(ic, ip);
      } else {
        const DirBC bc = dir_bc(steps_done + s, 1);
        e = launch_mmfd_step<T>(consts, G, B[ic], B[ip], B[io], tb, stream, &bc);
        if (e != hipSuccess) return hip(e, "mmfd step launch");
        const int t = ip;
        ip = ic;
        ic = io;
        io = t;
      }
    } else if (d > 1 && plan_supported(pl) && s + d <= nsteps) {
      // blocked MesoFD: d steps; moments of t + d into B[io]; the held
      // previous level is d steps old.  The populations of t + d go to
      // pop[pn] only when no step follows in this call: a step reads the one
      // before through its moments alone, so only the call's last
      // populations are ever read.
      const bool final_launch = s + d == nsteps;
      e = launch_mesofd_tb<T>(consts, G, pl, B[ic], B[io], final_launch ? B[pn] : nullptr, stream);
      if (e != hipSuccess) return hip(e, "blocked mesofd launch");
      if (final_launch) std::swap(pc, pn);
      const int t = ip;
      ip = ic;
      ic = io;
      io = t;
      s += d - 1;
      prev_gap = d;
    } else {
      // MesoFD: moments of t in B[ic] and of t-dt in B[ip]; writes the new
      // moments into B[io] and, at the call's last step, the populations
      // they sum into pop[pn] (no step reads populations); then rotate.
      const bool final_step = s + 1 == nsteps;
      e = launch_mesofd_step<T>(consts, G, B[ic], B[ip], final_step ? B[pn] : nullptr, B[io],
                                stream);
      if (e != hipSuccess) return hip(e, "mesofd step launch");
      if (final_step) std::swap(pc, pn);
      const int t = ip;
      ip = ic;
      ic = io;
      io = t;
      prev_gap = 1;
    }
  }
  steps_done += nsteps;
  return MFD_OK;
}

// Dirichlet values of the launch that writes steps first_step + 1 .. +nsteps
DirBC Solver::dir_bc(int64_t first_step, int nsteps) const {
  DirBC b;
  std::memset(&b, 0, sizeof(b));
  if (!dirichlet) return b;
  b.on = 1;
  b.Gb = (const double *)d_bnd;
  for (int s = 1; s <= nsteps && s <= kMaxBcSteps; ++s)
    b.E[s] = std::exp(bnd_lambda * ((double)(first_step + s) * cfg.dt));
  return b;
}

// Theta steps solved to a tolerance.  2D grids the fused window takes: the
// chunk sequence is decided on the device (no host round trip per step);
// others: one host check per chunk of sweeps.
template <typename T>
int Solver::theta_solve_steps(int64_t nsteps) {
  T *B[kNumBuf];
  for (int i = 0; i < kNumBuf; ++i) B[i] = (T *)buf[i];
  const int K = theta_chunk;
  const int cap = cfg.theta_iters;
  const int nchunk = (cap + K - 1) / K;
  const int64_t part_cap = (theta_buf_bytes() - kThetaCtlBytes) / 16;
  const int tiles = theta_solve_tiles(consts, G, K, (int)sizeof(T));
  if (tiles > 0 && tiles <= part_cap) {
    ThetaCtl *ctl = (ThetaCtl *)buf[kThetaBuf];
    double *part = (double *)((char *)buf[kThetaBuf] + kThetaCtlBytes);
    T *const ring[4] = {B[ic], B[ip], B[5], B[6]};
    hipError_t e = launch_theta_ctl_init<T>(ctl, stream);
    if (e != hipSuccess) return hip(e, "theta control launch");
    for (int64_t s = 0; s < nsteps; ++s)
      for (int c = 0; c < nchunk; ++c) {
        e = launch_theta_chunk<T>(consts, G, K, ring, ctl, part, theta_tol, cap, c == 0, stream);
        if (e != hipSuccess) return hip(e, "theta chunk launch");
      }
    e = launch_theta_gather<T>(ring, ctl, G.N, stream);
    if (e != hipSuccess) return hip(e, "theta gather launch");
    steps_done += nsteps;
    prev_gap = 1;
    return MFD_OK;
  }
  // host-checked chunks: rhs into B[5]; iterates alternate B[io] / B[6]
  double *part = (double *)buf[kRedBuf];
  double *out = part + kReduceBlocks * 8;
  const double den = theta_den(consts);
  for (int64_t s = 0; s < nsteps; ++s) {
    hipError_t e = launch_theta_rhs<T>(consts, G, B[ic], B[5], stream);
    if (e != hipSuccess) return hip(e, "theta rhs launch");
    const T *src = B[ic];
    int k = 0;
    bool conv = false;
    while (true) {
      const T *before = src;
      for (int it = 0; it < K; ++it) {
        T *dst = (k % 2 == 0) ? B[io] : B[6];
        e = launch_theta_sweep<T>(consts, G, src, B[5], dst, stream);
        if (e != hipSuccess) return hip(e, "theta sweep launch");
        before = src;
        src = dst;
        ++k;
      }
      e = launch_sq_sums<T>(src, before, B[5], 1, G.N, part, out, stream);
      if (e != hipSuccess) return hip(e, "theta residual launch");
      double h[2];
      int rc = copy_out(h, out, sizeof(h), 0);
      if (rc) return rc;
      if (!std::isfinite(h[0]) || !std::isfinite(h[1]))
        return fail(MFD_E_UNSTABLE, "non-finite theta residual");
      conv = den * den * h[0] <= theta_tol * theta_tol * h[1];
      if (conv || k >= cap) break;
    }
    if (src == B[6]) {  // the result is kept in the io role
      std::swap(buf[io], buf[6]);
      std::swap(B[io], B[6]);
    }
    std::swap(ic, io);
    ip = io;
    ++steps_done;
    th_total += k;
    ++th_steps;
    th_max = std::max(th_max, k);
    if (!conv) ++th_unconv;
  }
  prev_gap = 1;
  return MFD_OK;
}

// Theta steps of Burgers' equation (beta = 1) and of the NSE: Picard
// iteration with the Jacobi splitting of the linear part's diagonal, per
// field (chunks of theta_chunk sweeps checked on the host when a tolerance
// is set, else theta_iters sweeps).
//   density (and the scalar):  A0,  dd = 2 sum_p (a_1 + a_-1) w_p
//   momentum component a:      Ab0, dd = 2 sum_{p: e_pa != 0} (ab_1 + ab_-1) (w_p / d0)
// (pairs in lattice order): the own-node coefficient of the second
// differences of the linear parts, w_p rho of F+ and (w_p / d0) e_p . j of
// F-; the off-diagonal and nonlinear terms stay in S(x) - A0 x.
template <typename T>
int Solver::theta_picard_steps(int64_t nsteps) {
  T *B[kNumBuf];
  for (int i = 0; i < kNumBuf; ++i) B[i] = (T *)buf[i];
  const bool tol_on = theta_tol > 0.0;
  const int cap = cfg.theta_iters;
  const int K = tol_on ? theta_chunk : cap;
  const int third = 3 - ic - io;  // the ring level neither phi^n nor the io role holds
  const double th = consts.theta, th1 = consts.th1;
  const int F = nf();
  double A0[4], dd[4], den[4], inv_den[4];
  {
    double sp = 0.0;
    for (int p = 0; p < consts.npair; ++p) sp = sp + consts.ap * consts.w[consts.pair[p]];
    A0[0] = consts.A0;
    dd[0] = 2.0 * sp;
    const double abp = consts.abp;
    for (int f = 1; f < F; ++f) {
      double sj = 0.0;
      for (int p = 0; p < consts.npair; ++p) {
        const int j = consts.pair[p];
        if (consts.e[j][f - 1] != 0) sj = sj + abp * (consts.w[j] / consts.d0);
      }
      A0[f] = consts.Ab0;
      dd[f] = 2.0 * sj;
    }
    for (int f = 0; f < F; ++f) {
      den[f] = 1.0 + th1 * dd[f];
      inv_den[f] = 1.0 / den[f];
    }
  }
  // Burgers on 1D / 2D grids and the 2D NSE: the sweep fused into the
  // explicit step's tile
  const bool fused = (consts.eq == kBurgers && consts.dim <= 2) ||
                     (consts.eq == kNSE && consts.dim == 2);
  double *part = (double *)buf[kRedBuf];
  double *out = part + kReduceBlocks * 8;
  const int64_t N = G.N;
  for (int64_t s = 0; s < nsteps; ++s) {
    hipError_t e;
    if (fused && consts.eq == kNSE) {
      e = launch_picard_rhs_step<T>(consts, G, B[ic], B[5], A0, th, th1, stream);
    } else {
      e = launch_mmfd_step<T>(consts, G, B[ic], nullptr, B[6], 1, stream);
      if (e == hipSuccess) e = launch_picard_rhs<T>(B[6], B[ic], B[5], th, th1, F, A0, N, stream);
    }
    if (e != hipSuccess) return hip(e, "picard rhs launch");
    const T *src = B[ic];
    int k = 0;
    bool conv = false;
    while (true) {
      const T *before = src;
      int rows = 0;  // residual rows the chunk's last sweep wrote (fused NSE sweep)
      for (int it = 0; it < K; ++it) {
        T *dst = (k % 2 == 0) ? B[io] : B[third];
        if (fused) {
          e = launch_picard_sweep<T>(consts, G, src, B[5], dst, A0, dd, th1, inv_den,
                                     tol_on && it == K - 1 ? part : nullptr, &rows, stream);
        } else {
          e = launch_mmfd_step<T>(consts, G, src, nullptr, B[6], 1, stream);
          if (e == hipSuccess)
            e = launch_picard_update<T>(B[6], src, B[5], dst, F, A0, dd, th1, inv_den, N, stream);
        }
        if (e != hipSuccess) return hip(e, "picard sweep launch");
        before = src;
        src = dst;
        ++k;
      }
      if (!tol_on) break;
      // sum_f den_f^2 |x_k - x_(k-1)|_f^2 <= tol^2 sum_f |R|_f^2 (field f's two
      // sums in out[2 f], out[2 f + 1]; one copy to the host)
      e = rows > 0 ? launch_final_sums(part, rows, 2 * F, out, stream)
                   : launch_sq_sums<T>(src, before, B[5], F, N, part, out, stream);
      if (e != hipSuccess) return hip(e, "picard residual launch");
      double hsum[8];
      const int rc = copy_out(hsum, out, 2 * F * sizeof(double), 0);
      if (rc) return rc;
      double lhs = 0.0, rhs = 0.0;
      for (int f = 0; f < F; ++f) {
        if (!std::isfinite(hsum[2 * f]) || !std::isfinite(hsum[2 * f + 1]))
          return fail(MFD_E_UNSTABLE, "non-finite theta residual");
        lhs = lhs + den[f] * den[f] * hsum[2 * f];
        rhs = rhs + hsum[2 * f + 1];
      }
      conv = lhs <= theta_tol * theta_tol * rhs;
      if (conv || k >= cap) break;
    }
    if (src == B[third]) {  // the result is kept in the io role
      std::swap(buf[io], buf[third]);
      std::swap(B[io], B[third]);
    }
    std::swap(ic, io);
    ip = io;
    ++steps_done;
    if (tol_on) {
      th_total += k;
      ++th_steps;
      th_max = std::max(th_max, k);
      if (!conv) ++th_unconv;
    }
  }
  prev_gap = 1;
  return MFD_OK;
}

// Theta steps of the 2D linear CDE by multigrid V-cycles (kernels_mg.hip):
// per step the right-hand side R = A0 phi + theta L phi, then V(pre, post)
// cycles from x = phi, each followed by the binary64 check
//   sum (R - A x)^2 <= tol^2 sum R^2
// (tol = 0: exactly theta_iters cycles); theta_iters caps the cycles.
template <typename T>
int Solver::theta_mg_steps(int64_t nsteps) {
  T *B[kNumBuf];
  for (int i = 0; i < kNumBuf; ++i) B[i] = (T *)buf[i];
  const int L = mg_levels;
  const int lat = consts.lattice;
  const bool tol_on = theta_tol > 0.0;
  const int cap = cfg.theta_iters;
  int nxl[kMgMaxLevels], nyl[kMgMaxLevels];
  MgOp<T> op[kMgMaxLevels];
  T *xl[kMgMaxLevels], *tl[kMgMaxLevels], *Rl[kMgMaxLevels];
  {
    T *m = B[kMgBuf];
    nxl[0] = (int)G.n[0];
    nyl[0] = (int)G.n[1];
    tl[0] = B[6];  // the fine level's second iterate array
    Rl[0] = B[5];
    for (int l = 1; l < L; ++l) {
      nxl[l] = nxl[l - 1] / 2;
      nyl[l] = nyl[l - 1] / 2;
      const int64_t n = (int64_t)nxl[l] * nyl[l];
      xl[l] = m;
      Rl[l] = m + n;
      tl[l] = m + 2 * n;
      m += 3 * n;
    }
    for (int l = 0; l < L; ++l) op[l] = mg_op<T>(consts, l, nxl[l], nyl[l]);
  }
  // the coarsest level's sweeps: enough to reduce its error 1000-fold at the
  // weighted Jacobi bound (1 - w) + w (den - 1) / den (its off-diagonal sum
  // is at most den - 1 while |Cm| <= Cp), between 2 and kMgCoarseSweeps
  int coarse_sweeps = kMgCoarseSweeps;
  {
    const double den = (double)op[L - 1].den;
    const double rho = (1.0 - kMgOmega) + kMgOmega * (den - 1.0) / den;
    if (rho > 0.0 && rho < 1.0)
      coarse_sweeps = std::max(2, std::min(kMgCoarseSweeps, (int)std::ceil(std::log(1e-3) / std::log(rho))));
  }
  double *part = (double *)buf[kRedBuf];
  double *out = part + kReduceBlocks * 8;
  const int64_t N = G.N;
  hipError_t e = hipSuccess;
  // smoothing sweeps on level l between its iterate and scratch arrays
  auto smooth = [&](int l, T *&cur, T *&oth, int sweeps, bool from_zero) {
    for (int k = 0; k < sweeps && e == hipSuccess; ++k) {
      e = launch_mg_smooth<T>(lat, cur, Rl[l], oth, op[l], kMgOmega, from_zero && k == 0, stream);
      std::swap(cur, oth);
    }
  };
  for (int64_t s = 0; s < nsteps; ++s) {
    e = launch_theta_rhs<T>(consts, G, B[ic], B[5], stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(B[io], B[ic], (size_t)(N * sizeof(T)), hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip(e, "multigrid rhs");
    T *cur[kMgMaxLevels], *oth[kMgMaxLevels];
    cur[0] = B[io];
    oth[0] = tl[0];
    int k = 0;
    bool conv = false;
    while (true) {
      // down: pre-smooth, restrict the residual; coarse levels start from 0
      for (int l = 0; l + 1 < L; ++l) {
        if (l > 0) {
          cur[l] = xl[l];
          oth[l] = tl[l];
        }
        smooth(l, cur[l], oth[l], mg_pre, l > 0);
        // the residual into the free array, then its restriction
        if (e == hipSuccess) e = launch_mg_residual<T>(lat, cur[l], Rl[l], oth[l], op[l], stream);
        if (e == hipSuccess) e = launch_mg_restrict_r<T>(oth[l], Rl[l + 1], nxl[l], nyl[l], stream);
      }
      cur[L - 1] = xl[L - 1];
      oth[L - 1] = tl[L - 1];
      smooth(L - 1, cur[L - 1], oth[L - 1], coarse_sweeps, true);
      // up: add the prolongated correction, post-smooth
      for (int l = L - 2; l >= 0; --l) {
        if (e == hipSuccess) e = launch_mg_prolong_add<T>(cur[l + 1], cur[l], nxl[l], nyl[l], stream);
        smooth(l, cur[l], oth[l], mg_post, false);
      }
      if (e != hipSuccess) return hip(e, "multigrid cycle launch");
      ++k;
      if (tol_on) {
        e = launch_mg_resid_norm<T>(lat, cur[0], B[5], op[0], part, out, stream);
        if (e != hipSuccess) return hip(e, "multigrid residual launch");
        double h[2];
        int rc = copy_out(h, out, sizeof(h), 0);
        if (rc) return rc;
        if (!std::isfinite(h[0]) || !std::isfinite(h[1]))
          return fail(MFD_E_UNSTABLE, "non-finite theta residual");
        conv = h[0] <= theta_tol * theta_tol * h[1];
        if (conv || k >= cap) break;
      } else if (k >= cap) {
        break;
      }
    }
    if (cur[0] != B[io]) {  // the result is kept in the io role
      std::swap(buf[io], buf[6]);
      std::swap(B[io], B[6]);
      tl[0] = B[6];
    }
    std::swap(ic, io);
    ip = io;
    ++steps_done;
    if (tol_on) {
      th_total += k;
      ++th_steps;
      th_max = std::max(th_max, k);
      if (!conv) ++th_unconv;
    }
  }
  prev_gap = 1;
  return MFD_OK;
}

bool Solver::source_supported() const {
  if (cfg.kind == MFD_THETA || consts.eq != kLCDE || consts.wave || dirichlet || cfg.rect)
    return false;
  return grid.form == MFD_MMFD || grid.dim <= 2;  // MesoFD: 1D / 2D
}

int Solver::step(int64_t nsteps) {
  if (sticky) return fail(MFD_E_HIP, "solver is in a failed HIP state: %s", err.c_str());
  if (nsteps < 0) return fail(MFD_E_ARG, "nsteps < 0");
  if (!state_set) return fail(MFD_E_ORDER, "state not set");
  if (dirichlet && !bnd_set) return fail(MFD_E_ORDER, "Dirichlet values not set (mfd_set_boundary)");
  if (nsteps == 0) return MFD_OK;
  if (check_every <= 0)
    return grid.precision == MFD_FP64 ? step_t<double>(nsteps) : step_t<float>(nsteps);
  // the steps in runs of check_every, each followed by the FP64 reduction;
  // a run ends as it would inside one call (the blocked kernels give the
  // single-step values), so the check changes no result
  for (int64_t done = 0; done < nsteps;) {
    const int64_t k = std::min(check_every, nsteps - done);
    int rc = grid.precision == MFD_FP64 ? step_t<double>(k) : step_t<float>(k);
    if (rc) return rc;
    done += k;
    rc = reduce(nullptr, nullptr);
    if (rc) return rc;
  }
  return MFD_OK;
}

int Solver::reduce(double sums[4], double *residual) {
  if (sticky) return fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!state_set) return fail(MFD_E_ORDER, "state not set");
  double *part = (double *)buf[kRedBuf];
  double *out = part + kReduceBlocks * 8;
  const bool have_prev = steps_done > 0;
  hipError_t e;
  if (grid.precision == MFD_FP64) {
    const double *cur = (const double *)buf[ic];
    const double *prev = have_prev ? (const double *)buf[ip] : nullptr;
    e = launch_reduce<double>(cur, prev, (int)nf(), G.N, part, out, stream);
  } else {
    const float *cur = (const float *)buf[ic];
    const float *prev = have_prev ? (const float *)buf[ip] : nullptr;
    e = launch_reduce<float>(cur, prev, (int)nf(), G.N, part, out, stream);
  }
  if (e != hipSuccess) return hip(e, "reduce launch");
  double host[8];
  int rc = copy_out(host, out, sizeof(host), 0);
  if (rc) return rc;
  bool finite = std::isfinite(host[4]);
  for (int f = 0; f < nf(); ++f) finite = finite && std::isfinite(host[f]);
  if (!finite) return fail(MFD_E_UNSTABLE, "non-finite moment sum or residual");
  if (sums)
    for (int f = 0; f < 4; ++f) sums[f] = f < nf() ? host[f] : 0.0;
  if (residual) *residual = std::sqrt(host[4]) / (double)prev_gap;
  return MFD_OK;
}

}  // namespace mfd

// ================================================================ C ABI

#define SOLVER_OR_ARG(s) \
  if (!(s)) return MFD_E_ARG;

extern "C" int mfd_create(mfd_solver **out, const mfd_grid *g) {
  if (!out || !g) return MFD_E_ARG;
  if (g->dim < 1 || g->dim > 3) return MFD_E_ARG;
  if (g->boundary != MFD_PERIODIC && g->boundary != MFD_DIRICHLET) return MFD_E_ARG;
  if (g->boundary == MFD_DIRICHLET && (g->dim != 2 || g->form != MFD_MMFD))
    return MFD_E_UNSUPPORTED;
  if (g->precision != MFD_FP64 && g->precision != MFD_FP32) return MFD_E_ARG;
  if (g->form != MFD_MMFD && g->form != MFD_MESOFD) return MFD_E_ARG;
  if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return MFD_E_ARG;
  int64_t N = 1;
  for (int a = 0; a < 3; ++a) {
    const int64_t n = a < g->dim ? g->n[a] : 1;
    if (a < g->dim && (n < 3 || n > (int64_t)1 << 30)) return MFD_E_ARG;
    if (a >= g->dim && g->n[a] != 1 && g->n[a] != 0) return MFD_E_ARG;
    N *= n;
    if (N > ((int64_t)1 << 34)) return MFD_E_ARG;
  }
  Solver *s = new (std::nothrow) Solver();
  if (!s) return MFD_E_OOM;
  s->grid = *g;
  s->dirichlet = g->boundary == MFD_DIRICHLET;
  for (int a = 0; a < 3; ++a) s->G.n[a] = a < g->dim ? g->n[a] : 1;
  s->G.N = N;
  *out = reinterpret_cast<mfd_solver *>(s);
  return MFD_OK;
}

extern "C" int mfd_destroy(mfd_solver *h) {
  if (!h) return MFD_OK;
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->buf[0] || s->d_src || s->d_bnd) (void)hipStreamSynchronize(s->stream);
  s->release();
  if (s->d_src) dev_free(s->d_src);
  if (s->d_bnd) dev_free(s->d_bnd);
  delete s;
  return MFD_OK;
}

extern "C" int mfd_memory_stats(int64_t *in_use, int64_t *peak, int reset_peak) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (in_use) *in_use = g_alloc_now;
  if (peak) *peak = g_alloc_peak;
  if (reset_peak) g_alloc_peak = g_alloc_now;
  return MFD_OK;
}

extern "C" const char *mfd_last_error(const mfd_solver *h) {
  if (!h) return "null solver";
  return reinterpret_cast<const Solver *>(h)->err.c_str();
}

static int rebuild(Solver *s) {
  s->configured = false;
  if (!s->have_lattice || !s->have_eq || !s->have_scheme) return MFD_OK;
  SchemeInput in;
  std::memset(&in, 0, sizeof(in));
  in.lattice = s->cfg.lattice;
  in.d0 = s->cfg.d0;
  in.eq = s->cfg.eq;
  in.kind = s->cfg.kind;
  for (int k = 0; k < 3; ++k) {
    in.a[k] = s->cfg.a[k];
    in.ah[k] = s->cfg.kind == MFD_THREE_LEVEL ? s->cfg.ah[k] : 0.0;
    in.ab[k] = s->cfg.ab[k];
    in.abh[k] = s->cfg.kind == MFD_THREE_LEVEL ? s->cfg.abh[k] : 0.0;
  }
  in.theta = s->cfg.theta;
  in.dt = s->cfg.dt;
  in.dx = s->grid.dx;
  for (int a = 0; a < 3; ++a) in.u[a] = s->cfg.ep.u[a];
  for (int i = 0; i < 9; ++i) in.K[i] = s->cfg.ep.K[i];
  in.lambda_bar = s->cfg.ep.lambda_bar;
  in.beta = s->cfg.ep.beta;
  in.rho0 = s->cfg.ep.rho0;
  in.he_luo = s->cfg.ep.he_luo;
  in.multiset = s->cfg.multiset;
  in.rect = s->cfg.rect;
  for (int k = 0; k < 3; ++k) {
    in.d0v[k] = s->cfg.d0v[k];
    in.dxv[k] = s->cfg.dxv[k];
  }
  for (int k = 0; k < 3; ++k) {
    in.ae[k] = s->cfg.ae[k];
    in.ao[k] = s->cfg.ao[k];
    in.aeh[k] = s->cfg.kind == MFD_THREE_LEVEL ? s->cfg.aeh[k] : 0.0;
    in.aoh[k] = s->cfg.kind == MFD_THREE_LEVEL ? s->cfg.aoh[k] : 0.0;
  }
  int rc = build_consts(in, s->consts);
  if (rc) return s->fail(rc, "scheme constants could not be formed");
  s->configured = true;
  s->state_set = false;
  return MFD_OK;
}

extern "C" int mfd_set_lattice(mfd_solver *h, int lattice, double d0) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (d0 <= 0.0) d0 = 1.0 / 3.0;
  Consts c;
  std::memset(&c, 0, sizeof(c));
  if (lattice_weights(lattice, d0, c) != MFD_OK)
    return s->fail(MFD_E_ARG, "lattice %d with d0 = %g has a non-positive weight", lattice, d0);
  if (c.dim != s->grid.dim)
    return s->fail(MFD_E_ARG, "lattice dimension %d differs from grid dimension %d", c.dim,
                   s->grid.dim);
  if (!(d0 < 1.0)) return s->fail(MFD_E_ARG, "d0 must lie in (0, 1)");
  if (lattice == MFD_D3Q27)
    return s->fail(MFD_E_UNSUPPORTED, "rD3Q27 runs through the general-scheme solver (mfd_general_*)");
  s->cfg.lattice = lattice;
  s->cfg.d0 = d0;
  s->cfg.rect = 0;  // a new lattice is square until mfd_set_rectangular
  s->have_lattice = true;
  return rebuild(s);
}

extern "C" int mfd_set_rectangular(mfd_solver *h, const double dx[3], const double d0[3]) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!dx || !d0) return s->fail(MFD_E_ARG, "null spacing or d0");
  if (!s->have_lattice) return s->fail(MFD_E_ORDER, "mfd_set_lattice must precede mfd_set_rectangular");
  if (s->have_eq && s->cfg.eq != MFD_LCDE)
    return s->fail(MFD_E_UNSUPPORTED, "rectangular lattices are implemented for the linear CDE");
  if (s->src_on)
    return s->fail(MFD_E_UNSUPPORTED, "the source term is implemented for square lattices");
  const int dim = s->grid.dim;
  double dv[3], xv[3];
  for (int a = 0; a < 3; ++a) {
    dv[a] = a < dim ? d0[a] : d0[0];
    xv[a] = a < dim ? dx[a] : dx[0];
    if (!(dv[a] > 0.0 && dv[a] < 1.0) || !(xv[a] > 0.0) || !std::isfinite(xv[a]))
      return s->fail(MFD_E_ARG, "d0 per axis must lie in (0, 1) and the spacing be positive");
  }
  Consts c;
  std::memset(&c, 0, sizeof(c));
  const int rc = lattice_weights_v(s->cfg.lattice, dv, c);
  if (rc == MFD_E_UNSUPPORTED)
    return s->fail(rc, "rD2Q5II and rD3Q9 take one d0 on every axis");
  if (rc) return s->fail(MFD_E_ARG, "a weight of the lattice is not positive for these d0");
  s->cfg.rect = 1;
  for (int a = 0; a < 3; ++a) {
    s->cfg.d0v[a] = dv[a];
    s->cfg.dxv[a] = xv[a];
  }
  return rebuild(s);
}

extern "C" int mfd_set_equation(mfd_solver *h, int eq, const mfd_eq_params *p) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!p) return s->fail(MFD_E_ARG, "null equation parameters");
  if (eq != MFD_LCDE && eq != MFD_BURGERS && eq != MFD_NSE && eq != MFD_WAVE)
    return s->fail(MFD_E_ARG, "unknown equation %d", eq);
  if (s->cfg.rect && eq != MFD_LCDE)
    return s->fail(MFD_E_UNSUPPORTED, "rectangular lattices are implemented for the linear CDE");
  if (eq == MFD_NSE && s->dirichlet)
    return s->fail(MFD_E_UNSUPPORTED, "Dirichlet boundaries are implemented for scalar equations");
  if (eq == MFD_WAVE && !(p->beta == 0.0 || (p->beta > 0.0 && std::isfinite(p->beta))))
    return s->fail(MFD_E_ARG, "the wave EDF needs beta > 0");
  if (eq == MFD_NSE && s->grid.dim == 1)
    return s->fail(MFD_E_UNSUPPORTED, "the NSE needs a 2D or 3D lattice");
  if (eq == MFD_NSE && !p->he_luo && p->rho0 != 0.0 && !std::isfinite(p->rho0))
    return s->fail(MFD_E_ARG, "rho0 must be finite");
  if (eq == MFD_NSE && p->he_luo && !(p->rho0 > 0.0))
    return s->fail(MFD_E_ARG, "He-Luo EDF needs rho0 > 0");
  s->cfg.eq = eq;
  s->cfg.ep = *p;
  if ((eq == MFD_BURGERS || eq == MFD_WAVE) && p->beta == 0.0) s->cfg.ep.beta = 1.0;
  s->have_eq = true;
  int rc = rebuild(s);
  if (rc < 0) return rc;
  if (eq == MFD_LCDE && s->have_lattice && s->cfg.lattice == MFD_D2Q5 && s->configured) {
    const double *C = s->consts.Ch;
    if (C[0] != 0.0 || C[4] != 0.0 || C[1] != 0.0) {
      s->fail(MFD_W_INCONSISTENT, "D2Q5 cannot represent a non-zero EDF tensor C");
      return MFD_W_INCONSISTENT;
    }
  }
  return MFD_OK;
}

extern "C" int mfd_set_scheme(mfd_solver *h, int kind, const double a[3], const double ah[3],
                              const double ab[3], const double abh[3], double theta,
                              int32_t theta_iters, double dt) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!s->have_lattice || !s->have_eq)
    return s->fail(MFD_E_ORDER, "mfd_set_lattice and mfd_set_equation must precede mfd_set_scheme");
  if (!a) return s->fail(MFD_E_ARG, "null coefficients");
  if (kind != MFD_TWO_LEVEL && kind != MFD_THETA && kind != MFD_THREE_LEVEL)
    return s->fail(MFD_E_ARG, "unknown scheme kind %d", kind);
  if (kind == MFD_THREE_LEVEL && !ah) return s->fail(MFD_E_ARG, "three-level scheme needs ah");
  if (!(dt > 0.0) || !std::isfinite(dt)) return s->fail(MFD_E_ARG, "dt must be positive");
  if (kind == MFD_THETA) {
    if (s->dirichlet)
      return s->fail(MFD_E_UNSUPPORTED, "the theta scheme runs on periodic grids");
    if (s->cfg.eq != MFD_LCDE && s->cfg.eq != MFD_NSE &&
        !(s->cfg.eq == MFD_BURGERS && (s->cfg.ep.beta == 1.0 || s->cfg.ep.beta == 0.0)))
      return s->fail(MFD_E_UNSUPPORTED, "the theta scheme is implemented for the LCDE, "
                                        "Burgers' equation (beta = 1) and the NSE");
    if (!(theta >= 0.0 && theta <= 1.0) || theta_iters < 0)
      return s->fail(MFD_E_ARG, "theta must lie in [0,1] and theta_iters >= 0");
    if (s->grid.form != MFD_MMFD)
      return s->fail(MFD_E_UNSUPPORTED, "the theta scheme is a moment (MMFD) scheme");
  }
  for (int k = 0; k < 3; ++k) {
    const double v[4] = {a[k], ah ? ah[k] : 0.0, ab ? ab[k] : a[k], abh ? abh[k] : (ah ? ah[k] : 0.0)};
    for (double x : v)
      if (!std::isfinite(x)) return s->fail(MFD_E_ARG, "non-finite coefficient");
  }
  if (kind == MFD_THREE_LEVEL && s->grid.precision == MFD_FP32) {
    // the binary32 kernels form the base as phi - Ah0 (phi - phi^(n-1))
    // (in binary64, or with one fused multiply-add in the binary32 NSE pair
    // form), which is A0 phi + Ah0 phi^(n-1) only when A0 + Ah0 = 1
    // (A00 = 1 of Eq. (4-2-00a)); the momentum set likewise
    const double *sets[2][2] = {{a, ah}, {ab ? ab : a, abh ? abh : ah}};
    for (auto &st : sets) {
      const double A0 = st[0][0] + st[0][1] + st[0][2];
      const double Ah0 = st[1][0] + st[1][1] + st[1][2];
      if (std::fabs(A0 + Ah0 - 1.0) > 1e-12)
        return s->fail(MFD_E_UNSUPPORTED,
                       "binary32 three-level schemes need A0 + Ah0 = 1 (got %.17g)", A0 + Ah0);
    }
  }
  if (s->grid.form == MFD_MESOFD && (ab || abh)) {
    for (int k = 0; k < 3; ++k)
      if ((ab && ab[k] != a[k]) || (abh && ah && abh[k] != ah[k]))
        return s->fail(MFD_E_UNSUPPORTED, "MesoFD uses one parameter set (Eq. (2-3))");
  }
  s->cfg.kind = kind;
  for (int k = 0; k < 3; ++k) {
    s->cfg.a[k] = a[k];
    s->cfg.ah[k] = ah ? ah[k] : 0.0;
    s->cfg.ab[k] = ab ? ab[k] : a[k];
    s->cfg.abh[k] = abh ? abh[k] : s->cfg.ah[k];
  }
  s->cfg.theta = kind == MFD_THETA ? theta : 1.0;
  s->cfg.theta_iters = kind == MFD_THETA ? theta_iters : 0;
  s->mg_levels = 0;  // a new scheme solves its theta steps by sweeps until set again
  s->cfg.dt = dt;
  s->cfg.multiset = 0;
  s->have_scheme = true;
  int rc = rebuild(s);
  if (rc < 0) return rc;
  double m[6];
  mfd_coeff_moments(s->cfg.a, s->cfg.ah, m);
  if (std::fabs(m[0] - 1.0) > 1e-12) {
    s->fail(MFD_W_INCONSISTENT, "A00 = %.17g differs from 1", m[0]);
    return MFD_W_INCONSISTENT;
  }
  if (!stability_proven(s->consts)) {
    s->fail(MFD_W_STABILITY_UNPROVEN, "sufficient stability conditions do not hold");
    return MFD_W_STABILITY_UNPROVEN;
  }
  return MFD_OK;
}

extern "C" int mfd_set_stream(mfd_solver *h, void *stream) {
  SOLVER_OR_ARG(h);
  reinterpret_cast<Solver *>(h)->stream = (hipStream_t)stream;
  return MFD_OK;
}

extern "C" int mfd_state_size(const mfd_solver *h, int64_t *moment_elems,
                              int64_t *population_elems, int64_t *device_bytes) {
  SOLVER_OR_ARG(h);
  const Solver *s = reinterpret_cast<const Solver *>(h);
  if (!s->configured) return MFD_E_ORDER;
  if (moment_elems) *moment_elems = s->mom_elems();
  if (population_elems) *population_elems = s->pop_elems();
  if (device_bytes) *device_bytes = s->device_bytes_needed();
  return MFD_OK;
}

extern "C" int mfd_set_state(mfd_solver *h, int level, const void *src, int64_t bytes,
                             int on_device, int populations) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!s->configured) return s->fail(MFD_E_ORDER, "configure the solver first");
  if (!src) return s->fail(MFD_E_ARG, "null source");
  if (level != 0 && level != 1) return s->fail(MFD_E_ARG, "level must be 0 or 1");
  if (level == 1 && !s->consts.three)
    return s->fail(MFD_E_ARG, "level 1 exists only for three-level schemes");
  const bool meso = s->grid.form == MFD_MESOFD;
  if (populations && (!meso || level != 0))
    return s->fail(MFD_E_ARG, "populations exist only for MesoFD level 0");
  const int64_t es = s->elem();
  const int64_t want = (populations ? s->pop_elems() : s->mom_elems()) * es;
  if (bytes != want)
    return s->fail(MFD_E_ARG, "expected %lld bytes, got %lld", (long long)want, (long long)bytes);
  int rc;
  if (level == 0 || !s->buf[0]) {
    // (re)allocate on the first state of a configuration
    rc = s->ensure_buffers();
    if (rc) return rc;
  }
  if (level == 1) {
    rc = s->copy_in(s->buf[s->ip], src, bytes, on_device);
    if (rc) return rc;
    s->prev_set = true;
    return MFD_OK;
  }
  if (!meso) {
    rc = s->copy_in(s->buf[s->ic], src, bytes, on_device);
    if (rc) return rc;
    // phi^(-1) = phi^0 start; also the residual reference
    rc = s->copy_in(s->buf[s->ip], src, bytes, on_device);
    if (rc) return rc;
  } else {
    // MesoFD level t: populations pop[pc] and their moments B[ic]; level
    // t-dt: B[ip] = the moments given (or those of the populations given).
    hipError_t e;
    const bool f64 = s->grid.precision == MFD_FP64;
    if (populations) {
      rc = s->copy_in(s->buf[s->pc], src, bytes, on_device);
      if (rc) return rc;
      e = f64 ? launch_moments<double>(s->consts, s->G, (const double *)s->buf[s->pc],
                                       (double *)s->buf[s->ip], s->stream)
              : launch_moments<float>(s->consts, s->G, (const float *)s->buf[s->pc],
                                      (float *)s->buf[s->ip], s->stream);
      if (e != hipSuccess) return s->hip(e, "moments launch");
    } else {
      rc = s->copy_in(s->buf[s->ip], src, bytes, on_device);
      if (rc) return rc;
      e = f64 ? launch_init_populations<double>(s->consts, s->G, (const double *)s->buf[s->ip],
                                                (double *)s->buf[s->pc], s->stream)
              : launch_init_populations<float>(s->consts, s->G, (const float *)s->buf[s->ip],
                                               (float *)s->buf[s->pc], s->stream);
      if (e != hipSuccess) return s->hip(e, "init populations launch");
    }
    e = f64 ? launch_moments<double>(s->consts, s->G, (const double *)s->buf[s->pc],
                                     (double *)s->buf[s->ic], s->stream)
            : launch_moments<float>(s->consts, s->G, (const float *)s->buf[s->pc],
                                    (float *)s->buf[s->ic], s->stream);
    if (e != hipSuccess) return s->hip(e, "moments launch");
    rc = s->hip(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    if (rc) return rc;
  }
  s->state_set = true;
  s->prev_set = false;
  s->steps_done = 0;
  return MFD_OK;
}

extern "C" int mfd_get_state(mfd_solver *h, int level, void *dst, int64_t bytes, int on_device,
                             int populations) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!s->state_set) return s->fail(MFD_E_ORDER, "state not set");
  if (!dst) return s->fail(MFD_E_ARG, "null destination");
  if (level != 0 && level != 1) return s->fail(MFD_E_ARG, "level must be 0 or 1");
  const bool meso = s->grid.form == MFD_MESOFD;
  if (populations && (!meso || level != 0))
    return s->fail(MFD_E_ARG, "populations exist only for MesoFD level 0");
  const int64_t es = s->elem();
  const int64_t want = (populations ? s->pop_elems() : s->mom_elems()) * es;
  if (bytes != want)
    return s->fail(MFD_E_ARG, "expected %lld bytes, got %lld", (long long)want, (long long)bytes);
  if (level == 1) return s->copy_out(dst, s->buf[s->ip], bytes, on_device);
  if (populations) return s->copy_out(dst, s->buf[s->pc], bytes, on_device);
  // MMFD state, or the moments of the current MesoFD populations (kept
  // beside them by every step)
  return s->copy_out(dst, s->buf[s->ic], bytes, on_device);
}

extern "C" int mfd_step(mfd_solver *h, int64_t nsteps) {
  SOLVER_OR_ARG(h);
  return reinterpret_cast<Solver *>(h)->step(nsteps);
}

extern "C" int mfd_synchronize(mfd_solver *h) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  return s->hip(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
}

extern "C" int mfd_reduce(mfd_solver *h, double sums[4], double *residual) {
  SOLVER_OR_ARG(h);
  return reinterpret_cast<Solver *>(h)->reduce(sums, residual);
}

extern "C" int mfd_set_check_interval(mfd_solver *h, int64_t every) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (every < 0) return s->fail(MFD_E_ARG, "check interval < 0");
  s->check_every = every;
  return MFD_OK;
}

extern "C" int mfd_set_blocking(mfd_solver *h, int32_t tb_depth) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (tb_depth < 0 || tb_depth > 16) return s->fail(MFD_E_ARG, "blocking depth out of range");
  const int old = s->tb;
  s->tb = tb_depth;
  if (tb_depth > 1 && s->configured && s->effective_plan().tb != tb_depth) {
    s->tb = old;
    return s->fail(MFD_E_UNSUPPORTED, "depth %d cannot be used by this configuration", tb_depth);
  }
  return MFD_OK;
}

extern "C" int mfd_set_plan(mfd_solver *h, int32_t tb_depth, int32_t window_rows,
                            int32_t window_cols) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!s->configured) return s->fail(MFD_E_ORDER, "set the scheme first");
  if (tb_depth == 1) {
    s->tb = 1;
    return MFD_OK;
  }
  const TbPlan p{tb_depth, window_rows, window_cols};
  if (!s->plan_supported(p))
    return s->fail(MFD_E_UNSUPPORTED, "plan (%d, %d, %d) cannot be used by this configuration",
                   tb_depth, window_rows, window_cols);
  s->tb = tb_depth;
  s->tuned = p;
  return MFD_OK;
}

extern "C" int mfd_launch_plan(const mfd_solver *h, int32_t *tb_depth, int32_t *window_rows,
                               int32_t *window_cols) {
  if (!h) return MFD_E_ARG;
  const Solver *s = reinterpret_cast<const Solver *>(h);
  if (!s->configured) return MFD_E_ORDER;
  const TbPlan p = s->effective_plan();
  if (tb_depth) *tb_depth = p.tb;
  if (window_rows) *window_rows = p.tb > 1 ? p.h : 0;
  if (window_cols) *window_cols = p.tb > 1 ? p.w : 0;
  return MFD_OK;
}

extern "C" int mfd_set_source(mfd_solver *h, const double *G, int64_t count, int on_device,
                              double lambda, const double b[3], const double bh[3],
                              const double v[3]) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!s->configured) return s->fail(MFD_E_ORDER, "set the scheme first");
  if (!s->source_supported())
    return s->fail(MFD_E_UNSUPPORTED, "the source term needs the linear CDE with an explicit "
                                      "scheme (MesoFD form: 1D / 2D)");
  if (!G || !b || !bh || !v) return s->fail(MFD_E_ARG, "null argument");
  if (count != s->G.N)
    return s->fail(MFD_E_ARG, "expected %lld source values, got %lld", (long long)s->G.N,
                   (long long)count);
  if (!std::isfinite(lambda)) return s->fail(MFD_E_ARG, "lambda is not finite");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(b[k]) || !std::isfinite(bh[k]) || !std::isfinite(v[k]))
      return s->fail(MFD_E_ARG, "non-finite coefficient");
  const int64_t N = s->G.N;
  std::vector<double> host;
  const double *hg = G;
  if (on_device) {
    host.resize((size_t)N);
    int rc = s->hip(hipMemcpy(host.data(), G, (size_t)N * 8, hipMemcpyDeviceToHost),
                    "hipMemcpy (source)");
    if (rc) return rc;
    hg = host.data();
  }
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(hg[i])) return s->fail(MFD_E_ARG, "source value %lld is not finite", (long long)i);
  const int64_t es = s->elem();
  if (s->d_src) {
    (void)hipStreamSynchronize(s->stream);
    dev_free(s->d_src);
    s->d_src = nullptr;
    s->src_on = false;
  }
  if (dev_malloc(&s->d_src, (size_t)(N * es)) != hipSuccess) {
    (void)hipGetLastError();
    s->d_src = nullptr;
    return s->fail(MFD_E_OOM, "no device memory for the source field");
  }
  int rc;
  if (es == 8) {
    rc = s->hip(hipMemcpy(s->d_src, hg, (size_t)N * 8, hipMemcpyHostToDevice), "hipMemcpy (source)");
  } else {
    std::vector<float> f((size_t)N);
    for (int64_t i = 0; i < N; ++i) f[(size_t)i] = (float)hg[i];
    rc = s->hip(hipMemcpy(s->d_src, f.data(), (size_t)N * 4, hipMemcpyHostToDevice),
                "hipMemcpy (source)");
  }
  if (rc) return rc;
  for (int k = 0; k < 3; ++k) {
    s->src.b[k] = b[k];
    s->src.bh[k] = bh[k];
    s->src.v[k] = k < s->grid.dim ? v[k] : 0.0;
  }
  s->src.lambda = lambda;
  s->src_on = true;
  return MFD_OK;
}

extern "C" int mfd_clear_source(mfd_solver *h) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->d_src) {
    (void)hipStreamSynchronize(s->stream);
    dev_free(s->d_src);
  }
  s->d_src = nullptr;
  s->src_on = false;
  return MFD_OK;
}

extern "C" int mfd_autotune(mfd_solver *h, int32_t *chosen_tb) {
  SOLVER_OR_ARG(h);
  return reinterpret_cast<Solver *>(h)->autotune(chosen_tb);
}

extern "C" int mfd_max_amplification(mfd_solver *h, double *out) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!out) return MFD_E_ARG;
  if (!s->configured) return s->fail(MFD_E_ORDER, "configure the solver first");
  if (s->consts.eq != kLCDE) return s->fail(MFD_E_UNSUPPORTED, "linear (LCDE) schemes only");
  if (s->G.N > ((int64_t)1 << 24)) return s->fail(MFD_E_ARG, "grid too large for a mode sweep");
  *out = max_amplification(s->consts, s->G.n);
  return MFD_OK;
}

extern "C" int mfd_linear_tables(mfd_solver *h, double *w, double *ubar, double *out6) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!s->configured) return s->fail(MFD_E_ORDER, "configure the solver first");
  const Consts &c = s->consts;
  for (int j = 0; j < c.q; ++j) {
    if (w) w[j] = c.w[j];
    if (ubar) ubar[j] = c.ubar[j];
  }
  if (out6)
    for (int p = 0; p < c.npair; ++p) {
      out6[0 * kMaxP + p] = c.ubp[p];
      out6[1 * kMaxP + p] = c.ubm[p];
      out6[2 * kMaxP + p] = c.Cp[p];
      out6[3 * kMaxP + p] = c.Cm[p];
      out6[4 * kMaxP + p] = c.Chp[p];
      out6[5 * kMaxP + p] = c.Chm[p];
    }
  return c.q;
}

extern "C" int mfd_max_stable_dt(int lattice, double d0, double dx, const double u[3],
                                 double alpha, const int64_t n[3], double *dt_sufficient,
                                 double *dt_exact) {
  if (!u || !dt_sufficient || !(dx > 0.0) || !(alpha > 0.0) || !std::isfinite(dx) ||
      !std::isfinite(alpha))
    return MFD_E_ARG;
  if (d0 <= 0.0) d0 = 1.0 / 3.0;
  if (!(d0 < 1.0)) return MFD_E_ARG;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(u[a])) return MFD_E_ARG;
  int64_t N = 1;
  if (n && dt_exact) {
    Consts c;
    std::memset(&c, 0, sizeof(c));
    if (lattice_weights(lattice, d0, c) != MFD_OK) return MFD_E_ARG;
    for (int a = 0; a < c.dim; ++a) {
      if (n[a] < 1) return MFD_E_ARG;
      N *= n[a];
    }
    if (N > ((int64_t)1 << 24)) return MFD_E_ARG;
  }
  double s = 0.0, e = 0.0;
  if (max_stable_dt(lattice, d0, dx, u, alpha, dt_exact ? n : nullptr, &s, &e) != 0)
    return MFD_E_ARG;
  *dt_sufficient = s;
  if (n && dt_exact) *dt_exact = e;
  return MFD_OK;
}

extern "C" int mfd_level_ptr(mfd_solver *h, int level, int field, int populations, void **ptr) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!ptr) return s->fail(MFD_E_ARG, "null output");
  if (!s->state_set) return s->fail(MFD_E_ORDER, "state not set");
  if (level != 0 && level != 1) return s->fail(MFD_E_ARG, "level must be 0 or 1");
  if (level == 1 && !s->consts.three)
    return s->fail(MFD_E_ARG, "level 1 exists only for three-level schemes");
  const bool meso = s->grid.form == MFD_MESOFD;
  if (populations && (!meso || level != 0))
    return s->fail(MFD_E_ARG, "populations exist only for MesoFD level 0");
  const int64_t nfld = populations ? s->q() : s->nf();
  if (field < 0 || field >= nfld) return s->fail(MFD_E_ARG, "field %d out of range", field);
  char *base = (char *)s->buf[populations ? s->pc : (level == 0 ? s->ic : s->ip)];
  *ptr = base + (int64_t)field * s->G.N * s->elem();
  return MFD_OK;
}

extern "C" int mfd_set_theta_tolerance(mfd_solver *h, double tol, int32_t chunk) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!s->configured || s->cfg.kind != MFD_THETA)
    return s->fail(MFD_E_ORDER, "set a theta scheme first");
  if (!std::isfinite(tol) || tol < 0.0) return s->fail(MFD_E_ARG, "tolerance must be >= 0");
  if (chunk == 0) chunk = 8;
  if (chunk < 1 || chunk > 16) return s->fail(MFD_E_ARG, "chunk must lie in [1, 16]");
  if (tol > 0.0 && s->cfg.theta_iters < 1)
    return s->fail(MFD_E_ARG, "the sweep cap (theta_iters) must be >= 1");
  s->theta_tol = tol;
  s->theta_chunk = chunk;
  return MFD_OK;
}

extern "C" int mfd_set_theta_multigrid(mfd_solver *h, int32_t levels, int32_t pre,
                                       int32_t post) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!s->configured || s->cfg.kind != MFD_THETA)
    return s->fail(MFD_E_ORDER, "set a theta scheme first");
  int L = 0;
  if (levels != 0) {
    if (s->consts.eq != kLCDE || s->grid.dim != 2 ||
        (s->consts.lattice != MFD_D2Q5 && s->consts.lattice != MFD_D2Q9))
      return s->fail(MFD_E_UNSUPPORTED, "multigrid theta solves: the linear CDE on D2Q5 / D2Q9");
    if (pre < 1 || pre > 8 || post < 0 || post > 8)
      return s->fail(MFD_E_ARG, "pre-smoothing sweeps in [1, 8], post-smoothing in [0, 8]");
    // levels the grid allows: halve while both sides stay even and >= the
    // minimum; the automatic choice stops at the first level of at most
    // kMgAutoCoarseNodes nodes (below it a level costs launches, not work)
    int most = 1, autol = 0;
    for (int64_t nx = s->G.n[0], ny = s->G.n[1];
         most < kMgMaxLevels && nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= kMgMinSide &&
         ny / 2 >= kMgMinSide;
         nx /= 2, ny /= 2) {
      if (!autol && nx * ny <= kMgAutoCoarseNodes) autol = most;
      ++most;
    }
    if (!autol) autol = most;
    L = levels < 0 ? std::max(2, std::min(autol, most)) : levels;
    if (L < 2 || L > most)
      return s->fail(MFD_E_ARG, "this grid takes 2 .. %d multigrid levels (got %d)", most, levels);
  }
  const int64_t old_bytes = s->mg_bytes();
  s->mg_levels = L;
  s->mg_pre = pre;
  s->mg_post = post;
  const int64_t new_bytes = s->mg_bytes();
  // buffers already allocated (state set): replace the multigrid buffer only
  if (s->buf[0] && new_bytes != old_bytes) {
    if (s->buf[Solver::kMgBuf]) {
      hipError_t e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return s->hip(e, "hipStreamSynchronize");
      dev_free(s->buf[Solver::kMgBuf]);
      s->buf[Solver::kMgBuf] = nullptr;
    }
    if (new_bytes > 0) {
      hipError_t e = dev_malloc(&s->buf[Solver::kMgBuf], (size_t)new_bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        s->mg_levels = 0;
        s->allocated_bytes += -old_bytes;
        return s->fail(MFD_E_OOM, "hipMalloc of %lld bytes failed", (long long)new_bytes);
      }
    }
    s->allocated_bytes += new_bytes - old_bytes;
  }
  return MFD_OK;
}

extern "C" int mfd_theta_stats(mfd_solver *h, int64_t *total_sweeps, int64_t *steps,
                               int32_t *max_sweeps, int32_t *unconverged, int reset) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  ThetaCtl c;
  std::memset(&c, 0, sizeof(c));
  if (s->buf[Solver::kThetaBuf]) {
    int rc = s->copy_out(&c, s->buf[Solver::kThetaBuf], sizeof(c), 0);
    if (rc) return rc;
  }
  if (total_sweeps) *total_sweeps = c.total_sweeps + s->th_total;
  if (steps) *steps = c.steps + s->th_steps;
  if (max_sweeps) *max_sweeps = std::max(c.max_sweeps, s->th_max);
  if (unconverged) *unconverged = c.unconverged + s->th_unconv;
  if (reset) {
    s->th_total = s->th_steps = 0;
    s->th_max = s->th_unconv = 0;
    if (s->buf[Solver::kThetaBuf]) {
      c.total_sweeps = c.steps = 0;
      c.max_sweeps = c.unconverged = 0;
      int rc = s->copy_in(s->buf[Solver::kThetaBuf], &c, sizeof(c), 0);
      if (rc) return rc;
    }
  }
  return MFD_OK;
}

extern "C" int mfd_step_noalloc(mfd_solver *h, void *level0, void *level1, int64_t nsteps) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!s->configured) return s->fail(MFD_E_ORDER, "configure the solver first");
  if (s->grid.form != MFD_MMFD || s->cfg.kind == MFD_THETA || s->src_on)
    return s->fail(MFD_E_UNSUPPORTED,
                   "mfd_step_noalloc takes explicit MMFD schemes without a source term");
  const bool three = s->consts.three != 0;
  if (!level0 || (three && !level1) || (!three && level1))
    return s->fail(MFD_E_ARG, "level0 (and for three-level schemes only, level1) must be given");
  if (nsteps < 0) return s->fail(MFD_E_ARG, "nsteps < 0");
  if (nsteps == 0) return MFD_OK;
  const int64_t me = s->mom_elems() * s->elem();
  if (2 * me > (int64_t)kNoAllocScratchBytes)
    return s->fail(MFD_E_ARG, "state of %lld bytes per level exceeds the %lld-byte limit "
                              "(two work levels in %lld bytes of scratch)",
                   (long long)me, (long long)(kNoAllocScratchBytes / 2),
                   (long long)kNoAllocScratchBytes);
  void *scr = nullptr;
  int rc = s->hip(noalloc_scratch(&scr), "hipGetSymbolAddress (scratch)");
  if (rc) return rc;
  char *w0 = (char *)scr, *w1 = (char *)scr + me;
  // run the ordinary step loop on the caller's levels and the scratch
  void *saved_buf[Solver::kNumBuf];
  for (int i = 0; i < Solver::kNumBuf; ++i) saved_buf[i] = s->buf[i];
  const int sic = s->ic, sip = s->ip, sio = s->io, spc = s->pc, spn = s->pn, six = s->ix;
  const int64_t ssteps = s->steps_done;
  const int sgap = s->prev_gap;
  const bool sset = s->state_set;
  for (int i = 0; i < Solver::kNumBuf; ++i) s->buf[i] = nullptr;
  s->buf[0] = level0;
  if (three) {
    s->buf[1] = level1;
    s->buf[2] = w0;
    s->buf[8] = w1;
  } else {
    s->buf[1] = w0;
    s->buf[2] = w1;
  }
  s->ic = 0;
  s->ip = 1;
  s->io = 2;
  s->ix = 8;
  s->steps_done = 0;
  s->prev_gap = 1;
  s->state_set = true;
  rc = s->step(nsteps);
  // the final levels back into the caller's buffers (plain device copies)
  const int ic = s->ic, ip = s->ip;
  void *B[Solver::kNumBuf];
  for (int i = 0; i < Solver::kNumBuf; ++i) B[i] = s->buf[i];
  auto cp = [&](int dst, int src) {
    if (rc == MFD_OK)
      rc = s->hip(hipMemcpyAsync(B[dst], B[src], (size_t)me, hipMemcpyDeviceToDevice, s->stream),
                  "hipMemcpyAsync (noalloc level)");
  };
  if (rc == MFD_OK) {
    if (!three) {
      if (ic != 0) cp(0, ic);
    } else if (ic == 1 && ip == 0) {
      const int free_buf = 2;  // both work levels are free here
      cp(free_buf, 1);
      cp(1, 0);
      cp(0, free_buf);
    } else if (ic == 1) {
      cp(0, 1);
      cp(1, ip);
    } else {
      if (ip != 1) cp(1, ip);
      if (ic != 0) cp(0, ic);
    }
  }
  for (int i = 0; i < Solver::kNumBuf; ++i) s->buf[i] = saved_buf[i];
  s->ic = sic;
  s->ip = sip;
  s->io = sio;
  s->pc = spc;
  s->pn = spn;
  s->ix = six;
  s->steps_done = ssteps;
  s->prev_gap = sgap;
  s->state_set = sset;
  return rc;
}

extern "C" int mfd_set_boundary(mfd_solver *h, const double *G, int64_t count, int on_device,
                                double lambda) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!s->dirichlet) return s->fail(MFD_E_ORDER, "the grid was created periodic");
  if (!G) return s->fail(MFD_E_ARG, "null boundary values");
  if (count != s->G.N)
    return s->fail(MFD_E_ARG, "expected %lld values, got %lld", (long long)s->G.N,
                   (long long)count);
  if (!std::isfinite(lambda)) return s->fail(MFD_E_ARG, "lambda is not finite");
  const int nx = (int)s->G.n[0], ny = (int)s->G.n[1];
  std::vector<double> full;
  const double *hg = G;
  if (on_device) {
    full.resize((size_t)s->G.N);
    int rc = s->hip(hipMemcpy(full.data(), G, (size_t)s->G.N * 8, hipMemcpyDeviceToHost),
                    "hipMemcpy (boundary)");
    if (rc) return rc;
    hg = full.data();
  }
  const int64_t nb = dir_count(nx, ny);
  std::vector<double> comp((size_t)nb);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      if (!dir_node(x, y, nx, ny)) continue;
      const double v = hg[(int64_t)y * nx + x];
      if (!std::isfinite(v)) return s->fail(MFD_E_ARG, "boundary value (%d, %d) is not finite", x, y);
      comp[(size_t)dir_index(x, y, nx, ny)] = v;
    }
  if (!s->d_bnd) {
    if (dev_malloc(&s->d_bnd, (size_t)nb * 8) != hipSuccess) {
      (void)hipGetLastError();
      s->d_bnd = nullptr;
      return s->fail(MFD_E_OOM, "no device memory for the boundary values");
    }
  } else {
    (void)hipStreamSynchronize(s->stream);
  }
  int rc = s->hip(hipMemcpy(s->d_bnd, comp.data(), (size_t)nb * 8, hipMemcpyHostToDevice),
                  "hipMemcpy (boundary)");
  if (rc) return rc;
  s->bnd_lambda = lambda;
  s->bnd_set = true;
  return MFD_OK;
}

extern "C" int mfd_wave_start(mfd_solver *h, const double *phi_t, int64_t count, int on_device) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (s->sticky) return s->fail(MFD_E_HIP, "solver is in a failed HIP state");
  if (!s->configured || !s->consts.wave || !s->consts.three)
    return s->fail(MFD_E_ORDER, "configure a three-level wave scheme first");
  if (s->grid.form != MFD_MMFD)
    return s->fail(MFD_E_UNSUPPORTED, "the special first step is a moment (MMFD) step");
  if (!s->state_set || s->steps_done != 0)
    return s->fail(MFD_E_ORDER, "set level 0 (phi at t = 0) just before the first step");
  if (s->dirichlet && !s->bnd_set)
    return s->fail(MFD_E_ORDER, "Dirichlet values not set (mfd_set_boundary)");
  if (!phi_t) return s->fail(MFD_E_ARG, "null phi_t");
  if (count != s->G.N)
    return s->fail(MFD_E_ARG, "expected %lld values, got %lld", (long long)s->G.N,
                   (long long)count);
  void *dphit = nullptr;
  const size_t bytes = (size_t)s->G.N * 8;
  if (dev_malloc(&dphit, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return s->fail(MFD_E_OOM, "no device memory for phi_t");
  }
  int rc = s->hip(hipMemcpyAsync(dphit, phi_t, bytes,
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 s->stream),
                  "hipMemcpyAsync (phi_t)");
  // alpha = A22 beta c_s^2 of the wave equation: the Taylor start
  // phi + dt phi_t + (dt^2 / 2) alpha Laplacian phi in lattice units
  const double A22 = 0.5 * (s->consts.ap + s->consts.ahp);
  const double cw = ((0.5 * A22) * s->cfg.ep.beta) * s->consts.d0;
  const DirBC bc = s->dir_bc(0, 1);
  if (!rc) {
    hipError_t e = s->grid.precision == MFD_FP64
                       ? launch_wave_start<double>(s->consts, s->G, (const double *)s->buf[s->ic],
                                                   (const double *)dphit, (double *)s->buf[s->io],
                                                   s->cfg.dt, cw, bc, s->stream)
                       : launch_wave_start<float>(s->consts, s->G, (const float *)s->buf[s->ic],
                                                  (const double *)dphit, (float *)s->buf[s->io],
                                                  s->cfg.dt, cw, bc, s->stream);
    rc = s->hip(e, "wave start launch");
  }
  if (!rc) rc = s->hip(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  dev_free(dphit);
  if (rc) return rc;
  const int oc = s->ic, op = s->ip;
  s->ic = s->io;
  s->ip = oc;
  s->io = op;
  s->steps_done = 1;
  s->prev_gap = 1;
  s->prev_set = true;
  return MFD_OK;
}

extern "C" int mfd_set_scheme_sets(mfd_solver *h, int kind, const double a[3], const double ah[3],
                                   const double ae[3], const double aeh[3], const double ao[3],
                                   const double aoh[3], double dt) {
  SOLVER_OR_ARG(h);
  Solver *s = reinterpret_cast<Solver *>(h);
  if (!s->have_lattice || !s->have_eq)
    return s->fail(MFD_E_ORDER, "mfd_set_lattice and mfd_set_equation must precede the scheme");
  if (kind != MFD_TWO_LEVEL && kind != MFD_THREE_LEVEL)
    return s->fail(MFD_E_UNSUPPORTED, "multiple-set schemes are explicit two- or three-level");
  if (s->cfg.eq == MFD_NSE || s->grid.form != MFD_MMFD)
    return s->fail(MFD_E_UNSUPPORTED, "multiple-set schemes: scalar equations, MMFD form");
  const bool three = kind == MFD_THREE_LEVEL;
  if (!a || !ae || !ao || (three && (!ah || !aeh || !aoh)))
    return s->fail(MFD_E_ARG, "null coefficient set");
  for (int k = 0; k < 3; ++k) {
    const double v[6] = {a[k], ae[k], ao[k], three ? ah[k] : 0.0, three ? aeh[k] : 0.0,
                         three ? aoh[k] : 0.0};
    for (double x : v)
      if (!std::isfinite(x)) return s->fail(MFD_E_ARG, "non-finite coefficient");
  }
  // the base set through the single-set call (checks, A00, stability report)
  int rc = mfd_set_scheme(h, kind, a, three ? ah : nullptr, nullptr, nullptr, 1.0, 0, dt);
  if (rc < 0) return rc;
  s->cfg.multiset = 1;
  for (int k = 0; k < 3; ++k) {
    s->cfg.ae[k] = ae[k];
    s->cfg.ao[k] = ao[k];
    s->cfg.aeh[k] = three ? aeh[k] : 0.0;
    s->cfg.aoh[k] = three ? aoh[k] : 0.0;
  }
  int rc2 = rebuild(s);
  if (rc2 < 0) return rc2;
  return rc;
}
