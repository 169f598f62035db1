// The single-grid solver object behind the opaque mfd_solver handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mfd.h"
#include "mfd_internal.h"

namespace mfd {

struct Config {
  int lattice = 0;
  double d0 = 1.0 / 3.0;
  int eq = 0;
  mfd_eq_params ep{};
  int kind = MFD_TWO_LEVEL;
  double a[3] = {0, 0, 0}, ah[3] = {0, 0, 0}, ab[3] = {0, 0, 0}, abh[3] = {0, 0, 0};
  double theta = 1.0;
  int theta_iters = 0;
  double dt = 0.0;
  int multiset = 0;
  double ae[3] = {0, 0, 0}, aeh[3] = {0, 0, 0}, ao[3] = {0, 0, 0}, aoh[3] = {0, 0, 0};
  int rect = 0;  // rectangular lattice: d0 and spacing per axis
  double d0v[3] = {0, 0, 0}, dxv[3] = {0, 0, 0};
};

struct Solver {
  // device buffers: 0..2 moment ring, 3..4 population ping-pong, 5..6 theta
  // rhs / Jacobi work, 7 reduction scratch, 8 fourth moment buffer (blocked
  // three-level steps write two levels), 9 control block and tile partials of
  // the to-tolerance theta solve, 10 multigrid levels (fine-level scratch,
  // then iterate, right-hand side and scratch of every coarser level)
  static constexpr int kNumBuf = 11;
  static constexpr int kRedBuf = 7;
  static constexpr int kThetaBuf = 9;
  static constexpr int kMgBuf = 10;
  static constexpr int64_t kThetaCtlBytes = 256;

  mfd_grid grid{};
  Grid G{};
  Config cfg;
  Consts consts{};
  bool have_lattice = false, have_eq = false, have_scheme = false;
  bool configured = false, state_set = false, prev_set = false;
  bool sticky = false;
  hipStream_t stream = nullptr;
  void *buf[kNumBuf] = {nullptr};
  int64_t allocated_bytes = 0;
  int ic = 0, ip = 1, io = 2, pc = 3, pn = 4, ix = 8;  // roles in the rings
  int64_t steps_done = 0;
  // theta step solved to a tolerance (tol > 0; theta_iters is then the cap)
  double theta_tol = 0.0;
  int theta_chunk = 8;
  int64_t th_total = 0, th_steps = 0;  // host-checked solves (unfused path)
  int th_max = 0, th_unconv = 0;
  // multigrid V-cycles for the theta step (0 levels: Jacobi sweeps)
  int mg_levels = 0, mg_pre = 2, mg_post = 2;
  int prev_gap = 1;  // steps between the current and the held previous level
  int64_t check_every = 0;  // finiteness check every this many steps (0: off)
  int tb = 0;           // temporal-blocking depth requested (0 = automatic)
  TbPlan tuned{0, 0};   // plan chosen by the autotuner (tb = 0: not tuned)
  // Dirichlet boundary (2D): compact binary64 values G_b on the device,
  // prescribed value G_b exp(lambda t) with t = n dt as for the source term
  bool dirichlet = false, bnd_set = false;
  void *d_bnd = nullptr;
  double bnd_lambda = 0.0;
  DirBC dir_bc(int64_t first_step, int nsteps) const;
  // source term (linear CDE): G in the solver's precision, on the device
  bool src_on = false;
  SourceSpec src{};
  void *d_src = nullptr;
  std::string err;

  int fail(int code, const char *fmt, ...);
  int hip(hipError_t e, const char *what);
  int64_t elem() const { return grid.precision == MFD_FP64 ? 8 : 4; }
  int64_t nf() const;
  int64_t q() const;
  int64_t mom_elems() const;
  int64_t pop_elems() const;
  int64_t device_bytes_needed() const;
  int64_t theta_buf_bytes() const;
  int64_t mg_bytes() const;
  void release();
  int ensure_buffers();
  int copy_in(void *dst, const void *src, int64_t bytes, int on_device);
  int copy_out(void *dst, const void *src, int64_t bytes, int on_device);
  int step(int64_t nsteps);
  int reduce(double sums[4], double *residual);
  bool source_supported() const;
  TbPlan effective_plan() const;
  bool plan_supported(const TbPlan &p) const;  // the blocked kernel of this form can run p
  int autotune(int32_t *chosen);
  template <typename T>
  int step_t(int64_t nsteps);
  template <typename T>
  int theta_solve_steps(int64_t nsteps);
  template <typename T>
  int theta_picard_steps(int64_t nsteps);
  template <typename T>
  int theta_mg_steps(int64_t nsteps);
};

}  // namespace mfd
