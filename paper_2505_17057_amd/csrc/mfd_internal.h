// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfd {

constexpr int kMaxQ = 19;  // the kernels' constant block (KC): up to rD3Q19
constexpr int kMaxP = 9;
constexpr int kHostMaxQ = 27;  // host tables (Consts): up to rD3Q27
constexpr int kHostMaxP = 13;

// --------------------------------------------------------------- lattices
// Appendix A velocity sets.  D1Q3 is the one-axis member of the family
// (w_j = d0/2, w_0 = 1 - 2 sum w_j).  In D3Q19 the xz-edge block follows the
// (+,+),(-,+),(-,-),(+,-) pattern of the xy and yz blocks (the printed xz
// block repeats two velocities).
struct LatD1Q3 {
  static constexpr int id = 1, D = 1, Q = 3, P = 1;
  static constexpr int E[Q][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
  static constexpr int PR[P] = {1};
};
struct LatD2Q5 {
  static constexpr int id = 2, D = 2, Q = 5, P = 2;
  static constexpr int E[Q][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}};
  static constexpr int PR[P] = {1, 2};
};
struct LatD2Q9 {
  static constexpr int id = 3, D = 2, Q = 9, P = 4;
  static constexpr int E[Q][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                  {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  static constexpr int PR[P] = {1, 2, 5, 6};
};
struct LatD3Q19 {
  static constexpr int id = 4, D = 3, Q = 19, P = 9;
  static constexpr int E[Q][3] = {
      {0, 0, 0},   {1, 0, 0},   {0, 1, 0},  {0, 0, 1},   {-1, 0, 0},  {0, -1, 0}, {0, 0, -1},
      {1, 1, 0},   {-1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {1, 0, 1},   {-1, 0, 1}, {-1, 0, -1},
      {1, 0, -1},  {0, 1, 1},   {0, -1, 1}, {0, -1, -1}, {0, 1, -1}};
  static constexpr int PR[P] = {1, 2, 3, 7, 8, 11, 12, 15, 16};
};

struct LatD2Q5II {
  static constexpr int id = 5, D = 2, Q = 5, P = 2;
  static constexpr int E[Q][3] = {{0, 0, 0}, {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  static constexpr int PR[P] = {1, 2};
};
struct LatD3Q7 {
  static constexpr int id = 6, D = 3, Q = 7, P = 3;
  static constexpr int E[Q][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0}, {0, 0, 1},
                                  {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}};
  static constexpr int PR[P] = {1, 2, 3};
};
struct LatD3Q9 {
  static constexpr int id = 7, D = 3, Q = 9, P = 4;
  static constexpr int E[Q][3] = {{0, 0, 0},    {1, 1, 1},   {1, 1, -1},  {1, -1, 1}, {-1, 1, 1},
                                  {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
  static constexpr int PR[P] = {1, 2, 3, 4};
};
// rD3Q27: the rest velocity, the axes, the edges as in D3Q19 and the eight
// corners in the printed order (run by the general-scheme kernel only)
struct LatD3Q27 {
  static constexpr int id = 8, D = 3, Q = 27, P = 13;
  static constexpr int E[Q][3] = {
      {0, 0, 0},   {1, 0, 0},   {0, 1, 0},   {0, 0, 1},   {-1, 0, 0},   {0, -1, 0},  {0, 0, -1},
      {1, 1, 0},   {-1, 1, 0},  {-1, -1, 0}, {1, -1, 0},  {1, 0, 1},    {-1, 0, 1},  {-1, 0, -1},
      {1, 0, -1},  {0, 1, 1},   {0, -1, 1},  {0, -1, -1}, {0, 1, -1},   {1, 1, 1},   {1, 1, -1},
      {1, -1, 1},  {-1, 1, 1},  {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
  static constexpr int PR[P] = {1, 2, 3, 7, 8, 11, 12, 15, 16, 19, 20, 21, 22};
};

// ---------------------------------------------------------- configuration
enum Eq { kLCDE = 0, kBurgers = 1, kNSE = 2 };
// equation code of the wave equation as given by the caller; its constants
// are those of a linear EDF, so its steps run as kLCDE
constexpr int kWaveInput = 3;

// All derived constants of one solver, in binary64 (host side).
struct Consts {
  int lattice, dim, q, npair, eq;
  int e[kHostMaxQ][3];
  int pair[kHostMaxP];
  double d0, inv_d0;
  double w[kHostMaxQ], w1[kHostMaxQ];
  double qd[kHostMaxQ][3], qo[kHostMaxQ][3];
  double A0, Ah0, Ab0, Abh0;
  double ap, am, ahp, ahm, abp, abm, abhp, abhm;
  double a[3], ah[3];
  // linear CDE
  double uh[3], kh[9], Ch[9];
  double ubar[kHostMaxQ], ubp[kHostMaxP], ubm[kHostMaxP], Cp[kHostMaxP], Cm[kHostMaxP],
      Chp[kHostMaxP], Chm[kHostMaxP];
  // Burgers
  double bh, cbeta;
  int beta_one;
  // NSE
  double rho0, rinv0;
  int he_luo;
  // theta
  double theta, th1, den, inv_den;  // den = 1 + (1 - theta) 2 sum_p Cp_p
  int wave;           // the linear EDF of the wave equation (eq = kLCDE)
  int multiset;       // a+-/ah+- from the even / odd sets of Eq. (2-2-1b)
  int three;          // three-level scheme
  int three_stencil;  // level t - dt enters through central differences
};

// Kernel-side constants of one step (by value in the kernel argument block).
template <typename T>
struct KC {
  T w[kMaxQ], w1[kMaxQ], qd[kMaxQ][3], qo[kMaxQ][3], inv_d0;
  T ubar[kMaxQ];
  T ap, am, ahp, ahm, abp, abm, abhp, abhm;
  T nw[kMaxP][4];  // binary32 NSE pair form: a+ w_p, a- w_p / d0, abar+ w_p / d0, abar- w_p
  T a[3], ah[3];              // k = -1, 0, +1 (MesoFD)
  T Cp[kMaxP], Cm[kMaxP], Chp[kMaxP], Chm[kMaxP];
  T Ap[kMaxP], Am[kMaxP], Ahp[kMaxP], Ahm[kMaxP];  // Cp +- Cm, Chp +- Chm (binary32 form)
  T bh, cbeta, rho0, rinv0;
  double A0, Ah0, Ab0, Abh0;  // binary64 base coefficients
  T A0t, Ah0t, Ab0t, Abh0t;   // the same in T
  T th, th1, inv_den;
  int beta_one, he_luo;
};

template <typename T>
KC<T> make_kc(const Consts &c);

// ------------------------------------------------------ device allocations
// Every device allocation of the library goes through these two calls, which
// count the bytes held (now and at peak) for mfd_memory_stats.
hipError_t dev_malloc(void **p, size_t bytes);
void dev_free(void *p);

// ------------------------------------------------------ kernel launchers
// Each returns a hipError_t of the launch.  `cur`/`prev`/`out` are moment
// levels (field-major); n = (nx, ny, nz).

struct Grid {
  int64_t n[3];
  int64_t N;
};

// Dirichlet boundary of a 2D grid: the nodes with x or y on the grid's edge
// hold prescribed values G_b(x) exp(lambda t).  G_b is stored compactly in
// binary64: row y = 0 (x = 0..nx-1), row y = ny-1, then column x = 0 and
// column x = nx-1 (y = 1..ny-2 each).  A launch that writes the levels
// t + s dt, s = 1..tb, takes E[s] = exp(lambda (t + s dt)); binary32 levels
// hold the binary64 product rounded once.
constexpr int kMaxBcSteps = 16;
struct DirBC {
  const double *Gb;
  double E[kMaxBcSteps + 1];
  int on;
};
__host__ __device__ inline bool dir_node(int gx, int gy, int nx, int ny) {
  return gx == 0 || gy == 0 || gx == nx - 1 || gy == ny - 1;
}
__host__ __device__ inline int64_t dir_index(int gx, int gy, int nx, int ny) {
  if (gy == 0) return gx;
  if (gy == ny - 1) return (int64_t)nx + gx;
  if (gx == 0) return 2 * (int64_t)nx + (gy - 1);
  return 2 * (int64_t)nx + (ny - 2) + (gy - 1);
}
inline int64_t dir_count(int64_t nx, int64_t ny) { return 2 * nx + 2 * (ny - 2); }

template <typename T>
hipError_t launch_mmfd_step(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                            int tb_depth, hipStream_t st, const DirBC *bc = nullptr);

// special first step of the three-level wave scheme: out = phi^0 + dt phi_t
// + cw sum_axes D2_axis phi^0 (binary64 arithmetic, rounded once), with the
// Dirichlet values of t = dt on the boundary when bc is on
template <typename T>
hipError_t launch_wave_start(const Consts &c, const Grid &g, const T *phi0, const double *phit,
                             T *out, double dt, double cw, const DirBC &bc, hipStream_t st);

// source term of the linear CDE (kernels_source.hip): S(x, t) = exp(lambda t)
// G(x), M_1F = v S, coefficients b (level t) and bh (level t - dt)
struct SourceSpec {
  double b[3], bh[3], v[3];
  double lambda, dt, dx;
};
// one MMFD step from t = n dt with the source term: level t (cur), t - dt
// (prev, three-level) in, t + dt out; G the source field
template <typename T>
hipError_t launch_mmfd_source_step(const Consts &c, const Grid &g, const SourceSpec &s, int64_t n,
                                   const T *cur, const T *prev, T *out, const T *G,
                                   hipStream_t st);
// the same for the MesoFD form (1D / 2D): moments of t (cur) and t - dt (prev)
// in; the populations of t + dt (pop_out, unless null) and their moments
// (mom_out) out
template <typename T>
hipError_t launch_mesofd_source_step(const Consts &c, const Grid &g, const SourceSpec &s,
                                     int64_t n, const T *cur, const T *prev, T *pop_out,
                                     T *mom_out, const T *G, hipStream_t st);

// one NSE step on D3Q19 without an older-level stencil, pair parts staged
// once per node (kernels_nse3d.hip)
template <typename T>
hipError_t launch_nse3d_pp(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                           hipStream_t st);

// LDS-resident 1D run: nsteps steps inside one workgroup; ring buffers
// a (level t) / b (level t - dt) are updated in place; returns the index of
// the buffer holding the final level among {a, b, c}.
template <typename T>
hipError_t launch_mmfd_1d_resident(const Consts &c, const Grid &g, T *a, T *b, T *cbuf,
                                   int64_t nsteps, hipStream_t st);
bool mmfd_1d_resident_fits(const Consts &c, const Grid &g, int elem_bytes);
// whole run of a small periodic 1D two-level LCDE grid (64, 128, 256, 512 or
// 1024 nodes) in the registers of one workgroup (kernels_1d_wave.hip); levels
// stay in place (ga: last level, gb: the one before), MesoFD populations to
// pop
bool wave1d_applies(const Consts &c, const Grid &g);
template <typename T>
hipError_t launch_1d_wave(const Consts &c, const Grid &g, bool mesofd, T *ga, T *gb, T *pop,
                          int64_t nsteps, hipStream_t st);

// Temporally blocked MMFD step (linear CDE, Burgers) on D2Q5 / D2Q9: one
// launch advances tb steps
// over windows of 64 x h nodes.  Reads levels t (cur) and t - dt (prev,
// three-level), writes t + tb (out_cur) and, for three-level schemes,
// t + tb - 1 (out_prev).
struct TbPlan {
  int tb;       // steps per launch
  int h;        // window rows
  int w = 64;   // window columns: 64 or 128
};
size_t tb_lds_bytes(const Consts &c, const TbPlan &pl, int elem);
// plan limits (depth, window height, LDS) for `levels` LDS levels
bool tb_plan_valid(const TbPlan &pl, int levels, int elem);

// blocked MMFD steps of the linear CDE with the source term (D2Q5 / D2Q9,
// 64-column windows, 2 .. kMaxBcSteps steps per launch): the launch starts
// from level n0 (cur; prev = level n0 - 1 for three-level schemes) and
// writes n0 + tb (out_cur) and, three-level, n0 + tb - 1 (out_prev)
bool source_tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem);
template <typename T>
hipError_t launch_mmfd_source_tb(const Consts &c, const Grid &g, const SourceSpec &s, int64_t n0,
                                 const TbPlan &pl, const T *cur, const T *prev, T *out_cur,
                                 T *out_prev, const T *G, hipStream_t st);
// equations / lattices the blocked kernels implement
bool tb_equation_supported(const Consts &c);
// the single-grid blocked kernel can run this plan on this grid
bool tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem);
int tb_window_cols();
// lane-shared two-level steps of the linear CDE and Burgers' equation
// (kernels_lane_tb.hip): 128-column windows updated in place; level t in,
// level t + tb out; binary32 and binary64
bool lane_tb_applies(const Consts &c, int elem);
// the binary32 constants suit the specialized linear CDE / Burgers segments
// (also the batched lane kernel's condition)
bool lane_shared_fp32(const Consts &c);
bool lane_tb_window_fits(const TbPlan &pl);
// the same window for the two-level MesoFD form: moments of level t in;
// moments and (pop_out not null) populations of level t + tb out
bool lane_meso_applies(const Consts &c, int elem);
template <typename T>
hipError_t launch_lane_mesofd_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                                 T *mom_out, T *pop_out, hipStream_t st);
template <typename T>
hipError_t launch_lane_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *out,
                          hipStream_t st);
// blocked MesoFD step, two-level linear CDE / Burgers (kernels_mesofd_tb.hip):
// moments of level t in, moments and (pop_out not null) populations of level
// t + tb out
bool mesofd_tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem);
template <typename T>
hipError_t launch_mesofd_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                            T *mom_out, T *pop_out, hipStream_t st);
// blocked NSE step (kernels_nse_tb.hip): 64 x 32 or 64 x 64 windows
bool nse_tb_plan_valid(const TbPlan &pl, int npair, int elem);
template <typename T>
hipError_t launch_nse_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                         const T *prev, T *out_cur, T *out_prev, hipStream_t st);
template <typename T>
hipError_t launch_mmfd_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                          const T *prev, T *out_cur, T *out_prev, hipStream_t st,
                          const DirBC *bc = nullptr);

// MesoFD step: moments of level t (mom) and t-dt (prev_mom) in; moments and
// (pop_out not null) populations of level t+1 out.
template <typename T>
hipError_t launch_mesofd_step(const Consts &c, const Grid &g, const T *mom, const T *prev_mom,
                              T *pop_out, T *mom_out, hipStream_t st);

// MesoFD 1D grids that fit in LDS: all steps in one workgroup (ga / gb:
// moments of levels t and t - dt, in and out; pop: final populations)
bool mesofd_1d_resident_fits(const Consts &c, const Grid &g, int elem);
template <typename T>
hipError_t launch_mesofd_1d_resident(const Consts &c, const Grid &g, T *ga, T *gb, T *pop,
                                     int64_t nsteps, hipStream_t st);

template <typename T>
hipError_t launch_init_populations(const Consts &c, const Grid &g, const T *mom, T *pop,
                                   hipStream_t st);

template <typename T>
hipError_t launch_moments(const Consts &c, const Grid &g, const T *pop, T *mom, hipStream_t st);

// Fused theta step (2D): right-hand side and K Jacobi sweeps in one launch;
// theta_fused_rows gives its window height, 0 when it cannot run.
int theta_fused_rows(const Consts &c, const Grid &g, int K, int elem);
template <typename T>
hipError_t launch_theta_fused(const Consts &c, const Grid &g, int K, const T *cur, T *out,
                              hipStream_t st);

// Theta step solved to a tolerance (kernels_misc.hip).  The control block
// lives in device memory; its roles index four level buffers: 0 and 1 hold
// phi^n and phi^(n-1) between mfd_step calls, 2 and 3 are work buffers.
struct ThetaCtl {
  int role[4];    // buffer of: phi^n, phi^(n-1), next destination, spare
  int nsrc, ndst; // iterate source / destination of the next continuation chunk
  int done;       // the running step's solve has stopped
  int sweeps;     // sweeps of the running step so far
  unsigned count; // workgroups finished in the running chunk
  int max_sweeps, unconverged;
  int pad;
  long long total_sweeps, steps;
};
inline double theta_den(const Consts &c) { return c.den; }
// tiles of one chunk of K sweeps (0 when the fused window cannot run)
int theta_solve_tiles(const Consts &c, const Grid &g, int K, int elem);
template <typename T>
hipError_t launch_theta_ctl_init(ThetaCtl *ctl, hipStream_t st);
// one chunk of K sweeps; first = the step's first chunk (starts from phi^n)
template <typename T>
hipError_t launch_theta_chunk(const Consts &c, const Grid &g, int K, T *const bufs[4],
                              ThetaCtl *ctl, double *part, double tol, int cap, bool first,
                              hipStream_t st);
template <typename T>
hipError_t launch_theta_gather(T *const bufs[4], const ThetaCtl *ctl, int64_t N, hipStream_t st);
// Picard-Jacobi theta step of Burgers' equation and the NSE: the elementwise
// parts of F (<= 4) fields of N nodes each (field f at offset f N), with the
// per-field constants A0[f], dd[f], inv_den[f]
template <typename T>
hipError_t launch_picard_rhs(const T *S0, const T *phi, T *R, double th, double th1, int F,
                             const double *A0, int64_t N, hipStream_t st);
template <typename T>
hipError_t launch_picard_update(const T *Sx, const T *x, const T *R, T *out, int F,
                                const double *A0, const double *dd, double th1,
                                const double *inv_den, int64_t N, hipStream_t st);
// one Picard-Jacobi sweep of the theta step fused with the explicit step of
// the iterate: Burgers' equation on 1D / 2D grids (field 0's constants) and
// the NSE on 2D grids (per-field constants); hipErrorInvalidValue otherwise
// part (may be null): the sweep also writes per-workgroup binary64 rows of
// (x_new - x)^2 and R^2 per field (8 doubles a row) and sets *rows to their
// count, when the workgroups fit kReduceBlocks rows (else *rows = 0)
template <typename T>
hipError_t launch_picard_sweep(const Consts &c, const Grid &g, const T *x, const T *R, T *out,
                               const double *A0, const double *dd, double th1,
                               const double *inv_den, double *part, int *rows, hipStream_t st);
// the 2D NSE's theta right-hand side R = theta S(x) + (1 - theta) (A0 x) per
// field, formed at the store of the explicit step (hipErrorInvalidValue for
// other equations and grids)
template <typename T>
hipError_t launch_picard_rhs_step(const Consts &c, const Grid &g, const T *x, T *R,
                                  const double *A0, double th, double th1, hipStream_t st);
// out[q] = sum of the rows' quantity q (q < nq <= 8) in a fixed order
hipError_t launch_final_sums(const double *partial, int rows, int nq, double *out, hipStream_t st);
// per field f < F (<= 4; field f at offset f N): sum (a - b)^2 and sum c^2 in
// binary64 (out[2 f], out[2 f + 1]); partial as launch_reduce
template <typename T>
hipError_t launch_sq_sums(const T *a, const T *b, const T *c, int F, int64_t N, double *partial,
                          double *out, hipStream_t st);

template <typename T>
hipError_t launch_theta_rhs(const Consts &c, const Grid &g, const T *cur, T *rhs, hipStream_t st);
template <typename T>
hipError_t launch_theta_sweep(const Consts &c, const Grid &g, const T *src, const T *rhs, T *dst,
                              hipStream_t st);

// FP64 reductions: sums of nf fields of `cur` and ||cur - prev||_2 of field 0
// (prev may be null).  partial: >= kReduceBlocks * 8 doubles of scratch;
// out: 8 doubles (device).
constexpr int kReduceBlocks = 2048;
template <typename T>
hipError_t launch_reduce(const T *cur, const T *prev, int nf, int64_t N, double *partial,
                         double *out, hipStream_t st);

}  // namespace mfd
