/*
 * mfd.h -- C ABI of the MI355X (gfx950) MesoFD / MMFD stepping library.
 *
 * The library advances the explicit multi-level schemes of the EDF-based
 * mesoscopic finite-difference method (MesoFD, Eq. (2-1) and (3layer-1)) and
 * its macroscopic central-difference form (MMFD, Eq. (2-2-1), (2-4-1),
 * (3layerMMFD-2), linear form Eq. (LMMFD-3)) on periodic rDdQb lattices
 * (Appendix A), for the linear convection-diffusion equation (LCDE,
 * Eq. (LCDE) with the EDF of Eq. (TforMMFD-0)), the Burgers-type nonlinear
 * CDE (Eq. (NCDEfeq) with flux phi^2/2 per axis) and the Navier-Stokes
 * equations (Eq. (NSEfeq); He-Luo variant of Remark 4).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Return value: 0 = success; > 0 = success with a warning (MFD_W_*);
 * < 0 = error (MFD_E_*), in which case no out-parameter is written.
 * mfd_last_error() returns a library-owned message for the last error of a
 * solver.  A HIP runtime failure is sticky: every later call on that solver
 * returns MFD_E_HIP.  No C++ exception crosses this interface.  A solver is
 * not thread-safe; use one per host thread (different solvers may share a
 * device and a stream).
 *
 * Units: lattice units c = dx/dt = 1, c_s^2 = d0.  The state of a scalar NCDE
 * is phi.  The NSE state holds (rho - rho0, j_x, j_y[, j_z]) with
 * j = rho u dt/dx; rho0 is a parameter (0 gives plain rho).
 *
 * Layout: structure of arrays, field-major, x fastest:
 *   moments     [field][nz][ny][nx],  nf = 1 (NCDE) or 1 + dim (NSE) fields;
 *   populations [j][nz][ny][nx],      b = 3, 5, 9, 19 directions (Appendix-A
 *                                     order; for the NSE, f_j - w_j rho0).
 * Precision: MFD_FP64 stores and computes in binary64; MFD_FP32 stores and
 * computes in binary32, except that the three-level base
 * phi^n - Ah0 (phi^n - phi^(n-1)) and all reductions are formed in binary64.
 *
 * Memory: the solver owns its state buffers (device memory allocated when
 * the configuration is complete).  State is exchanged through plain host or
 * device pointers (mfd_set_state / mfd_get_state); a device pointer must be
 * device memory of the solver's device (e.g. a torch tensor's data_ptr()).
 * All device work is enqueued on the solver's stream (mfd_set_stream;
 * default: the null stream); calls documented as synchronous wait for it.
 */
#ifndef MFD_H
#define MFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define MFD_OK 0
#define MFD_W_STABILITY_UNPROVEN 1  /* sufficient stability conditions fail  */
#define MFD_W_INCONSISTENT 2        /* A00 != 1 or A10 != A11 (Eq. (4-2-0)) */
#define MFD_E_ARG (-1)              /* invalid argument                      */
#define MFD_E_ORDER (-2)            /* call-order violation                  */
#define MFD_E_UNSUPPORTED (-3)      /* combination not implemented           */
#define MFD_E_OOM (-4)              /* device allocation failed              */
#define MFD_E_HIP (-5)              /* HIP runtime failure (sticky)          */
#define MFD_E_UNSTABLE (-6)         /* NaN / Inf found by a reduction        */
#define MFD_E_BUDGET (-7)           /* request exceeds a memory budget       */
#define MFD_E_CANCELLED (-8)        /* served request cancelled              */
#define MFD_E_TIMEOUT (-9)          /* served request exceeded its timeout   */

/* --------------------------------------------------------------- enums     */
#define MFD_D1Q3 1   /* rD1Q3: e = 0, +1, -1;  w = 1-d0, d0/2, d0/2           */
#define MFD_D2Q5 2   /* rD2Q5I of Appendix A                                  */
#define MFD_D2Q9 3   /* rD2Q9 of Appendix A                                   */
#define MFD_D3Q19 4  /* rD3Q19 of Appendix A                                  */
/* The lattices below carry the single-step kernels only (no temporally
 * blocked plans, batches or fused theta windows).  Their EDF meets the
 * second-moment identity of Eq. (3-5) only for C = 0 (isotropic diffusion
 * with lambda_bar = 0, or the wave equation at beta = 1). */
#define MFD_D2Q5II 5 /* rD2Q5II: the rest velocity and the four diagonals,
                        w = 1-d0, d0/4 (x4)                                  */
#define MFD_D3Q7 6   /* rD3Q7: rest and the six axis velocities,
                        w = 1-3d0, d0/2 (x6); 0 < d0 < 1/3                   */
#define MFD_D3Q9 7   /* rD3Q9: rest and the eight cube corners,
                        w = 1-d0, d0/8 (x8)                                  */
#define MFD_D3Q27 8  /* rD3Q27: rest, axes, edges and corners, the product
                        weights of Appendix A; the general-scheme solver
                        (mfd_general_*) runs it, mfd_set_lattice does not    */

#define MFD_FP64 0
#define MFD_FP32 1

#define MFD_MMFD 0   /* moments only: central-difference form                */
#define MFD_MESOFD 1 /* populations: Eq. (2-1) / (3layer-1)                  */

#define MFD_LCDE 0
#define MFD_BURGERS 1
#define MFD_NSE 2
#define MFD_WAVE 3   /* wave equation, Eq. (ME-NCDE-W-1): EDF of Example 3   */

#define MFD_PERIODIC 0
#define MFD_DIRICHLET 1 /* 2D MMFD: edge nodes hold prescribed values        */

#define MFD_TWO_LEVEL 0   /* explicit, level t only (ah = 0)                 */
#define MFD_THETA 1       /* two-level theta scheme, Eq. (GCN): LCDE, Burgers (beta = 1), NSE */
#define MFD_THREE_LEVEL 2 /* explicit, levels t and t - dt, Eq. (3layer-1)   */

/* presets of the three-level family (after Eq. (4-2-00)) and Eq. (LMMFD-2-2) */
#define MFD_PRESET_SRT 0        /* SRT LB, tau = 1 (param unused)            */
#define MFD_PRESET_TRT 1        /* TRT LB with s+ + s- = 2, param = s-        */
#define MFD_PRESET_ONE_STAGE 2  /* one-stage simplified LB, param = tau       */
#define MFD_PRESET_TWO_LEVEL 3  /* m = 1 two-level family, param = s          */

typedef struct mfd_solver mfd_solver;

typedef struct {
    int32_t dim;        /* 1, 2 or 3; must match the lattice                 */
    int32_t precision;  /* MFD_FP64 / MFD_FP32                               */
    int32_t form;       /* MFD_MMFD / MFD_MESOFD                             */
    int32_t boundary;   /* MFD_PERIODIC, or MFD_DIRICHLET (2D, MMFD form)    */
    int64_t n[3];       /* nodes along x, y, z (unused axes: 1); >= 3 each   */
    double dx;          /* node spacing (square / cubic grid), > 0           */
} mfd_grid;

/* Rectangular lattice of Appendix A for the linear CDE: spacing dx[a] along
 * axis a and d0[a] = c_s,a^2 / c_a^2 (c_a = dx[a] / dt) per axis (entries
 * beyond the grid's dimension are ignored).  The weights are Appendix A's
 * with d0 per axis (e.g. rD2Q9: w0 = (1 - d01)(1 - d02),
 * w_x = d01 (1 - d02) / 2, w_y = (1 - d01) d02 / 2, w_diag = d01 d02 / 4;
 * rD2Q5II and rD3Q9 take one d0), the EDF of Eq. (3-3)/(3-4) takes
 * c~_ja = e_ja / d0_a and Q~ per axis, and the equation's u and K map per
 * axis (u_a dt / dx_a, K_ab dt / (dx_a dx_b)); the grid's dx is then unused.
 * The kernels are those of the square lattice (the per-axis values live in
 * the constant tables).  Call after mfd_set_lattice (which returns to the
 * square lattice); MFD_E_ORDER before it, MFD_E_UNSUPPORTED for an
 * equation other than the linear CDE (set before or after), for unequal d0
 * on rD2Q5II / rD3Q9 and with a source term, MFD_E_ARG for d0 outside
 * (0, 1), a non-positive spacing or a non-positive weight. */
int mfd_set_rectangular(mfd_solver *s, const double dx[3], const double d0[3]);

/* Equation parameters.  MFD_WAVE (phi_tt = alpha Laplacian phi) uses the EDF
 * f_j = w_j phi [1 + (beta - 1)(|e_j|^2 - dim d0) / (2 d0)] printed with
 * Example 3 (beta > 0; 0 selects 1) and the linear-CDE kernels; its wave
 * coefficient is alpha = A22 beta c_s^2 (Eq. (ME-NCDE-W-1)), set through the
 * coefficients (e.g. a = (gamma, 2(1 - gamma), gamma), ah = (0, -1, 0),
 * gamma = alpha / (beta c_s^2), after Eq. (4-2-00)). */
typedef struct {
    double u[3];        /* LCDE: constant advection velocity (physical)      */
    double K[9];        /* LCDE: diffusion tensor, row-major 3 x 3           */
    int32_t lambda_bar; /* LCDE: 0 or 1, the u u term of Eq. (TforMMFD-0)    */
    int32_t he_luo;     /* NSE: 1 selects g(rho, rho0 u, rho0 u u)           */
    double beta;        /* Burgers: D = phi I scaled by beta (1 = default);  */
                        /* wave: the EDF's beta                              */
    double rho0;        /* NSE: reference density stored apart from rho      */
} mfd_eq_params;

/* ---------------------------------------------------------- solver set-up */

/* Create a solver for a periodic grid, or (boundary = MFD_DIRICHLET, 2D,
 * MMFD form) a grid whose edge nodes (x or y = 0 or n - 1) hold prescribed
 * values (mfd_set_boundary) and whose other nodes are updated by the scheme.
 * *out receives an owned handle to be released with mfd_destroy.  Errors:
 * MFD_E_ARG (null pointers, dim/n/dx out of range, unknown precision, form or
 * boundary), MFD_E_UNSUPPORTED (Dirichlet outside 2D MMFD). */
int mfd_create(mfd_solver **out, const mfd_grid *g);

/* Release the solver and every device buffer it owns.  Never frees memory
 * passed in by the caller.  Accepts NULL. */
int mfd_destroy(mfd_solver *s);

/* Library-owned, NUL-terminated description of the solver's last error
 * ("" if none).  Valid until the next call on the solver. */
const char *mfd_last_error(const mfd_solver *s);

/* Lattice of Appendix A with d0 = c_s^2/c^2 on every axis (d0 <= 0 selects
 * 1/3).  Rejects weights outside the Appendix ranges (MFD_E_ARG) and lattices
 * whose dimension differs from the grid's (MFD_E_ARG). */
int mfd_set_lattice(mfd_solver *s, int lattice, double d0);

/* Equation and its parameters (copied).  MFD_E_UNSUPPORTED for the NSE on
 * D1Q3.  On D2Q5 the quadratic EDF term cannot represent cross-axis
 * diagonal C (no e_x^2 e_y^2 moment); the call then returns
 * MFD_W_INCONSISTENT. */
int mfd_set_equation(mfd_solver *s, int eq, const mfd_eq_params *p);

/* Scheme: kind (MFD_TWO_LEVEL, MFD_THETA, MFD_THREE_LEVEL), coefficients
 * a[k+1] (k = -1, 0, 1) for level t and ah[k+1] for level t - dt
 * (three-level notation of Eq. (3layer-1); ah is ignored unless
 * MFD_THREE_LEVEL), optional momentum set ab / abh of Eq. (2-4) (NULL: equal
 * to a / ah), theta in [0,1] with theta_iters sweeps (MFD_THETA) and the
 * time step dt > 0.  The theta step (periodic grids, MMFD form) is solved by
 * Jacobi sweeps for the linear CDE and by Picard sweeps for Burgers' equation
 * (beta = 1) and the NSE: each sweep takes the explicit step of the iterate
 * and moves the own-node coefficient of the linear EDF parts to the left,
 * per field (density / scalar: 2 sum_p (a_1 + a_-1) w_p; momentum j_a:
 * 2 sum_{p: e_pa != 0} (ab_1 + ab_-1) w_p / d0); MFD_E_UNSUPPORTED for other
 * equations.  Must follow mfd_set_lattice and mfd_set_equation.
 * Returns MFD_W_INCONSISTENT if A00 != 1 (Eq. (4-2-00a)) and
 * MFD_W_STABILITY_UNPROVEN if the linear(ised) scheme fails the sufficient
 * conditions (Theorem 1 / Corollary 2); both are warnings. */
int mfd_set_scheme(mfd_solver *s, int kind, const double a[3], const double ah[3],
                   const double ab[3], const double abh[3], double theta,
                   int32_t theta_iters, double dt);

/* Multiple-set (TRT-type) explicit scheme of Eq. (2-2-1b) for a scalar
 * equation (linear CDE, Burgers, wave) in the MMFD form: the base terms
 * sum_k a_k phi (+ sum_k ah_k phi^(n-1)) take the set a / ah, the second
 * differences of the even EDF parts take the even set ae / aeh (through
 * ae_1 + ae_-1), the first differences of the odd parts the odd set ao / aoh
 * (through ao_1 - ao_-1); index k + 1 for k = -1, 0, +1, level t and t - dt
 * (ah, aeh, aoh only for MFD_THREE_LEVEL).  With ae = ao = a it is the scheme
 * of mfd_set_scheme; with a = ae its moments are those of the populations of
 * Eq. (2-1b).  The linear CDE maps K with A10 of the base set and A22 of the
 * even set.  Checks and warnings as mfd_set_scheme on the base set;
 * MFD_E_UNSUPPORTED for the NSE, the MesoFD form or kinds other than two-
 * and three-level. */
int mfd_set_scheme_sets(mfd_solver *s, int kind, const double a[3], const double ah[3],
                        const double ae[3], const double aeh[3], const double ao[3],
                        const double aoh[3], double dt);

/* Solve every theta step (Eq. (GCN), Theorem 2) to a residual tolerance:
 * Jacobi sweeps started from phi(t), checked after every `chunk` sweeps
 * (0: 8; at most 16), stopping at the first check where
 *     den^2 sum_x (x_k - x_(k-1))^2 <= tol^2 sum_x rhs^2
 * (den (x_k - x_(k-1)) is the residual rhs - (I - (1-theta) L) x_(k-1);
 * den = 1 + (1-theta) 2 sum_p (a_1 + a_-1) ubar+_p; sums in binary64; for
 * the NSE the two sums run over all fields, each field's squared differences
 * weighted by its own den^2), or at the first check at or beyond theta_iters
 * sweeps (the cap), returning x_k.
 * tol = 0 restores the fixed count of theta_iters sweeps.  On 2D D2Q5 / D2Q9
 * grids of at least 64 x 32 nodes the stop is decided on the device (no host
 * round trip per step); other grids check on the host after each chunk.
 * Suggested tolerances: 1e-12 (binary64), 1e-6 (binary32).  MFD_E_ORDER
 * unless a theta scheme is set, MFD_E_ARG for tol < 0, chunk outside
 * [0, 16] or a cap below 1. */
int mfd_set_theta_tolerance(mfd_solver *s, double tol, int32_t chunk);

/* Solve the theta steps of the linear CDE on a periodic 2D D2Q5 / D2Q9 grid
 * by geometric multigrid V-cycles instead of Jacobi sweeps (Eq. (GCN): the
 * same step, (I - (1-theta) L) x = A0 phi + theta L phi).  Level l has
 * (nx >> l) x (ny >> l) nodes and the operator discretised again on the
 * coarser spacing (second differences Cp_p / 4^l, first differences
 * Cm_p / 2^l); weighted Jacobi smoothing (weight 0.8), full-weighting
 * restriction of the residual, bilinear prolongation; on the coarsest level
 * as many sweeps (2 .. 64) as cut its error 1000-fold at the weighted Jacobi
 * bound.  The grid allows levels while both sides stay even and at least 4
 * when halved.  levels: 0 switches multigrid off (Jacobi sweeps), -1 takes
 * them down to the first level of at most 4096 nodes (at least 2 levels),
 * 2 .. the allowed number takes as many; pre in [1, 8] and post in
 * [0, 8] smoothing sweeps per level and cycle.  Each step starts from
 * phi(t) and, with a tolerance set (mfd_set_theta_tolerance), stops after the
 * first cycle with sum (rhs - A x)^2 <= tol^2 sum rhs^2 (binary64 sums), at
 * most theta_iters cycles; without one it runs theta_iters cycles.
 * mfd_theta_stats then counts cycles.  Device memory: one more level of
 * scratch plus three arrays per coarser level (about 2 x one field).  A new
 * mfd_set_scheme switches it off.  MFD_E_ORDER unless a theta scheme is set,
 * MFD_E_UNSUPPORTED for other equations or lattices, MFD_E_ARG for levels the
 * grid does not allow or sweep counts out of range, MFD_E_OOM. */
int mfd_set_theta_multigrid(mfd_solver *s, int32_t levels, int32_t pre, int32_t post);

/* Sweeps taken by the to-tolerance theta solves since the last reset: total,
 * time steps, the most in one step and the steps stopped by the cap before
 * the tolerance held.  Synchronous; reset = 1 zeroes the counters. */
int mfd_theta_stats(mfd_solver *s, int64_t *total_sweeps, int64_t *steps, int32_t *max_sweeps,
                    int32_t *unconverged, int reset);

/* Enqueue all further work of this solver on the HIP stream `stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL =
 * null stream).  The stream must outlive its use by the solver. */
int mfd_set_stream(mfd_solver *s, void *stream);

/* Element counts of one time level: moments (nf * nodes) and populations
 * (b * nodes, 0 for MMFD), and the bytes of device memory the solver holds
 * or will hold once configured. */
int mfd_state_size(const mfd_solver *s, int64_t *moment_elems, int64_t *population_elems,
                   int64_t *device_bytes);

/* ------------------------------------------------------------- state I/O */

/* Set a time level: level 0 = t^n, level 1 = t^(n-1) (three-level only).
 * MMFD: moments of that level.  MesoFD, level 0: moments, from which the
 * populations are initialised to the EDF (f_j = f_j^eq), or, with
 * `populations` = 1, the populations themselves; level 1: moments.
 * Elements are of the solver's precision; `bytes` must equal their total
 * size.  `on_device` = 1 if src is device memory.  Synchronous.  Setting
 * level 0 of a three-level scheme also sets level 1 to the same values
 * (the phi^(-1) = phi^0 start) unless level 1 is set afterwards. */
int mfd_set_state(mfd_solver *s, int level, const void *src, int64_t bytes, int on_device,
                  int populations);

/* Copy a time level out (same level / population conventions; for MesoFD
 * level 0 with populations = 0 the moments are computed on the device by
 * Eq. (2-1-1)).  Synchronous. */
int mfd_get_state(mfd_solver *s, int level, void *dst, int64_t bytes, int on_device,
                  int populations);

/* --------------------------------------------------------------- stepping */

/* Enqueue nsteps >= 0 time steps; asynchronous with respect to the host. */
int mfd_step(mfd_solver *s, int64_t nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mfd_step on
 * caller-owned levels, allocating nothing.  `level0` (phi^n) and, for
 * three-level schemes only, `level1` (phi^(n-1)) are device buffers of the
 * solver's precision and layout (mfd_state_size moment elements each), read
 * and overwritten in place with phi^(n+nsteps) and phi^(n+nsteps-1)
 * (level1 must be NULL for two-level schemes).  The solver needs its
 * lattice, equation and scheme (explicit MMFD, no source term) but no state:
 * its own buffers and level roles are not touched.  The work levels live in
 * a fixed 64 MiB device array per GPU, held until the process ends, so a
 * level may hold at most 32 MiB (e.g. 2048^2 binary64 scalar fields or
 * 1448^2 binary32 NSE fields).  Every call on a GPU shares that array:
 * calls that overlap on one GPU (other streams or host threads) race and must
 * be serialised by the caller.  Asynchronous on the solver's stream, like
 * mfd_step.  MFD_E_ORDER before the scheme is set, MFD_E_UNSUPPORTED for
 * MesoFD, theta or source-term solvers, MFD_E_ARG for missing / extra level
 * pointers, nsteps < 0 or a state larger than the limit. */
int mfd_step_noalloc(mfd_solver *s, void *level0, void *level1, int64_t nsteps);

/* Source term of the linear CDE (explicit two- or three-level scheme; MMFD
 * form on every lattice, MesoFD form on 1D / 2D lattices): the b terms of
 * Eq. (2-1) / (3layerMMFD-1) with the source distribution F_j of
 * Eq. (SourceF) for the NCDE, F_j = w_j (S + c_j.M_1F / c_s^2), added to each
 * population (MesoFD) or taken in the central-difference form of
 * Eq. (2-2-1) (MMFD):
 *   S(x, t)  = exp(lambda t) G(x), t = n dt with n the steps taken since the
 *              last level-0 mfd_set_state (the step from t to t + dt reads S
 *              at t and at t - dt, whatever the scheme's levels of phi);
 *   M_1F     = v S, v[0..dim-1] a constant vector in physical units;
 *   b[3]     = b_k at level t, bh[3] = b_k at level t - dt, k = -1, 0, +1
 *              (Example 1 of the paper: b = (3/2, 0, 0), bh = (-1/2, 0, 0)).
 * G holds count = nx ny nz binary64 values, x fastest (host memory, or
 * device memory when on_device); it is copied (converted to the solver's
 * precision) into a device buffer the solver owns until mfd_clear_source or
 * mfd_destroy.  Each step is then a single-step launch followed by the source
 * launch: temporal blocking and the resident 1D paths are not used while a
 * source is set.  Returns MFD_E_ORDER before the scheme is set,
 * MFD_E_UNSUPPORTED for another equation, the theta scheme or a 3D MesoFD grid,
 * MFD_E_ARG for a null G, a wrong count or non-finite values, MFD_E_OOM. */
int mfd_set_source(mfd_solver *s, const double *G, int64_t count, int on_device, double lambda,
                   const double b[3], const double bh[3], const double v[3]);

/* Dirichlet values of a boundary = MFD_DIRICHLET grid (the grids of Example 3
 * of the paper): at time t = n dt (n the steps taken since the last level-0
 * mfd_set_state, as for the source term) every edge node holds
 * G(x) exp(lambda t); each step writes the values of its new level (binary32
 * grids: the binary64 product rounded once).  G holds nx * ny binary64
 * values, x fastest (host, or device memory when on_device); only the edge
 * nodes are read and copied (2 nx + 2 (ny - 2) values, owned by the solver).
 * The values of the levels passed to mfd_set_state are the caller's.
 * Supported steps: explicit two- and three-level MMFD of the linear CDE,
 * Burgers' equation and the wave equation (64-column blocked windows or one
 * step per launch).  MFD_E_ORDER on a periodic grid, MFD_E_ARG for a null G,
 * a wrong count or non-finite values, MFD_E_OOM.  mfd_step returns
 * MFD_E_ORDER on a Dirichlet grid until the values are set. */
int mfd_set_boundary(mfd_solver *s, const double *G, int64_t count, int on_device, double lambda);

/* Special first step of the three-level wave scheme (Example 3): from
 * phi^0 = level 0 as just set (no step taken yet) and phi_t = d phi / dt at
 * t = 0 (count = nodes binary64 values, host or device memory),
 *   phi^1 = phi^0 + dt phi_t + cw sum_axes [phi^0(x+e_a) - 2 phi^0 + phi^0(x-e_a)],
 *   cw = A22 beta d0 / 2  (the Taylor start phi + dt phi_t + dt^2 alpha
 *                          Laplacian(phi) / 2 with alpha = A22 beta c_s^2),
 * evaluated in binary64 and rounded once to the solver's precision, with the
 * Dirichlet values of t = dt on the edge of a Dirichlet grid.  Afterwards
 * level 1 holds phi^0, level 0 phi^1 and one step counts as taken.
 * Synchronous.  MFD_E_ORDER unless a three-level MFD_WAVE scheme is set and
 * level 0 was set with no step since (and on a Dirichlet grid the values),
 * MFD_E_ARG for a null phi_t or a wrong count. */
int mfd_wave_start(mfd_solver *s, const double *phi_t, int64_t count, int on_device);

/* Remove the source term (frees its buffer). */
int mfd_clear_source(mfd_solver *s);

/* Wait for all work the solver has enqueued. */
int mfd_synchronize(mfd_solver *s);

/* FP64 reductions over the current level (synchronous):
 * sums[f] = sum over nodes of moment field f (f < nf, others 0): the
 * conserved totals implied by the moment identities after Eq. (2-1-FD1);
 * *residual = || phi^n - phi^(n-m) ||_2 / m of field 0, where m is the number
 * of steps between the current level and the previous level the solver holds
 * (m = 1 except after a temporally blocked two-level launch of depth m);
 * 0 before the first step.
 * Returns MFD_E_UNSTABLE if a sum or the residual is not finite. */
int mfd_reduce(mfd_solver *s, double sums[4], double *residual);

/* Growth check of a solve (the moment sums of the reductions above are the
 * conserved quantities of Sec. 2; a blow-up of an unstable scheme makes them
 * overflow to Inf or NaN): with every > 0, mfd_step runs its steps in runs of
 * `every` and after each run performs the reductions of mfd_reduce, returning
 * MFD_E_UNSTABLE at the first non-finite sum or residual (the state then
 * holds the level that failed the check; the steps after it are not taken).
 * Each check synchronises the solver's stream.  The results of the steps are
 * those without the check, bit for bit.  every = 0 (the default) turns it
 * off; every < 0 is MFD_E_ARG. */
int mfd_set_check_interval(mfd_solver *s, int64_t every);

/* Autotune the launch plan (tile shape, temporal-blocking depth) of this
 * solver's configuration by timing candidates on its own state (restored
 * afterwards); the choice is cached per (lattice, equation, form, precision,
 * levels, size) for the process.  Synchronous. *chosen_tb receives the depth. */
int mfd_autotune(mfd_solver *s, int32_t *chosen_tb);

/* Force a temporal-blocking depth (1 = none; 0 = automatic).  Blocking is
 * implemented on D2Q5 / D2Q9 grids of at least 64 x (2 depth + 4) nodes
 * (depth <= 16, window LDS <= 160 KiB) for the MMFD form of the linear CDE,
 * Burgers' equation (two- and three-level) and the NSE (without an older-level
 * stencil), and for the two-level MesoFD form of the linear CDE and Burgers'
 * equation (the populations are then written at the last step of each
 * mfd_step call only: every step depends on the one before through its
 * moments alone, and the populations read back after mfd_step are those of
 * the final step);
 * MFD_E_UNSUPPORTED for other configured solvers. */
int mfd_set_blocking(mfd_solver *s, int32_t tb_depth);

/* Force a full launch plan: tb_depth steps per launch over windows of
 * window_rows x window_cols (64 or 128) nodes; tb_depth = 1 is one launch per
 * step.  MFD_E_UNSUPPORTED when the blocked kernel cannot run it on this
 * solver (see mfd_set_blocking; the grid needs at least window_cols x
 * window_rows nodes), MFD_E_ORDER before the scheme is set. */
int mfd_set_plan(mfd_solver *s, int32_t tb_depth, int32_t window_rows, int32_t window_cols);

/* The launch plan mfd_step uses now: *tb_depth time steps per launch of the
 * step kernel (1 = one launch per step), *window_rows and *window_cols, the
 * height and width of the temporally blocked kernel's LDS window (0 when
 * tb_depth is 1).  Any pointer may be NULL.  MFD_E_ORDER before the scheme
 * is set. */
int mfd_launch_plan(const mfd_solver *s, int32_t *tb_depth, int32_t *window_rows,
                    int32_t *window_cols);

/* ---------------------------------------------------------------- batches */

/* A batch advances many solvers (independent periodic grids of any sizes,
 * coefficients and step counts) together: the solvers of one kind (lattice,
 * equation, levels, precision) form a group, each time step of a group is one
 * kernel launch over the tiles of the solvers still running (or, under a
 * temporally blocked plan, each launch advances every running solver by up to
 * tb steps), and the whole launch sequence is captured once into a hipGraph
 * and replayed by every mfd_batch_run.  Each solver's result equals the one
 * of stepping it alone (the same node update, value for value).  Only 2D
 * explicit MMFD solvers (D2Q5, D2Q9) can be batched.
 * A batch references its solvers: they must outlive it, must not be
 * stepped by other calls while a run is in flight, and their own streams
 * must be idle when a run is enqueued. */
typedef struct mfd_batch mfd_batch;

int mfd_batch_create(mfd_batch **out);
int mfd_batch_destroy(mfd_batch *b);
const char *mfd_batch_last_error(const mfd_batch *b);

/* Stream the runs are enqueued on (non-null: graph capture needs one; default
 * is a stream the batch creates). */
int mfd_batch_set_stream(mfd_batch *b, void *stream);

/* 1 (default): capture the step sequence in a hipGraph; 0: plain launches. */
int mfd_batch_set_graph(mfd_batch *b, int use_graph);

/* Add a configured solver with its state set, to be advanced nsteps >= 0 per
 * run.  *slot receives its index.  MFD_E_UNSUPPORTED for solvers that are not
 * 2D explicit MMFD or that have a source term. */
int mfd_batch_add(mfd_batch *b, mfd_solver *s, int64_t nsteps, int32_t *slot);

/* Remove every solver. */
int mfd_batch_clear(mfd_batch *b);

/* Enqueue one run (asynchronous); afterwards each solver holds its advanced
 * state as if mfd_step(s, nsteps) had been called. */
int mfd_batch_run(mfd_batch *b);

/* Wait for the batch's stream. */
int mfd_batch_wait(mfd_batch *b);

/* Kernel launches per run, lattice-node updates per run, tiles. */
int mfd_batch_stats(const mfd_batch *b, int64_t *launches, int64_t *lups, int64_t *tiles);

/* LDS-resident instances: binary32 two-level linear CDE and Burgers
 * instances of at most max_nodes nodes (nx ny; capped at 20480, where their
 * two levels fill the 160 KiB of LDS) run all of their steps in one
 * workgroup each, in one launch per kind on a branch of the run beside the
 * windowed launches (the run's graph forks and joins it), with the
 * single-step node function: results are those of the windowed path value
 * for value.  max_nodes = 0 sends every instance to the windowed launches;
 * the default is 4096 (grids up to 64 x 64, which a blocked window would
 * mostly spend on wrapped copies of the grid; larger resident grids hold a
 * CU's whole LDS for all of their steps).  MFD_E_ARG for max_nodes < 0.
 * Takes effect at the next run. */
int mfd_batch_set_resident(mfd_batch *b, int32_t max_nodes);

/* Number of instances the last build sent to the LDS-resident kernel. */
int mfd_batch_resident(const mfd_batch *b, int32_t *count);

/* Launch plan of the groups that can be temporally blocked (two-level linear
 * CDE and Burgers groups, NSE groups without an older-level stencil; others
 * always take one launch per step): tb_depth = 1 one launch per step,
 * tb_depth > 1 up to tb_depth steps per launch over windows of window_cols x
 * window_rows nodes, 0 automatic (the plan chosen by mfd_batch_autotune, else
 * one launch per step).  window_cols: 64 (0 means 64), or 128 for the
 * lane-shared kernel of binary32 two-level linear CDE and Burgers (beta = 1)
 * groups (other groups then take the same plan in 64-column windows).  Any
 * grid size can be blocked in a batch (the window wraps periodically).
 * MFD_E_ARG for a plan beyond the kernels' limits: depth <= 16,
 * window_cols - 2 depth >= 8, window_rows >= 2 depth + 4, two window levels
 * (64 columns) or one (128 columns, window_rows <= 128) within 160 KiB of
 * LDS. */
int mfd_batch_set_plan(mfd_batch *b, int32_t tb_depth, int32_t window_rows, int32_t window_cols);

/* Pick the plan of every blockable group by timing each candidate's first
 * launch over all the group's instances (their current states; the spare
 * level each trial overwrites is restored).  Synchronous; the choice holds
 * for later runs of groups of the same kind. */
int mfd_batch_autotune(mfd_batch *b);

/* Plan of group `group` (groups in a fixed order of kind) after the last
 * run or autotune (window sizes 0 when tb_depth is 1).  Any pointer may be
 * NULL. */
int mfd_batch_plan(const mfd_batch *b, int32_t group, int32_t *tb_depth, int32_t *window_rows,
                   int32_t *window_cols);

/* ---------------------------------------------------------------- serving */

/* A server runs MMFD solves submitted by any thread with continuous
 * batching: a scheduler thread advances all admitted requests together in
 * quanta of `quantum_steps` steps (a batch run per quantum: one launch per
 * step, or per blocked group of steps for two-level linear CDE / Burgers
 * kinds, whose plan the batch autotuner picks on the first quantum that holds
 * the kind), admits queued requests (arrival order) whenever a slot and the
 * HBM budget allow, while the previous quantum is on the GPU, and retires
 * finished requests by copying their final level to the caller's buffer.
 * Each request's result equals the solve of the same request alone. */
typedef struct mfd_server mfd_server;

typedef struct {
    int32_t lattice;          /* MFD_D2Q9 or MFD_D2Q5                          */
    int32_t eq;               /* MFD_LCDE, MFD_BURGERS, MFD_NSE                */
    int32_t precision;        /* MFD_FP32 / MFD_FP64                           */
    int32_t kind;             /* MFD_TWO_LEVEL or MFD_THREE_LEVEL              */
    int64_t n[2];             /* grid nodes (x, y), >= 3                       */
    double d0;                /* lattice parameter (<= 0: 1/3)                 */
    double dx, dt;
    mfd_eq_params ep;
    double a[3], ah[3];       /* coefficients as for mfd_set_scheme            */
    int64_t nsteps;
    const void *state0;       /* level t moments (host, solver precision);     */
    const void *prev0;        /* level t - dt or NULL; both must stay valid    */
                              /* until the request has left the queue          */
    void *result_out;         /* host buffer for the final moments, or NULL    */
    int64_t result_bytes;
    int32_t exclude_from_stats; /* 1: not counted in the latency percentiles  */
    int32_t reserved;
    double timeout_s;         /* > 0: fail with MFD_E_TIMEOUT once this long   */
                              /* has passed since submission (checked at       */
                              /* quantum boundaries); 0: no timeout            */
} mfd_request;

/* Create a server with a device-memory budget, a slot limit and a quantum.
 * Starts the scheduler thread.  A request holds, from admission to
 * retirement, the device bytes of its solver (mfd_state_size: level ring,
 * fourth level of blocked three-level steps, reduction scratch) plus one
 * state level for the batch autotuner's copy and its batch tables; the sum
 * over admitted requests never exceeds hbm_budget_bytes. */
int mfd_server_create(mfd_server **out, int64_t hbm_budget_bytes, int32_t max_slots,
                      int64_t quantum_steps);

/* Queue a request (thread-safe, non-blocking); *ticket identifies it.  The
 * request's configuration is checked here (host only): errors of
 * mfd_create / mfd_set_lattice / mfd_set_equation / mfd_set_scheme are
 * returned, MFD_E_UNSUPPORTED for a kind other than MFD_TWO_LEVEL /
 * MFD_THREE_LEVEL or a lattice other than D2Q5 / D2Q9, MFD_E_ARG for a
 * result buffer of the wrong size.  A request whose bytes can never fit the
 * budget fails with MFD_E_BUDGET; one whose final level is not finite fails
 * with MFD_E_UNSTABLE; a failed batch run fails the requests it held with its
 * error.  A failed request frees its slot and budget without touching the
 * others. */
int mfd_server_submit(mfd_server *srv, const mfd_request *req, int64_t *ticket);

/* Device bytes a request holds while admitted (the figure the budget is
 * checked against); host only.  Errors as mfd_server_submit. */
int mfd_server_request_bytes(const mfd_request *req, int64_t *bytes);

/* Cancel a ticket: a queued request fails at once with MFD_E_CANCELLED, a
 * running one at the next quantum boundary (its slot and budget are freed).
 * MFD_E_ORDER if the request has already finished. */
int mfd_server_cancel(mfd_server *srv, int64_t ticket);

/* State of a ticket: 0 queued, 1 running, 2 done (result written), -1 failed
 * (the return value is then the error).  *latency_s: submission to result,
 * or -1 if not done. */
int mfd_server_poll(mfd_server *srv, int64_t ticket, int32_t *state, double *latency_s);

/* Block until every submitted request is done or failed (MFD_E_ORDER on
 * timeout). */
int mfd_server_drain(mfd_server *srv, double timeout_s);

/* Latency percentiles of the completed requests, completed requests per
 * second and lattice-node updates per second over the span from the first
 * counted submission to the last completion. */
int mfd_server_stats(mfd_server *srv, double *p50_s, double *p99_s, double *req_per_s,
                     int64_t *completed, double *glups);

/* Stop accepting work, finish the running requests, free everything. */
int mfd_server_destroy(mfd_server *srv);

/* Device bytes held now by every object of the library in this process, and
 * the peak since the last reset (reset_peak = 1 sets the peak to the current
 * figure after reading it).  Thread-safe. */
int mfd_memory_stats(int64_t *in_use, int64_t *peak, int reset_peak);

/* ------------------------------------------------------ host-side algebra */

/* Coefficient moments of Eq. (4-2-00): out = {A00, A10, A11, A20, A21, A22}. */
int mfd_coeff_moments(const double a[3], const double ah[3], double out[6]);

/* Coefficients meeting A00 = 1 and given (a0, A10, A11, A21, A22),
 * closed form Eq. (X).  Writes a[3], ah[3]. */
int mfd_coeffs_from_constraints(double a0, double A10, double A11, double A21, double A22,
                                double a[3], double ah[3]);

/* Preset coefficient sets (MFD_PRESET_*). */
int mfd_preset(int preset, double param, double a[3], double ah[3]);

/* Transport coefficient of a coefficient set on a lattice:
 * -(A22/A10) dt beta d0 dx^2/dt^2 (diffusivity alpha for the NCDE, kinematic
 * viscosity nu for the NSE with beta = 1). */
int mfd_transport_coefficient(const double a[3], const double ah[3], double dx, double dt,
                              double d0, double beta, double *out);

/* Largest modulus over the grid's Fourier modes of the amplification
 * factor(s) of the configured linear (LCDE) scheme, Eq. (TforMMFD-3)
 * (roots of lambda^2 - p1 lambda - p0 for three-level schemes, the theta
 * factor of Eq. (Tcond1-1) for MFD_THETA). */
int mfd_max_amplification(mfd_solver *s, double *out);

/* Largest stable time step of the two-level m = 1 MMFD scheme for the linear
 * CDE with the linear EDF (D0 = I, beta = 1, lambda_bar = 0; Eq. (LMMFD-1))
 * whose coefficients follow Eq. (LMMFD-2-2) for each dt (a_0 = 1 - s,
 * a_{+-1} = (s -+ 1)/2, s = 2 alpha dt / (d0 dx^2)), isotropic diffusivity
 * alpha > 0 and velocity u[3] (physical units; unused axes 0) on `lattice`
 * with d0 (<= 0: 1/3):
 *   *dt_sufficient = the bound of Eq. (LMMFD-2-3),
 *                    min(d0 dx^2 / (2 alpha (1 - w0)), 2 alpha / |u|^2);
 *   *dt_exact      = (when n and dt_exact are non-NULL) the largest dt with
 *                    |lambda| <= 1 for every Fourier mode of the periodic
 *                    grid n[0..dim-1] (Eq. (TforMMFD-3)), in closed form per
 *                    mode; n may hold at most 2^24 nodes.
 * Host only.  MFD_E_ARG for a bad lattice, d0, dx, alpha, u or n. */
int mfd_max_stable_dt(int lattice, double d0, double dx, const double u[3], double alpha,
                      const int64_t n[3], double *dt_sufficient, double *dt_exact);

/* Device address of the current storage of a time level: level 0 = t^n,
 * level 1 = t^(n-1) (three-level schemes), moment field `field` (0..nf-1),
 * or with populations = 1 (MesoFD, level 0) population j = field.  The
 * address is owned by the solver and stays valid until the next call that
 * steps or sets the state (mfd_step rotates the level roles among the
 * solver's buffers); it is device memory holding G.N elements of the
 * solver's precision, x fastest.  MFD_E_ORDER before the state is set,
 * MFD_E_ARG for a level, field or population request that does not exist. */
int mfd_level_ptr(mfd_solver *s, int level, int field, int populations, void **ptr);

/* Per-pair linear EDF constants of the configured LCDE (for checks):
 * ubar[b] (full EDF per unit phi), and per opposite pair p:
 * out6[0..5][p] = ubar+_p, ubar-_p, (a_1+a_-1) ubar+_p, (a_1-a_-1) ubar-_p,
 * (ah_1+ah_-1) ubar+_p, (ah_1-ah_-1) ubar-_p; stride 9 per row. */
int mfd_linear_tables(mfd_solver *s, double *w, double *ubar, double *out6);

/* ------------------------------------------------ general-scheme solver
 * The MMFD scheme of Eq. (2-2-1) / (2-4-1) with any stencil reach m and any
 * number n of time levels (the index ranges -m <= k <= m and the levels
 * t - l dt, l = 0 .. n - 1, of Eq. (2-1)), periodic:
 *   scalar / density: sum_l A_l phi_l + sum_l sum_p sum_{k=1..m}
 *                     [(a_lk + a_l,-k) D2_{p,k} F+_p + (a_lk - a_l,-k) D1_{p,k} F-_p]
 *   momentum (NSE):   sum_l Ab_l j_l + sum_l sum_p e_p sum_{k=1..m}
 *                     [(ab_lk + ab_l,-k) D2_{p,k} F-_p + (ab_lk - ab_l,-k) D1_{p,k} F+_p]
 * on the pair parts F+-_p of each level's EDF, A_l = sum_k a_lk,
 * D2_{p,k} g = g(x + k e_p) - 2 g + g(x - k e_p), D1_{p,k} g = g(x + k e_p)
 * - g(x - k e_p).  eq_code: MFD_LCDE (the linear EDF of Eq. (TforMMFD-0);
 * every lattice including rD3Q27, square or rectangular; its diffusion
 * tensor follows the scheme's own moments of Eq. (4-2-00a) with the new level
 * at q = 0: C = (-A10 / A22) K dt / dx^2 - diag(d0) + lambda_bar u u in
 * lattice units, A10 = sum_lk -(l + 1) a_lk, A22 = (1/2) sum_lk k^2 a_lk, so
 * A10 < 0 < A22 is required), MFD_BURGERS or MFD_NSE (square lattices of up
 * to 19 velocities; the NSE's viscosity follows the momentum set's own
 * moments).  mfd_general_create: grid (MMFD form, periodic, FP64 / FP32),
 * lattice (MFD_D1Q3 .. MFD_D3Q27), d0 (d0[0] on a square grid, one per axis
 * with spacing; NULL: 1/3), spacing (NULL: the square grid of grid->dx; else
 * the spacing per axis of a rectangular lattice, linear CDE only), eq_code,
 * the equation's parameters (u, K, lambda_bar; beta; rho0, he_luo),
 * 1 <= m <= 3, 1 <= n <= 4, a and ab (NSE momentum set; NULL: a): n rows
 * of 2m + 1 (row l = level t - l dt, entry k + m), dt > 0; n[1] <= 262140
 * and n[2] <= 65535 (launch-grid limits).  Returns MFD_OK
 * or MFD_W_INCONSISTENT (A00 != 1, or for the linear CDE A11 != A10) with
 * *out set; MFD_E_ARG for bad sizes or coefficients, MFD_E_UNSUPPORTED for
 * another form, boundary or equation, or a lattice / spacing the equation
 * does not take, MFD_E_OOM.  Levels hold the equation's fields (1, or
 * 1 + dim for the NSE: rho - rho0, then j), field-major, x fastest:
 * set_level(0) fills every level with the data (phi^(-l) = phi^0),
 * set_level(l) then overrides level t - l dt; get_level(l) reads it
 * (synchronous, host or device pointers).  step advances nsteps steps on
 * the solver's stream (the default stream unless set). */
typedef struct mfd_general mfd_general;
int mfd_general_create(mfd_general **out, const mfd_grid *grid, int lattice, const double d0[3],
                       const double spacing[3], int eq_code, const mfd_eq_params *eq, int32_t m,
                       int32_t n, const double *a, const double *ab, double dt);
int mfd_general_destroy(mfd_general *g);
const char *mfd_general_last_error(const mfd_general *g);
int mfd_general_set_stream(mfd_general *g, void *stream);
int mfd_general_set_level(mfd_general *g, int32_t level, const void *src, int64_t bytes,
                          int on_device);
int mfd_general_get_level(mfd_general *g, int32_t level, void *dst, int64_t bytes, int on_device);
int mfd_general_step(mfd_general *g, int64_t nsteps);
int mfd_general_synchronize(mfd_general *g);

#ifdef __cplusplus
}
#endif
#endif /* MFD_H */
