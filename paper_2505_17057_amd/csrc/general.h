// The general MMFD scheme of Eq. (2-2-1) for linear EDFs: any stencil reach
// m (<= kGenMaxM) and number of time levels n (<= kGenMaxLevels), any
// lattice of Appendix A (rD3Q27 included), periodic grids.
#pragma once

#include <hip/hip_runtime.h>

#include "mfd_internal.h"

namespace mfd {

constexpr int kGenMaxM = 3;
constexpr int kGenMaxLevels = 4;

// per level l: A[l] = sum_k a_lk; per level, k = 1..m and pair p:
// Cp = (a_lk + a_l,-k) ubp_p, Cm = (a_lk - a_l,-k) ubm_p (device memory)
template <typename T>
struct GenC {
  int m, nl;
  T A[kGenMaxLevels];
  T Cp[kGenMaxLevels][kGenMaxM][kHostMaxP];
  T Cm[kGenMaxLevels][kGenMaxM][kHostMaxP];
};

// Burgers' equation and the NSE: per level l the base sums A_l (density /
// scalar) and Ab_l (momentum), per level and k = 1..m the pair sums
// a+ = a_lk + a_l,-k, a- = a_lk - a_l,-k and the momentum set's ab+, ab-
// (the pair parts carry the weights); device memory
template <typename T>
struct GenNL {
  int m, nl;
  T A[kGenMaxLevels], Ab[kGenMaxLevels];
  T ap[kGenMaxLevels][kGenMaxM], am[kGenMaxLevels][kGenMaxM];
  T abp[kGenMaxLevels][kGenMaxM], abm[kGenMaxLevels][kGenMaxM];
};

// the levels t, t - dt, ... of one step, by value
template <typename T>
struct GenLevels {
  const T *p[kGenMaxLevels];
};

// one step of every node (m: the reach gc holds): out = sum_l A_l phi_l + sum_l sum_p sum_k
// [Cp D2_{p,k} phi_l + Cm D1_{p,k} phi_l]; gc in device memory
template <typename T>
hipError_t launch_general_step(int lattice, int m, GenLevels<T> lev, T *out, const int64_t n[3],
                               const GenC<T> *gc, hipStream_t st);
// the same for Burgers' equation (eq = kBurgers) and the NSE (kNSE, fields
// field-major) on lattices of at most 19 velocities: each neighbour's pair
// part from its moments (make_record, fplus, fminus of edf.h, as the
// single-step kernels form them)
template <typename T>
hipError_t launch_general_nl_step(const Consts &c, int m, GenLevels<T> lev, T *out,
                                  const int64_t n[3], const GenNL<T> *g, hipStream_t st);

}  // namespace mfd
