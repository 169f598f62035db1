// Multigrid V-cycles for the linear CDE's theta step on periodic 2D grids:
// the per-level operator and the kernel launches (kernels_mg.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mfd_internal.h"

namespace mfd {

constexpr int kMgMaxLevels = 16;
constexpr int kMgMinSide = 4;        // coarsest level: at least 4 x 4 nodes
constexpr int kMgCoarseSweeps = 64;  // most weighted Jacobi sweeps on the coarsest level
constexpr int64_t kMgAutoCoarseNodes = 4096;  // automatic levels: coarsest <= this many nodes
constexpr double kMgOmega = 0.8;     // Jacobi weight of the smoother

// A x = den x - sum_p [cpos_p x(+e_p) + cneg_p x(-e_p)] on an nx x ny level
template <typename T>
struct MgOp {
  T cpos[kMaxP], cneg[kMaxP];
  T den, inv_den;
  int nx, ny;
};

template <typename T>
MgOp<T> mg_op(const Consts &c, int level, int nx, int ny);
// out = x + omega ((R + nbr(x)) / den - x); zero: x = 0 (x is not read)
template <typename T>
hipError_t launch_mg_smooth(int lattice, const T *x, const T *R, T *out, const MgOp<T> &op,
                            double omega, bool zero, hipStream_t st);
// x += bilinear prolongation of the coarse correction e (x: nx x ny, e: half)
template <typename T>
hipError_t launch_mg_prolong_add(const T *e, T *x, int nx, int ny, hipStream_t st);
// r = R - A x
template <typename T>
hipError_t launch_mg_residual(int lattice, const T *x, const T *R, T *r, const MgOp<T> &op,
                              hipStream_t st);
// Rc = full-weighting restriction of r (nx x ny) to (nx / 2) x (ny / 2)
template <typename T>
hipError_t launch_mg_restrict_r(const T *r, T *Rc, int nx, int ny, hipStream_t st);
// out[0] = sum (R - A x)^2, out[1] = sum R^2 in binary64 (partial: 2 kMgNormBlocks doubles)
constexpr int kMgNormBlocks = 2048;
template <typename T>
hipError_t launch_mg_resid_norm(int lattice, const T *x, const T *R, const MgOp<T> &op,
                                double *partial, double *out, hipStream_t st);

}  // namespace mfd
