// Geometric multigrid V-cycles for the linear CDE's theta step (Eq. (GCN))
// on periodic 2D grids (D2Q5 / D2Q9):
//   A x = R,   A = I - (1 - theta) L,   L x = sum_p [Cp_p D2_p x + Cm_p D1_p x],
// D2_p x = x(+e_p) - 2 x + x(-e_p), D1_p x = x(+e_p) - x(-e_p).
//
// Level l has (nx >> l) x (ny >> l) nodes of spacing 2^l dx and the operator
// discretised again on that spacing: the second differences take Cp_p / 4^l
// and the first differences Cm_p / 2^l, so every level carries the same
// continuous operator.  On every level
//   A x = den x - sum_p [cpos_p x(+e_p) + cneg_p x(-e_p)],
//   cpos_p = (1 - theta)(Cp_p + Cm_p), cneg_p = (1 - theta)(Cp_p - Cm_p),
//   den = 1 + (1 - theta) 2 sum_p Cp_p        (level-scaled Cp, Cm).
// Smoother: weighted Jacobi, x <- x + omega ((R + nbr(x)) / den - x).
// Transfer: the residual R - A x restricted by full weighting,
// (1 2 1) x (1 2 1) / 16 around fine node (2I, 2J); the coarse correction
// prolongated bilinearly and added.  One thread per node, periodic wrap.
#include <cstring>

#include "edf.h"
#include "mg.h"

namespace mfd {

namespace {

template <class L, typename T>
__device__ __forceinline__ T mg_nbr(const T *__restrict__ x, const MgOp<T> &op, int i, int j) {
  const int nx = op.nx, ny = op.ny;
  const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
  const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
  T acc = 0;
  static_for<L::P>([&](auto PI) {
    constexpr int P = decltype(PI)::value;
    constexpr int J = L::PR[P];
    constexpr int ex = L::E[J][0], ey = L::E[J][1];
    const int xp = ex > 0 ? ip : (ex < 0 ? im : i), yp = ey > 0 ? jp : (ey < 0 ? jm : j);
    const int xm = ex > 0 ? im : (ex < 0 ? ip : i), ym = ey > 0 ? jm : (ey < 0 ? jp : j);
    acc = acc + op.cpos[P] * x[(int64_t)yp * nx + xp];
    acc = acc + op.cneg[P] * x[(int64_t)ym * nx + xm];
  });
  return acc;
}

template <class L, typename T>
__device__ __forceinline__ T mg_resid(const T *__restrict__ x, const T *__restrict__ R,
                                      const MgOp<T> &op, int i, int j) {
  const int64_t k = (int64_t)j * op.nx + i;
  return R[k] - (op.den * x[k] - mg_nbr<L, T>(x, op, i, j));
}

// ZERO: the iterate is 0 (a coarse level's first sweep): out = omega R / den
template <class L, bool ZERO, typename T>
__global__ __launch_bounds__(256) void k_mg_smooth(const T *__restrict__ x, const T *__restrict__ R,
                                                   T *__restrict__ out, MgOp<T> op, T omega) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= op.nx || j >= op.ny) return;
  const int64_t k = (int64_t)j * op.nx + i;
  if constexpr (ZERO) {
    out[k] = omega * (R[k] * op.inv_den);
  } else {
    const T xk = x[k];
    const T xj = (R[k] + mg_nbr<L, T>(x, op, i, j)) * op.inv_den;
    out[k] = xk + omega * (xj - xk);
  }
}

// x(i, j) += the bilinear interpolation of the coarse correction e at the
// fine node: e(I, J) at (2I, 2J), the mean of the two (four) coarse nodes
// around an edge (cell) midpoint
template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong_add(const T *__restrict__ e, T *__restrict__ x,
                                                        int nx, int ny) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const int ncx = nx >> 1, ncy = ny >> 1;
  const int I = i >> 1, J = j >> 1;
  const int I1 = I + 1 == ncx ? 0 : I + 1, J1 = J + 1 == ncy ? 0 : J + 1;
  const bool ox = i & 1, oy = j & 1;
  const T e00 = e[(int64_t)J * ncx + I];
  T v;
  if (!ox && !oy) {
    v = e00;
  } else if (ox && !oy) {
    v = (e00 + e[(int64_t)J * ncx + I1]) * T(0.5);
  } else if (!ox && oy) {
    v = (e00 + e[(int64_t)J1 * ncx + I]) * T(0.5);
  } else {
    v = ((e00 + e[(int64_t)J * ncx + I1]) + (e[(int64_t)J1 * ncx + I] + e[(int64_t)J1 * ncx + I1])) *
        T(0.25);
  }
  const int64_t k = (int64_t)j * nx + i;
  x[k] = x[k] + v;
}

// r = R - A x
template <class L, typename T>
__global__ __launch_bounds__(256) void k_mg_residual(const T *__restrict__ x, const T *__restrict__ R,
                                                     T *__restrict__ r, MgOp<T> op) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= op.nx || j >= op.ny) return;
  r[(int64_t)j * op.nx + i] = mg_resid<L, T>(x, R, op, i, j);
}

// Rc(I, J) = sum_{a, b = -1..1} w_a w_b r(2I + a, 2J + b) / 16, w = (1, 2, 1)
template <typename T>
__global__ __launch_bounds__(256) void k_mg_restrict_r(const T *__restrict__ r, T *__restrict__ Rc,
                                                       int nx, int ny, int ncx, int ncy) {
  const int I = blockIdx.x * 64 + threadIdx.x, J = blockIdx.y * 4 + threadIdx.y;
  if (I >= ncx || J >= ncy) return;
  T acc = 0;
#pragma unroll
  for (int b = -1; b <= 1; ++b) {
    int j = 2 * J + b;
    j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
    T row = 0;
#pragma unroll
    for (int a = -1; a <= 1; ++a) {
      int i = 2 * I + a;
      i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
      const T v = r[(int64_t)j * nx + i];
      row = row + (a == 0 ? T(2) * v : v);
    }
    acc = acc + (b == 0 ? T(2) * row : row);
  }
  Rc[(int64_t)J * ncx + I] = acc * T(0.0625);
}

__device__ __forceinline__ double mg_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// binary64 sums of (R - A x)^2 and R^2: per workgroup (grid-stride rows),
// then one workgroup adds the partials in a fixed order
template <class L, typename T>
__global__ __launch_bounds__(256) void k_mg_resid_norm(const T *__restrict__ x,
                                                       const T *__restrict__ R, MgOp<T> op,
                                                       double *__restrict__ partial) {
  double s0 = 0.0, s1 = 0.0;
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < op.nx) {
    for (int j = blockIdx.y * 4 + threadIdx.y; j < op.ny; j += gridDim.y * 4) {
      const double r = (double)mg_resid<L, T>(x, R, op, i, j);
      const double b = (double)R[(int64_t)j * op.nx + i];
      s0 += r * r;
      s1 += b * b;
    }
  }
  s0 = mg_wave_sum(s0);
  s1 = mg_wave_sum(s1);
  __shared__ double red[2][4];
  const int t = threadIdx.y * 64 + threadIdx.x;
  if ((t & 63) == 0) {
    red[0][t >> 6] = s0;
    red[1][t >> 6] = s1;
  }
  __syncthreads();
  if (t < 2) {
    partial[2 * (blockIdx.y * gridDim.x + blockIdx.x) + t] =
        ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
  }
}

__global__ __launch_bounds__(256) void k_mg_norm_final(const double *__restrict__ partial, int nblk,
                                                       double *__restrict__ out) {
  double s0 = 0.0, s1 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    s0 += partial[2 * b];
    s1 += partial[2 * b + 1];
  }
  s0 = mg_wave_sum(s0);
  s1 = mg_wave_sum(s1);
  __shared__ double red[2][4];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s0;
    red[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    out[threadIdx.x] = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) +
                       red[threadIdx.x][3];
}

dim3 mg_grid(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }

template <class L, typename T>
hipError_t smooth_l(const T *x, const T *R, T *out, const MgOp<T> &op, double omega, bool zero,
                    hipStream_t st) {
  if (zero)
    hipLaunchKernelGGL((k_mg_smooth<L, true, T>), mg_grid(op.nx, op.ny), dim3(64, 4), 0, st, x, R,
                       out, op, (T)omega);
  else
    hipLaunchKernelGGL((k_mg_smooth<L, false, T>), mg_grid(op.nx, op.ny), dim3(64, 4), 0, st, x,
                       R, out, op, (T)omega);
  return hipGetLastError();
}

}  // namespace

template <typename T>
MgOp<T> mg_op(const Consts &c, int level, int nx, int ny) {
  MgOp<T> op;
  std::memset(&op, 0, sizeof(op));
  double s2 = 1.0, s1 = 1.0;
  for (int l = 0; l < level; ++l) {
    s2 = s2 * 0.25;
    s1 = s1 * 0.5;
  }
  double sp = 0.0;
  for (int p = 0; p < c.npair; ++p) {
    const double Cp = c.Cp[p] * s2, Cm = c.Cm[p] * s1;
    op.cpos[p] = (T)(c.th1 * (Cp + Cm));
    op.cneg[p] = (T)(c.th1 * (Cp - Cm));
    sp = sp + Cp;
  }
  const double den = 1.0 + c.th1 * (2.0 * sp);
  op.den = (T)den;
  op.inv_den = (T)(1.0 / den);
  op.nx = nx;
  op.ny = ny;
  return op;
}

template <typename T>
hipError_t launch_mg_smooth(int lattice, const T *x, const T *R, T *out, const MgOp<T> &op,
                            double omega, bool zero, hipStream_t st) {
  if (lattice == 3) return smooth_l<LatD2Q9, T>(x, R, out, op, omega, zero, st);
  if (lattice == 2) return smooth_l<LatD2Q5, T>(x, R, out, op, omega, zero, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_mg_prolong_add(const T *e, T *x, int nx, int ny, hipStream_t st) {
  hipLaunchKernelGGL((k_mg_prolong_add<T>), mg_grid(nx, ny), dim3(64, 4), 0, st, e, x, nx, ny);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_residual(int lattice, const T *x, const T *R, T *r, const MgOp<T> &op,
                              hipStream_t st) {
  if (lattice == 3)
    hipLaunchKernelGGL((k_mg_residual<LatD2Q9, T>), mg_grid(op.nx, op.ny), dim3(64, 4), 0, st, x, R,
                       r, op);
  else if (lattice == 2)
    hipLaunchKernelGGL((k_mg_residual<LatD2Q5, T>), mg_grid(op.nx, op.ny), dim3(64, 4), 0, st, x, R,
                       r, op);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_restrict_r(const T *r, T *Rc, int nx, int ny, hipStream_t st) {
  const int ncx = nx / 2, ncy = ny / 2;
  hipLaunchKernelGGL((k_mg_restrict_r<T>), mg_grid(ncx, ncy), dim3(64, 4), 0, st, r, Rc, nx, ny,
                     ncx, ncy);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_resid_norm(int lattice, const T *x, const T *R, const MgOp<T> &op,
                                double *partial, double *out, hipStream_t st) {
  const int bx = (op.nx + 63) / 64;
  int by = (op.ny + 3) / 4;
  while (bx * by > kMgNormBlocks) by = (by + 1) / 2;
  if (lattice == 3)
    hipLaunchKernelGGL((k_mg_resid_norm<LatD2Q9, T>), dim3(bx, by), dim3(64, 4), 0, st, x, R, op,
                       partial);
  else if (lattice == 2)
    hipLaunchKernelGGL((k_mg_resid_norm<LatD2Q5, T>), dim3(bx, by), dim3(64, 4), 0, st, x, R, op,
                       partial);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mg_norm_final, dim3(1), dim3(256), 0, st, partial, bx * by, out);
  return hipGetLastError();
}

#define MFD_MG_INST(T)                                                                          \
  template MgOp<T> mg_op<T>(const Consts &, int, int, int);                                     \
  template hipError_t launch_mg_smooth<T>(int, const T *, const T *, T *, const MgOp<T> &,     \
                                          double, bool, hipStream_t);                           \
  template hipError_t launch_mg_prolong_add<T>(const T *, T *, int, int, hipStream_t);           \
  template hipError_t launch_mg_residual<T>(int, const T *, const T *, T *, const MgOp<T> &,    \
                                            hipStream_t);                                       \
  template hipError_t launch_mg_restrict_r<T>(const T *, T *, int, int, hipStream_t);           \
  template hipError_t launch_mg_resid_norm<T>(int, const T *, const T *, const MgOp<T> &,       \
                                              double *, double *, hipStream_t);
MFD_MG_INST(float)
MFD_MG_INST(double)
#undef MFD_MG_INST

}  // namespace mfd
