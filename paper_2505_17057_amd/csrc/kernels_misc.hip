// Theta-scheme kernels (LCDE, Eq. (GCN)) and FP64 reductions.
//
// theta step: (I - (1-theta) L) phi' = A0 phi + theta L phi,
//   L g = sum_p [Cp_p D2_p g + Cm_p D1_p g]   (the explicit increment)
// solved by Jacobi sweeps started from phi:
//   phi_{k+1} = (rhs + (1-theta) Loff phi_k) / (1 + (1-theta) 2 sum_p Cp_p),
//   Loff g = sum_p [Cp_p (g(x+e_p) + g(x-e_p)) + Cm_p (g(x+e_p) - g(x-e_p))].
//
// Reductions: sums over nodes accumulated in binary64 per thread (grid
// stride), reduced across the 64-lane wavefront with shuffles, across the
// workgroup through LDS, and across a fixed set of workgroups by a second
// single-workgroup pass in a fixed order: the result is deterministic.
#include "edf.h"

namespace mfd {

__device__ __forceinline__ int64_t nbr_index(int64_t i, const int64_t n[3], int ex, int ey,
                                             int ez) {
  int64_t x = i % n[0];
  int64_t y = (i / n[0]) % n[1];
  int64_t z = i / (n[0] * n[1]);
  x += ex;
  y += ey;
  z += ez;
  x = x < 0 ? x + n[0] : (x >= n[0] ? x - n[0] : x);
  y = y < 0 ? y + n[1] : (y >= n[1] ? y - n[1] : y);
  z = z < 0 ? z + n[2] : (z >= n[2] ? z - n[2] : z);
  return (z * n[1] + y) * n[0] + x;
}

struct Dims {
  int64_t n[3];
};

template <class L, typename T>
__global__ __launch_bounds__(256) void k_theta_rhs(const T *__restrict__ cur, T *__restrict__ rhs,
                                                   Dims d, int64_t N, KC<T> kc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    T acc = T(0);
    const T g0 = cur[i];
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      const T gp = cur[nbr_index(i, d.n, L::E[J][0], L::E[J][1], L::E[J][2])];
      const T gm = cur[nbr_index(i, d.n, -L::E[J][0], -L::E[J][1], -L::E[J][2])];
      acc = madd(kc.Cp[P], (gp - T(2) * g0) + gm, acc);
      acc = madd(kc.Cm[P], gp - gm, acc);
    });
    const T b = kc.A0t * g0;
    rhs[i] = madd(kc.th, acc, b);
  }
}

template <class L, typename T>
__global__ __launch_bounds__(256) void k_theta_sweep(const T *__restrict__ src,
                                                     const T *__restrict__ rhs,
                                                     T *__restrict__ dst, Dims d, int64_t N,
                                                     KC<T> kc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    T acc = T(0);
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      const T gp = src[nbr_index(i, d.n, L::E[J][0], L::E[J][1], L::E[J][2])];
      const T gm = src[nbr_index(i, d.n, -L::E[J][0], -L::E[J][1], -L::E[J][2])];
      acc = madd(kc.Cp[P], gp + gm, acc);
      acc = madd(kc.Cm[P], gp - gm, acc);
    });
    dst[i] = madd(kc.th1, acc, rhs[i]) * kc.inv_den;
  }
}

namespace {
inline int blocks_for(int64_t N) {
  int64_t b = (N + 255) / 256;
  return (int)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}
}  // namespace

template <typename T>
hipError_t launch_theta_rhs(const Consts &c, const Grid &g, const T *cur, T *rhs, hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  Dims d{{g.n[0], g.n[1], g.n[2]}};
  const dim3 gr(blocks_for(g.N)), bl(256);
  switch (c.lattice) {
    case 1: hipLaunchKernelGGL((k_theta_rhs<LatD1Q3, T>), gr, bl, 0, st, cur, rhs, d, g.N, kc); break;
    case 2: hipLaunchKernelGGL((k_theta_rhs<LatD2Q5, T>), gr, bl, 0, st, cur, rhs, d, g.N, kc); break;
    case 3: hipLaunchKernelGGL((k_theta_rhs<LatD2Q9, T>), gr, bl, 0, st, cur, rhs, d, g.N, kc); break;
    case 4: hipLaunchKernelGGL((k_theta_rhs<LatD3Q19, T>), gr, bl, 0, st, cur, rhs, d, g.N, kc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_theta_sweep(const Consts &c, const Grid &g, const T *src, const T *rhs, T *dst,
                              hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  Dims d{{g.n[0], g.n[1], g.n[2]}};
  const dim3 gr(blocks_for(g.N)), bl(256);
  switch (c.lattice) {
    case 1: hipLaunchKernelGGL((k_theta_sweep<LatD1Q3, T>), gr, bl, 0, st, src, rhs, dst, d, g.N, kc); break;
    case 2: hipLaunchKernelGGL((k_theta_sweep<LatD2Q5, T>), gr, bl, 0, st, src, rhs, dst, d, g.N, kc); break;
    case 3: hipLaunchKernelGGL((k_theta_sweep<LatD2Q9, T>), gr, bl, 0, st, src, rhs, dst, d, g.N, kc); break;
    case 4: hipLaunchKernelGGL((k_theta_sweep<LatD3Q19, T>), gr, bl, 0, st, src, rhs, dst, d, g.N, kc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ reductions
constexpr int kRedQ = 8;  // quantities per pass: 4 field sums, squared diff, spare

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_reduce_partial(const T *__restrict__ cur,
                                                        const T *__restrict__ prev, int nf,
                                                        int64_t N, double *__restrict__ partial) {
  double acc[kRedQ];
#pragma unroll
  for (int q = 0; q < kRedQ; ++q) acc[q] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int f = 0; f < nf; ++f) acc[f] += (double)cur[f * N + i];
    if (prev) {
      const double d = (double)cur[i] - (double)prev[i];
      acc[4] += d * d;
    }
  }
  __shared__ double red[kRedQ][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kRedQ; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kRedQ) {
    const int q = threadIdx.x;
    partial[blockIdx.x * kRedQ + q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
  }
}

__global__ __launch_bounds__(256) void k_reduce_final(const double *__restrict__ partial, int nblk,
                                                      double *__restrict__ out) {
  __shared__ double red[kRedQ][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < kRedQ; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) v += partial[b * kRedQ + q];
    v = wave_sum(v);
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kRedQ) {
    const int q = threadIdx.x;
    out[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
  }
}

template <typename T>
hipError_t launch_reduce(const T *cur, const T *prev, int nf, int64_t N, double *partial,
                         double *out, hipStream_t st) {
  int nblk = (int)((N + 255) / 256);
  if (nblk > kReduceBlocks) nblk = kReduceBlocks;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL((k_reduce_partial<T>), dim3(nblk), dim3(256), 0, st, cur, prev, nf, N,
                     partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partial, nblk, out);
  return hipGetLastError();
}

#define MFD_INST(T)                                                                               \
  template hipError_t launch_theta_rhs<T>(const Consts &, const Grid &, const T *, T *,           \
                                          hipStream_t);                                           \
  template hipError_t launch_theta_sweep<T>(const Consts &, const Grid &, const T *, const T *,   \
                                            T *, hipStream_t);                                    \
  template hipError_t launch_reduce<T>(const T *, const T *, int, int64_t, double *, double *,    \
                                       hipStream_t);
MFD_INST(float)
MFD_INST(double)
#undef MFD_INST

}  // namespace mfd
