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

// Launch shape of the theta kernels: x in blocks of 256 threads, one grid row
// per (y, z) line (grid-stride in y and z beyond the grid limits), so that a
// thread finds its node and its neighbours without any division.
struct Dims {
  int n[3];
};

__device__ __forceinline__ int wrap_step(int i, int n) {
  i += i < 0 ? n : 0;
  return i - (i >= n ? n : 0);
}

template <class L, bool RHS, typename T, class F>
__device__ __forceinline__ void theta_lines(const Dims &d, F &&node) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= d.n[0]) return;
  for (int z = blockIdx.z; z < d.n[2]; z += gridDim.z)
    for (int y = blockIdx.y; y < d.n[1]; y += gridDim.y) {
      const int64_t row = ((int64_t)z * d.n[1] + y) * d.n[0];
      auto at = [&](int ex, int ey, int ez) {
        const int xx = wrap_step(x + ex, d.n[0]);
        const int yy = wrap_step(y + ey, d.n[1]);
        const int zz = wrap_step(z + ez, d.n[2]);
        return ((int64_t)zz * d.n[1] + yy) * d.n[0] + xx;
      };
      node(row + x, at);
    }
}

template <class L, typename T>
__global__ __launch_bounds__(256) void k_theta_rhs(const T *__restrict__ cur, T *__restrict__ rhs,
                                                   Dims d, KC<T> kc) {
  theta_lines<L, true, T>(d, [&](int64_t i, auto &at) {
    T acc = T(0);
    const T g0 = cur[i];
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      const T gp = cur[at(L::E[J][0], L::E[J][1], L::E[J][2])];
      const T gm = cur[at(-L::E[J][0], -L::E[J][1], -L::E[J][2])];
      acc = madd(kc.Cp[P], (gp - T(2) * g0) + gm, acc);
      acc = madd(kc.Cm[P], gp - gm, acc);
    });
    const T b = kc.A0t * g0;
    rhs[i] = madd(kc.th, acc, b);
  });
}

template <class L, typename T>
__global__ __launch_bounds__(256) void k_theta_sweep(const T *__restrict__ src,
                                                     const T *__restrict__ rhs,
                                                     T *__restrict__ dst, Dims d, KC<T> kc) {
  theta_lines<L, false, T>(d, [&](int64_t i, auto &at) {
    T acc = T(0);
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      const T gp = src[at(L::E[J][0], L::E[J][1], L::E[J][2])];
      const T gm = src[at(-L::E[J][0], -L::E[J][1], -L::E[J][2])];
      acc = madd(kc.Cp[P], gp + gm, acc);
      acc = madd(kc.Cm[P], gp - gm, acc);
    });
    dst[i] = madd(kc.th1, acc, rhs[i]) * kc.inv_den;
  });
}

// Fused theta step for 2D lattices: one launch per time step.  A workgroup
// loads a W x H window of phi^n into LDS, forms the right-hand side on the
// window less one node on each side, then runs the K Jacobi sweeps in LDS,
// each on a region one node smaller (the stencil reaches one node), and
// stores the (W - 2(K+1)) x (H - 2(K+1)) interior of the last sweep.  Each
// node's arithmetic is that of k_theta_rhs / k_theta_sweep, so the result is
// the same value for value.  The host guarantees nx >= W and ny >= H.
template <class L, int W, int RG, typename T>
__global__ __launch_bounds__(W *RG) void k_theta_fused(const T *__restrict__ cur,
                                                      T *__restrict__ out, int nx, int ny, int H,
                                                      int K, int tiles_x, int ntiles, KC<T> kc) {
  constexpr int NT = W * RG;
  constexpr int KB = 8;
  extern __shared__ unsigned char smem_theta[];
  T *lds = reinterpret_cast<T *>(smem_theta);  // [3][H][W]: phi / sweep, rhs, sweep
  const int WH = W * H;
  const int halo = K + 1;
  const int TX = W - 2 * halo, TY = H - 2 * halo;
  const int tile = blockIdx.x;
  const int x0 = (tile % tiles_x) * TX - halo, y0 = (tile / tiles_x) * TY - halo;

  for (int base = 0; base < WH; base += KB * NT) {
    T v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < WH) {
        int gx = x0 + (i % W), gy = y0 + i / W;
        gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
        gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        v[k] = cur[(int64_t)gy * nx + gx];
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < WH) lds[i] = v[k];
    }
  }
  __syncthreads();

  const int xx = threadIdx.x % W, rg = threadIdx.x / W;
  // Walk this thread's column segment of the region t nodes in with a 3 x 3
  // register window of `src` (three LDS reads per node instead of nine);
  // f(y, w) gets the window centred on row y.
  auto slide = [&](const T *src, int t, auto &&f) {
    if (xx < t || xx >= W - t) return;
    const int Hr = H - 2 * t;
    const int seg = (Hr + RG - 1) / RG;
    const int ya = t + rg * seg, yb = min(ya + seg, H - t);
    if (ya >= yb) return;
    T w[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      w[0][c] = src[(ya - 1) * W + xx - 1 + c];
      w[1][c] = src[ya * W + xx - 1 + c];
    }
#pragma unroll 2
    for (int y = ya; y < yb; ++y) {
#pragma unroll
      for (int c = 0; c < 3; ++c) w[2][c] = src[(y + 1) * W + xx - 1 + c];
      f(y, w);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[0][c] = w[1][c];
        w[1][c] = w[2][c];
      }
    }
  };
  T *R = lds + WH;
  slide(lds, 1, [&](int y, const T (&w)[3][3]) {
    T acc = T(0);
    const T g0 = w[1][1];
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      constexpr int ex = L::E[J][0], ey = L::E[J][1];
      const T gp = w[1 + ey][1 + ex];
      const T gm = w[1 - ey][1 - ex];
      acc = madd(kc.Cp[P], (gp - T(2) * g0) + gm, acc);
      acc = madd(kc.Cm[P], gp - gm, acc);
    });
    const T b = kc.A0t * g0;
    R[y * W + xx] = madd(kc.th, acc, b);
  });
  __syncthreads();
  int src = 0;
#pragma unroll 1
  for (int k = 1; k <= K; ++k) {
    T *D = lds + (src == 0 ? 2 : 0) * WH;
    slide(lds + src * WH, 1 + k, [&](int y, const T (&w)[3][3]) {
      T acc = T(0);
      static_for<L::P>([&](auto PI) {
        constexpr int P = decltype(PI)::value;
        constexpr int J = L::PR[P];
        constexpr int ex = L::E[J][0], ey = L::E[J][1];
        const T gp = w[1 + ey][1 + ex];
        const T gm = w[1 - ey][1 - ex];
        acc = madd(kc.Cp[P], gp + gm, acc);
        acc = madd(kc.Cm[P], gp - gm, acc);
      });
      D[y * W + xx] = madd(kc.th1, acc, R[y * W + xx]) * kc.inv_den;
    });
    __syncthreads();
    src = src == 0 ? 2 : 0;
  }

  const T *C = lds + src * WH;
  for (int i = threadIdx.x; i < TX * TY; i += NT) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + halo + lx, gy = y0 + halo + ly;
    if (gx >= nx || gy >= ny) continue;
    out[(int64_t)gy * nx + gx] = C[(halo + ly) * W + halo + lx];
  }
}

namespace {
inline void theta_shape(const Grid &g, Dims *d, dim3 *gr) {
  *d = Dims{{(int)g.n[0], (int)g.n[1], (int)g.n[2]}};
  const int64_t gy = g.n[1] < 65535 ? g.n[1] : 65535;
  const int64_t gz = g.n[2] < 65535 ? g.n[2] : 65535;
  *gr = dim3((unsigned)((g.n[0] + 255) / 256), (unsigned)gy, (unsigned)gz);
}
}  // namespace

template <typename T>
hipError_t launch_theta_rhs(const Consts &c, const Grid &g, const T *cur, T *rhs, hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  Dims d;
  dim3 gr;
  theta_shape(g, &d, &gr);
  const dim3 bl(256);
  switch (c.lattice) {
    case 1: hipLaunchKernelGGL((k_theta_rhs<LatD1Q3, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
    case 2: hipLaunchKernelGGL((k_theta_rhs<LatD2Q5, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
    case 3: hipLaunchKernelGGL((k_theta_rhs<LatD2Q9, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
    case 4: hipLaunchKernelGGL((k_theta_rhs<LatD3Q19, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_theta_sweep(const Consts &c, const Grid &g, const T *src, const T *rhs, T *dst,
                              hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  Dims d;
  dim3 gr;
  theta_shape(g, &d, &gr);
  const dim3 bl(256);
  switch (c.lattice) {
    case 1: hipLaunchKernelGGL((k_theta_sweep<LatD1Q3, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
    case 2: hipLaunchKernelGGL((k_theta_sweep<LatD2Q5, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
    case 3: hipLaunchKernelGGL((k_theta_sweep<LatD2Q9, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
    case 4: hipLaunchKernelGGL((k_theta_sweep<LatD3Q19, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
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

template <typename T, int NF>
__global__ __launch_bounds__(256) void k_reduce_partial(const T *__restrict__ cur,
                                                        const T *__restrict__ prev, int64_t N,
                                                        double *__restrict__ partial) {
  constexpr int U = 4;  // grid-stride elements in flight per thread
  double acc[kRedQ];
#pragma unroll
  for (int q = 0; q < kRedQ; ++q) acc[q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < N; i += U * stride) {
    T c[U][NF], p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int f = 0; f < NF; ++f) c[u][f] = cur[f * N + i + u * stride];
      p[u] = prev ? prev[i + u * stride] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f] += (double)c[u][f];
      if (prev) {
        const double d = (double)c[u][0] - (double)p[u];
        acc[4] += d * d;
      }
    }
  }
  for (; i < N; i += stride) {
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] += (double)cur[f * N + i];
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
  switch (nf) {
    case 1:
      hipLaunchKernelGGL((k_reduce_partial<T, 1>), dim3(nblk), dim3(256), 0, st, cur, prev, N,
                         partial);
      break;
    case 2:
      hipLaunchKernelGGL((k_reduce_partial<T, 2>), dim3(nblk), dim3(256), 0, st, cur, prev, N,
                         partial);
      break;
    case 3:
      hipLaunchKernelGGL((k_reduce_partial<T, 3>), dim3(nblk), dim3(256), 0, st, cur, prev, N,
                         partial);
      break;
    case 4:
      hipLaunchKernelGGL((k_reduce_partial<T, 4>), dim3(nblk), dim3(256), 0, st, cur, prev, N,
                         partial);
      break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partial, nblk, out);
  return hipGetLastError();
}

constexpr int kThetaW = 64, kThetaRG = 8;

// window rows of the fused theta step for K sweeps, or 0 when it cannot run
int theta_fused_rows(const Consts &c, const Grid &g, int K, int elem) {
  if (c.dim != 2 || (c.lattice != 2 && c.lattice != 3) || K < 1) return 0;
  const int halo = K + 1;
  if (kThetaW - 2 * halo < 8 || g.n[0] < kThetaW) return 0;
  for (int h : {64, 48, 32}) {
    if (h - 2 * halo < 8 || g.n[1] < h) continue;
    if ((size_t)3 * h * kThetaW * elem > 64 * 1024) continue;
    return h;
  }
  return 0;
}

template <typename T>
hipError_t launch_theta_fused(const Consts &c, const Grid &g, int K, const T *cur, T *out,
                              hipStream_t st) {
  const int H = theta_fused_rows(c, g, K, (int)sizeof(T));
  if (!H) return hipErrorInvalidValue;
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int halo = K + 1, TX = kThetaW - 2 * halo, TY = H - 2 * halo;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)3 * H * kThetaW * sizeof(T);
  auto fn = c.lattice == 3 ? k_theta_fused<LatD2Q9, kThetaW, kThetaRG, T>
                           : k_theta_fused<LatD2Q5, kThetaW, kThetaRG, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(kThetaW * kThetaRG), lds, st, cur, out, nx, ny, H, K,
                     tx, tx * ty, kc);
  return hipGetLastError();
}

#define MFD_INST(T)                                                                               \
  template hipError_t launch_theta_fused<T>(const Consts &, const Grid &, int, const T *, T *,    \
                                            hipStream_t);                                         \
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
