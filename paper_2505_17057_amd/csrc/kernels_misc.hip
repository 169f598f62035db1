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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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
//
// Solved to a tolerance (SOLVE): the launch is one chunk of K sweeps of a
// step's Jacobi solve.  The level phi^n, the iterate a chunk starts from and
// the buffer it writes are chosen on the device by a control block, so the
// host enqueues the same chunk sequence for every step (the first chunk of a
// step starts from phi^n; later chunks continue from the last iterate and
// return at once when the solve has stopped).  Each tile adds its interior's
// sum (x_K - x_{K-1})^2 and sum rhs^2 (binary64) to its slot of `part`; the
// last workgroup to finish (atomic count, no waiting) sums the slots in tile
// order and stops the solve when den^2 sum d^2 <= tol^2 sum rhs^2 (the
// residual of x_{K-1} is den (x_K - x_{K-1})) or the sweep cap is reached,
// rotating the level roles: prev <- phi^n, phi^n <- the last iterate.
template <typename T>
struct ThetaRing {
  T *b[4];  // the four level buffers the control block's roles index
};

struct ThetaSolveArgs {
  ThetaCtl *ctl;
  double *part;  // 2 per tile
  double tol2, den2;
  int cap, first;
};

template <class L, int W, int RG, typename T, bool SOLVE>
__global__ __launch_bounds__(W *RG) void k_theta_fused(const T *__restrict__ cur_in,
                                                      T *__restrict__ out_in, ThetaRing<T> ring,
                                                      ThetaSolveArgs sa, int nx, int ny, int H,
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
  __shared__ int s_sel[4];  // skip, level, iterate source, destination

  const T *cur = cur_in, *itsrc = cur_in;
  T *out = out_in;
  if constexpr (SOLVE) {
    if (threadIdx.x == 0) {
      const ThetaCtl *c = sa.ctl;
      s_sel[0] = (!sa.first && c->done) ? 1 : 0;
      s_sel[1] = c->role[0];
      s_sel[2] = sa.first ? c->role[0] : c->nsrc;
      s_sel[3] = sa.first ? c->role[2] : c->ndst;
    }
    __syncthreads();
    if (s_sel[0]) return;
    cur = ring.b[s_sel[1]];
    itsrc = ring.b[s_sel[2]];
    out = ring.b[s_sel[3]];
  }

  auto load_window = [&](const T *__restrict__ g) {
    for (int base = 0; base < WH; base += KB * NT) {
      T v[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int i = base + threadIdx.x + k * NT;
        if (i < WH) {
          int gx = x0 + (i % W), gy = y0 + i / W;
          gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
          gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
          v[k] = g[(int64_t)gy * nx + gx];
        }
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int i = base + threadIdx.x + k * NT;
        if (i < WH) lds[i] = v[k];
      }
    }
  };
  load_window(cur);
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
  if constexpr (SOLVE) {
    if (sa.first == 0) {  // continue from the last iterate
      load_window(itsrc);
      __syncthreads();
    }
  }
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
  const T *Pv = lds + (src == 0 ? 2 : 0) * WH;  // the sweep before the last
  double d2 = 0.0, b2 = 0.0;
  for (int i = threadIdx.x; i < TX * TY; i += NT) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + halo + lx, gy = y0 + halo + ly;
    if (gx >= nx || gy >= ny) continue;
    const int li = (halo + ly) * W + halo + lx;
    out[(int64_t)gy * nx + gx] = C[li];
    if constexpr (SOLVE) {
      const double d = (double)C[li] - (double)Pv[li];
      const double r = (double)R[li];
      d2 += d * d;
      b2 += r * r;
    }
  }
  if constexpr (SOLVE) {
    // tile sums (fixed order: lanes, then wavefronts), then the last
    // workgroup's pass over the tiles
    __shared__ double red[2][NT / 64];
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    d2 = wave_sum(d2);
    b2 = wave_sum(b2);
    if (lane == 0) {
      red[0][wave] = d2;
      red[1][wave] = b2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NT / 64; ++w) {
        a += red[0][w];
        b += red[1][w];
      }
      sa.part[2 * tile] = a;
      sa.part[2 * tile + 1] = b;
      __threadfence();
      s_last = atomicAdd(&sa.ctl->count, 1u) == (unsigned)(ntiles - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += NT) {
      a += __builtin_nontemporal_load(&sa.part[2 * t]);
      b += __builtin_nontemporal_load(&sa.part[2 * t + 1]);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane == 0) {
      red[0][wave] = a;
      red[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double D2 = 0.0, B2 = 0.0;
      for (int w = 0; w < NT / 64; ++w) {
        D2 += red[0][w];
        B2 += red[1][w];
      }
      ThetaCtl *c = sa.ctl;
      const int sweeps = (sa.first ? 0 : c->sweeps) + K;
      const bool conv = sa.den2 * D2 <= sa.tol2 * B2;
      const int dst = s_sel[3];
      const int other = dst == c->role[2] ? c->role[3] : c->role[2];
      if (conv || sweeps >= sa.cap) {
        const int oc = c->role[0], op = c->role[1];
        c->role[0] = dst;
        c->role[1] = oc;
        c->role[2] = op;
        c->role[3] = other;
        c->done = 1;
        c->total_sweeps += sweeps;
        c->steps += 1;
        if (sweeps > c->max_sweeps) c->max_sweeps = sweeps;
        if (!conv) c->unconverged += 1;
      } else {
        c->done = 0;
        c->nsrc = dst;
        c->ndst = other;
      }
      c->sweeps = sweeps;
      c->count = 0u;
      __threadfence();
    }
  }
}

// start of an mfd_step call of the to-tolerance solve: identity roles
__global__ void k_theta_ctl_init(ThetaCtl *c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int i = 0; i < 4; ++i) c->role[i] = i;
    c->done = 1;
    c->nsrc = 0;
    c->ndst = 2;
    c->sweeps = 0;
    c->count = 0u;
  }
}

// end of the call: phi^n and phi^(n-1) back into buffers 0 and 1 (each node
// reads both sources before writing, so any permutation of roles is safe)
template <typename T>
__global__ __launch_bounds__(256) void k_theta_gather(ThetaRing<T> ring, const ThetaCtl *c,
                                                      int64_t N) {
  const int r0 = c->role[0], r1 = c->role[1];
  if (r0 == 0 && r1 == 1) return;
  const T *s0 = ring.b[r0], *s1 = ring.b[r1];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T v0 = s0[i], v1 = s1[i];
    ring.b[0][i] = v0;
    ring.b[1][i] = v1;
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
    case 5: hipLaunchKernelGGL((k_theta_rhs<LatD2Q5II, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
    case 6: hipLaunchKernelGGL((k_theta_rhs<LatD3Q7, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
    case 7: hipLaunchKernelGGL((k_theta_rhs<LatD3Q9, T>), gr, bl, 0, st, cur, rhs, d, kc); break;
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
    case 5: hipLaunchKernelGGL((k_theta_sweep<LatD2Q5II, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
    case 6: hipLaunchKernelGGL((k_theta_sweep<LatD3Q7, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
    case 7: hipLaunchKernelGGL((k_theta_sweep<LatD3Q9, T>), gr, bl, 0, st, src, rhs, dst, d, kc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ reductions
constexpr int kRedQ = 8;  // quantities per pass: 4 field sums, squared diff, spare


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

// out[q] = sum over the nblk rows of partial[b kRedQ + q], q < nq (<= kRedQ):
// thread t adds rows t, t + 256, ... in order (all quantities of a row in one
// pass, so the loads of the quantities overlap), then per quantity a wave sum
// and the four waves in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_final(const double *__restrict__ partial, int nblk,
                                                      int nq, double *__restrict__ out) {
  __shared__ double red[kRedQ][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[kRedQ];
#pragma unroll
  for (int q = 0; q < kRedQ; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int q = 0; q < kRedQ; ++q)
      if (q < nq) v[q] += partial[b * kRedQ + q];
  }
#pragma unroll
  for (int q = 0; q < kRedQ; ++q) {
    if (q < nq) {
      const double w = wave_sum(v[q]);
      if (lane == 0) red[q][wave] = w;
    }
  }
  __syncthreads();
  if (threadIdx.x < nq) {
    const int q = threadIdx.x;
    out[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
  }
}

hipError_t launch_final_sums(const double *partial, int rows, int nq, double *out, hipStream_t st) {
  if (rows < 1 || rows > kReduceBlocks || nq < 1 || nq > kRedQ) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partial, rows, nq, out);
  return hipGetLastError();
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
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partial, nblk, kRedQ, out);
  return hipGetLastError();
}

constexpr int kThetaW = 64, kThetaRG = 8;

// window rows of the fused theta step for K sweeps, or 0 when it cannot run
int theta_fused_rows(const Consts &c, const Grid &g, int K, int elem) {
  if (c.dim != 2 || (c.lattice != 2 && c.lattice != 3) || K < 1) return 0;
  const int halo = K + 1;
  if (kThetaW - 2 * halo < 8 || g.n[0] < kThetaW) return 0;
  for (int h : {96, 64, 48, 32}) {
    if (h - 2 * halo < 8 || g.n[1] < h) continue;
    // three W x h arrays; at most half of the 160 KiB of a CU (two workgroups)
    if ((size_t)3 * h * kThetaW * elem > 80 * 1024) continue;
    // at least a fifth of the window stored (else the recomputed halo costs
    // more than the separate sweeps save)
    if (5 * (kThetaW - 2 * halo) * (h - 2 * halo) < kThetaW * h) continue;
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
  auto fn = c.lattice == 3 ? k_theta_fused<LatD2Q9, kThetaW, kThetaRG, T, false>
                           : k_theta_fused<LatD2Q5, kThetaW, kThetaRG, T, false>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  ThetaRing<T> ring{{nullptr, nullptr, nullptr, nullptr}};
  ThetaSolveArgs sa{nullptr, nullptr, 0.0, 0.0, 0, 1};
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(kThetaW * kThetaRG), lds, st, cur, out, ring, sa, nx,
                     ny, H, K, tx, tx * ty, kc);
  return hipGetLastError();
}

int theta_solve_tiles(const Consts &c, const Grid &g, int K, int elem) {
  const int H = theta_fused_rows(c, g, K, elem);
  if (!H) return 0;
  const int halo = K + 1, TX = kThetaW - 2 * halo, TY = H - 2 * halo;
  return (int)(((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY));
}

template <typename T>
hipError_t launch_theta_ctl_init(ThetaCtl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_theta_ctl_init, dim3(1), dim3(64), 0, st, ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_theta_chunk(const Consts &c, const Grid &g, int K, T *const bufs[4],
                              ThetaCtl *ctl, double *part, double tol, int cap, bool first,
                              hipStream_t st) {
  const int H = theta_fused_rows(c, g, K, (int)sizeof(T));
  if (!H) return hipErrorInvalidValue;
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int halo = K + 1, TX = kThetaW - 2 * halo, TY = H - 2 * halo;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)3 * H * kThetaW * sizeof(T);
  auto fn = c.lattice == 3 ? k_theta_fused<LatD2Q9, kThetaW, kThetaRG, T, true>
                           : k_theta_fused<LatD2Q5, kThetaW, kThetaRG, T, true>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  ThetaRing<T> ring{{bufs[0], bufs[1], bufs[2], bufs[3]}};
  const double den = theta_den(c);
  ThetaSolveArgs sa{ctl, part, tol * tol, den * den, cap, first ? 1 : 0};
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(kThetaW * kThetaRG), lds, st, nullptr, nullptr, ring,
                     sa, nx, ny, H, K, tx, tx * ty, kc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_theta_gather(T *const bufs[4], const ThetaCtl *ctl, int64_t N, hipStream_t st) {
  ThetaRing<T> ring{{bufs[0], bufs[1], bufs[2], bufs[3]}};
  int nblk = (int)std::min<int64_t>((N + 255) / 256, 4096);
  hipLaunchKernelGGL((k_theta_gather<T>), dim3(nblk), dim3(256), 0, st, ring, ctl, N);
  return hipGetLastError();
}

// sums sum (a - b)^2 and sum c^2 in binary64 over N nodes (deterministic):
// out[0], out[1]
template <typename T>
__global__ __launch_bounds__(256) void k_sq_partial(const T *__restrict__ a,
                                                    const T *__restrict__ b,
                                                    const T *__restrict__ cc, int64_t N,
                                                    double *__restrict__ partial) {
  const int64_t o = blockIdx.y * N;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)a[o + i] - (double)b[o + i];
    const double r = (double)cc[o + i];
    s0 += d * d;
    s1 += r * r;
  }
  __shared__ double red[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    partial[blockIdx.x * kRedQ + 2 * blockIdx.y + q] =
        ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
  }
}

template <typename T>
hipError_t launch_sq_sums(const T *a, const T *b, const T *c, int F, int64_t N, double *partial,
                          double *out, hipStream_t st) {
  if (F < 1 || 2 * F > kRedQ) return hipErrorInvalidValue;
  int nblk = (int)((N + 255) / 256);
  if (nblk > kReduceBlocks) nblk = kReduceBlocks;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL((k_sq_partial<T>), dim3(nblk, F), dim3(256), 0, st, a, b, c, N, partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partial, nblk, 2 * F, out);
  return hipGetLastError();
}

// Picard-Jacobi theta step of Burgers' equation (Eq. (GCN)): the elementwise
// parts around the explicit step kernel S,
//   R       = theta S(phi^n) + (1 - theta) (A0 phi^n),
//   x_{k+1} = (R + (1 - theta) ((S(x_k) - A0 x_k) + dd x_k)) / den,
// one rounding per operation in the order written.
// Fields are stored one after another (field f at f N); blockIdx.y is the
// field, whose constants come in PicardF.
template <typename T>
struct PicardF {
  T A0[4], dd[4], inv_den[4];
};

template <typename T>
__global__ __launch_bounds__(256) void k_picard_rhs(const T *__restrict__ S0,
                                                    const T *__restrict__ phi, T *__restrict__ R,
                                                    T th, T th1, PicardF<T> pf, int64_t N) {
  const int64_t o = blockIdx.y * N;
  const T A0 = pf.A0[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T a = th * S0[o + i];
    const T b = A0 * phi[o + i];
    R[o + i] = a + th1 * b;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_picard_update(const T *__restrict__ Sx,
                                                       const T *__restrict__ x,
                                                       const T *__restrict__ R,
                                                       T *__restrict__ out, T th1, PicardF<T> pf,
                                                       int64_t N) {
  const int64_t o = blockIdx.y * N;
  const T A0 = pf.A0[blockIdx.y], dd = pf.dd[blockIdx.y], inv_den = pf.inv_den[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T xi = x[o + i];
    const T t = (Sx[o + i] - A0 * xi) + dd * xi;
    const T c = th1 * t;
    out[o + i] = (R[o + i] + c) * inv_den;
  }
}

template <typename T>
PicardF<T> picard_f(int F, const double *A0, const double *dd, const double *inv_den) {
  PicardF<T> pf{};
  for (int f = 0; f < F; ++f) {
    pf.A0[f] = (T)A0[f];
    pf.dd[f] = dd ? (T)dd[f] : (T)0;
    pf.inv_den[f] = inv_den ? (T)inv_den[f] : (T)0;
  }
  return pf;
}

template <typename T>
hipError_t launch_picard_rhs(const T *S0, const T *phi, T *R, double th, double th1, int F,
                             const double *A0, int64_t N, hipStream_t st) {
  if (F < 1 || F > 4) return hipErrorInvalidValue;
  const int nblk = (int)std::min<int64_t>((N + 255) / 256, 8192 / F);
  hipLaunchKernelGGL((k_picard_rhs<T>), dim3(nblk, F), dim3(256), 0, st, S0, phi, R, (T)th, (T)th1,
                     picard_f<T>(F, A0, nullptr, nullptr), N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_picard_update(const T *Sx, const T *x, const T *R, T *out, int F,
                                const double *A0, const double *dd, double th1,
                                const double *inv_den, int64_t N, hipStream_t st) {
  if (F < 1 || F > 4) return hipErrorInvalidValue;
  const int nblk = (int)std::min<int64_t>((N + 255) / 256, 8192 / F);
  hipLaunchKernelGGL((k_picard_update<T>), dim3(nblk, F), dim3(256), 0, st, Sx, x, R, out, (T)th1,
                     picard_f<T>(F, A0, dd, inv_den), N);
  return hipGetLastError();
}

// Special first step of the three-level wave scheme (Example 3 of the paper):
// phi(t + dt) = phi + dt phi_t + cw sum_axes [(phi(x+e_a) - 2 phi) + phi(x-e_a)]
// at every node (periodic wrap), in binary64 and rounded once; on a
// Dirichlet grid the boundary nodes take G_b E[1].
template <typename T>
__global__ __launch_bounds__(256) void k_wave_start(const T *__restrict__ phi0,
                                                    const double *__restrict__ phit,
                                                    T *__restrict__ out, Dims d, int dim,
                                                    double dt, double cw, DirBC bc) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= d.n[0]) return;
  for (int z = blockIdx.z; z < d.n[2]; z += gridDim.z)
    for (int y = blockIdx.y; y < d.n[1]; y += gridDim.y) {
      const int64_t i = ((int64_t)z * d.n[1] + y) * d.n[0] + x;
      double v;
      if (bc.on && dir_node(x, y, d.n[0], d.n[1])) {
        v = bc.Gb[dir_index(x, y, d.n[0], d.n[1])] * bc.E[1];
      } else {
        const double c = (double)phi0[i];
        double lap = 0.0;
        for (int a = 0; a < dim; ++a) {
          const int ex = a == 0, ey = a == 1, ez = a == 2;
          const int64_t ip = ((int64_t)wrap_step(z + ez, d.n[2]) * d.n[1] + wrap_step(y + ey, d.n[1])) *
                                 d.n[0] + wrap_step(x + ex, d.n[0]);
          const int64_t im = ((int64_t)wrap_step(z - ez, d.n[2]) * d.n[1] + wrap_step(y - ey, d.n[1])) *
                                 d.n[0] + wrap_step(x - ex, d.n[0]);
          lap = lap + (((double)phi0[ip] - 2.0 * c) + (double)phi0[im]);
        }
        v = (c + dt * phit[i]) + cw * lap;
      }
      out[i] = (T)v;
    }
}

template <typename T>
hipError_t launch_wave_start(const Consts &c, const Grid &g, const T *phi0, const double *phit,
                             T *out, double dt, double cw, const DirBC &bc, hipStream_t st) {
  if (bc.on && c.dim != 2) return hipErrorInvalidValue;
  Dims d;
  dim3 gr;
  theta_shape(g, &d, &gr);
  hipLaunchKernelGGL((k_wave_start<T>), gr, dim3(256), 0, st, phi0, phit, out, d, c.dim, dt, cw,
                     bc);
  return hipGetLastError();
}

#define MFD_INST(T)                                                                               \
  template hipError_t launch_picard_rhs<T>(const T *, const T *, T *, double, double, int,        \
                                           const double *, int64_t, hipStream_t);                 \
  template hipError_t launch_picard_update<T>(const T *, const T *, const T *, T *, int,          \
                                              const double *, const double *, double,             \
                                              const double *, int64_t, hipStream_t);              \
  template hipError_t launch_wave_start<T>(const Consts &, const Grid &, const T *,               \
                                           const double *, T *, double, double, const DirBC &,    \
                                           hipStream_t);                                          \
  template hipError_t launch_theta_fused<T>(const Consts &, const Grid &, int, const T *, T *,    \
                                            hipStream_t);                                         \
  template hipError_t launch_theta_rhs<T>(const Consts &, const Grid &, const T *, T *,           \
                                          hipStream_t);                                           \
  template hipError_t launch_theta_sweep<T>(const Consts &, const Grid &, const T *, const T *,   \
                                            T *, hipStream_t);                                    \
  template hipError_t launch_reduce<T>(const T *, const T *, int, int64_t, double *, double *,    \
                                       hipStream_t);                                              \
  template hipError_t launch_theta_ctl_init<T>(ThetaCtl *, hipStream_t);                          \
  template hipError_t launch_theta_chunk<T>(const Consts &, const Grid &, int, T *const[4],       \
                                            ThetaCtl *, double *, double, int, bool,              \
                                            hipStream_t);                                         \
  template hipError_t launch_theta_gather<T>(T *const[4], const ThetaCtl *, int64_t,              \
                                             hipStream_t);                                        \
  template hipError_t launch_sq_sums<T>(const T *, const T *, const T *, int, int64_t, double *,  \
                                        double *, hipStream_t);
MFD_INST(float)
MFD_INST(double)
#undef MFD_INST

}  // namespace mfd
