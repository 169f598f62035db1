// MMFD step of the linear CDE with a source term: the b terms of Eq. (2-1) /
// (3layerMMFD-1) with F_j of Eq. (SourceF) for the NCDE, M_1F = v S, in the
// central-difference (MMFD) form of Eq. (2-2-1).  The step's value is that of
// the plain step (mmfd_node), rounded to the working precision, plus
//
//   dt [ (B0 S(x, t) + Bh0 S(x, t - dt))
//        + sum over pairs p, level t then t - dt, of
//            b+ ((F+(x + e_p) - 2 F+(x)) + F+(x - e_p)) + b- (F-(x + e_p) - F-(x - e_p)) ]
//
// with B0 = sum_k b_k, b+- = b_1 +- b_-1 (and the same for bh at t - dt), the
// pair parts F+_p = w_p S and F-_p = (w_p / d0)(e_p . vh) S, vh = v dt / dx,
// and S(x, t) = exp(lambda t) G(x).  Every operation is a plain rounded one,
// in the order written, so binary64 results equal the step followed by this
// sum value for value.
//
// The MesoFD form adds to each population f_j dt times its direction's b
// terms, sum_k b_k F_j(x + k e_j, t) + sum_k bh_k F_j(x + k e_j, t - dt); the
// moments of the new populations equal the MMFD value to round-off.
//
// 1D / 2D: one fused launch per step.  A workgroup stages phi at t (and at
// t - dt when that level has a stencil) and G for a TX x TY tile and a
// one-node halo into LDS, then each node forms its step value and its source
// term from LDS and stores once.  3D (MMFD only): the plain step launch, then
// a launch that adds the source term to the level it wrote.
#include <cmath>

#include "mesofd_node.h"
#include "mfd_internal.h"
#include "mmfd_node.h"
#include "tb_window.h"

namespace mfd {

namespace {

template <typename T>
struct SrcC {
  T wp[kMaxP], wm[kMaxP];
  T B0, Bh0, bp, bm, bhp, bhm;
  T dt, sig_t, sig_m;
  // MesoFD: F_j(y) = wj (S(y) + evj S(y)) per direction, b_k and bh_k
  T wj[kMaxQ], evj[kMaxQ];
  T b[3], bh[3];
};

// the source term at one node; g(dz, dy, dx) reads G at the node's
// neighbour; sig_t, sig_m the factors exp(lambda t) of the step's two levels
template <class L, typename T, class Gat>
__device__ __forceinline__ T source_at(const Gat &g, const SrcC<T> &sc, T sig_t, T sig_m) {
  const T g0 = g(0, 0, 0);
  const T sv = sc.B0 * (sig_t * g0) + sc.Bh0 * (sig_m * g0);
  T sa = T(0);
#pragma unroll
  for (int lev = 0; lev < 2; ++lev) {
    const T sig = lev == 0 ? sig_t : sig_m;
    const T cp = lev == 0 ? sc.bp : sc.bhp, cm = lev == 0 ? sc.bm : sc.bhm;
    const T s0 = sig * g0;
#pragma unroll
    for (int p = 0; p < L::P; ++p) {
      const int j = L::PR[p];
      const T sp = sig * g(L::E[j][2], L::E[j][1], L::E[j][0]);
      const T sm = sig * g(-L::E[j][2], -L::E[j][1], -L::E[j][0]);
      const T d2v = (sc.wp[p] * sp - T(2) * (sc.wp[p] * s0)) + sc.wp[p] * sm;
      const T d1v = sc.wm[p] * sp - sc.wm[p] * sm;
      sa = sa + cp * d2v;
      sa = sa + cm * d1v;
    }
  }
  return sc.dt * (sv + sa);
}
template <class L, typename T, class Gat>
__device__ __forceinline__ T source_at(const Gat &g, const SrcC<T> &sc) {
  return source_at<L, T>(g, sc, sc.sig_t, sc.sig_m);
}

// the source term as a hook of the blocked window (tb_window.h): G staged
// once per launch beside the levels (a static field), each step's factors
// from sig[]: step t of the launch reads level n0 + t - 1, so sig_t =
// sig[t] and sig_m = sig[t - 1] with sig[k] = exp(lambda (n0 + k - 1) dt)
template <class L, typename T>
struct SrcTbHook {
  static constexpr int kExtra = 1;
  const T *G;
  SrcC<T> sc;
  T sig[kMaxBcSteps + 1];
  __device__ __forceinline__ void load(T *extra, int W, int H, int x0, int y0, int nx, int ny,
                                       int tid, int nt) const {
    for (int i = tid; i < W * H; i += nt) {
      int gx = x0 + (i % W), gy = y0 + i / W;
      gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
      gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
      extra[i] = G[(int64_t)gy * nx + gx];
    }
  }
  __device__ __forceinline__ T apply(int t, const T *extra, int W, int y, int x, T v) const {
    auto g = [&](int, int dy, int dx) { return extra[(y + dy) * W + x + dx]; };
    return v + source_at<L, T>(g, sc, sig[t], sig[t - 1]);
  }
};

// 1D / 2D fused step + source over one TX x TY tile per workgroup
template <class L, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_lcde_source_plane(const T *__restrict__ cur,
                                                           const T *__restrict__ prev,
                                                           const T *__restrict__ G,
                                                           T *__restrict__ out, int nx, int ny,
                                                           int tiles_x, int ntiles, KC<T> kc,
                                                           SrcC<T> sc) {
  constexpr int HYL = L::D >= 2 ? 1 : 0;
  constexpr int HX = TX + 2, HY = TY + 2 * HYL;
  __shared__ T ph[HY][HX];
  __shared__ T hp[THREE_ST ? HY : 1][THREE_ST ? HX : 1];
  __shared__ T gs[HY][HX];
  const int tile = xcd_remap(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  for (int i = threadIdx.x; i < HX * HY; i += 256) {
    const int lx = i % HX, ly = i / HX;
    const int gx = wrapi(x0 - 1 + lx, nx), gy = wrapi(y0 - HYL + ly, ny);
    const int64_t gi = (int64_t)gy * nx + gx;
    ph[ly][lx] = cur[gi];
    if constexpr (THREE_ST) hp[ly][lx] = prev[gi];
    gs[ly][lx] = G[gi];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TX * TY; i += 256) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= nx || gy >= ny) continue;
    const int cx = lx + 1, cy = ly + HYL;
    const int64_t gi = (int64_t)gy * nx + gx;
    auto at = [&](int, int, int dy, int dx) { return ph[cy + dy][cx + dx]; };
    auto ath = [&](int, int, int dy, int dx) {
      if constexpr (THREE_ST) return hp[cy + dy][cx + dx];
      else return T(0);
    };
    T cc[1] = {ph[cy][cx]}, pc[1] = {THREE ? prev[gi] : T(0)}, oc[1];
    mmfd_node<L, kLCDE, THREE, THREE_ST, T>(at, ath, cc, pc, oc, kc);
    auto gat = [&](int, int dy, int dx) { return gs[cy + dy][cx + dx]; };
    out[gi] = oc[0] + source_at<L, T>(gat, sc);
  }
}

// MesoFD form (1D / 2D), one launch per step: the same staging; each node
// forms its b populations with the single-step node function (mesofd_pops),
// adds to each dt times its direction's source term
//   sum_k b_k F_j(x + k e_j, t) + sum_k bh_k F_j(x + k e_j, t - dt)
// (zero coefficients skipped, level t first), stores them (pop_out not null)
// and their sum, the new moment (Eq. (2-1-1)).
template <class L, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_lcde_mesofd_source_plane(
    const T *__restrict__ cur, const T *__restrict__ prev, const T *__restrict__ G,
    T *__restrict__ pop_out, T *__restrict__ mom_out, int nx, int ny, int tiles_x, int ntiles,
    KC<T> kc, SrcC<T> sc) {
  constexpr int HYL = L::D >= 2 ? 1 : 0;
  constexpr int HX = TX + 2, HY = TY + 2 * HYL;
  __shared__ T ph[HY][HX];
  __shared__ T hp[THREE_ST ? HY : 1][THREE_ST ? HX : 1];
  __shared__ T gs[HY][HX];
  const int tile = xcd_remap(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  const int64_t N = (int64_t)nx * ny;
  for (int i = threadIdx.x; i < HX * HY; i += 256) {
    const int lx = i % HX, ly = i / HX;
    const int gx = wrapi(x0 - 1 + lx, nx), gy = wrapi(y0 - HYL + ly, ny);
    const int64_t gi = (int64_t)gy * nx + gx;
    ph[ly][lx] = cur[gi];
    if constexpr (THREE_ST) hp[ly][lx] = prev[gi];
    gs[ly][lx] = G[gi];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TX * TY; i += 256) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= nx || gy >= ny) continue;
    const int cx = lx + 1, cy = ly + HYL;
    const int64_t gi = (int64_t)gy * nx + gx;
    auto at = [&](int, int, int dy, int dx) { return ph[cy + dy][cx + dx]; };
    auto ath = [&](int, int, int dy, int dx) {
      if constexpr (THREE_ST) return hp[cy + dy][cx + dx];
      else return T(0);
    };
    T hc[1] = {THREE && !THREE_ST ? prev[gi] : T(0)};
    T fo[L::Q], m[1];
    mesofd_pops<L, kLCDE, THREE_ST>(at, ath, hc, THREE, fo, kc);
#pragma unroll
    for (int j = 0; j < L::Q; ++j) {
      T sj = T(0);
#pragma unroll
      for (int lev = 0; lev < 2; ++lev) {
        const T sig = lev == 0 ? sc.sig_t : sc.sig_m;
#pragma unroll
        for (int k = -1; k <= 1; ++k) {
          const T bk = lev == 0 ? sc.b[k + 1] : sc.bh[k + 1];
          if (bk != T(0)) {
            const T sy = sig * gs[cy + k * L::E[j][1]][cx + k * L::E[j][0]];
            sj = sj + bk * (sc.wj[j] * (sy + sc.evj[j] * sy));
          }
        }
      }
      fo[j] = fo[j] + sc.dt * sj;
    }
    if (pop_out) {
#pragma unroll
      for (int j = 0; j < L::Q; ++j) pop_out[j * N + gi] = fo[j];
    }
    moments_of<L, kLCDE>(fo, m);
    mom_out[gi] = m[0];
  }
}

// 3D: adds the source term to the level the step kernel wrote; blocks of
// 256 nodes along x, grid (x blocks, y, z)
template <class L, typename T>
__global__ __launch_bounds__(256) void k_add_source_3d(T *__restrict__ out,
                                                       const T *__restrict__ G, int nx, int ny,
                                                       int nz, SrcC<T> sc) {
  const int x = (int)blockIdx.x * 256 + (int)threadIdx.x;
  const int y = (int)blockIdx.y, z = (int)blockIdx.z;
  if (x >= nx) return;
  auto gat = [&](int dz, int dy, int dx) {
    const int xs = wrapi(x + dx, nx), ys = wrapi(y + dy, ny), zs = wrapi(z + dz, nz);
    return G[((int64_t)zs * ny + ys) * nx + xs];
  };
  const int64_t i = ((int64_t)z * ny + y) * nx + x;
  out[i] = out[i] + source_at<L, T>(gat, sc);
}

template <class L, bool THREE, bool THREE_ST, typename T>
hipError_t plane_cfg(const Consts &c, const Grid &g, const T *cur, const T *prev, const T *G,
                     T *out, const SrcC<T> &sc, hipStream_t st) {
  constexpr int TX = L::D >= 2 ? 64 : 256, TY = L::D >= 2 ? 16 : 1;
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  hipLaunchKernelGGL((k_lcde_source_plane<L, THREE, THREE_ST, TX, TY, T>), dim3(tx * ty),
                     dim3(256), 0, st, cur, prev, G, out, nx, ny, tx, tx * ty, make_kc<T>(c), sc);
  return hipGetLastError();
}

template <class L, typename T>
hipError_t step_l(const Consts &c, const Grid &g, const T *cur, const T *prev, const T *G, T *out,
                  const SrcC<T> &sc, hipStream_t st) {
  if constexpr (L::D <= 2) {
    if (!c.three) return plane_cfg<L, false, false, T>(c, g, cur, prev, G, out, sc, st);
    if (!c.three_stencil) return plane_cfg<L, true, false, T>(c, g, cur, prev, G, out, sc, st);
    return plane_cfg<L, true, true, T>(c, g, cur, prev, G, out, sc, st);
  } else {
    hipError_t e = launch_mmfd_step<T>(c, g, cur, prev, out, 1, st);
    if (e != hipSuccess) return e;
    const int nx = (int)g.n[0], ny = (int)g.n[1], nz = (int)g.n[2];
    hipLaunchKernelGGL((k_add_source_3d<L, T>), dim3((nx + 255) / 256, ny, nz), dim3(256), 0, st,
                       out, G, nx, ny, nz, sc);
    return hipGetLastError();
  }
}

}  // namespace

namespace {
template <typename T>
SrcC<T> src_consts(const Consts &c, const SourceSpec &s, int64_t n) {
  SrcC<T> sc{};
  double vh[3];
  for (int a = 0; a < 3; ++a) vh[a] = s.v[a] * s.dt / s.dx;
  for (int p = 0; p < c.npair; ++p) {
    const int j = c.pair[p];
    double ev = 0.0;  // e_j . vh, signed accumulation from zero
    for (int a = 0; a < c.dim; ++a) {
      if (c.e[j][a] == 1) ev = ev + vh[a];
      else if (c.e[j][a] == -1) ev = ev - vh[a];
    }
    sc.wp[p] = (T)c.w[j];
    sc.wm[p] = (T)(c.w1[j] * ev);
  }
  sc.B0 = (T)(s.b[0] + s.b[1] + s.b[2]);
  sc.Bh0 = (T)(s.bh[0] + s.bh[1] + s.bh[2]);
  sc.bp = (T)(s.b[2] + s.b[0]);
  sc.bm = (T)(s.b[2] - s.b[0]);
  sc.bhp = (T)(s.bh[2] + s.bh[0]);
  sc.bhm = (T)(s.bh[2] - s.bh[0]);
  sc.dt = (T)s.dt;
  // S at the step's two levels, t = n dt and t - dt
  sc.sig_t = (T)std::exp(s.lambda * ((double)n * s.dt));
  sc.sig_m = (T)std::exp(s.lambda * ((double)(n - 1) * s.dt));
  for (int j = 0; j < c.q; ++j) {
    double ev = 0.0;
    for (int a = 0; a < c.dim; ++a) {
      if (c.e[j][a] == 1) ev = ev + vh[a];
      else if (c.e[j][a] == -1) ev = ev - vh[a];
    }
    sc.wj[j] = (T)c.w[j];
    sc.evj[j] = (T)(ev * c.inv_d0);
  }
  for (int k = 0; k < 3; ++k) {
    sc.b[k] = (T)s.b[k];
    sc.bh[k] = (T)s.bh[k];
  }
  return sc;
}

template <class L, bool THREE, bool THREE_ST, typename T>
hipError_t meso_cfg(const Consts &c, const Grid &g, const T *cur, const T *prev, const T *G,
                    T *pop_out, T *mom_out, const SrcC<T> &sc, hipStream_t st) {
  constexpr int TX = L::D >= 2 ? 64 : 256, TY = L::D >= 2 ? 16 : 1;
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  hipLaunchKernelGGL((k_lcde_mesofd_source_plane<L, THREE, THREE_ST, TX, TY, T>), dim3(tx * ty),
                     dim3(256), 0, st, cur, prev, G, pop_out, mom_out, nx, ny, tx, tx * ty,
                     make_kc<T>(c), sc);
  return hipGetLastError();
}

template <class L, typename T>
hipError_t meso_l(const Consts &c, const Grid &g, const T *cur, const T *prev, const T *G,
                  T *pop_out, T *mom_out, const SrcC<T> &sc, hipStream_t st) {
  if (!c.three) return meso_cfg<L, false, false, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
  if (!c.three_stencil)
    return meso_cfg<L, true, false, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
  return meso_cfg<L, true, true, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
}
}  // namespace

template <typename T>
hipError_t launch_mmfd_source_step(const Consts &c, const Grid &g, const SourceSpec &s, int64_t n,
                                   const T *cur, const T *prev, T *out, const T *G,
                                   hipStream_t st) {
  if (c.eq != kLCDE) return hipErrorInvalidValue;
  // the 3D source launch is a (x blocks, y, z) grid
  if (c.dim == 3 && (g.n[1] > 65535 || g.n[2] > 65535)) return hipErrorInvalidValue;
  const SrcC<T> sc = src_consts<T>(c, s, n);
  switch (c.lattice) {
    case 1: return step_l<LatD1Q3, T>(c, g, cur, prev, G, out, sc, st);
    case 2: return step_l<LatD2Q5, T>(c, g, cur, prev, G, out, sc, st);
    case 3: return step_l<LatD2Q9, T>(c, g, cur, prev, G, out, sc, st);
    case 4: return step_l<LatD3Q19, T>(c, g, cur, prev, G, out, sc, st);
    case 5: return step_l<LatD2Q5II, T>(c, g, cur, prev, G, out, sc, st);
    case 6: return step_l<LatD3Q7, T>(c, g, cur, prev, G, out, sc, st);
    case 7: return step_l<LatD3Q9, T>(c, g, cur, prev, G, out, sc, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_mesofd_source_step(const Consts &c, const Grid &g, const SourceSpec &s,
                                     int64_t n, const T *cur, const T *prev, T *pop_out,
                                     T *mom_out, const T *G, hipStream_t st) {
  if (c.eq != kLCDE || c.dim == 3) return hipErrorInvalidValue;
  const SrcC<T> sc = src_consts<T>(c, s, n);
  switch (c.lattice) {
    case 1: return meso_l<LatD1Q3, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
    case 2: return meso_l<LatD2Q5, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
    case 3: return meso_l<LatD2Q9, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
    case 5: return meso_l<LatD2Q5II, T>(c, g, cur, prev, G, pop_out, mom_out, sc, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_mesofd_source_step<float>(const Consts &, const Grid &,
                                                     const SourceSpec &, int64_t, const float *,
                                                     const float *, float *, float *,
                                                     const float *, hipStream_t);
template hipError_t launch_mesofd_source_step<double>(const Consts &, const Grid &,
                                                      const SourceSpec &, int64_t, const double *,
                                                      const double *, double *, double *,
                                                      const double *, hipStream_t);
// ------------------------------------------------------------ blocked
// Linear CDE with the source on D2Q5 / D2Q9, MMFD, TB steps per launch: the
// blocked window of tb_window.h with G staged beside the levels; each step's
// value is the plain step's plus its source term, as in the one-step launch.
template <class L, bool THREE, bool THREE_ST, int W, int RG, typename T>
__global__ __launch_bounds__(W *RG) void k_lcde_source_tb(const T *__restrict__ cur,
                                                         const T *__restrict__ prev,
                                                         T *__restrict__ out_cur,
                                                         T *__restrict__ out_prev, int nx, int ny,
                                                         int H, int TB, int tiles_x, int ntiles,
                                                         KC<T> kc, SrcTbHook<L, T> hook) {
  extern __shared__ unsigned char smem_srctb[];
  T *lds = reinterpret_cast<T *>(smem_srctb);  // [levels + G][H][W]
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int tile = xcd_remap_tb(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  tb_window<L, kLCDE, THREE, THREE_ST, W, 8, false, false, T, SrcTbHook<L, T>>(
      cur, prev, out_cur, out_prev, nx, ny, H, TB, TB, x0, y0, kc, lds, nullptr, hook);
}

namespace {
template <class L, bool THREE, bool THREE_ST, typename T>
hipError_t src_tb_cfg(const Consts &c, const Grid &g, const SourceSpec &s, int64_t n0,
                      const TbPlan &pl, const T *cur, const T *prev, T *oc, T *op, const T *G,
                      hipStream_t st) {
  constexpr int W = 64;
  SrcTbHook<L, T> hook;
  hook.G = G;
  hook.sc = src_consts<T>(c, s, n0);
  for (int k = 0; k <= pl.tb; ++k)
    hook.sig[k] = (T)std::exp(s.lambda * ((double)(n0 + k - 1) * s.dt));
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int TX = W - 2 * pl.tb, TY = pl.h - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)((THREE ? 3 : 2) + 1) * pl.h * W * sizeof(T);
  auto fn = k_lcde_source_tb<L, THREE, THREE_ST, W, 8, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(W * 8), lds, st, cur, prev, oc, op, nx, ny, pl.h,
                     pl.tb, tx, tx * ty, make_kc<T>(c), hook);
  return hipGetLastError();
}

template <class L, typename T>
hipError_t src_tb_l(const Consts &c, const Grid &g, const SourceSpec &s, int64_t n0,
                    const TbPlan &pl, const T *cur, const T *prev, T *oc, T *op, const T *G,
                    hipStream_t st) {
  if (!c.three) return src_tb_cfg<L, false, false, T>(c, g, s, n0, pl, cur, prev, oc, op, G, st);
  if (!c.three_stencil)
    return src_tb_cfg<L, true, false, T>(c, g, s, n0, pl, cur, prev, oc, op, G, st);
  return src_tb_cfg<L, true, true, T>(c, g, s, n0, pl, cur, prev, oc, op, G, st);
}
}  // namespace

bool source_tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem) {
  if (c.dim != 2 || (c.lattice != 2 && c.lattice != 3) || c.eq != kLCDE) return false;
  if (pl.w != 64 || pl.tb < 2 || pl.tb > kMaxBcSteps) return false;
  if (!tb_plan_valid(pl, (c.three ? 3 : 2) + 1, elem)) return false;
  return g.n[0] >= pl.w && g.n[1] >= pl.h;
}

template <typename T>
hipError_t launch_mmfd_source_tb(const Consts &c, const Grid &g, const SourceSpec &s, int64_t n0,
                                 const TbPlan &pl, const T *cur, const T *prev, T *out_cur,
                                 T *out_prev, const T *G, hipStream_t st) {
  if (!source_tb_supported(c, g, pl, (int)sizeof(T))) return hipErrorInvalidValue;
  if (c.lattice == 3) return src_tb_l<LatD2Q9, T>(c, g, s, n0, pl, cur, prev, out_cur, out_prev, G, st);
  return src_tb_l<LatD2Q5, T>(c, g, s, n0, pl, cur, prev, out_cur, out_prev, G, st);
}

template hipError_t launch_mmfd_source_tb<float>(const Consts &, const Grid &, const SourceSpec &,
                                                 int64_t, const TbPlan &, const float *,
                                                 const float *, float *, float *, const float *,
                                                 hipStream_t);
template hipError_t launch_mmfd_source_tb<double>(const Consts &, const Grid &, const SourceSpec &,
                                                  int64_t, const TbPlan &, const double *,
                                                  const double *, double *, double *,
                                                  const double *, hipStream_t);

template hipError_t launch_mmfd_source_step<float>(const Consts &, const Grid &,
                                                   const SourceSpec &, int64_t, const float *,
                                                   const float *, float *, const float *,
                                                   hipStream_t);
template hipError_t launch_mmfd_source_step<double>(const Consts &, const Grid &,
                                                    const SourceSpec &, int64_t, const double *,
                                                    const double *, double *, const double *,
                                                    hipStream_t);

}  // namespace mfd
