// Temporally blocked MMFD kernel for the linear CDE on 2D lattices
// (D2Q5, D2Q9): one launch advances TB time steps.
//
// A workgroup loads a (TX + 2 TB) x (TY + 2 TB) window of level t (and t-dt
// for three-level schemes) into LDS, then performs TB updates in LDS, each on
// a region one node smaller on every side (the stencil reaches one node), and
// finally stores the TX x TY interior of the last level (and of the level
// before it, which the next three-level launch needs).  Every node update is
// the same expression as the single-step kernel (mmfd_node), so results are
// bitwise independent of TB.
//
// Inside a step each thread owns one column of the window (a 64-wide
// wavefront reads one LDS row: no bank conflicts) and a contiguous segment of
// rows, and slides a 3 x 3 register window down it: 3 LDS reads per node
// instead of 9.  The window loads are all issued before the first LDS store.
#include "mmfd_node.h"

namespace mfd {

__device__ __forceinline__ int xcd_remap_tb(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

template <class L, bool THREE, bool THREE_ST, int W, int RG, typename T>
__global__ __launch_bounds__(W *RG) void k_lcde_tb(const T *__restrict__ cur,
                                                  const T *__restrict__ prev,
                                                  T *__restrict__ out_cur,
                                                  T *__restrict__ out_prev, int nx, int ny,
                                                  int H, int TB, int tiles_x, int ntiles,
                                                  KC<T> kc) {
  constexpr int NT = W * RG;
  constexpr int NB = THREE ? 3 : 2;
  constexpr int KB = 8;  // window loads in flight per thread
  extern __shared__ unsigned char smem_tb[];
  T *lds = reinterpret_cast<T *>(smem_tb);  // [NB][H][W]
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int WH = W * H;

  const int tile = xcd_remap_tb(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;

  // ---- load level t (buffer 0) and t - dt (buffer 1), KB loads in flight;
  // the host guarantees nx >= W and ny >= H, so one conditional wrap suffices
  for (int base = 0; base < WH; base += KB * NT) {
    T v[KB], vp[THREE ? KB : 1];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < WH) {
        int gx = x0 + (i % W), gy = y0 + i / W;
        gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
        gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        const int64_t gi = (int64_t)gy * nx + gx;
        v[k] = cur[gi];
        if constexpr (THREE) vp[k] = prev[gi];
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < WH) {
        lds[i] = v[k];
        if constexpr (THREE) lds[WH + i] = vp[k];
      }
    }
  }
  __syncthreads();

  // one column per thread, RG row groups
  const int xx = threadIdx.x % W, rg = threadIdx.x / W;
  int ic = 0, ip = 1, io = THREE ? 2 : 1;
#pragma unroll 1
  for (int t = 1; t <= TB; ++t) {
    const T *A = lds + ic * WH;
    const T *P = lds + ip * WH;
    T *O = lds + io * WH;
    const int Hr = H - 2 * t;
    const int seg = (Hr + RG - 1) / RG;
    const int ya = t + rg * seg, yb = min(ya + seg, H - t);
    if (xx >= t && xx < W - t && ya < yb) {
      T w[3][3], h[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[0][c] = A[(ya - 1) * W + xx - 1 + c];
        w[1][c] = A[ya * W + xx - 1 + c];
        if constexpr (THREE_ST) {
          h[0][c] = P[(ya - 1) * W + xx - 1 + c];
          h[1][c] = P[ya * W + xx - 1 + c];
        }
      }
#pragma unroll 2
      for (int y = ya; y < yb; ++y) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[2][c] = A[(y + 1) * W + xx - 1 + c];
          if constexpr (THREE_ST) h[2][c] = P[(y + 1) * W + xx - 1 + c];
        }
        auto at = [&](int, int, int dy, int dx) { return w[1 + dy][1 + dx]; };
        auto ath = [&](int, int, int dy, int dx) {
          if constexpr (THREE_ST) return h[1 + dy][1 + dx];
          else return T(0);
        };
        T cc[1] = {w[1][1]};
        T pc[1] = {THREE ? P[y * W + xx] : T(0)};
        T oc[1];
        mmfd_node<L, kLCDE, THREE, THREE_ST, T>(at, ath, cc, pc, oc, kc);
        O[y * W + xx] = oc[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[0][c] = w[1][c];
          w[1][c] = w[2][c];
          if constexpr (THREE_ST) {
            h[0][c] = h[1][c];
            h[1][c] = h[2][c];
          }
        }
      }
    }
    __syncthreads();
    if constexpr (THREE) {
      const int tt = ip;
      ip = ic;
      ic = io;
      io = tt;
    } else {
      const int tt = ic;
      ic = io;
      io = tt;
    }
  }

  // ---- store the interior of the last level (and the one before it)
  const T *C = lds + ic * WH;
  const T *Pv = lds + ip * WH;
  for (int i = threadIdx.x; i < TX * TY; i += NT) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + TB + lx, gy = y0 + TB + ly;
    if (gx >= nx || gy >= ny) continue;
    const int64_t gi = (int64_t)gy * nx + gx;
    out_cur[gi] = C[(TB + ly) * W + TB + lx];
    if constexpr (THREE) out_prev[gi] = Pv[(TB + ly) * W + TB + lx];
  }
}

namespace {

// Window: W = 64 columns (one per thread, a wavefront reads one LDS row),
// H rows in RG = 4 row groups; the tile advanced is (W - 2 TB) x (H - 2 TB).
constexpr int kTbW = 64, kTbRG = 4;

template <class L, bool THREE, bool THREE_ST, typename T>
hipError_t tb_cfg(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, const T *prev,
                  T *oc, T *op, hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int TX = kTbW - 2 * pl.tb, TY = pl.h - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)(THREE ? 3 : 2) * pl.h * kTbW * sizeof(T);
  auto fn = k_lcde_tb<L, THREE, THREE_ST, kTbW, kTbRG, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(kTbW * kTbRG), lds, st, cur, prev, oc, op, nx, ny,
                     pl.h, pl.tb, tx, tx * ty, kc);
  return hipGetLastError();
}

template <class L, typename T>
hipError_t tb_levels(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                     const T *prev, T *oc, T *op, hipStream_t st) {
  if (!c.three) return tb_cfg<L, false, false, T>(c, g, pl, cur, prev, oc, op, st);
  if (!c.three_stencil) return tb_cfg<L, true, false, T>(c, g, pl, cur, prev, oc, op, st);
  return tb_cfg<L, true, true, T>(c, g, pl, cur, prev, oc, op, st);
}

}  // namespace

size_t lcde_tb_lds_bytes(const Consts &c, int h, int elem) {
  return (size_t)(c.three ? 3 : 2) * h * kTbW * elem;
}

bool lcde_tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem) {
  if (c.eq != kLCDE || c.dim != 2) return false;
  if (c.lattice != 2 && c.lattice != 3) return false;
  if (pl.tb < 1 || pl.tb > 16 || pl.h < 2 * pl.tb + 4) return false;
  if (kTbW - 2 * pl.tb < 8) return false;
  if (lcde_tb_lds_bytes(c, pl.h, elem) > 160 * 1024) return false;
  // one conditional wrap per coordinate covers the window
  return g.n[0] >= kTbW && g.n[1] >= pl.h;
}

template <typename T>
hipError_t launch_lcde_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                          const T *prev, T *out_cur, T *out_prev, hipStream_t st) {
  if (c.lattice == 3) return tb_levels<LatD2Q9, T>(c, g, pl, cur, prev, out_cur, out_prev, st);
  if (c.lattice == 2) return tb_levels<LatD2Q5, T>(c, g, pl, cur, prev, out_cur, out_prev, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_lcde_tb<float>(const Consts &, const Grid &, const TbPlan &,
                                          const float *, const float *, float *, float *,
                                          hipStream_t);
template hipError_t launch_lcde_tb<double>(const Consts &, const Grid &, const TbPlan &,
                                           const double *, const double *, double *, double *,
                                           hipStream_t);

}  // namespace mfd
