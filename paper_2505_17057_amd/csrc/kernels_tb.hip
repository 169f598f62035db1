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
// Inside a step each thread owns a column segment of RY rows and slides a
// 3 x 3 register window down it: 3 LDS reads per node instead of 9.
#include "mmfd_node.h"

namespace mfd {

__device__ __forceinline__ int wrap_tb(int i, int n) {
  if (i < 0) {
    i += n;
    if (i < 0) i = ((i % n) + n) % n;
  } else if (i >= n) {
    i -= n;
    if (i >= n) i %= n;
  }
  return i;
}

__device__ __forceinline__ int xcd_remap_tb(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

template <class L, bool THREE, bool THREE_ST, int TX, int TY, int TB, int RY, typename T>
__global__ __launch_bounds__(256) void k_lcde_tb(const T *__restrict__ cur,
                                                 const T *__restrict__ prev,
                                                 T *__restrict__ out_cur,
                                                 T *__restrict__ out_prev, int nx, int ny,
                                                 int tiles_x, int ntiles, KC<T> kc) {
  constexpr int W = TX + 2 * TB, H = TY + 2 * TB;
  constexpr int NB = THREE ? 3 : 2;
  __shared__ T lds[NB][H][W];

  const int tile = xcd_remap_tb(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;

  // ---- load level t (buffer 0) and t - dt (buffer 1)
  for (int i = threadIdx.x; i < W * H; i += 256) {
    const int lx = i % W, ly = i / W;
    const int gx = wrap_tb(x0 + lx, nx), gy = wrap_tb(y0 + ly, ny);
    const int64_t gi = (int64_t)gy * nx + gx;
    lds[0][ly][lx] = cur[gi];
    if constexpr (THREE) lds[1][ly][lx] = prev[gi];
  }
  __syncthreads();

  int ic = 0, ip = 1, io = THREE ? 2 : 1;
#pragma unroll 1
  for (int t = 1; t <= TB; ++t) {
    const int Wr = W - 2 * t, Hr = H - 2 * t;
    const int nseg = (Hr + RY - 1) / RY;
    const T(*A)[W] = lds[ic];
    const T(*P)[W] = lds[ip];
    T(*O)[W] = lds[io];
    for (int item = threadIdx.x; item < Wr * nseg; item += 256) {
      const int xx = t + item % Wr;
      const int ya = t + (item / Wr) * RY;
      const int yb = min(ya + RY, H - t);
      // register windows: rows y-1, y, y+1 of columns xx-1, xx, xx+1
      T w[3][3], h[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[0][c] = A[ya - 1][xx - 1 + c];
        w[1][c] = A[ya][xx - 1 + c];
        if constexpr (THREE_ST) {
          h[0][c] = P[ya - 1][xx - 1 + c];
          h[1][c] = P[ya][xx - 1 + c];
        }
      }
#pragma unroll 4
      for (int y = ya; y < yb; ++y) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[2][c] = A[y + 1][xx - 1 + c];
          if constexpr (THREE_ST) h[2][c] = P[y + 1][xx - 1 + c];
        }
        auto at = [&](int, int, int dy, int dx) { return w[1 + dy][1 + dx]; };
        auto ath = [&](int, int, int dy, int dx) {
          if constexpr (THREE_ST) return h[1 + dy][1 + dx];
          else return T(0);
        };
        T cc[1] = {w[1][1]};
        T pc[1] = {THREE ? P[y][xx] : T(0)};
        T oc[1];
        mmfd_node<L, kLCDE, THREE, THREE_ST, T>(at, ath, cc, pc, oc, kc);
        O[y][xx] = oc[0];
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
  for (int i = threadIdx.x; i < TX * TY; i += 256) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + TB + lx, gy = y0 + TB + ly;
    if (gx >= nx || gy >= ny) continue;
    const int64_t gi = (int64_t)gy * nx + gx;
    out_cur[gi] = lds[ic][TB + ly][TB + lx];
    if constexpr (THREE) out_prev[gi] = lds[ip][TB + ly][TB + lx];
  }
}

namespace {

template <class L, bool THREE, bool THREE_ST, int TB, typename T>
hipError_t tb_cfg(const Consts &c, const Grid &g, const T *cur, const T *prev, T *oc, T *op,
                  hipStream_t st) {
  constexpr int TX = 64, TY = sizeof(T) == 8 ? 24 : 32, RY = 8;
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  hipLaunchKernelGGL((k_lcde_tb<L, THREE, THREE_ST, TX, TY, TB, RY, T>), dim3(tx * ty), dim3(256), 0,
                     st, cur, prev, oc, op, nx, ny, tx, tx * ty, kc);
  return hipGetLastError();
}

template <class L, int TB, typename T>
hipError_t tb_levels(const Consts &c, const Grid &g, const T *cur, const T *prev, T *oc, T *op,
                     hipStream_t st) {
  if (!c.three) return tb_cfg<L, false, false, TB, T>(c, g, cur, prev, oc, op, st);
  if (!c.three_stencil) return tb_cfg<L, true, false, TB, T>(c, g, cur, prev, oc, op, st);
  return tb_cfg<L, true, true, TB, T>(c, g, cur, prev, oc, op, st);
}

template <class L, typename T>
hipError_t tb_depth(const Consts &c, const Grid &g, int tb, const T *cur, const T *prev, T *oc,
                    T *op, hipStream_t st) {
  switch (tb) {
    case 2: return tb_levels<L, 2, T>(c, g, cur, prev, oc, op, st);
    case 4: return tb_levels<L, 4, T>(c, g, cur, prev, oc, op, st);
    case 6: return tb_levels<L, 6, T>(c, g, cur, prev, oc, op, st);
    case 8: return tb_levels<L, 8, T>(c, g, cur, prev, oc, op, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool lcde_tb_supported(const Consts &c, const Grid &g, int tb) {
  if (c.eq != kLCDE || c.dim != 2) return false;
  if (c.lattice != 2 && c.lattice != 3) return false;
  if (tb != 2 && tb != 4 && tb != 6 && tb != 8) return false;
  // the window must not wrap onto itself
  return g.n[0] >= 2 * tb + 1 && g.n[1] >= 2 * tb + 1;
}

template <typename T>
hipError_t launch_lcde_tb(const Consts &c, const Grid &g, int tb, const T *cur, const T *prev,
                          T *out_cur, T *out_prev, hipStream_t st) {
  if (c.lattice == 3) return tb_depth<LatD2Q9, T>(c, g, tb, cur, prev, out_cur, out_prev, st);
  if (c.lattice == 2) return tb_depth<LatD2Q5, T>(c, g, tb, cur, prev, out_cur, out_prev, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_lcde_tb<float>(const Consts &, const Grid &, int, const float *,
                                          const float *, float *, float *, hipStream_t);
template hipError_t launch_lcde_tb<double>(const Consts &, const Grid &, int, const double *,
                                           const double *, double *, double *, hipStream_t);

}  // namespace mfd
