// The temporally blocked window of the 2D linear CDE / Burgers MMFD step
// (shared by the blocked kernels of kernels_tb.hip and the blocked source
// step of kernels_source.hip).
//
// A workgroup loads a W x H window of level t (and t-dt for three-level
// schemes) into LDS, then performs TBS updates in LDS, each on a region one
// node smaller on every side (the stencil reaches one node), and finally
// stores the interior of the last level (and of the level before it, which
// the next three-level launch needs).  Every node update is the same
// expression as the single-step kernel (mmfd_node), so results are bitwise
// independent of the steps per launch.
#pragma once

#include "mmfd_node.h"

namespace mfd {

__device__ __forceinline__ int xcd_remap_tb(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// Window whose origin is (x0, y0) (global, may be negative): load, TBS steps,
// store of the interior that starts TBW nodes in.  WRAP_ANY: grids of any
// size (modular wrap); otherwise nx >= W and ny >= H (one conditional wrap).
// A window hook adds per-node work to the steps: kExtra more W x H LDS arrays
// are staged by load() with the window's levels (same origin and wrap), and
// every new node value v of step t (1-based) becomes apply(t, extra, W, y,
// x, v).  TbNoHook adds nothing.
struct TbNoHook {
  static constexpr int kExtra = 0;
  template <typename T>
  __device__ __forceinline__ void load(T *, int, int, int, int, int, int, int, int) const {}
  template <typename T>
  __device__ __forceinline__ T apply(int, const T *, int, int, int, T v) const {
    return v;
  }
};

template <class L, int EQ, bool THREE, bool THREE_ST, int W, int RG, bool WRAP_ANY, bool B1,
          typename T, class Hook = TbNoHook>
__device__ __forceinline__ void tb_window(const T *__restrict__ cur, const T *__restrict__ prev,
                                          T *__restrict__ out_cur, T *__restrict__ out_prev,
                                          int nx, int ny, int H, int TBW, int TBS, int x0, int y0,
                                          const KC<T> &kc, T *lds, const DirBC *bc = nullptr,
                                          const Hook &hook = Hook()) {
  constexpr int NT = W * RG;
  constexpr int KB = 8;  // window loads in flight per thread
  constexpr bool BURG = EQ == kBurgers;
  const int WH = W * H;

  // ---- load level t (buffer 0) and t - dt (buffer 1)
  for (int base = 0; base < WH; base += KB * NT) {
    T v[KB], vp[THREE ? KB : 1];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < WH) {
        int gx = x0 + (i % W), gy = y0 + i / W;
        if constexpr (WRAP_ANY) {
          gx = wrapi(gx, nx);
          gy = wrapi(gy, ny);
        } else {
          gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
          gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        }
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
  T *const extra = lds + (THREE ? 3 : 2) * WH;
  if constexpr (Hook::kExtra > 0) hook.load(extra, W, H, x0, y0, nx, ny, (int)threadIdx.x, NT);
  __syncthreads();

  // one column per thread, RG row groups
  const int xx = threadIdx.x % W, rg = threadIdx.x / W;
  int ic = 0, ip = 1, io = THREE ? 2 : 1;
#pragma unroll 1
  for (int t = 1; t <= TBS; ++t) {
    const T *A = lds + ic * WH;
    const T *P = lds + ip * WH;
    T *O = lds + io * WH;
    const int Hr = H - 2 * t;
    const int seg = (Hr + RG - 1) / RG;
    const int ya = t + rg * seg, yb = min(ya + seg, H - t);
    if (xx >= t && xx < W - t && ya < yb) {
      // phi (w, h) and, for Burgers, the second record field (wb, hb)
      T w[3][3], h[3][3], wb[BURG ? 3 : 1][3], hb[BURG && THREE_ST ? 3 : 1][3];
      auto second = [&](T v) { return (v * v) * kc.bh; };
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[0][c] = A[(ya - 1) * W + xx - 1 + c];
        w[1][c] = A[ya * W + xx - 1 + c];
        if constexpr (BURG) {
          wb[0][c] = second(w[0][c]);
          wb[1][c] = second(w[1][c]);
        }
        if constexpr (THREE_ST) {
          h[0][c] = P[(ya - 1) * W + xx - 1 + c];
          h[1][c] = P[ya * W + xx - 1 + c];
          if constexpr (BURG) {
            hb[0][c] = second(h[0][c]);
            hb[1][c] = second(h[1][c]);
          }
        }
      }
#pragma unroll 2
      for (int y = ya; y < yb; ++y) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[2][c] = A[(y + 1) * W + xx - 1 + c];
          if constexpr (BURG) wb[2][c] = second(w[2][c]);
          if constexpr (THREE_ST) {
            h[2][c] = P[(y + 1) * W + xx - 1 + c];
            if constexpr (BURG) hb[2][c] = second(h[2][c]);
          }
        }
        auto at = [&](int k, int, int dy, int dx) {
          if constexpr (BURG) return k == 0 ? w[1 + dy][1 + dx] : wb[1 + dy][1 + dx];
          else return w[1 + dy][1 + dx];
        };
        auto ath = [&](int k, int, int dy, int dx) {
          if constexpr (THREE_ST) {
            if constexpr (BURG) return k == 0 ? h[1 + dy][1 + dx] : hb[1 + dy][1 + dx];
            else return h[1 + dy][1 + dx];
          } else {
            return T(0);
          }
        };
        T cc[1] = {w[1][1]};
        T pc[1] = {THREE ? P[y * W + xx] : T(0)};
        T oc[1];
        mmfd_node<L, EQ, THREE, THREE_ST, T, B1>(at, ath, cc, pc, oc, kc);
        if (bc && bc->on) {
          // Dirichlet nodes take the value prescribed for step t of this
          // launch (window nodes outside the grid are wrapped copies that
          // only ever feed boundary nodes)
          const int gx = x0 + xx, gy = y0 + y;
          if (gx >= 0 && gy >= 0 && gx < nx && gy < ny && dir_node(gx, gy, nx, ny))
            oc[0] = (T)(bc->Gb[dir_index(gx, gy, nx, ny)] * bc->E[t]);
        }
        if constexpr (Hook::kExtra > 0) oc[0] = hook.apply(t, (const T *)extra, W, y, xx, oc[0]);
        O[y * W + xx] = oc[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[0][c] = w[1][c];
          w[1][c] = w[2][c];
          if constexpr (BURG) {
            wb[0][c] = wb[1][c];
            wb[1][c] = wb[2][c];
          }
          if constexpr (THREE_ST) {
            h[0][c] = h[1][c];
            h[1][c] = h[2][c];
            if constexpr (BURG) {
              hb[0][c] = hb[1][c];
              hb[1][c] = hb[2][c];
            }
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
  const int TX = W - 2 * TBW, TY = H - 2 * TBW;
  for (int i = threadIdx.x; i < TX * TY; i += NT) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + TBW + lx, gy = y0 + TBW + ly;
    if (gx >= nx || gy >= ny) continue;
    const int64_t gi = (int64_t)gy * nx + gx;
    out_cur[gi] = C[(TBW + ly) * W + TBW + lx];
    if constexpr (THREE) out_prev[gi] = Pv[(TBW + ly) * W + TBW + lx];
  }
}

}  // namespace mfd
