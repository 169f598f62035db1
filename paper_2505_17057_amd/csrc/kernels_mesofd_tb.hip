// Temporally blocked MesoFD step for the two-level linear CDE and Burgers'
// equation on D2Q5 / D2Q9: one launch advances TB time steps.
//
// A workgroup loads a W x H window of the moments of level t into LDS; each
// step every node of a region one node smaller than the last evaluates its b
// new populations (Eq. (2-1), the node function of the single-step kernel)
// in registers and sums them into its moment of the new level (Eq. (2-1-1)),
// which goes to LDS for the next step.  The populations of the launch's last
// step (unless pop_out is null) and their moments are stored for the window's
// interior.  The
// populations of the intermediate steps are formed like every other and
// summed, but not written to memory (no later step reads populations: each
// step depends on the previous one only through its moments).  Results
// equal the single-step kernel's value for value.
//
// Each thread owns one column of the window and a segment of rows and slides
// a 3 x 3 register window of the moment (and, for Burgers, of the second
// record field) down it.
#include "mesofd_node.h"

namespace mfd {

namespace {
__device__ __forceinline__ int xcd_remap_mtb(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}
}  // namespace

template <class L, int EQ, int W, int RG, bool B1, typename T>
__global__ __launch_bounds__(W *RG) void k_mesofd_tb(const T *__restrict__ cur,
                                                    T *__restrict__ mom_out,
                                                    T *__restrict__ pop_out, int nx, int ny,
                                                    int H, int TB, int tiles_x, int ntiles,
                                                    KC<T> kc) {
  constexpr int NT = W * RG;
  constexpr int KB = 8;
  constexpr bool BURG = EQ == kBurgers;
  extern __shared__ unsigned char smem_mtb[];
  T *lds = reinterpret_cast<T *>(smem_mtb);  // [2][H][W]
  const int WH = W * H;
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int tile = xcd_remap_mtb(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  const int64_t N = (int64_t)nx * ny;

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
  int ic = 0;
#pragma unroll 1
  for (int t = 1; t <= TB; ++t) {
    const T *A = lds + ic * WH;
    T *O = lds + (1 - ic) * WH;
    const int Hr = H - 2 * t;
    const int seg = (Hr + RG - 1) / RG;
    const int ya = t + rg * seg, yb = min(ya + seg, H - t);
    const bool last = t == TB;
    if (xx >= t && xx < W - t && ya < yb) {
      T w[3][3], wb[BURG ? 3 : 1][3];
      auto second = [&](T v) { return (v * v) * kc.bh; };
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[0][c] = A[(ya - 1) * W + xx - 1 + c];
        w[1][c] = A[ya * W + xx - 1 + c];
        if constexpr (BURG) {
          wb[0][c] = second(w[0][c]);
          wb[1][c] = second(w[1][c]);
        }
      }
#pragma unroll 2
      for (int y = ya; y < yb; ++y) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[2][c] = A[(y + 1) * W + xx - 1 + c];
          if constexpr (BURG) wb[2][c] = second(w[2][c]);
        }
        auto at = [&](int q, int, int dy, int dx) {
          if constexpr (BURG) return q == 0 ? w[1 + dy][1 + dx] : wb[1 + dy][1 + dx];
          else return w[1 + dy][1 + dx];
        };
        auto ath = [&](int, int, int, int) { return T(0); };
        T fo[L::Q], m[1];
        mesofd_pops<L, EQ, false, B1>(at, ath, (const T *)nullptr, false, fo, kc);
        moments_of<L, EQ>(fo, m);
        O[y * W + xx] = m[0];
        if (last) {
          // the launch's final populations and moments, interior nodes only
          const int gx = x0 + xx, gy = y0 + y;
          if (xx >= TB && xx < W - TB && y >= TB && y < H - TB && gx < nx && gy < ny) {
            const int64_t gi = (int64_t)gy * nx + gx;
            if (pop_out) {  // null: moments only
#pragma unroll
              for (int j = 0; j < L::Q; ++j) pop_out[j * N + gi] = fo[j];
            }
            mom_out[gi] = m[0];
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[0][c] = w[1][c];
          w[1][c] = w[2][c];
          if constexpr (BURG) {
            wb[0][c] = wb[1][c];
            wb[1][c] = wb[2][c];
          }
        }
      }
    }
    __syncthreads();
    ic = 1 - ic;
  }
}

// ------------------------------------------------------------ host side
bool mesofd_tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem) {
  if (c.dim != 2 || (c.lattice != 2 && c.lattice != 3)) return false;
  if ((c.eq != kLCDE && c.eq != kBurgers) || c.three) return false;
  if (pl.w == 128 && lane_meso_applies(c, elem)) {
    // the in-place lane-shared window (one LDS level)
    if (!tb_plan_valid(pl, 1, elem) || !lane_tb_window_fits(pl)) return false;
  } else if (!tb_plan_valid(pl, 2, elem)) {
    return false;
  }
  return g.n[0] >= pl.w && g.n[1] >= pl.h;
}

namespace {
template <class L, int EQ, bool B1, int W, typename T>
hipError_t mtb_cfg(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *mo, T *po,
                   hipStream_t st) {
  constexpr int RG = 4;
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int TX = W - 2 * pl.tb, TY = pl.h - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)2 * pl.h * W * sizeof(T);
  auto fn = k_mesofd_tb<L, EQ, W, RG, B1, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(W * RG), lds, st, cur, mo, po, nx, ny, pl.h, pl.tb, tx,
                     tx * ty, kc);
  return hipGetLastError();
}

template <class L, int EQ, bool B1, typename T>
hipError_t mtb_w(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *mo, T *po,
                 hipStream_t st) {
  if (pl.w == 128) return mtb_cfg<L, EQ, B1, 128, T>(c, g, pl, cur, mo, po, st);
  return mtb_cfg<L, EQ, B1, 64, T>(c, g, pl, cur, mo, po, st);
}

template <class L, typename T>
hipError_t mtb_eq(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *mo, T *po,
                  hipStream_t st) {
  if (c.eq == kLCDE) return mtb_w<L, kLCDE, false, T>(c, g, pl, cur, mo, po, st);
  if (c.beta_one) return mtb_w<L, kBurgers, true, T>(c, g, pl, cur, mo, po, st);
  return mtb_w<L, kBurgers, false, T>(c, g, pl, cur, mo, po, st);
}
}  // namespace

template <typename T>
hipError_t launch_mesofd_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                            T *mom_out, T *pop_out, hipStream_t st) {
  if (pl.w == 128 && lane_meso_applies(c, sizeof(T)))
    return launch_lane_mesofd_tb<T>(c, g, pl, cur, mom_out, pop_out, st);
  if (c.lattice == 3) return mtb_eq<LatD2Q9, T>(c, g, pl, cur, mom_out, pop_out, st);
  if (c.lattice == 2) return mtb_eq<LatD2Q5, T>(c, g, pl, cur, mom_out, pop_out, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_mesofd_tb<float>(const Consts &, const Grid &, const TbPlan &,
                                            const float *, float *, float *, hipStream_t);
template hipError_t launch_mesofd_tb<double>(const Consts &, const Grid &, const TbPlan &,
                                             const double *, double *, double *, hipStream_t);

}  // namespace mfd
