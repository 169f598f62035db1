// Temporally blocked MMFD kernels for the two-level / three-level scheme on
// 2D lattices (D2Q5, D2Q9) for the linear CDE and Burgers' equation: one
// launch advances several time steps.
//
// A workgroup loads a W x H window of level t (and t-dt for three-level
// schemes) into LDS, then performs TB updates in LDS, each on a region one
// node smaller on every side (the stencil reaches one node), and finally
// stores the (W - 2 TB) x (H - 2 TB) interior of the last level (and of the
// level before it, which the next three-level launch needs).  Every node
// update is the same expression as the single-step kernel (mmfd_node), so
// results are bitwise independent of TB.
//
// Inside a step each thread owns one column of the window (a 64-wide
// wavefront reads one LDS row: no bank conflicts) and a contiguous segment of
// rows, and slides a 3 x 3 register window down it: 3 LDS reads per node
// instead of 9.  For Burgers' equation the window also carries the second
// record field phi^2 dt/(2 dx), formed from phi as each row enters.  The
// window loads are all issued before the first LDS store.
//
// The batched kernel runs the same window body for every tile of a table of
// independent grids; each instance advances min(TB, its remaining steps) in a
// window sized for TB.
#include "batch_kernels.h"
#include "mmfd_node.h"
#include "tb_window.h"

namespace mfd {

template <class L, int EQ, bool THREE, bool THREE_ST, int W, int RG, bool B1, typename T>
__global__ __launch_bounds__(W *RG) void k_mmfd_tb(const T *__restrict__ cur,
                                                  const T *__restrict__ prev,
                                                  T *__restrict__ out_cur,
                                                  T *__restrict__ out_prev, int nx, int ny,
                                                  int H, int TB, int tiles_x, int ntiles,
                                                  KC<T> kc, DirBC bc) {
  extern __shared__ unsigned char smem_tb[];
  T *lds = reinterpret_cast<T *>(smem_tb);  // [levels][H][W]
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int tile = xcd_remap_tb(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  tb_window<L, EQ, THREE, THREE_ST, W, RG, false, B1, T>(cur, prev, out_cur, out_prev, nx, ny, H,
                                                         TB, TB, x0, y0, kc, lds, &bc);
}

// Batched two-level variant: launch `launch` of a run whose launches advance
// TB steps; tiles of instances with steps left form the prefix [0, ntiles).
template <class L, int EQ, int W, int RG, bool B1, typename T>
__global__ __launch_bounds__(W *RG) void k_batch_tb(const BatchInst<T> *__restrict__ inst,
                                                   const int *__restrict__ tile_inst, int ntiles,
                                                   int64_t launch, int H, int TB) {
  extern __shared__ unsigned char smem_btb[];
  T *lds = reinterpret_cast<T *>(smem_btb);
  const int t = xcd_remap_tb(blockIdx.x, ntiles);
  const BatchInst<T> &I = inst[tile_inst[t]];
  const int64_t left = I.nsteps - launch * TB;
  const int TBS = left < TB ? (int)left : TB;
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int lt = t - I.tile0;
  const int x0 = (lt % I.tiles_x) * TX - TB, y0 = (lt / I.tiles_x) * TY - TB;
  const int64_t r = I.c0 + launch;
  const T *cur = I.ring[r & 1];
  T *out = I.ring[(r + 1) & 1];
  tb_window<L, EQ, false, false, W, RG, true, B1, T>(cur, nullptr, out, nullptr, I.nx, I.ny, H,
                                                     TB, TBS, x0, y0, I.kc, lds);
}

namespace {

// Window: W = 64 or 128 columns (one per thread; a wavefront reads 64
// consecutive LDS words of a row), H rows in RG = 8 row groups; the tile
// advanced is (W - 2 TB) x (H - 2 TB).  The batched kernel uses W = 64.
constexpr int kTbW = 64, kTbRG = 8;

template <class L, int EQ, bool THREE, bool THREE_ST, bool B1, int W, typename T>
hipError_t tb_cfg_w(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, const T *prev,
                    T *oc, T *op, const DirBC &bc, hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int TX = W - 2 * pl.tb, TY = pl.h - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)(THREE ? 3 : 2) * pl.h * W * sizeof(T);
  auto fn = k_mmfd_tb<L, EQ, THREE, THREE_ST, W, kTbRG, B1, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(W * kTbRG), lds, st, cur, prev, oc, op, nx, ny,
                     pl.h, pl.tb, tx, tx * ty, kc, bc);
  return hipGetLastError();
}

template <class L, int EQ, bool THREE, bool THREE_ST, bool B1, typename T>
hipError_t tb_cfg(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, const T *prev,
                  T *oc, T *op, const DirBC &bc, hipStream_t st) {
  if (pl.w == 128)
    return tb_cfg_w<L, EQ, THREE, THREE_ST, B1, 128, T>(c, g, pl, cur, prev, oc, op, bc, st);
  return tb_cfg_w<L, EQ, THREE, THREE_ST, B1, 64, T>(c, g, pl, cur, prev, oc, op, bc, st);
}

template <class L, int EQ, bool B1, typename T>
hipError_t tb_levels(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                     const T *prev, T *oc, T *op, const DirBC &bc, hipStream_t st) {
  if (!c.three) return tb_cfg<L, EQ, false, false, B1, T>(c, g, pl, cur, prev, oc, op, bc, st);
  if (!c.three_stencil)
    return tb_cfg<L, EQ, true, false, B1, T>(c, g, pl, cur, prev, oc, op, bc, st);
  return tb_cfg<L, EQ, true, true, B1, T>(c, g, pl, cur, prev, oc, op, bc, st);
}

template <class L, typename T>
hipError_t tb_eq(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, const T *prev,
                 T *oc, T *op, const DirBC &bc, hipStream_t st) {
  if (c.eq == kNSE) {
    if (bc.on) return hipErrorInvalidValue;
    return launch_nse_tb<T>(c, g, pl, cur, prev, oc, op, st);
  }
  if (c.eq == kLCDE) return tb_levels<L, kLCDE, false, T>(c, g, pl, cur, prev, oc, op, bc, st);
  if (c.eq == kBurgers) {
    if (c.beta_one) return tb_levels<L, kBurgers, true, T>(c, g, pl, cur, prev, oc, op, bc, st);
    return tb_levels<L, kBurgers, false, T>(c, g, pl, cur, prev, oc, op, bc, st);
  }
  return hipErrorInvalidValue;
}

template <class L, int EQ, bool B1, typename T>
hipError_t btb_cfg(const BatchInst<T> *inst, const int *tile_inst, int ntiles, int64_t launch,
                   const TbPlan &pl, hipStream_t st) {
  const size_t lds = (size_t)2 * pl.h * kTbW * sizeof(T);
  auto fn = k_batch_tb<L, EQ, kTbW, kTbRG, B1, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(ntiles), dim3(kTbW * kTbRG), lds, st, inst, tile_inst, ntiles,
                     launch, pl.h, pl.tb);
  return hipGetLastError();
}

}  // namespace

size_t tb_lds_bytes(const Consts &c, const TbPlan &pl, int elem) {
  if (c.eq == kNSE) return (size_t)2 * c.npair * pl.h * pl.w * elem;  // pair parts only
  if (pl.w == 128 && lane_tb_applies(c, elem)) return (size_t)pl.h * 128 * elem;  // in place
  return (size_t)(c.three ? 3 : 2) * pl.h * pl.w * elem;
}

bool tb_plan_valid(const TbPlan &pl, int levels, int elem) {
  if (pl.w != 64 && pl.w != 128) return false;
  if (pl.tb < 1 || pl.tb > 16 || pl.h < 2 * pl.tb + 4) return false;
  if (pl.w - 2 * pl.tb < 8) return false;
  return (size_t)levels * pl.h * pl.w * elem <= 160 * 1024;
}

bool tb_equation_supported(const Consts &c) {
  if (c.dim != 2 || (c.lattice != 2 && c.lattice != 3)) return false;
  if (c.eq == kNSE) return !c.three_stencil;
  return c.eq == kLCDE || c.eq == kBurgers;
}

bool tb_supported(const Consts &c, const Grid &g, const TbPlan &pl, int elem) {
  if (!tb_equation_supported(c)) return false;
  if (c.eq == kNSE) {
    if (!nse_tb_plan_valid(pl, c.npair, elem)) return false;
  } else if (pl.w == 128 && lane_tb_applies(c, elem)) {
    // the in-place binary32 LCDE window: one LDS level
    if (!tb_plan_valid(pl, 1, elem) || !lane_tb_window_fits(pl)) return false;
  } else if (!tb_plan_valid(pl, c.three ? 3 : 2, elem)) {
    return false;
  }
  // one conditional wrap per coordinate covers the window
  return g.n[0] >= pl.w && g.n[1] >= pl.h;
}

template <typename T>
hipError_t launch_mmfd_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                          const T *prev, T *out_cur, T *out_prev, hipStream_t st,
                          const DirBC *bcp) {
  DirBC bc{};
  if (bcp) bc = *bcp;
  if (bc.on && pl.tb > kMaxBcSteps) return hipErrorInvalidValue;
  if (pl.w == 128 && lane_tb_applies(c, sizeof(T))) {
    if (bc.on) return hipErrorInvalidValue;  // the in-place window has no boundary nodes
    return launch_lane_tb<T>(c, g, pl, cur, out_cur, st);
  }
  if (c.lattice == 3) return tb_eq<LatD2Q9, T>(c, g, pl, cur, prev, out_cur, out_prev, bc, st);
  if (c.lattice == 2) return tb_eq<LatD2Q5, T>(c, g, pl, cur, prev, out_cur, out_prev, bc, st);
  return hipErrorInvalidValue;
}

int tb_window_cols() { return kTbW; }

template <typename T>
hipError_t launch_batch_tb(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst,
                           int ntiles, int64_t launch, const TbPlan &pl, hipStream_t st) {
  if (k.three || pl.w != kTbW) return hipErrorInvalidValue;
  if (k.lattice == 3) {
    if (k.eq == kLCDE)
      return btb_cfg<LatD2Q9, kLCDE, false, T>(inst, tile_inst, ntiles, launch, pl, st);
    if (k.eq == kBurgers && k.b1)
      return btb_cfg<LatD2Q9, kBurgers, true, T>(inst, tile_inst, ntiles, launch, pl, st);
    if (k.eq == kBurgers)
      return btb_cfg<LatD2Q9, kBurgers, false, T>(inst, tile_inst, ntiles, launch, pl, st);
  } else if (k.lattice == 2) {
    if (k.eq == kLCDE)
      return btb_cfg<LatD2Q5, kLCDE, false, T>(inst, tile_inst, ntiles, launch, pl, st);
    if (k.eq == kBurgers && k.b1)
      return btb_cfg<LatD2Q5, kBurgers, true, T>(inst, tile_inst, ntiles, launch, pl, st);
    if (k.eq == kBurgers)
      return btb_cfg<LatD2Q5, kBurgers, false, T>(inst, tile_inst, ntiles, launch, pl, st);
  }
  return hipErrorInvalidValue;
}

#define MFD_INST(T)                                                                               \
  template hipError_t launch_mmfd_tb<T>(const Consts &, const Grid &, const TbPlan &, const T *, \
                                        const T *, T *, T *, hipStream_t, const DirBC *);         \
  template hipError_t launch_batch_tb<T>(const BatchKey &, const BatchInst<T> *, const int *,    \
                                         int, int64_t, const TbPlan &, hipStream_t);
MFD_INST(float)
MFD_INST(double)
#undef MFD_INST

}  // namespace mfd
