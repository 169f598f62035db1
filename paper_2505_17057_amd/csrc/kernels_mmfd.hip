// MMFD step kernels: the central-difference form of the scheme on moments,
// Eq. (2-2-1) / (2-4-1) (two-level: level t only), Eq. (3layerMMFD-2)
// (three-level), and the linear pair form Eq. (LMMFD-1/3) for the LCDE.
//
// Per node x and opposite pair p = (j, jbar) with representative e_p:
//   D2_p g = (g(x+e_p) - 2 g(x)) + g(x-e_p),   D1_p g = g(x+e_p) - g(x-e_p)
//   zeroth moment: acc += a+ D2_p F+_p;  acc += a- D1_p F-_p      (pairs in order,
//                  level t then level t-dt), out = (A0 m + Ah0 m_prev) + acc
//   first moments (NSE), axis a with e_pa != 0:
//                  acc_a +-= ab+ D2_p F-_p;  acc_a +-= ab- D1_p F+_p
//   LCDE: acc += Cp_p D2_p phi; acc += Cm_p D1_p phi with Cp = a+ ubar+, Cm = a- ubar-.
// In binary32 the three-level base phi - Ah0 (phi - phi_prev) and its sum
// with acc are formed in binary64 and rounded once.
//
// Tiling: a workgroup of 256 threads owns a TX x TY tile of one xy plane
// (1D/2D) or a TX x TY column of planes marched along z (3D).  The EDF
// record of every node of the tile plus a one-node halo is built once into
// LDS (structure of arrays, x fastest: bank-conflict free), then every
// interior node reads its stencil from LDS.  Periodic wrap is applied to the
// global indices of the halo.  Workgroup ids are remapped so that each of
// the 8 XCDs owns a contiguous band of tiles (L2 reuse of halos).
#include "mmfd_node.h"

namespace mfd {

// ------------------------------------------------------ 1D / 2D kernel
template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_mmfd_plane(const T *__restrict__ cur,
                                                    const T *__restrict__ prev,
                                                    T *__restrict__ out, int nx, int ny,
                                                    int tiles_x, int ntiles, KC<T> kc,
                                                    DirBC bc) {
  const int tile = xcd_remap(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  mmfd_plane_tile<L, EQ, THREE, THREE_ST, TX, TY, T>(cur, prev, out, nx, ny, x0, y0, kc, &bc);
}

// one sweep of Burgers' theta step (1D / 2D): the explicit step of the
// iterate x and the Picard-Jacobi update in one pass
template <class L, bool B1, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_picard_plane(const T *__restrict__ x,
                                                      T *__restrict__ out, int nx, int ny,
                                                      int tiles_x, int ntiles, KC<T> kc,
                                                      PicardEp<T> pe) {
  const int tile = xcd_remap(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  mmfd_plane_tile<L, kBurgers, false, false, TX, TY, T>(x, nullptr, out, nx, ny, x0, y0, kc,
                                                        nullptr, &pe);
  (void)B1;
}

// ------------------------------------- 2D NSE, persistent workgroups
// Each workgroup walks a contiguous run of tiles (XCD-aware: the runs of one
// XCD are adjacent, so halo rows are shared in its L2) and loads the next
// tile's moments while it updates the current one.
// PIC: one Picard-Jacobi sweep of the theta step (the explicit step of the
// iterate cur, then the per-field update of pe at the store).
template <class L, bool THREE, bool THREE_ST, int TX, int TY, bool FAST, typename T,
          bool PIC = false, bool SUMS = false>
__global__ __launch_bounds__(256) void k_nse_plane_pp(const T *__restrict__ cur,
                                                      const T *__restrict__ prev,
                                                      T *__restrict__ out, int nx, int ny,
                                                      int tiles_x, int ntiles, KC<T> kc,
                                                      PicardNse<T> pe) {
  using P = PfTile<L, THREE, THREE_ST, TX, TY, T, FAST>;
  __shared__ typename P::Lds sm;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int t0 = w * per, t1 = min(ntiles, t0 + per);
  constexpr bool sums = PIC && SUMS;
  double sq[2 * P::NF];
#pragma unroll
  for (int q = 0; q < 2 * P::NF; ++q) sq[q] = 0.0;
  if (t0 >= t1) {  // the whole workgroup: no barrier is skipped by part of it
    if (sums && threadIdx.x < 2 * P::NF) pe.part[blockIdx.x * 8 + threadIdx.x] = 0.0;
    return;
  }
  typename P::Regs g;
  P::load(cur, prev, nx, ny, (t0 % tiles_x) * TX, (t0 / tiles_x) * TY, g);
  for (int t = t0; t < t1; ++t) {
    P::stage(g, sm, kc);
    T pcv[P::KI][P::NF];
#pragma unroll
    for (int k = 0; k < P::KI; ++k)
#pragma unroll
      for (int q = 0; q < P::NF; ++q) pcv[k][q] = g.pcv[k][q];
    __syncthreads();
    if (t + 1 < t1) P::load(cur, prev, nx, ny, ((t + 1) % tiles_x) * TX, ((t + 1) / tiles_x) * TY, g);
    P::update(sm, pcv, out, nx, ny, (t % tiles_x) * TX, (t / tiles_x) * TY, kc,
              PIC ? &pe : nullptr, sums ? sq : nullptr);
    __syncthreads();
  }
  if constexpr (sums) {
    {  // the workgroup's row: wave sums, then the four waves in order
      __shared__ double red[2 * P::NF][4];
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
      for (int q = 0; q < 2 * P::NF; ++q) {
        double v = sq[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[q][wave] = v;
      }
      __syncthreads();
      if (threadIdx.x < 2 * P::NF) {
        const int q = threadIdx.x;
        pe.part[blockIdx.x * 8 + q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
      }
    }
  }
}

// ---------------------------------------------------------- 3D kernel
template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_mmfd_3d(const T *__restrict__ cur,
                                                 const T *__restrict__ prev,
                                                 T *__restrict__ out, int nx, int ny, int nz,
                                                 int tiles_x, int tiles_y, int zchunk,
                                                 int ntiles, KC<T> kc) {
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR, NF = R::NF;
  constexpr int HX = TX + 2, HY = TY + 2;
  __shared__ T rec[3][NR][HY][HX];
  __shared__ T hrec[THREE_ST ? 3 : 1][THREE_ST ? NR : 1][THREE_ST ? HY : 1][THREE_ST ? HX : 1];

  const int tile = xcd_remap(blockIdx.x, ntiles);
  const int txy = tiles_x * tiles_y;
  const int tz = tile / txy, trem = tile % txy;
  const int x0 = (trem % tiles_x) * TX, y0 = (trem / tiles_x) * TY;
  const int z0 = tz * zchunk, z1 = min(nz, z0 + zchunk);
  const int64_t N = (int64_t)nx * ny * nz;

  auto load_plane = [&](int z, int slot) {
    const int gz = wrapi(z, nz);
    for (int i = threadIdx.x; i < HX * HY; i += 256) {
      const int lx = i % HX, ly = i / HX;
      const int gx = wrapi(x0 - 1 + lx, nx), gy = wrapi(y0 - 1 + ly, ny);
      const int64_t gi = ((int64_t)gz * ny + gy) * nx + gx;
      T m[NF], r[NR];
#pragma unroll
      for (int f = 0; f < NF; ++f) m[f] = cur[f * N + gi];
      make_record<L, EQ>(m, r, kc);
#pragma unroll
      for (int k = 0; k < NR; ++k) rec[slot][k][ly][lx] = r[k];
      if constexpr (THREE_ST) {
#pragma unroll
        for (int f = 0; f < NF; ++f) m[f] = prev[f * N + gi];
        make_record<L, EQ>(m, r, kc);
#pragma unroll
        for (int k = 0; k < NR; ++k) hrec[slot][k][ly][lx] = r[k];
      }
    }
  };

  load_plane(z0 - 1, 0);
  load_plane(z0, 1);
  for (int z = z0; z < z1; ++z) {
    const int rel = z - z0;
    load_plane(z + 1, (rel + 2) % 3);
    __syncthreads();
    const int sm = rel % 3, s0 = (rel + 1) % 3, sp = (rel + 2) % 3;
    for (int i = threadIdx.x; i < TX * TY; i += 256) {
      const int lx = i % TX, ly = i / TX;
      const int gx = x0 + lx, gy = y0 + ly;
      if (gx >= nx || gy >= ny) continue;
      const int cx = lx + 1, cy = ly + 1;
      const int64_t gi = ((int64_t)z * ny + gy) * nx + gx;
      auto slot = [&](int dz) { return dz == 0 ? s0 : (dz > 0 ? sp : sm); };
      auto at = [&](int k, int dz, int dy, int dx) { return rec[slot(dz)][k][cy + dy][cx + dx]; };
      auto ath = [&](int k, int dz, int dy, int dx) {
        if constexpr (THREE_ST) return hrec[slot(dz)][k][cy + dy][cx + dx];
        else return T(0);
      };
      T cc[NF], pc[NF], oc[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        cc[f] = at(f, 0, 0, 0);
        pc[f] = THREE ? prev[f * N + gi] : T(0);
      }
      mmfd_node<L, EQ, THREE, THREE_ST, T>(at, ath, cc, pc, oc, kc);
#pragma unroll
      for (int f = 0; f < NF; ++f) out[f * N + gi] = oc[f];
    }
    __syncthreads();
  }
}

// ------------------------------------------------ LDS-resident 1D run
// One workgroup holds every time level of a 1D grid in LDS and runs all
// steps: the C1 workload (1024 nodes) is latency-bound, so one launch.
constexpr int kResidentBytes = 96 * 1024;

template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
__global__ __launch_bounds__(1024) void k_mmfd_1d_resident(T *__restrict__ ga,
                                                           T *__restrict__ gb,
                                                           T *__restrict__ gc, int nx,
                                                           int64_t nsteps, KC<T> kc) {
  extern __shared__ unsigned char smem[];
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR;
  // three moment levels (a = t, b = t - dt, c = next) and two record planes
  // level k at L0 + k * nx (arithmetic on the LDS base keeps every access a
  // local-data-share access)
  T *const L0 = (T *)smem;
  auto lev = [&](int k) { return L0 + k * nx; };
  T *rec = (T *)smem + 3 * nx;       // NR * nx
  T *hrec = rec + NR * nx;           // NR * nx (three-level stencil)
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    lev(0)[i] = ga[i];
    lev(1)[i] = THREE ? gb[i] : T(0);
  }
  __syncthreads();
  // the linear CDE's record is the moment itself: it reads the levels
  // directly (one barrier per step instead of two)
  constexpr bool LIN = EQ == kLCDE;
  int ic = 0, ip = 1, io = 2;
  for (int64_t s = 0; s < nsteps; ++s) {
    if constexpr (!LIN) {
      for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        T m[1], r[NR];
        m[0] = lev(ic)[i];
        make_record<L, EQ>(m, r, kc);
#pragma unroll
        for (int k = 0; k < NR; ++k) rec[k * nx + i] = r[k];
        if constexpr (THREE_ST) {
          m[0] = lev(ip)[i];
          make_record<L, EQ>(m, r, kc);
#pragma unroll
          for (int k = 0; k < NR; ++k) hrec[k * nx + i] = r[k];
        }
      }
      __syncthreads();
    }
    const T *rc = LIN ? lev(ic) : rec;
    const T *rh = LIN ? lev(ip) : hrec;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      auto idx = [&](int dx) {
        int j = i + dx;
        return j < 0 ? j + nx : (j >= nx ? j - nx : j);
      };
      auto at = [&](int k, int, int, int dx) { return rc[k * nx + idx(dx)]; };
      auto ath = [&](int k, int, int, int dx) {
        if constexpr (THREE_ST) return rh[k * nx + idx(dx)];
        else return T(0);
      };
      T cc[1] = {lev(ic)[i]}, pc[1] = {THREE ? lev(ip)[i] : T(0)}, oc[1];
      mmfd_node<L, EQ, THREE, THREE_ST, T>(at, ath, cc, pc, oc, kc);
      lev(io)[i] = oc[0];
    }
    __syncthreads();
    const int t = ip;
    ip = ic;
    ic = io;
    io = t;
  }
  // final level -> ga, previous level -> gb
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    ga[i] = lev(ic)[i];
    gb[i] = lev(ip)[i];
  }
  (void)gc;
}

// ------------------------------------------------------------ launchers
namespace {

// compute units of an MI355X (persistent grids)
constexpr int kNumCUs = 256;

template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
hipError_t launch_cfg(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                      const DirBC &bc,
                      hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1], nz = (int)g.n[2];
  if constexpr (L::D == 1) {
    constexpr int TX = 1024, TY = 1;
    const int tx = (nx + TX - 1) / TX;
    hipLaunchKernelGGL((k_mmfd_plane<L, EQ, THREE, THREE_ST, TX, TY, T>), dim3(tx), dim3(256), 0,
                       st, cur, prev, out, nx, 1, tx, tx, kc, bc);
  } else if constexpr (L::D == 2 && EQ == kNSE) {
    constexpr int TX = 64, TY = sizeof(T) == 4 ? 16 : 4;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    const int ntiles = tx * ty;
    // persistent groups: as many as the tile's LDS lets reside on each CU
    constexpr int per_cu = (int)((160 * 1024) / sizeof(typename PfTile<L, THREE, THREE_ST, TX, TY, T>::Lds));
    constexpr int groups = kNumCUs * (per_cu < 1 ? 1 : per_cu);
    const int grid = ntiles < groups ? ntiles : groups;
    if (nx >= TX + 2 && ny >= TY + 2)
      hipLaunchKernelGGL((k_nse_plane_pp<L, THREE, THREE_ST, TX, TY, true, T>), dim3(grid),
                         dim3(256), 0, st, cur, prev, out, nx, ny, tx, ntiles, kc,
                         PicardNse<T>{});
    else
      hipLaunchKernelGGL((k_nse_plane_pp<L, THREE, THREE_ST, TX, TY, false, T>), dim3(grid),
                         dim3(256), 0, st, cur, prev, out, nx, ny, tx, ntiles, kc,
                         PicardNse<T>{});
  } else if constexpr (L::D == 2) {
    constexpr int TX = 64, TY = 16;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    hipLaunchKernelGGL((k_mmfd_plane<L, EQ, THREE, THREE_ST, TX, TY, T>), dim3(tx * ty), dim3(256),
                       0, st, cur, prev, out, nx, ny, tx, tx * ty, kc, bc);
  } else if constexpr (L::D == 3 && EQ == kNSE && !THREE_ST && L::id == 4) {
    return launch_nse3d_pp<T>(c, g, cur, prev, out, st);
  } else {
    constexpr int TX = 32, TY = (THREE_ST && sizeof(T) == 8) ? 4 : 8;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    const int zc = nz >= 64 ? 32 : nz;
    const int tz = (nz + zc - 1) / zc;
    hipLaunchKernelGGL((k_mmfd_3d<L, EQ, THREE, THREE_ST, TX, TY, T>), dim3(tx * ty * tz),
                       dim3(256), 0, st, cur, prev, out, nx, ny, nz, tx, ty, zc, tx * ty * tz, kc);
  }
  return hipGetLastError();
}

template <class L, int EQ, typename T>
hipError_t launch_levels(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                         const DirBC &bc, hipStream_t st) {
  if (!c.three) return launch_cfg<L, EQ, false, false, T>(c, g, cur, prev, out, bc, st);
  if (!c.three_stencil) return launch_cfg<L, EQ, true, false, T>(c, g, cur, prev, out, bc, st);
  return launch_cfg<L, EQ, true, true, T>(c, g, cur, prev, out, bc, st);
}

template <class L, typename T>
hipError_t launch_eq(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                     const DirBC &bc, hipStream_t st) {
  switch (c.eq) {
    case kLCDE: return launch_levels<L, kLCDE, T>(c, g, cur, prev, out, bc, st);
    case kBurgers: return launch_levels<L, kBurgers, T>(c, g, cur, prev, out, bc, st);
    case kNSE:
      if constexpr (L::D >= 2) return launch_levels<L, kNSE, T>(c, g, cur, prev, out, bc, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
hipError_t launch_res(const Consts &c, const Grid &g, T *a, T *b, T *cc, int64_t nsteps,
                      hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0];
  const size_t bytes = (size_t)(3 + 2 * Rec<L, EQ>::NR) * nx * sizeof(T);
  auto fn = k_mmfd_1d_resident<L, EQ, THREE, THREE_ST, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(1), dim3(1024), bytes, st, a, b, cc, nx, nsteps, kc);
  return hipGetLastError();
}

}  // namespace

bool mmfd_1d_resident_fits(const Consts &c, const Grid &g, int elem_bytes) {
  if (c.dim != 1 || c.eq == kNSE) return false;
  const int nr = c.eq == kLCDE ? 1 : 2;
  return (size_t)(3 + 2 * nr) * g.n[0] * elem_bytes <= (size_t)kResidentBytes;
}

template <typename T>
hipError_t launch_mmfd_1d_resident(const Consts &c, const Grid &g, T *a, T *b, T *cbuf,
                                   int64_t nsteps, hipStream_t st) {
  using L = LatD1Q3;
  const bool three = c.three, ts = c.three_stencil;
  if (c.eq == kLCDE) {
    if (!three) return launch_res<L, kLCDE, false, false, T>(c, g, a, b, cbuf, nsteps, st);
    if (!ts) return launch_res<L, kLCDE, true, false, T>(c, g, a, b, cbuf, nsteps, st);
    return launch_res<L, kLCDE, true, true, T>(c, g, a, b, cbuf, nsteps, st);
  }
  if (!three) return launch_res<L, kBurgers, false, false, T>(c, g, a, b, cbuf, nsteps, st);
  if (!ts) return launch_res<L, kBurgers, true, false, T>(c, g, a, b, cbuf, nsteps, st);
  return launch_res<L, kBurgers, true, true, T>(c, g, a, b, cbuf, nsteps, st);
}

template <typename T>
hipError_t launch_mmfd_step(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                            int tb_depth, hipStream_t st, const DirBC *bcp) {
  (void)tb_depth;
  DirBC bc{};
  if (bcp) bc = *bcp;
  // the Dirichlet override lives in the 2D scalar plane kernel only
  if (bc.on && (c.dim != 2 || c.eq == kNSE)) return hipErrorInvalidValue;
  switch (c.lattice) {
    case 1: return launch_eq<LatD1Q3, T>(c, g, cur, prev, out, bc, st);
    case 2: return launch_eq<LatD2Q5, T>(c, g, cur, prev, out, bc, st);
    case 3: return launch_eq<LatD2Q9, T>(c, g, cur, prev, out, bc, st);
    case 4: return launch_eq<LatD3Q19, T>(c, g, cur, prev, out, bc, st);
    case 5: return launch_eq<LatD2Q5II, T>(c, g, cur, prev, out, bc, st);
    case 6: return launch_eq<LatD3Q7, T>(c, g, cur, prev, out, bc, st);
    case 7: return launch_eq<LatD3Q9, T>(c, g, cur, prev, out, bc, st);
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <class L, typename T>
hipError_t picard_l(const Consts &c, const Grid &g, const T *x, const T *R, T *out, double A0,
                    double dd, double th1, double inv_den, double *part, int *rows,
                    hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  PicardEp<T> pe{R, (T)A0, (T)dd, (T)th1, (T)inv_den, nullptr};
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  if constexpr (L::D == 1) {
    constexpr int TX = 1024, TY = 1;
    const int tx = (nx + TX - 1) / TX;
    if (part && tx <= kReduceBlocks) {  // one row of residual sums per workgroup
      pe.part = part;
      *rows = tx;
    }
    hipLaunchKernelGGL((k_picard_plane<L, true, TX, TY, T>), dim3(tx), dim3(256), 0, st, x, out,
                       nx, 1, tx, tx, kc, pe);
  } else {
    constexpr int TX = 64, TY = 16;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    const int ty2 = (ny + 2 * TY - 1) / (2 * TY);
    if (part && tx * ty <= kReduceBlocks) {
      pe.part = part;
      *rows = tx * ty;
    } else if (part && tx * ty2 <= kReduceBlocks) {  // taller tiles: one row per workgroup
      pe.part = part;
      *rows = tx * ty2;
      hipLaunchKernelGGL((k_picard_plane<L, true, TX, 2 * TY, T>), dim3(tx * ty2), dim3(256), 0,
                         st, x, out, nx, ny, tx, tx * ty2, kc, pe);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((k_picard_plane<L, true, TX, TY, T>), dim3(tx * ty), dim3(256), 0, st, x,
                       out, nx, ny, tx, tx * ty, kc, pe);
  }
  return hipGetLastError();
}

// the 2D NSE: the persistent tile kernel of the explicit step with the
// per-field update at the store (the explicit step's launch shape)
template <class L, typename T>
hipError_t picard_nse_l(const Consts &c, const Grid &g, const T *x, const T *R, T *out,
                        const double *A0, const double *dd, double th1, const double *inv_den,
                        double *part, int *rows, hipStream_t st, bool rhs = false,
                        double th = 0.0) {
  const KC<T> kc = make_kc<T>(c);
  PicardNse<T> pe{};
  pe.R = R;
  pe.th1 = (T)th1;
  pe.th = (T)th;
  pe.rhs = rhs ? 1 : 0;
  for (int q = 0; q < Rec<L, kNSE>::NF; ++q) {
    pe.A0[q] = (T)A0[q];
    pe.dd[q] = dd ? (T)dd[q] : (T)0;
    pe.inv_den[q] = inv_den ? (T)inv_den[q] : (T)0;
  }
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  constexpr int TX = 64, TY = sizeof(T) == 4 ? 16 : 4;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const int ntiles = tx * ty;
  constexpr int per_cu = (int)((160 * 1024) / sizeof(typename PfTile<L, false, false, TX, TY, T>::Lds));
  constexpr int groups = kNumCUs * (per_cu < 1 ? 1 : per_cu);
  const int grid = ntiles < groups ? ntiles : groups;
  // the residual sums ride along when the workgroups' rows fit the scratch
  if (part && grid <= kReduceBlocks) {
    pe.part = part;
    *rows = grid;
  }
  const bool fast = nx >= TX + 2 && ny >= TY + 2;
  if (pe.part) {
    if (fast)
      hipLaunchKernelGGL((k_nse_plane_pp<L, false, false, TX, TY, true, T, true, true>),
                         dim3(grid), dim3(256), 0, st, x, nullptr, out, nx, ny, tx, ntiles, kc, pe);
    else
      hipLaunchKernelGGL((k_nse_plane_pp<L, false, false, TX, TY, false, T, true, true>),
                         dim3(grid), dim3(256), 0, st, x, nullptr, out, nx, ny, tx, ntiles, kc, pe);
  } else if (fast) {
    hipLaunchKernelGGL((k_nse_plane_pp<L, false, false, TX, TY, true, T, true>), dim3(grid),
                       dim3(256), 0, st, x, nullptr, out, nx, ny, tx, ntiles, kc, pe);
  } else {
    hipLaunchKernelGGL((k_nse_plane_pp<L, false, false, TX, TY, false, T, true>), dim3(grid),
                       dim3(256), 0, st, x, nullptr, out, nx, ny, tx, ntiles, kc, pe);
  }
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t launch_picard_rhs_step(const Consts &c, const Grid &g, const T *x, T *R,
                                  const double *A0, double th, double th1, hipStream_t st) {
  if (c.three || c.eq != kNSE || c.dim != 2) return hipErrorInvalidValue;
  int rows = 0;
  switch (c.lattice) {
    case 2:
      return picard_nse_l<LatD2Q5, T>(c, g, x, nullptr, R, A0, nullptr, th1, nullptr, nullptr,
                                      &rows, st, true, th);
    case 3:
      return picard_nse_l<LatD2Q9, T>(c, g, x, nullptr, R, A0, nullptr, th1, nullptr, nullptr,
                                      &rows, st, true, th);
    case 5:
      return picard_nse_l<LatD2Q5II, T>(c, g, x, nullptr, R, A0, nullptr, th1, nullptr, nullptr,
                                        &rows, st, true, th);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_picard_sweep(const Consts &c, const Grid &g, const T *x, const T *R, T *out,
                               const double *A0, const double *dd, double th1,
                               const double *inv_den, double *part, int *rows, hipStream_t st) {
  *rows = 0;
  if (c.three) return hipErrorInvalidValue;
  if (c.eq == kNSE) {
    if (c.dim != 2) return hipErrorInvalidValue;
    switch (c.lattice) {
      case 2:
        return picard_nse_l<LatD2Q5, T>(c, g, x, R, out, A0, dd, th1, inv_den, part, rows, st);
      case 3:
        return picard_nse_l<LatD2Q9, T>(c, g, x, R, out, A0, dd, th1, inv_den, part, rows, st);
      case 5:
        return picard_nse_l<LatD2Q5II, T>(c, g, x, R, out, A0, dd, th1, inv_den, part, rows, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (c.eq != kBurgers) return hipErrorInvalidValue;
  switch (c.lattice) {
    case 1:
      return picard_l<LatD1Q3, T>(c, g, x, R, out, A0[0], dd[0], th1, inv_den[0], part, rows, st);
    case 2:
      return picard_l<LatD2Q5, T>(c, g, x, R, out, A0[0], dd[0], th1, inv_den[0], part, rows, st);
    case 3:
      return picard_l<LatD2Q9, T>(c, g, x, R, out, A0[0], dd[0], th1, inv_den[0], part, rows, st);
    case 5:
      return picard_l<LatD2Q5II, T>(c, g, x, R, out, A0[0], dd[0], th1, inv_den[0], part, rows,
                                    st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_picard_rhs_step<float>(const Consts &, const Grid &, const float *,
                                                  float *, const double *, double, double,
                                                  hipStream_t);
template hipError_t launch_picard_rhs_step<double>(const Consts &, const Grid &, const double *,
                                                   double *, const double *, double, double,
                                                   hipStream_t);
template hipError_t launch_picard_sweep<float>(const Consts &, const Grid &, const float *,
                                               const float *, float *, const double *,
                                               const double *, double, const double *, double *,
                                               int *, hipStream_t);
template hipError_t launch_picard_sweep<double>(const Consts &, const Grid &, const double *,
                                                const double *, double *, const double *,
                                                const double *, double, const double *, double *,
                                                int *, hipStream_t);

template hipError_t launch_mmfd_step<float>(const Consts &, const Grid &, const float *,
                                            const float *, float *, int, hipStream_t,
                                            const DirBC *);
template hipError_t launch_mmfd_step<double>(const Consts &, const Grid &, const double *,
                                             const double *, double *, int, hipStream_t,
                                             const DirBC *);
template hipError_t launch_mmfd_1d_resident<float>(const Consts &, const Grid &, float *, float *,
                                                   float *, int64_t, hipStream_t);
template hipError_t launch_mmfd_1d_resident<double>(const Consts &, const Grid &, double *,
                                                    double *, double *, int64_t, hipStream_t);

}  // namespace mfd
