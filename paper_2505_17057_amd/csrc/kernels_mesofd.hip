// MesoFD step kernels: the population form of the scheme, Eq. (2-1) /
// (3layer-1),
//   f_j(x, t+dt) = sum_k a_k f_j^eq(x + k e_j, t) + sum_k ah_k f_j^eq(x + k e_j, t-dt),
// k in (-1, 0, +1) order, level t first, zero coefficients skipped; f^eq at
// level t is the EDF of the moments of the populations (Eq. (2-1-1):
// phi = sum_j f_j, j_a = sum_j e_ja f_j, lattice order), at level t - dt the
// EDF of the stored moments of that level.
//
// The new populations depend on the old ones only through their moments.  So
// each launch reads the moments of level t (one to d+1 fields, not b
// populations), writes the b populations of level t+1 and, summed from the
// same values in registers in lattice order, the moments of level t+1: the
// input of the next launch.  Those sums are the ones a read-back of the
// populations would give, value for value.
//
// Same tiling as the MMFD kernels: EDF records of the tile plus a one-node
// halo in LDS, then every interior node evaluates its b directions.

#include "mesofd_node.h"

namespace mfd {

__device__ __forceinline__ int wrapm(int i, int n) {
  if (i < 0) {
    i += n;
    if (i < 0) i = ((i % n) + n) % n;
  } else if (i >= n) {
    i -= n;
    if (i >= n) i %= n;
  }
  return i;
}

__device__ __forceinline__ int xcd_remap_m(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_mesofd_plane(const T *__restrict__ mom,
                                                      const T *__restrict__ prev_mom,
                                                      T *__restrict__ pop_out,
                                                      T *__restrict__ mom_out, int nx, int ny,
                                                      int tiles_x, int ntiles, KC<T> kc) {
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR, NF = R::NF;
  constexpr int HYL = L::D >= 2 ? 1 : 0;
  constexpr int HX = TX + 2, HY = TY + 2 * HYL;
  __shared__ T rec[NR][HY][HX];
  __shared__ T hrec[THREE_ST ? NR : 1][THREE_ST ? HY : 1][THREE_ST ? HX : 1];
  const int tile = xcd_remap_m(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  const int64_t N = (int64_t)nx * ny;

  for (int i = threadIdx.x; i < HX * HY; i += 256) {
    const int lx = i % HX, ly = i / HX;
    const int gx = wrapm(x0 - 1 + lx, nx), gy = wrapm(y0 - HYL + ly, ny);
    const int64_t gi = (int64_t)gy * nx + gx;
    T m[NF], r[NR];
#pragma unroll
    for (int f = 0; f < NF; ++f) m[f] = mom[f * N + gi];
    make_record<L, EQ>(m, r, kc);
#pragma unroll
    for (int k = 0; k < NR; ++k) rec[k][ly][lx] = r[k];
    if constexpr (THREE_ST) {
#pragma unroll
      for (int f = 0; f < NF; ++f) m[f] = prev_mom[f * N + gi];
      make_record<L, EQ>(m, r, kc);
#pragma unroll
      for (int k = 0; k < NR; ++k) hrec[k][ly][lx] = r[k];
    }
  }
  __syncthreads();

  for (int i = threadIdx.x; i < TX * TY; i += 256) {
    const int lx = i % TX, ly = i / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= nx || gy >= ny) continue;
    const int cx = lx + 1, cy = ly + HYL;
    const int64_t gi = (int64_t)gy * nx + gx;
    auto at = [&](int k, int, int dy, int dx) { return rec[k][cy + dy][cx + dx]; };
    auto ath = [&](int k, int, int dy, int dx) {
      if constexpr (THREE_ST) return hrec[k][cy + dy][cx + dx];
      else return T(0);
    };
    T hc[NR];
    if constexpr (THREE && !THREE_ST) {
      T m[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) m[f] = prev_mom[f * N + gi];
      make_record<L, EQ>(m, hc, kc);
    }
    mesofd_node<L, EQ, THREE_ST, T>(at, ath, hc, THREE, pop_out, mom_out, N, gi, kc);
  }
}

template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_mesofd_3d(const T *__restrict__ mom,
                                                   const T *__restrict__ prev_mom,
                                                   T *__restrict__ pop_out,
                                                   T *__restrict__ mom_out, int nx, int ny,
                                                   int nz, int tiles_x, int tiles_y, int zchunk,
                                                   int ntiles, KC<T> kc) {
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR, NF = R::NF;
  constexpr int HX = TX + 2, HY = TY + 2;
  __shared__ T rec[3][NR][HY][HX];
  __shared__ T hrec[THREE_ST ? 3 : 1][THREE_ST ? NR : 1][THREE_ST ? HY : 1][THREE_ST ? HX : 1];
  const int tile = xcd_remap_m(blockIdx.x, ntiles);
  const int txy = tiles_x * tiles_y;
  const int tz = tile / txy, trem = tile % txy;
  const int x0 = (trem % tiles_x) * TX, y0 = (trem / tiles_x) * TY;
  const int z0 = tz * zchunk, z1 = min(nz, z0 + zchunk);
  const int64_t N = (int64_t)nx * ny * nz;

  auto load_plane = [&](int z, int slot) {
    const int gz = wrapm(z, nz);
    for (int i = threadIdx.x; i < HX * HY; i += 256) {
      const int lx = i % HX, ly = i / HX;
      const int gx = wrapm(x0 - 1 + lx, nx), gy = wrapm(y0 - 1 + ly, ny);
      const int64_t gi = ((int64_t)gz * ny + gy) * nx + gx;
      T m[NF], r[NR];
#pragma unroll
      for (int f = 0; f < NF; ++f) m[f] = mom[f * N + gi];
      make_record<L, EQ>(m, r, kc);
#pragma unroll
      for (int k = 0; k < NR; ++k) rec[slot][k][ly][lx] = r[k];
      if constexpr (THREE_ST) {
#pragma unroll
        for (int f = 0; f < NF; ++f) m[f] = prev_mom[f * N + gi];
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
      T hc[NR];
      if constexpr (THREE && !THREE_ST) {
        T m[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) m[f] = prev_mom[f * N + gi];
        make_record<L, EQ>(m, hc, kc);
      }
      mesofd_node<L, EQ, THREE_ST, T>(at, ath, hc, THREE, pop_out, mom_out, N, gi, kc);
    }
    __syncthreads();
  }
}

// ------------------------------------------------ LDS-resident 1D run
// One workgroup holds every level of a 1D grid in LDS and runs all steps (the
// 1024-node workload is latency-bound): each step evaluates all b
// populations of every node with the same node function as the tiled kernel,
// into LDS, sums their moments into the next level, and on the last step
// writes the populations to `pop`.  ga / gb: moments of levels t and t - dt
// in, of the last two levels out.
constexpr int kMesoResidentBytes = 96 * 1024;

template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
__global__ __launch_bounds__(1024) void k_mesofd_1d_resident(T *__restrict__ ga,
                                                             T *__restrict__ gb,
                                                             T *__restrict__ pop, int nx,
                                                             int64_t nsteps, KC<T> kc) {
  extern __shared__ unsigned char smem_m1[];
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR;
  static_assert(R::NF == 1, "1D equations carry one moment");
  // level k at L0 + k * nx (arithmetic on the LDS base keeps every access a
  // local-data-share access)
  T *const L0 = (T *)smem_m1;
  auto lev = [&](int k) { return L0 + k * nx; };
  T *rec = (T *)smem_m1 + 3 * nx;      // NR * nx
  T *hrec = rec + NR * nx;             // NR * nx (older level with a stencil)
  T *pl = hrec + NR * nx;              // Q * nx populations of the step
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    lev(0)[i] = ga[i];
    lev(1)[i] = gb[i];
  }
  __syncthreads();
  // the linear CDE's record is the moment itself (one barrier per step)
  constexpr bool LIN = EQ == kLCDE;
  int ic = 0, ip = 1, io = 2;
  for (int64_t s = 0; s < nsteps; ++s) {
    if constexpr (!LIN) {
      for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        T m[1] = {lev(ic)[i]}, r[NR];
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
        const int j = i + dx;
        return j < 0 ? j + nx : (j >= nx ? j - nx : j);
      };
      auto at = [&](int k, int, int, int dx) { return rc[k * nx + idx(dx)]; };
      auto ath = [&](int k, int, int, int dx) {
        if constexpr (THREE_ST) return rh[k * nx + idx(dx)];
        else return T(0);
      };
      T hc[NR];
      if constexpr (THREE && !THREE_ST) {
        T m[1] = {lev(ip)[i]};
        make_record<L, EQ>(m, hc, kc);
      }
      if (s + 1 < nsteps)  // populations of the step stay in LDS
        mesofd_node<L, EQ, THREE_ST, T>(at, ath, hc, THREE, pl, lev(io), nx, i, kc);
      else  // the last step's go to HBM
        mesofd_node<L, EQ, THREE_ST, T>(at, ath, hc, THREE, pop, lev(io), nx, i, kc);
    }
    __syncthreads();
    const int t = ip;
    ip = ic;
    ic = io;
    io = t;
  }
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    ga[i] = lev(ic)[i];
    gb[i] = lev(ip)[i];
  }
}

// ------------------------------------------------ init / moments kernels
template <class L, int EQ, typename T>
__global__ __launch_bounds__(256) void k_init_pop(const T *__restrict__ mom, T *__restrict__ pop,
                                                  int64_t N, KC<T> kc) {
  using R = Rec<L, EQ>;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    T m[R::NF], r[R::NR];
#pragma unroll
    for (int f = 0; f < R::NF; ++f) m[f] = mom[f * N + i];
    make_record<L, EQ>(m, r, kc);
    static_for<L::Q>([&](auto JI) {
      constexpr int J = decltype(JI)::value;
      pop[J * N + i] = g_dir<L, EQ, J>(r, kc);
    });
  }
}

template <class L, int EQ, typename T>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ pop, T *__restrict__ mom,
                                                 int64_t N) {
  using R = Rec<L, EQ>;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    T m[R::NF];
    pop_moments<L, EQ>(pop, N, i, m);
#pragma unroll
    for (int f = 0; f < R::NF; ++f) mom[f * N + i] = m[f];
  }
}

// ------------------------------------------------------------ launchers
namespace {

template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
hipError_t meso_cfg(const Consts &c, const Grid &g, const T *mc, const T *pm, T *po, T *mo,
                    hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1], nz = (int)g.n[2];
  if constexpr (L::D == 1) {
    constexpr int TX = 1024;
    const int tx = (nx + TX - 1) / TX;
    hipLaunchKernelGGL((k_mesofd_plane<L, EQ, THREE, THREE_ST, TX, 1, T>), dim3(tx), dim3(256), 0,
                       st, mc, pm, po, mo, nx, 1, tx, tx, kc);
  } else if constexpr (L::D == 2) {
    constexpr int TX = 64, TY = EQ == kNSE ? 8 : 16;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    hipLaunchKernelGGL((k_mesofd_plane<L, EQ, THREE, THREE_ST, TX, TY, T>), dim3(tx * ty),
                       dim3(256), 0, st, mc, pm, po, mo, nx, ny, tx, tx * ty, kc);
  } else {
    constexpr int TX = 32, TY = (THREE_ST && sizeof(T) == 8) ? 4 : 8;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    const int zc = nz >= 64 ? 32 : nz;
    const int tz = (nz + zc - 1) / zc;
    hipLaunchKernelGGL((k_mesofd_3d<L, EQ, THREE, THREE_ST, TX, TY, T>), dim3(tx * ty * tz),
                       dim3(256), 0, st, mc, pm, po, mo, nx, ny, nz, tx, ty, zc, tx * ty * tz, kc);
  }
  return hipGetLastError();
}

template <class L, int EQ, typename T>
hipError_t meso_levels(const Consts &c, const Grid &g, const T *mc, const T *pm, T *po, T *mo,
                       hipStream_t st) {
  if (!c.three) return meso_cfg<L, EQ, false, false, T>(c, g, mc, pm, po, mo, st);
  if (!c.three_stencil) return meso_cfg<L, EQ, true, false, T>(c, g, mc, pm, po, mo, st);
  return meso_cfg<L, EQ, true, true, T>(c, g, mc, pm, po, mo, st);
}

template <class L, typename T>
hipError_t meso_eq(const Consts &c, const Grid &g, const T *mc, const T *pm, T *po, T *mo,
                   hipStream_t st) {
  switch (c.eq) {
    case kLCDE: return meso_levels<L, kLCDE, T>(c, g, mc, pm, po, mo, st);
    case kBurgers: return meso_levels<L, kBurgers, T>(c, g, mc, pm, po, mo, st);
    case kNSE:
      if constexpr (L::D >= 2) return meso_levels<L, kNSE, T>(c, g, mc, pm, po, mo, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

inline int grid_blocks(int64_t N) {
  int64_t b = (N + 255) / 256;
  return (int)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

template <class L, typename T>
hipError_t init_eq(const Consts &c, const Grid &g, const T *mom, T *pop, hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  switch (c.eq) {
    case kLCDE:
      hipLaunchKernelGGL((k_init_pop<L, kLCDE, T>), dim3(grid_blocks(g.N)), dim3(256), 0, st, mom,
                         pop, g.N, kc);
      break;
    case kBurgers:
      hipLaunchKernelGGL((k_init_pop<L, kBurgers, T>), dim3(grid_blocks(g.N)), dim3(256), 0, st,
                         mom, pop, g.N, kc);
      break;
    case kNSE:
      if constexpr (L::D >= 2) {
        hipLaunchKernelGGL((k_init_pop<L, kNSE, T>), dim3(grid_blocks(g.N)), dim3(256), 0, st, mom,
                           pop, g.N, kc);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class L, typename T>
hipError_t mom_eq(const Consts &c, const Grid &g, const T *pop, T *mom, hipStream_t st) {
  if (c.eq == kNSE) {
    if constexpr (L::D >= 2) {
      hipLaunchKernelGGL((k_moments<L, kNSE, T>), dim3(grid_blocks(g.N)), dim3(256), 0, st, pop,
                         mom, g.N);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((k_moments<L, kLCDE, T>), dim3(grid_blocks(g.N)), dim3(256), 0, st, pop, mom,
                     g.N);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_mesofd_step(const Consts &c, const Grid &g, const T *mom, const T *prev_mom,
                              T *pop_out, T *mom_out, hipStream_t st) {
  switch (c.lattice) {
    case 1: return meso_eq<LatD1Q3, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    case 2: return meso_eq<LatD2Q5, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    case 3: return meso_eq<LatD2Q9, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    case 4: return meso_eq<LatD3Q19, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    case 5: return meso_eq<LatD2Q5II, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    case 6: return meso_eq<LatD3Q7, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    case 7: return meso_eq<LatD3Q9, T>(c, g, mom, prev_mom, pop_out, mom_out, st);
    default: return hipErrorInvalidValue;
  }
}

bool mesofd_1d_resident_fits(const Consts &c, const Grid &g, int elem) {
  if (c.dim != 1 || c.eq == kNSE) return false;
  const int nr = c.eq == kLCDE ? 1 : 2;
  return (size_t)(3 + 2 * nr + 3) * g.n[0] * elem <= (size_t)kMesoResidentBytes;
}

namespace {
template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
hipError_t meso_res(const Consts &c, const Grid &g, T *ga, T *gb, T *pop, int64_t nsteps,
                    hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0];
  const size_t bytes = (size_t)(3 + 2 * Rec<L, EQ>::NR + L::Q) * nx * sizeof(T);
  auto fn = k_mesofd_1d_resident<L, EQ, THREE, THREE_ST, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(1), dim3(1024), bytes, st, ga, gb, pop, nx, nsteps, kc);
  return hipGetLastError();
}
template <int EQ, typename T>
hipError_t meso_res_levels(const Consts &c, const Grid &g, T *ga, T *gb, T *pop, int64_t n,
                           hipStream_t st) {
  using L = LatD1Q3;
  if (!c.three) return meso_res<L, EQ, false, false, T>(c, g, ga, gb, pop, n, st);
  if (!c.three_stencil) return meso_res<L, EQ, true, false, T>(c, g, ga, gb, pop, n, st);
  return meso_res<L, EQ, true, true, T>(c, g, ga, gb, pop, n, st);
}
}  // namespace

template <typename T>
hipError_t launch_mesofd_1d_resident(const Consts &c, const Grid &g, T *ga, T *gb, T *pop,
                                     int64_t nsteps, hipStream_t st) {
  if (c.eq == kLCDE) return meso_res_levels<kLCDE, T>(c, g, ga, gb, pop, nsteps, st);
  if (c.eq == kBurgers) return meso_res_levels<kBurgers, T>(c, g, ga, gb, pop, nsteps, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_init_populations(const Consts &c, const Grid &g, const T *mom, T *pop,
                                   hipStream_t st) {
  switch (c.lattice) {
    case 1: return init_eq<LatD1Q3, T>(c, g, mom, pop, st);
    case 2: return init_eq<LatD2Q5, T>(c, g, mom, pop, st);
    case 3: return init_eq<LatD2Q9, T>(c, g, mom, pop, st);
    case 4: return init_eq<LatD3Q19, T>(c, g, mom, pop, st);
    case 5: return init_eq<LatD2Q5II, T>(c, g, mom, pop, st);
    case 6: return init_eq<LatD3Q7, T>(c, g, mom, pop, st);
    case 7: return init_eq<LatD3Q9, T>(c, g, mom, pop, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_moments(const Consts &c, const Grid &g, const T *pop, T *mom, hipStream_t st) {
  switch (c.lattice) {
    case 1: return mom_eq<LatD1Q3, T>(c, g, pop, mom, st);
    case 2: return mom_eq<LatD2Q5, T>(c, g, pop, mom, st);
    case 3: return mom_eq<LatD2Q9, T>(c, g, pop, mom, st);
    case 4: return mom_eq<LatD3Q19, T>(c, g, pop, mom, st);
    case 5: return mom_eq<LatD2Q5II, T>(c, g, pop, mom, st);
    case 6: return mom_eq<LatD3Q7, T>(c, g, pop, mom, st);
    case 7: return mom_eq<LatD3Q9, T>(c, g, pop, mom, st);
    default: return hipErrorInvalidValue;
  }
}

#define MFD_INST(T)                                                                               \
  template hipError_t launch_mesofd_step<T>(const Consts &, const Grid &, const T *, const T *,   \
                                            T *, T *, hipStream_t);                               \
  template hipError_t launch_init_populations<T>(const Consts &, const Grid &, const T *, T *,    \
                                                 hipStream_t);                                    \
  template hipError_t launch_moments<T>(const Consts &, const Grid &, const T *, T *, hipStream_t); \
  template hipError_t launch_mesofd_1d_resident<T>(const Consts &, const Grid &, T *, T *, T *,   \
                                                   int64_t, hipStream_t);
MFD_INST(float)
MFD_INST(double)
#undef MFD_INST

}  // namespace mfd
