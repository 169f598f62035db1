// Whole-run kernels for small periodic 1D grids (D1Q3, two-level linear CDE,
// MMFD and MesoFD form): NW wavefronts (one per SIMD) hold all 64 NW NPL nodes
// in registers (lane l of wavefront w owns the NPL nodes from (64 w + l) NPL
// on) and run every time step with one barrier and no other LDS traffic than
// the two end nodes of each wavefront: the neighbours a lane's block needs
// from the lanes beside it come by DPP lane shifts, and the first and last
// lanes take theirs from the LDS slots the neighbouring wavefronts wrote
// (double-buffered by step parity, so one barrier a step suffices).  Each
// node update is the single-step kernels' node function (mmfd_node,
// mesofd_pops), so results equal them value for value.  On return ga holds
// the last level, gb the one before it and, for MesoFD, pop the last step's
// populations.
#include "mesofd_node.h"
#include "mmfd_node.h"

namespace mfd {

namespace {

// value of lane l - 1 / l + 1; the first / last lane keeps `old`
template <int CTRL>
__device__ __forceinline__ float shift(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double shift(double old, double v) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffff), (int)(b & 0xffffffff), CTRL,
                                             0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kFromLeft = 0x138;   // wave_shr:1
constexpr int kFromRight = 0x130;  // wave_shl:1

}  // namespace

template <int NW, int NPL, bool MESO, typename T>
__global__ __launch_bounds__(64 * NW) void k_1d_wave(T *__restrict__ ga, T *__restrict__ gb,
                                                     T *__restrict__ pop, int64_t nsteps,
                                                     KC<T> kc) {
  using L = LatD1Q3;
  constexpr int NX = 64 * NW * NPL;
  __shared__ T edge[2][2][NW];  // [step parity][first, last node][wavefront]
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wl = (w + NW - 1) % NW, wr = (w + 1) % NW;
  const int i0 = (int)threadIdx.x * NPL;
  T phi[NPL], prv[NPL];
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    phi[k] = ga[i0 + k];
    prv[k] = gb[i0 + k];
  }
  auto step = [&](int par, bool last) {
    if (lane == 0) edge[par][0][w] = phi[0];
    if (lane == 63) edge[par][1][w] = phi[NPL - 1];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    const T left = shift<kFromLeft>(edge[par][1][wl], phi[NPL - 1]);
    const T right = shift<kFromRight>(edge[par][0][wr], phi[0]);
    T nxt[NPL];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      auto at = [&](int, int, int, int dx) {
        const int j = k + dx;
        return j < 0 ? left : (j >= NPL ? right : phi[j]);
      };
      auto ath = [&](int, int, int, int) { return T(0); };
      if constexpr (MESO) {
        T fo[L::Q], m[1];
        mesofd_pops<L, kLCDE, false>(at, ath, (const T *)nullptr, false, fo, kc);
        moments_of<L, kLCDE>(fo, m);
        nxt[k] = m[0];
        if (last) {
#pragma unroll
          for (int j = 0; j < L::Q; ++j) pop[j * NX + i0 + k] = fo[j];
        }
      } else {
        T cc[1] = {phi[k]}, pc[1] = {T(0)}, oc[1];
        mmfd_node<L, kLCDE, false, false, T>(at, ath, cc, pc, oc, kc);
        nxt[k] = oc[0];
      }
    }
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      prv[k] = phi[k];
      phi[k] = nxt[k];
    }
  };
  int64_t s = 0;
#pragma unroll 1
  for (; s + 1 < nsteps; ++s) step((int)(s & 1), false);
  if (nsteps > 0) step((int)(s & 1), true);
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    ga[i0 + k] = phi[k];
    gb[i0 + k] = prv[k];
  }
}

// ------------------------------------------------------------ host side
bool wave1d_applies(const Consts &c, const Grid &g) {
  if (c.dim != 1 || c.lattice != 1 || c.eq != kLCDE || c.three) return false;
  const int64_t n = g.n[0];
  return n == 64 || n == 128 || n == 256 || n == 512 || n == 1024;
}

namespace {
template <int NW, int NPL, bool MESO, typename T>
hipError_t wave_cfg(const Consts &c, T *ga, T *gb, T *pop, int64_t nsteps, hipStream_t st) {
  hipLaunchKernelGGL((k_1d_wave<NW, NPL, MESO, T>), dim3(1), dim3(64 * NW), 0, st, ga, gb, pop,
                     nsteps, make_kc<T>(c));
  return hipGetLastError();
}

// one wavefront per SIMD once the grid fills four
template <bool MESO, typename T>
hipError_t wave_n(const Consts &c, const Grid &g, T *ga, T *gb, T *pop, int64_t nsteps,
                  hipStream_t st) {
  switch (g.n[0]) {
    case 64: return wave_cfg<1, 1, MESO, T>(c, ga, gb, pop, nsteps, st);
    case 128: return wave_cfg<2, 1, MESO, T>(c, ga, gb, pop, nsteps, st);
    case 256: return wave_cfg<4, 1, MESO, T>(c, ga, gb, pop, nsteps, st);
    case 512: return wave_cfg<4, 2, MESO, T>(c, ga, gb, pop, nsteps, st);
    case 1024: return wave_cfg<4, 4, MESO, T>(c, ga, gb, pop, nsteps, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

template <typename T>
hipError_t launch_1d_wave(const Consts &c, const Grid &g, bool mesofd, T *ga, T *gb, T *pop,
                          int64_t nsteps, hipStream_t st) {
  if (!wave1d_applies(c, g)) return hipErrorInvalidValue;
  if (mesofd) return wave_n<true, T>(c, g, ga, gb, pop, nsteps, st);
  return wave_n<false, T>(c, g, ga, gb, pop, nsteps, st);
}

template hipError_t launch_1d_wave<float>(const Consts &, const Grid &, bool, float *, float *,
                                          float *, int64_t, hipStream_t);
template hipError_t launch_1d_wave<double>(const Consts &, const Grid &, bool, double *, double *,
                                           double *, int64_t, hipStream_t);

}  // namespace mfd
