// NSE step on D3Q19 (two-level, or three-level without an older-level
// stencil), one step per launch, with each node's pair parts F+-_p (Eq. (2-5)
// applied to Eq. (3-3)) evaluated once per node instead of once per
// neighbour that uses them.
//
// A workgroup owns a TX x TY column of the grid and marches it along z over
// a chunk of planes.  The pairs split by their direction: the five with a z
// component need their parts on the planes z - 1, z and z + 1; the four in
// the plane only on plane z.  So the LDS holds the z pairs' parts of three
// planes (a ring) and the in-plane pairs' parts of plane z, each for the tile
// and a one-node halo.  Thread k stages the interior node k (and, for the
// first 2 (TX + TY) + 4 threads, one halo node) and updates that same
// interior node, so the moments of its node at t (and t - dt) stay in its
// registers.  The moments of the plane after next are loaded into registers
// while a plane is updated.  The node update is mmfd_node on pair parts in
// binary64 (results equal the oracle's value for value) and the binary32 pair
// form of nse32_parts / nse32_node in binary32.
#include "mmfd_node.h"

namespace mfd {

namespace {

using L3 = LatD3Q19;

// pair p of D3Q19 (lattice pair order) has a z component
__host__ __device__ constexpr bool zpair(int p) { return L3::E[L3::PR[p]][2] != 0; }
// index of pair p among the z pairs / among the in-plane pairs
__host__ __device__ constexpr int zslot(int p) {
  int k = 0;
  for (int i = 0; i < p; ++i) k += zpair(i) ? 1 : 0;
  return k;
}
__host__ __device__ constexpr int islot(int p) {
  int k = 0;
  for (int i = 0; i < p; ++i) k += zpair(i) ? 0 : 1;
  return k;
}
constexpr int kZP = 5, kIP = 4;  // z pairs, in-plane pairs

}  // namespace

template <bool THREE, int TX, int TY, typename T>
__global__ __launch_bounds__(TX *TY) void k_nse3d_pp(const T *__restrict__ cur,
                                                    const T *__restrict__ prev,
                                                    T *__restrict__ out, int nx, int ny, int nz,
                                                    int tiles_x, int tiles_y, int zchunk,
                                                    int ntiles, KC<T> kc) {
  using Rc = Rec<L3, kNSE>;
  constexpr int NR = Rc::NR, NF = Rc::NF;
  constexpr int HX = TX + 2, HY = TY + 2, NT = TX * TY;
  constexpr int NHALO = 2 * HX + 2 * TY;
  static_assert(NHALO <= NT, "one halo node per thread at most");
  // binary32: the unweighted pair form of nse32_parts / nse32_node
  constexpr bool kF32 = std::is_same<T, float>::value;
  extern __shared__ unsigned char smem_nse3d[];
  // zb[3][2 kZP][HY][HX] then ib[2 kIP][HY][HX]
  T *const zb = reinterpret_cast<T *>(smem_nse3d);
  T *const ib = zb + 3 * 2 * kZP * HY * HX;
  auto zat = [&](int slot, int q, int y, int x) -> T & {
    return zb[((slot * 2 * kZP + q) * HY + y) * HX + x];
  };
  auto iat = [&](int q, int y, int x) -> T & { return ib[(q * HY + y) * HX + x]; };

  const int tile = xcd_remap(blockIdx.x, ntiles);
  const int txy = tiles_x * tiles_y;
  const int tz = tile / txy, trem = tile % txy;
  const int x0 = (trem % tiles_x) * TX, y0 = (trem / tiles_x) * TY;
  const int z0 = tz * zchunk, z1 = min(nz, z0 + zchunk);
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t plane = (int64_t)nx * ny;

  // this thread's nodes: the interior node (slot 0) and maybe one halo node
  const int tid = threadIdx.x;
  int hx[2], hy[2];
  hx[0] = tid % TX + 1;
  hy[0] = tid / TX + 1;
  const bool has_halo = tid < NHALO;
  {
    int k = tid;
    if (k < HX) {
      hx[1] = k, hy[1] = 0;
    } else if ((k -= HX) < HX) {
      hx[1] = k, hy[1] = HY - 1;
    } else if ((k -= HX) < TY) {
      hx[1] = 0, hy[1] = k + 1;
    } else {
      k -= TY;
      hx[1] = HX - 1, hy[1] = (k < TY ? k : 0) + 1;
    }
  }
  int64_t col[2];  // offset of each node's column within a plane
#pragma unroll
  for (int s = 0; s < 2; ++s)
    col[s] = (int64_t)wrapi(y0 - 1 + hy[s], ny) * nx + wrapi(x0 - 1 + hx[s], nx);
  const int gxi = x0 + hx[0] - 1, gyi = y0 + hy[0] - 1;
  const bool upd = gxi < nx && gyi < ny;

  T mc[2][NF] = {}, mn[2][NF] = {}, pc[NF] = {}, pn[NF] = {};
  auto load = [&](int z, T (&m)[2][NF], T (&p)[NF]) {
    const int64_t zo = (int64_t)wrapi(z, nz) * plane;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s == 0 || has_halo) {
#pragma unroll
        for (int f = 0; f < NF; ++f) m[s][f] = cur[f * N + zo + col[s]];
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) p[f] = THREE ? prev[f * N + zo + col[0]] : T(0);
  };
  // binary32: the parts of the thread's own node at plane z stay in
  // registers (own), those of its z pairs at plane z + 1 in ownn
  T own[kF32 ? 2 * L3::P : 1], ownn[kF32 ? 2 * L3::P : 1];
  // the parts of the z pairs (into ring slot `slot`) or of the in-plane pairs;
  // binary32: the own node's also into keep (when given)
  auto stage = [&](const T (&m)[2][NF], int slot, bool zpairs, T *keep) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s == 0 || has_halo) {
        if constexpr (kF32) {
          T g[2 * L3::P];
          nse32_parts<L3>(m[s], g, kc);
          static_for<L3::P>([&](auto PI) {
            constexpr int P = decltype(PI)::value;
            if constexpr (zpair(P)) {
              if (zpairs) {
                zat(slot, 2 * zslot(P), hy[s], hx[s]) = g[2 * P];
                zat(slot, 2 * zslot(P) + 1, hy[s], hx[s]) = g[2 * P + 1];
                if (s == 0 && keep) {
                  keep[2 * P] = g[2 * P];
                  keep[2 * P + 1] = g[2 * P + 1];
                }
              }
            } else {
              if (!zpairs) {
                iat(2 * islot(P), hy[s], hx[s]) = g[2 * P];
                iat(2 * islot(P) + 1, hy[s], hx[s]) = g[2 * P + 1];
                if (s == 0 && keep) {
                  keep[2 * P] = g[2 * P];
                  keep[2 * P + 1] = g[2 * P + 1];
                }
              }
            }
          });
        } else {
          T rec[NR];
          make_record<L3, kNSE>(m[s], rec, kc);
          static_for<L3::P>([&](auto PI) {
            constexpr int P = decltype(PI)::value;
            constexpr int J = L3::PR[P];
            if constexpr (zpair(P)) {
              if (zpairs) {
                zat(slot, 2 * zslot(P), hy[s], hx[s]) = fplus<L3, kNSE, J>(rec, kc);
                zat(slot, 2 * zslot(P) + 1, hy[s], hx[s]) = fminus<L3, kNSE, J>(rec, kc);
              }
            } else {
              if (!zpairs) {
                iat(2 * islot(P), hy[s], hx[s]) = fplus<L3, kNSE, J>(rec, kc);
                iat(2 * islot(P) + 1, hy[s], hx[s]) = fminus<L3, kNSE, J>(rec, kc);
              }
            }
          });
        }
      }
    }
  };

  // ring slot of plane z0 - 1 + k is k % 3
  load(z0 - 1, mn, pn);
  stage(mn, 0, true, nullptr);
  load(z0, mc, pc);
  stage(mc, 1, true, kF32 ? own : nullptr);
  load(z0 + 1, mn, pn);
  for (int z = z0; z < z1; ++z) {
    const int rel = z - z0;
    const int sm = rel % 3, s0 = (rel + 1) % 3, sp = (rel + 2) % 3;
    stage(mc, 0, false, kF32 ? own : nullptr);  // in-plane parts of plane z
    stage(mn, sp, true, kF32 ? ownn : nullptr);  // z parts of plane z + 1
    // moments of plane z + 1 for the next pass; plane z + 2 in flight
    T cc[NF], pcc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      cc[f] = mc[0][f];
      pcc[f] = pc[f];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int f = 0; f < NF; ++f) mc[s][f] = mn[s][f];
#pragma unroll
    for (int f = 0; f < NF; ++f) pc[f] = pn[f];
    if (z + 1 < z1) load(z + 2, mn, pn);
    __syncthreads();
    if (upd) {
      // the node's place in each ring slot and in the in-plane parts; every
      // access below is one of these plus a compile-time offset
      const int ctr = hy[0] * HX + hx[0];
      const T *const zpm = zb + sm * 2 * kZP * HY * HX + ctr;
      const T *const zp0 = zb + s0 * 2 * kZP * HY * HX + ctr;
      const T *const zpp = zb + sp * 2 * kZP * HY * HX + ctr;
      const T *const ipc = ib + ctr;
      auto at = [&](int q, int dz, int dy, int dx) {
        const int p = q >> 1, h = q & 1;
        const int off = dy * HX + dx;
        if (zpair(p)) {
          const T *b = dz == 0 ? zp0 : (dz > 0 ? zpp : zpm);
          return b[(2 * zslot(p) + h) * HY * HX + off];
        }
        return ipc[(2 * islot(p) + h) * HY * HX + off];
      };
      auto ath = [&](int, int, int, int) { return T(0); };
      T oc[NF];
      if constexpr (kF32) {
        nse32_node<L3, THREE>(at, own, cc, pcc, oc, kc);
      } else {
        mmfd_node<L3, kNSE, THREE, false, T, false, true>(at, ath, cc, pcc, oc, kc);
      }
      const int64_t gi = (int64_t)z * plane + (int64_t)gyi * nx + gxi;
#pragma unroll
      for (int f = 0; f < NF; ++f) out[f * N + gi] = oc[f];
    }
    __syncthreads();
    if constexpr (kF32) {
      // the z pairs' parts of plane z + 1 become the current plane's
      static_for<L3::P>([&](auto PI) {
        constexpr int P = decltype(PI)::value;
        if constexpr (zpair(P)) {
          own[2 * P] = ownn[2 * P];
          own[2 * P + 1] = ownn[2 * P + 1];
        }
      });
    }
  }
}

// ------------------------------------------------------------ host side
template <typename T>
hipError_t launch_nse3d_pp(const Consts &c, const Grid &g, const T *cur, const T *prev, T *out,
                           hipStream_t st) {
  if (c.lattice != 4 || c.eq != kNSE || c.three_stencil) return hipErrorInvalidValue;
  constexpr int TX = 32, TY = 8;
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1], nz = (int)g.n[2];
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const int zc = nz >= 64 ? 32 : nz;
  const int tzn = (nz + zc - 1) / zc;
  const size_t lds = (size_t)(3 * 2 * kZP + 2 * kIP) * (TY + 2) * (TX + 2) * sizeof(T);
  auto fn = c.three ? k_nse3d_pp<true, TX, TY, T> : k_nse3d_pp<false, TX, TY, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty * tzn), dim3(TX * TY), lds, st, cur, prev, out, nx, ny, nz,
                     tx, ty, zc, tx * ty * tzn, kc);
  return hipGetLastError();
}

template hipError_t launch_nse3d_pp<float>(const Consts &, const Grid &, const float *,
                                           const float *, float *, hipStream_t);
template hipError_t launch_nse3d_pp<double>(const Consts &, const Grid &, const double *,
                                            const double *, double *, hipStream_t);

}  // namespace mfd
