// The MMFD node update shared by the single-step and temporally blocked
// kernels (one expression tree for both, so TB does not change results).
#pragma once

#include "edf.h"

namespace mfd {

// ---------------------------------------------------------- node update
// `at(field, dz, dy, dx)` reads the level-t record, `ath` the level-(t-dt)
// record; cur_c / prev_c are the centre moments (global), out the outputs.
// B1: Burgers with beta = 1 known at compile time (see fplus).
template <class L, int EQ, bool THREE, bool THREE_ST, typename T, bool B1 = false, class At,
          class AtH>
__device__ __forceinline__ void mmfd_node(const At &at, const AtH &ath, const T *cur_c,
                                          const T *prev_c, T *out_c, const KC<T> &kc) {
  using R = Rec<L, EQ>;
  constexpr int D = L::D, NR = R::NR, NF = R::NF;
  T acc = T(0);
  T mom[D > 0 ? D : 1];
#pragma unroll
  for (int a = 0; a < D; ++a) mom[a] = T(0);

  auto level = [&](const auto &get, T cpl, T cmi, T bpl, T bmi, bool hat) {
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
      if constexpr (EQ == kLCDE) {
        const T gp = get(0, ez, ey, ex), g0 = get(0, 0, 0, 0), gm = get(0, -ez, -ey, -ex);
        if constexpr (std::is_same<T, double>::value) {
          const T cp = hat ? kc.Chp[P] : kc.Cp[P];
          const T cm = hat ? kc.Chm[P] : kc.Cm[P];
          acc = madd(cp, (gp - T(2) * g0) + gm, acc);
          acc = madd(cm, gp - gm, acc);
        } else {
          // binary32: Cp D2 g + Cm D1 g = (Cp + Cm)(g+ - g0) + (Cp - Cm)(g- - g0);
          // the differences of neighbouring values are exact or nearly so,
          // and the pair costs two subtractions and two fused multiply-adds
          const T al = hat ? kc.Ahp[P] : kc.Ap[P];
          const T be = hat ? kc.Ahm[P] : kc.Am[P];
          acc = madd(al, gp - g0, acc);
          acc = madd(be, gm - g0, acc);
        }
      } else {
        T rp[NR], r0[NR], rm[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          rp[k] = get(k, ez, ey, ex);
          r0[k] = get(k, 0, 0, 0);
          rm[k] = get(k, -ez, -ey, -ex);
        }
        const T Fpp = fplus<L, EQ, J, B1>(rp, kc), Fp0 = fplus<L, EQ, J, B1>(r0, kc),
                Fpm = fplus<L, EQ, J, B1>(rm, kc);
        const T Fmp = fminus<L, EQ, J>(rp, kc), Fmm = fminus<L, EQ, J>(rm, kc);
        acc = madd(cpl, (Fpp - T(2) * Fp0) + Fpm, acc);
        acc = madd(cmi, Fmp - Fmm, acc);
        if constexpr (EQ == kNSE) {
          const T Fm0 = fminus<L, EQ, J>(r0, kc);
          const T t1 = bpl * ((Fmp - T(2) * Fm0) + Fmm);
          const T t2 = bmi * (Fpp - Fpm);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (L::E[J][a] == 1) {
              mom[a] = mom[a] + t1;
              mom[a] = mom[a] + t2;
            } else if (L::E[J][a] == -1) {
              mom[a] = mom[a] - t1;
              mom[a] = mom[a] - t2;
            }
          }
        }
      }
    });
  };
  level(at, kc.ap, kc.am, kc.abp, kc.abm, false);
  if constexpr (THREE_ST) level(ath, kc.ahp, kc.ahm, kc.abhp, kc.abhm, true);

  // bases
  auto finish = [&](int f, T a_acc, double A0d, double Ah0d, T A0t, T Ah0t) {
    const T c = cur_c[f];
    if constexpr (std::is_same<T, double>::value) {
      double base = A0d * c;
      if constexpr (THREE) base = base + Ah0d * prev_c[f];
      out_c[f] = base + a_acc;
    } else {
      if constexpr (THREE) {
        const double cd = (double)c;
        const double base = cd - Ah0d * (cd - (double)prev_c[f]);
        out_c[f] = (T)(base + (double)a_acc);
      } else {
        out_c[f] = madd(A0t, c, a_acc);
      }
    }
  };
  finish(0, acc, kc.A0, kc.Ah0, kc.A0t, kc.Ah0t);
  if constexpr (EQ == kNSE) {
#pragma unroll
    for (int a = 0; a < D; ++a) finish(1 + a, mom[a], kc.Ab0, kc.Abh0, kc.Ab0t, kc.Abh0t);
  }
  (void)NF;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  if (i < 0) {
    i += n;
    if (i < 0) i = ((i % n) + n) % n;
  } else if (i >= n) {
    i -= n;
    if (i >= n) i %= n;
  }
  return i;
}

// Hardware dispatch sends consecutive workgroups round-robin to the 8 XCDs;
// give XCD x the contiguous tile range [x q + min(x, r), ...).
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// One TX x TY tile (origin x0, y0) of a 1D / 2D grid: EDF records of the tile
// and a one-node halo into LDS (periodic wrap), then the node updates.
template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__device__ __forceinline__ void mmfd_plane_tile(const T *__restrict__ cur,
                                                const T *__restrict__ prev,
                                                T *__restrict__ out, int nx, int ny, int x0,
                                                int y0, const KC<T> &kc) {
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR, NF = R::NF;
  constexpr int HYL = L::D >= 2 ? 1 : 0;
  constexpr int HX = TX + 2, HY = TY + 2 * HYL;
  __shared__ T rec[NR][HY][HX];
  __shared__ T hrec[THREE_ST ? NR : 1][THREE_ST ? HY : 1][THREE_ST ? HX : 1];
  const int64_t N = (int64_t)nx * ny;

  for (int i = threadIdx.x; i < HX * HY; i += 256) {
    const int lx = i % HX, ly = i / HX;
    const int gx = wrapi(x0 - 1 + lx, nx), gy = wrapi(y0 - HYL + ly, ny);
    const int64_t gi = (int64_t)gy * nx + gx;
    T m[NF], r[NR];
#pragma unroll
    for (int f = 0; f < NF; ++f) m[f] = cur[f * N + gi];
    make_record<L, EQ>(m, r, kc);
#pragma unroll
    for (int k = 0; k < NR; ++k) rec[k][ly][lx] = r[k];
    if constexpr (THREE_ST) {
#pragma unroll
      for (int f = 0; f < NF; ++f) m[f] = prev[f * N + gi];
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
    T cc[NF], pc[NF], oc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      cc[f] = at(f, 0, 0, 0);  // record fields 0..NF-1 are the moments
      pc[f] = THREE ? prev[f * N + gi] : T(0);
    }
    mmfd_node<L, EQ, THREE, THREE_ST, T>(at, ath, cc, pc, oc, kc);
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f * N + gi] = oc[f];
  }
}

}  // namespace mfd
