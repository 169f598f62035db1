// MesoFD node functions shared by the single-step, LDS-resident and blocked
// MesoFD kernels: the population form of the scheme, Eq. (2-1) /
// (3layer-1),
//   f_j(x, t+dt) = sum_k a_k f_j^eq(x + k e_j, t) + sum_k ah_k f_j^eq(x + k e_j, t-dt),
// k in (-1, 0, +1) order, level t first, zero coefficients skipped, and the
// moments of Eq. (2-1-1) (phi = sum_j f_j, j_a = sum_j e_ja f_j, lattice
// order).
#pragma once

#include "edf.h"

namespace mfd {

// moments of the b populations f[] of one node (lattice order)
template <class L, int EQ, typename T>
__device__ __forceinline__ void moments_of(const T *f, T *m) {
  constexpr int NF = Rec<L, EQ>::NF;
  T s = T(0);
#pragma unroll
  for (int j = 0; j < L::Q; ++j) s = s + f[j];
  m[0] = s;
#pragma unroll
  for (int a = 0; a + 1 < NF; ++a) {
    T t = T(0);
#pragma unroll
    for (int j = 0; j < L::Q; ++j) {
      if (L::E[j][a] == 1) t = t + f[j];
      else if (L::E[j][a] == -1) t = t - f[j];
    }
    m[1 + a] = t;
  }
}

template <class L, int EQ, typename T>
__device__ __forceinline__ void pop_moments(const T *pop, int64_t N, int64_t gi, T *m) {
  T f[L::Q];
#pragma unroll
  for (int j = 0; j < L::Q; ++j) f[j] = pop[j * N + gi];
  moments_of<L, EQ>(f, m);
}

// Rest-direction EDF.  binary64: g_0 of Eq. (3-3) like every direction.
// binary32: g_0 = A - sum_{j>=1} g_j, so that the populations of one node sum
// to A without the drift that the binary32-rounded weights (whose sum is not
// exactly 1) would add to the zeroth moment at every step.
template <class L, int EQ, bool B1 = false, typename T>
__device__ __forceinline__ T g_rest(const T *r, const KC<T> &kc) {
  if constexpr (std::is_same<T, double>::value) {
    return gfull<L, EQ, 0, B1>(r, kc);
  } else {
    T s = T(0);
    static_for<L::Q - 1>([&](auto JI) {
      constexpr int J = decltype(JI)::value + 1;
      s = s + gfull<L, EQ, J, B1>(r, kc);
    });
    return r[0] - s;
  }
}

template <class L, int EQ, int J, bool B1 = false, typename T>
__device__ __forceinline__ T g_dir(const T *r, const KC<T> &kc) {
  if constexpr (J == 0) return g_rest<L, EQ, B1>(r, kc);
  else return gfull<L, EQ, J, B1>(r, kc);
}

// the b new populations of one node (Eq. (2-1) / (3layer-1) in the order
// written above) into fo[]
template <class L, int EQ, bool THREE_ST, bool B1 = false, typename T, class At, class AtH>
__device__ __forceinline__ void mesofd_pops(const At &at, const AtH &ath, const T *hcentre,
                                            bool three, T *fo, const KC<T> &kc) {
  constexpr int NR = Rec<L, EQ>::NR;
  static_for<L::Q>([&](auto JI) {
    constexpr int J = decltype(JI)::value;
    constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
    T fj = T(0);
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
      const T ak = kc.a[k + 1];
      if (ak != T(0)) {
        T r[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) r[q] = at(q, k * ez, k * ey, k * ex);
        fj = madd(ak, g_dir<L, EQ, J, B1>(r, kc), fj);
      }
    }
    if (three) {
#pragma unroll
      for (int k = -1; k <= 1; ++k) {
        const T ak = kc.ah[k + 1];
        if (ak != T(0)) {
          T r[NR];
          if constexpr (THREE_ST) {
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = ath(q, k * ez, k * ey, k * ex);
          } else {
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = hcentre[q];  // only k = 0 is non-zero
          }
          fj = madd(ak, g_dir<L, EQ, J, B1>(r, kc), fj);
        }
      }
    }
    fo[J] = fj;
  });
}

// evaluate the b new populations of one node, store them (unless pout is
// null) and the moments of the new level
template <class L, int EQ, bool THREE_ST, typename T, class At, class AtH>
__device__ __forceinline__ void mesofd_node(const At &at, const AtH &ath, const T *hcentre,
                                            bool three, T *pout, T *mout, int64_t N, int64_t gi,
                                            const KC<T> &kc) {
  constexpr int NF = Rec<L, EQ>::NF;
  T fo[L::Q];
  mesofd_pops<L, EQ, THREE_ST>(at, ath, hcentre, three, fo, kc);
  if (pout) {  // null: the moments only
#pragma unroll
    for (int j = 0; j < L::Q; ++j) pout[j * N + gi] = fo[j];
  }
  T m[NF];
  moments_of<L, EQ>(fo, m);
#pragma unroll
  for (int f = 0; f < NF; ++f) mout[f * N + gi] = m[f];
}

}  // namespace mfd
