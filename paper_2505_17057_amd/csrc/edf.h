// Device-side EDF evaluation shared by the MMFD and MesoFD kernels.
//
// A node "record" holds what the EDF of Eq. (3-3) needs at that node:
//   LCDE    : phi                                  (f_j = ubar_j phi)
//   Burgers : phi, Bh = phi^2 (dt/2dx)             (B = Bh on every axis)
//   NSE     : rho - rho0, j_0..j_{D-1}, C_00..C_{D-1,D-1}, C_01[, C_02, C_12]
//             with C_ab = j_a j_b / rho (He-Luo: / rho0).
// Pair parts (Eq. (2-5) applied to Eq. (3-3)):
//   F+_p = w_p (A + Q~_p : C),   F-_p = (w_p / d0) e_p . B.
// Full EDF (MesoFD): g_j = w_j ((A + e_j . B / d0) + Q~_j : C).
// All sums run left to right in the order written (axis order; diagonal
// terms before off-diagonal ones).
#pragma once

#include <type_traits>

#include "mfd_internal.h"

namespace mfd {

template <typename T>
__device__ __forceinline__ T madd(T a, T b, T c);
// binary64: separate rounded multiply and add (the library is built with
// -ffp-contract=off), the same operations as the FP64 oracle.
template <>
__device__ __forceinline__ double madd<double>(double a, double b, double c) {
  return a * b + c;
}
// binary32: fused multiply-add.
template <>
__device__ __forceinline__ float madd<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// 1/x: binary64 a correctly rounded division (the oracle's operation);
// binary32 the hardware reciprocal (error within 1 ulp), an order of
// magnitude fewer instructions than the IEEE division sequence.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

template <class L, int EQ>
struct Rec {
  static constexpr int D = L::D;
  static constexpr int NF = EQ == kNSE ? 1 + D : 1;                    // moment fields
  static constexpr int NC = D == 1 ? 1 : (D == 2 ? 3 : 6);             // C components
  static constexpr int NR = EQ == kLCDE ? 1 : (EQ == kBurgers ? 2 : 1 + D + NC);
};

// index of C_ab in the record
template <int D>
__device__ __host__ constexpr int c_index(int a, int b) {
  // diagonal first, then (0,1), (0,2), (1,2)
  return a == b ? a : (D == 2 ? 2 : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5)));
}

template <class L, int EQ, typename T>
__device__ __forceinline__ void make_record(const T *m, T *r, const KC<T> &kc) {
  constexpr int D = L::D;
  if constexpr (EQ == kLCDE) {
    r[0] = m[0];
  } else if constexpr (EQ == kBurgers) {
    r[0] = m[0];
    r[1] = (m[0] * m[0]) * kc.bh;
  } else {
    r[0] = m[0];
    T rinv;
    if (kc.he_luo) rinv = kc.rinv0;
    else rinv = recip(kc.rho0 + m[0]);
#pragma unroll
    for (int a = 0; a < D; ++a) r[1 + a] = m[1 + a];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a; b < D; ++b) r[1 + D + c_index<D>(a, b)] = (m[1 + a] * m[1 + b]) * rinv;
  }
}

// Q~_j : C for direction j (compile-time), record r
template <class L, int EQ, int J, typename T>
__device__ __forceinline__ T quad(const T *r, const KC<T> &kc) {
  constexpr int D = L::D;
  if constexpr (EQ == kBurgers) {
    const T cb = kc.cbeta * r[0];
    T t = kc.qd[J][0] * cb;
#pragma unroll
    for (int a = 1; a < D; ++a) t = madd(kc.qd[J][a], cb, t);
    return t;
  } else {
    const T *C = r + 1 + D;
    T t = kc.qd[J][0] * C[0];
#pragma unroll
    for (int a = 1; a < D; ++a) t = madd(kc.qd[J][a], C[a], t);
    if constexpr (D >= 2) {
      constexpr int o01 = L::E[J][0] * L::E[J][1];
      if constexpr (o01 != 0) t = madd(kc.qo[J][0], C[c_index<D>(0, 1)], t);
    }
    if constexpr (D == 3) {
      constexpr int o02 = L::E[J][0] * L::E[J][2];
      constexpr int o12 = L::E[J][1] * L::E[J][2];
      if constexpr (o02 != 0) t = madd(kc.qo[J][1], C[c_index<D>(0, 2)], t);
      if constexpr (o12 != 0) t = madd(kc.qo[J][2], C[c_index<D>(1, 2)], t);
    }
    return t;
  }
}

// e_J . B with e in {-1,0,1}, signed accumulation
template <class L, int EQ, int J, typename T>
__device__ __forceinline__ T edotB(const T *r) {
  T s = T(0);
#pragma unroll
  for (int a = 0; a < L::D; ++a) {
    const T b = EQ == kBurgers ? r[1] : r[1 + a];
    if (L::E[J][a] == 1) s = s + b;
    else if (L::E[J][a] == -1) s = s - b;
  }
  return s;
}

// even pair part F+ of direction J (nonlinear EDFs).  B1: the caller knows
// that beta = 1 (Burgers), so the quadratic term, which is then absent, is
// not even tested for.
template <class L, int EQ, int J, bool B1 = false, typename T>
__device__ __forceinline__ T fplus(const T *r, const KC<T> &kc) {
  T t = r[0];
  if constexpr (EQ == kBurgers) {
    if constexpr (!B1) {
      if (!kc.beta_one) t = t + quad<L, EQ, J>(r, kc);
    }
  } else {
    t = t + quad<L, EQ, J>(r, kc);
  }
  return kc.w[J] * t;
}

// odd pair part F- of direction J
template <class L, int EQ, int J, typename T>
__device__ __forceinline__ T fminus(const T *r, const KC<T> &kc) {
  return kc.w1[J] * edotB<L, EQ, J>(r);
}

// full EDF g_J (MesoFD); B1 as for fplus
template <class L, int EQ, int J, bool B1 = false, typename T>
__device__ __forceinline__ T gfull(const T *r, const KC<T> &kc) {
  if constexpr (EQ == kLCDE) {
    return kc.ubar[J] * r[0];
  } else {
    T t = madd(edotB<L, EQ, J>(r), kc.inv_d0, r[0]);
    if constexpr (EQ == kBurgers) {
      if constexpr (!B1) {
        if (!kc.beta_one) t = t + quad<L, EQ, J>(r, kc);
      }
    } else {
      t = t + quad<L, EQ, J>(r, kc);
    }
    return kc.w[J] * t;
  }
}

// compile-time loop helper
template <int N, class F, int I = 0>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, F, I + 1>(static_cast<F &&>(f));
  }
}

}  // namespace mfd
