// The MMFD node update shared by the single-step and temporally blocked
// kernels (one expression tree for both, so TB does not change results).
#pragma once

#include "edf.h"

namespace mfd {

// ---------------------------------------------------------- node update
// `at(field, dz, dy, dx)` reads the level-t record, `ath` the level-(t-dt)
// record; cur_c / prev_c are the centre moments (global), out the outputs.
template <class L, int EQ, bool THREE, bool THREE_ST, typename T, class At, class AtH>
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
        const T Fpp = fplus<L, EQ, J>(rp, kc), Fp0 = fplus<L, EQ, J>(r0, kc),
                Fpm = fplus<L, EQ, J>(rm, kc);
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

}  // namespace mfd
