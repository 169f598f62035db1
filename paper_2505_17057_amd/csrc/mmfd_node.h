// The MMFD node update shared by the single-step and temporally blocked
// kernels (one expression tree for both, so TB does not change results).
#pragma once

#include "edf.h"

namespace mfd {

// ---------------------------------------------------------- node update
// `at(field, dz, dy, dx)` reads the level-t record, `ath` the level-(t-dt)
// record; cur_c / prev_c are the centre moments (global), out the outputs.
// B1: Burgers with beta = 1 known at compile time (see fplus).
// PF: the accessors return precomputed pair parts instead of records:
// at(2p, ...) = F+_p, at(2p + 1, ...) = F-_p of pair p at that offset (the
// same values fplus / fminus give for the node's record).
template <class L, int EQ, bool THREE, bool THREE_ST, typename T, bool B1 = false,
          bool PF = false, class At, class AtH>
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
        T Fpp, Fp0, Fpm, Fmp, Fmm, Fm0;
        if constexpr (PF) {
          Fpp = get(2 * P, ez, ey, ex);
          Fp0 = get(2 * P, 0, 0, 0);
          Fpm = get(2 * P, -ez, -ey, -ex);
          Fmp = get(2 * P + 1, ez, ey, ex);
          Fmm = get(2 * P + 1, -ez, -ey, -ex);
          if constexpr (EQ == kNSE) Fm0 = get(2 * P + 1, 0, 0, 0);
        } else {
          T rp[NR], r0[NR], rm[NR];
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            rp[k] = get(k, ez, ey, ex);
            r0[k] = get(k, 0, 0, 0);
            rm[k] = get(k, -ez, -ey, -ex);
          }
          Fpp = fplus<L, EQ, J, B1>(rp, kc);
          Fp0 = fplus<L, EQ, J, B1>(r0, kc);
          Fpm = fplus<L, EQ, J, B1>(rm, kc);
          Fmp = fminus<L, EQ, J>(rp, kc);
          Fmm = fminus<L, EQ, J>(rm, kc);
          if constexpr (EQ == kNSE) Fm0 = fminus<L, EQ, J>(r0, kc);
        }
        acc = madd(cpl, (Fpp - T(2) * Fp0) + Fpm, acc);
        acc = madd(cmi, Fmp - Fmm, acc);
        if constexpr (EQ == kNSE) {
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

// pair parts F+_p, F-_p of every opposite pair of one node record (lattice
// pair order), out[2p] = F+_p, out[2p + 1] = F-_p
template <class L, int EQ, typename T>
__device__ __forceinline__ void pair_parts(const T *r, T *out, const KC<T> &kc) {
  static_for<L::P>([&](auto PI) {
    constexpr int P = decltype(PI)::value;
    constexpr int J = L::PR[P];
    out[2 * P] = fplus<L, EQ, J>(r, kc);
    out[2 * P + 1] = fminus<L, EQ, J>(r, kc);
  });
}

// ------------------------------------------------ binary32 NSE pair form
// The binary32 NSE steps (2D, no older-level stencil) use unweighted pair
// parts, G+_p = (rho - rho0) + Q~_p : C and G-_p = e_p . j, so that
// F+_p = w_p G+_p and F-_p = (w_p / d0) G-_p; the weights are folded into
// the per-pair constants kc.nw[p] = {a+ w, a- w / d0, abar+ w / d0, abar- w}.
// Each difference of Eq. (2-2-1) is formed from the differences to the
// node's own part, dP = G(x + e_p) - G(x) and dM = G(x - e_p) - G(x)
// (second difference dP + dM, first difference dP - dM): neighbouring values
// differ in their low bits only, so these subtractions are exact or nearly
// so.  The time-level base A0 phi + Ah0 phi_hat is formed as
// phi + (acc - Ah0 (phi - phi_hat)) (A0 + Ah0 = 1), rounded once at the
// scale of phi.
// Every kernel that takes such a step uses these two functions, so the
// single-step, blocked and batched launches agree bit for bit.
template <class L>
__device__ __forceinline__ void nse32_parts(const float *m, float *g, const KC<float> &kc) {
  constexpr int D = L::D;
  static_assert(D >= 2, "2D and 3D lattices");
  const float rinv = kc.he_luo ? kc.rinv0 : __builtin_amdgcn_rcpf(kc.rho0 + m[0]);
  float u[D], cd[D], co[3];
#pragma unroll
  for (int a = 0; a < D; ++a) u[a] = m[1 + a] * rinv;
#pragma unroll
  for (int a = 0; a < D; ++a) cd[a] = m[1 + a] * u[a];
  co[0] = m[1] * u[1];
  co[1] = D == 3 ? m[1] * u[D - 1] : 0.f;
  co[2] = D == 3 ? m[2] * u[D - 1] : 0.f;
  static_for<L::P>([&](auto PI) {
    constexpr int P = decltype(PI)::value;
    constexpr int J = L::PR[P];
    float gp = __builtin_fmaf(kc.qd[J][0], cd[0], m[0]);
#pragma unroll
    for (int a = 1; a < D; ++a) gp = __builtin_fmaf(kc.qd[J][a], cd[a], gp);
    if constexpr (L::E[J][0] * L::E[J][1] != 0) gp = __builtin_fmaf(kc.qo[J][0], co[0], gp);
    if constexpr (D == 3) {
      if constexpr (L::E[J][0] * L::E[J][2] != 0) gp = __builtin_fmaf(kc.qo[J][1], co[1], gp);
      if constexpr (L::E[J][1] * L::E[J][2] != 0) gp = __builtin_fmaf(kc.qo[J][2], co[2], gp);
    }
    // e_J . j, from the first nonzero component on (no addition to zero)
    float gm = 0.f;
    bool started = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (L::E[J][a] == 0) continue;
      const float v = L::E[J][a] > 0 ? m[1 + a] : -m[1 + a];
      gm = started ? gm + v : v;
      started = true;
    }
    g[2 * P] = gp;
    g[2 * P + 1] = gm;
  });
}

// first pair (lattice pair order) whose direction has a nonzero component a
template <class L>
__device__ __host__ constexpr int nse32_first_pair(int a) {
  for (int p = 0; p < L::P; ++p)
    if (L::E[L::PR[p]][a] != 0) return p;
  return L::P;
}
template <class L, int P>
__device__ __host__ constexpr int nse32_ncomp() {
  int k = 0;
  for (int a = 0; a < L::D; ++a) k += L::E[L::PR[P]][a] != 0 ? 1 : 0;
  return k;
}

// `at(q, dz, dy, dx)` returns part q (2p: G+_p, 2p + 1: G-_p) of the node
// at that offset; g0 the node's own parts; cur_c / prev_c its moments at t
// and t - dt.
template <class L, bool THREE, class At>
__device__ __forceinline__ void nse32_node(const At &at, const float *g0, const float *cur_c,
                                           const float *prev_c, float *out_c,
                                           const KC<float> &kc) {
  constexpr int D = L::D;
  float acc = 0.f, mo[D];
#pragma unroll
  for (int a = 0; a < D; ++a) mo[a] = 0.f;
  static_for<L::P>([&](auto PI) {
    constexpr int P = decltype(PI)::value;
    constexpr int J = L::PR[P];
    constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
    const float cP = kc.nw[P][0], cM = kc.nw[P][1], bP = kc.nw[P][2], bM = kc.nw[P][3];
    const float pP = at(2 * P, ez, ey, ex) - g0[2 * P];  // G+ differences
    const float pM = at(2 * P, -ez, -ey, -ex) - g0[2 * P];
    const float mP = at(2 * P + 1, ez, ey, ex) - g0[2 * P + 1];  // G- differences
    const float mM = at(2 * P + 1, -ez, -ey, -ex) - g0[2 * P + 1];
    // rho: a+ D2 F+ + a- D1 F-
    if constexpr (P == 0) acc = cP * pP;
    else acc = __builtin_fmaf(cP, pP, acc);
    acc = __builtin_fmaf(cP, pM, acc);
    acc = __builtin_fmaf(cM, mP, acc);
    acc = __builtin_fmaf(-cM, mM, acc);
    // j: e_p (abar+ D2 F- + abar- D1 F+)
    if constexpr (nse32_ncomp<L, P>() == 1) {
      constexpr int a = ex != 0 ? 0 : (ey != 0 ? 1 : 2);
      constexpr int sg = L::E[J][a];
      const float sP = sg > 0 ? bP : -bP, sM = sg > 0 ? bM : -bM;
      if constexpr (nse32_first_pair<L>(a) == P) mo[a] = sM * pP;
      else mo[a] = __builtin_fmaf(sM, pP, mo[a]);
      mo[a] = __builtin_fmaf(-sM, pM, mo[a]);
      mo[a] = __builtin_fmaf(sP, mP, mo[a]);
      mo[a] = __builtin_fmaf(sP, mM, mo[a]);
    } else {
      float b = bM * pP;
      b = __builtin_fmaf(-bM, pM, b);
      b = __builtin_fmaf(bP, mP, b);
      b = __builtin_fmaf(bP, mM, b);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        if (L::E[J][a] == 0) continue;
        const bool pos = L::E[J][a] > 0;
        if (nse32_first_pair<L>(a) == P) mo[a] = pos ? b : -b;
        else mo[a] = pos ? mo[a] + b : mo[a] - b;
      }
    }
  });
#pragma unroll
  for (int f = 0; f <= D; ++f) {
    const float c = cur_c[f], d = f == 0 ? acc : mo[f - 1];
    if constexpr (THREE) {
      // c + (d - Ah0 (c - c_hat)): the bracket is of the size of one step's
      // change, so its rounding is far below an ulp of c, and the new value
      // is rounded once at the scale of c (as A0 c + Ah0 c_hat + d in
      // binary64 would be).  Rounding c - Ah0 (c - c_hat) first would add a
      // second rounding at that scale whose sign follows the slowly varying
      // change, i.e. a drift that grows linearly over a long run.
      const float t = __builtin_fmaf(f == 0 ? -kc.Ah0t : -kc.Abh0t, c - prev_c[f], d);
      out_c[f] = c + t;
    } else {
      out_c[f] = __builtin_fmaf(f == 0 ? kc.A0t : kc.Ab0t, c, d);
    }
  }
}

// One TX x TY tile of a 2D grid for the NSE, in three parts so that a
// persistent kernel can overlap the next tile's loads with this tile's work:
//   load   the moments of the tile and a one-node halo (both levels when the
//          older one has a stencil) and the older level at the interior
//          nodes, into registers (all loads of a thread in flight at once);
//   stage  the pair parts of every loaded node (each evaluated once, not once
//          per neighbour that uses it) and the tile's moments into LDS;
//   update the node updates of the interior, reading LDS.
// periodic index for i in [-n, 2n)
__device__ __forceinline__ int wrap1(int i, int n) {
  i += i < 0 ? n : 0;
  return i - (i >= n ? n : 0);
}

// Sweep of the Picard-Jacobi iteration of the NSE's theta step, applied per
// field q to the explicit step value S_q(x) of a node:
// out_q = (R_q + th1 ((S_q - A0_q x_q) + dd_q x_q)) inv_den_q (the operations
// and roundings of the separate elementwise update).
// part (may be null): the sweep also adds, per field, (x_new - x)^2 and R^2
// in binary64 into per-workgroup partial sums (rows of 8 doubles).
// rhs: instead of a sweep, the step's right-hand side
// R_q = th S_q(x) + th1 (A0_q x_q) (the operations of the separate pass).
template <typename T>
struct PicardNse {
  const T *R;
  T A0[4], dd[4], inv_den[4];
  T th1, th;
  int rhs;
  double *part;
};

// FAST: nx >= TX + 2 and ny >= TY + 2, so every halo index is within one
// period of the grid (cheap wrap); otherwise the general wrap.
template <class L, bool THREE, bool THREE_ST, int TX, int TY, typename T, bool FAST = false>
struct PfTile {
  using R = Rec<L, kNSE>;
  static constexpr int NR = R::NR, NF = R::NF, NPF = 2 * L::P;
  static constexpr int HX = TX + 2, HY = TY + 2;
  static constexpr int KH = (HX * HY + 255) / 256;  // halo-tile nodes per thread
  static constexpr int KI = (TX * TY + 255) / 256;  // interior nodes per thread
  // binary32 without an older-level stencil: the binary32 pair form above
  static constexpr bool kNse32 = std::is_same<T, float>::value && !THREE_ST;
  struct Lds {
    T pf[NPF][HY][HX];
    T hpf[THREE_ST ? NPF : 1][THREE_ST ? HY : 1][THREE_ST ? HX : 1];
    T mc[NF][TY][TX];
  };
  struct Regs {
    T mv[KH][NF];
    T hv[THREE_ST ? KH : 1][NF];
    T pcv[KI][NF];
  };

  static __device__ __forceinline__ void load(const T *__restrict__ cur,
                                              const T *__restrict__ prev, int nx, int ny, int x0,
                                              int y0, Regs &g) {
    const int64_t N = (int64_t)nx * ny;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < HX * HY) {
        const int lx = i % HX, ly = i / HX;
        const int gx = FAST ? wrap1(x0 - 1 + lx, nx) : wrapi(x0 - 1 + lx, nx);
        const int gy = FAST ? wrap1(y0 - 1 + ly, ny) : wrapi(y0 - 1 + ly, ny);
        const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
        for (int q = 0; q < NF; ++q) g.mv[k][q] = cur[q * N + gi];
        if constexpr (THREE_ST) {
#pragma unroll
          for (int q = 0; q < NF; ++q) g.hv[k][q] = prev[q * N + gi];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KI; ++k) {
      const int i = threadIdx.x + 256 * k;
      const int gx = x0 + i % TX, gy = y0 + i / TX;
      if (THREE && i < TX * TY && gx < nx && gy < ny) {
        const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
        for (int q = 0; q < NF; ++q) g.pcv[k][q] = prev[q * N + gi];
      }
    }
  }

  static __device__ __forceinline__ void stage(const Regs &g, Lds &s, const KC<T> &kc) {
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < HX * HY) {
        const int lx = i % HX, ly = i / HX;
        T r[NR], f[NPF];
        if (lx >= 1 && lx <= TX && ly >= 1 && ly <= TY) {
#pragma unroll
          for (int q = 0; q < NF; ++q) s.mc[q][ly - 1][lx - 1] = g.mv[k][q];
        }
        if constexpr (kNse32) {
          nse32_parts<L>(g.mv[k], f, kc);
        } else {
          make_record<L, kNSE>(g.mv[k], r, kc);
          pair_parts<L, kNSE>(r, f, kc);
        }
#pragma unroll
        for (int q = 0; q < NPF; ++q) s.pf[q][ly][lx] = f[q];
        if constexpr (THREE_ST) {
          make_record<L, kNSE>(g.hv[k], r, kc);
          pair_parts<L, kNSE>(r, f, kc);
#pragma unroll
          for (int q = 0; q < NPF; ++q) s.hpf[q][ly][lx] = f[q];
        }
      }
    }
  }

  static __device__ __forceinline__ void update(const Lds &s, const T (&pcv)[KI][NF],
                                                T *__restrict__ out, int nx, int ny, int x0,
                                                int y0, const KC<T> &kc,
                                                const PicardNse<T> *pe = nullptr,
                                                double *sq = nullptr) {
    const int64_t N = (int64_t)nx * ny;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i >= TX * TY) break;
      const int lx = i % TX, ly = i / TX;
      const int gx = x0 + lx, gy = y0 + ly;
      if (gx >= nx || gy >= ny) continue;
      const int cx = lx + 1, cy = ly + 1;
      const int64_t gi = (int64_t)gy * nx + gx;
      auto at = [&](int q, int, int dy, int dx) { return s.pf[q][cy + dy][cx + dx]; };
      auto ath = [&](int q, int, int dy, int dx) {
        if constexpr (THREE_ST) return s.hpf[q][cy + dy][cx + dx];
        else return T(0);
      };
      T cc[NF], pc[NF], oc[NF];
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        cc[q] = s.mc[q][ly][lx];
        pc[q] = THREE ? pcv[k][q] : T(0);
      }
      if constexpr (kNse32) {
        T g0[NPF];
#pragma unroll
        for (int q = 0; q < NPF; ++q) g0[q] = s.pf[q][cy][cx];
        auto at2 = [&](int q, int, int dy, int dx) { return s.pf[q][cy + dy][cx + dx]; };
        nse32_node<L, THREE>(at2, g0, cc, pc, oc, kc);
      } else {
        mmfd_node<L, kNSE, THREE, THREE_ST, T, false, true>(at, ath, cc, pc, oc, kc);
      }
      if (pe && pe->rhs) {
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const T a = pe->th * oc[q];
          const T b = pe->A0[q] * cc[q];
          oc[q] = a + pe->th1 * b;
        }
      } else if (pe) {
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const T xi = cc[q];
          const T t = (oc[q] - pe->A0[q] * xi) + pe->dd[q] * xi;
          const T c = pe->th1 * t;
          const T Rq = pe->R[q * N + gi];
          oc[q] = (Rq + c) * pe->inv_den[q];
          if (sq) {
            const double d = (double)oc[q] - (double)xi;
            sq[2 * q] += d * d;
            sq[2 * q + 1] += (double)Rq * (double)Rq;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NF; ++q) out[q * N + gi] = oc[q];
    }
  }
};

template <class L, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__device__ __forceinline__ void mmfd_plane_tile_pf(const T *__restrict__ cur,
                                                   const T *__restrict__ prev,
                                                   T *__restrict__ out, int nx, int ny, int x0,
                                                   int y0, const KC<T> &kc) {
  using P = PfTile<L, THREE, THREE_ST, TX, TY, T>;
  __shared__ typename P::Lds sm;
  typename P::Regs g;
  P::load(cur, prev, nx, ny, x0, y0, g);
  P::stage(g, sm, kc);
  __syncthreads();
  P::update(sm, g.pcv, out, nx, ny, x0, y0, kc);
}

// One TX x TY tile (origin x0, y0) of a 1D / 2D grid: EDF records of the tile
// and a one-node halo into LDS (periodic wrap), then the node updates.
// Sweep of the Picard-Jacobi iteration of Burgers' theta step, applied to
// the explicit step value S(x) of a node: out = (R + th1 ((S - A0 x) +
// dd x)) inv_den (the operations and roundings of the separate update).
// part (may be null): the sweep also forms (x_new - x)^2 and R^2 in binary64
// and writes the workgroup's sums to row blockIdx.x (8 doubles a row).
template <typename T>
struct PicardEp {
  const T *R;
  T A0, dd, th1, inv_den;
  double *part;
};

template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__device__ __forceinline__ void mmfd_plane_tile(const T *__restrict__ cur,
                                                const T *__restrict__ prev,
                                                T *__restrict__ out, int nx, int ny, int x0,
                                                int y0, const KC<T> &kc,
                                                const DirBC *bc = nullptr,
                                                const PicardEp<T> *pe = nullptr) {
  if constexpr (EQ == kNSE && L::D == 2) {
    mmfd_plane_tile_pf<L, THREE, THREE_ST, TX, TY, T>(cur, prev, out, nx, ny, x0, y0, kc);
  } else {
  using R = Rec<L, EQ>;
  constexpr int NR = R::NR, NF = R::NF;
  constexpr int HYL = L::D >= 2 ? 1 : 0;
  constexpr int HX = TX + 2, HY = TY + 2 * HYL;
  __shared__ T rec[NR][HY][HX];
  __shared__ T hrec[THREE_ST ? NR : 1][THREE_ST ? HY : 1][THREE_ST ? HX : 1];
  const int64_t N = (int64_t)nx * ny;

  // every load of the thread's halo-tile nodes is issued before the first
  // record is formed (the loads' latencies overlap)
  constexpr int KH = (HX * HY + 255) / 256;
  T mv[KH][NF], hv[THREE_ST ? KH : 1][NF];
#pragma unroll
  for (int j = 0; j < KH; ++j) {
    const int i = threadIdx.x + 256 * j;
    if (i < HX * HY) {
      const int lx = i % HX, ly = i / HX;
      const int gx = wrapi(x0 - 1 + lx, nx), gy = wrapi(y0 - HYL + ly, ny);
      const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
      for (int f = 0; f < NF; ++f) mv[j][f] = cur[f * N + gi];
      if constexpr (THREE_ST) {
#pragma unroll
        for (int f = 0; f < NF; ++f) hv[j][f] = prev[f * N + gi];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KH; ++j) {
    const int i = threadIdx.x + 256 * j;
    if (i < HX * HY) {
      const int lx = i % HX, ly = i / HX;
      T r[NR];
      make_record<L, EQ>(mv[j], r, kc);
#pragma unroll
      for (int k = 0; k < NR; ++k) rec[k][ly][lx] = r[k];
      if constexpr (THREE_ST) {
        make_record<L, EQ>(hv[j], r, kc);
#pragma unroll
        for (int k = 0; k < NR; ++k) hrec[k][ly][lx] = r[k];
      }
    }
  }
  __syncthreads();

  double sq0 = 0.0, sq1 = 0.0;  // residual sums of a Picard sweep with pe->part
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
    if constexpr (L::D == 2 && NF == 1) {
      // Dirichlet nodes take their prescribed value
      if (bc && bc->on && dir_node(gx, gy, nx, ny))
        oc[0] = (T)(bc->Gb[dir_index(gx, gy, nx, ny)] * bc->E[1]);
    }
    if constexpr (NF == 1) {
      if (pe) {
        const T xi = cc[0];
        const T t = (oc[0] - pe->A0 * xi) + pe->dd * xi;
        const T c = pe->th1 * t;
        const T Ri = pe->R[gi];
        oc[0] = (Ri + c) * pe->inv_den;
        if (pe->part) {
          const double d = (double)oc[0] - (double)xi;
          sq0 += d * d;
          sq1 += (double)Ri * (double)Ri;
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f * N + gi] = oc[f];
  }
  if (pe && pe->part) {  // the workgroup's row: wave sums, then the four waves in order
    __shared__ double red[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sq0 += __shfl_xor(sq0, o, 64);
      sq1 += __shfl_xor(sq1, o, 64);
    }
    if (lane == 0) {
      red[0][wave] = sq0;
      red[1][wave] = sq1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      const int q = threadIdx.x;
      pe->part[blockIdx.x * 8 + q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
    }
  }
  }
}

}  // namespace mfd
