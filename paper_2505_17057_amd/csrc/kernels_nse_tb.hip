// Temporally blocked NSE step (D2Q5 / D2Q9, two-level or three-level without
// an older-level stencil): one launch advances several time steps.
//
// Each thread owns one column of a W x H window and a fixed run of R rows,
// and keeps the moments of its nodes at levels t and t - dt in registers for
// the whole launch.  Every step:
//   A  each node one beyond the update region evaluates its pair parts F+-_p
//      (record, then the even / odd parts of Eq. (3-3) over the opposite pair,
//      Eq. (2-5)) into LDS;
//   B  each node of the update region reads its neighbours' pair parts and
//      updates its own moments with the single-step node function.
// The store writes the interior of the last two levels (the next three-level
// launch needs both).  Results equal the single-step kernel's value for value.
//
// Binary32 64 x 64 and 64 x 128 windows take a register window instead
// (nse_window_reg): the parts stay in registers, the lanes beside share them
// by DPP and only the first and last rows of each wavefront's run pass
// through LDS.
//
// The batched kernel runs the same window for every tile of a batch group's
// table; each instance advances min(TB, its remaining steps).
#include "batch_kernels.h"
#include "mmfd_node.h"

namespace mfd {

namespace {
constexpr int kNseW = 64;  // window columns (one per thread)
constexpr int kNseR = 4;   // window rows per thread for 64-row windows (32-row: 2)
constexpr int kNseRR = 8;  // rows per thread of the binary32 register window

// value of the lane one above (lane + 1) / one below (lane - 1) in the
// wavefront; lanes without a source read 0
__device__ __forceinline__ float nse_from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float nse_from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// The eight multiply-adds of one pair p whose direction has an x component,
// on two accumulators (a: density, m: momentum), with the terms that need
// the lane beside (dx = -1 / +1) reading it through DPP inside the
// multiply-add:
//   a += cP pP;  a += ncP dp[lane + dx];  a += cM mP;  a += cM dm[lane + dx]
//   m += sM pP;  m += sM dp[lane + dx];   m += sP mP;  m += nsP dm[lane + dx]
// AF / MF: a / m start here (the first term is a product).  One block, so
// that one pair of wait states covers every shifted read: dp and dm are
// written before the block and not inside it.  All operands are in VGPRs.
#define NSE_DPP_L "wave_shr:1 row_mask:0xf bank_mask:0xf"
#define NSE_DPP_R "wave_shl:1 row_mask:0xf bank_mask:0xf"
#define NSE_PAIR_ASM(A1, M1, SH)                                            \
  "s_nop 1\n\t" A1 "\n\t" M1 "\n\t"                                        \
  "v_fmac_f32_dpp %0, %4, %7 " SH "\n\t"                                    \
  "v_fmac_f32_dpp %1, %4, %9 " SH "\n\t"                                    \
  "v_fmac_f32 %0, %8, %3\n\t"                                               \
  "v_fmac_f32 %1, %10, %3\n\t"                                              \
  "v_fmac_f32_dpp %0, %5, %8 " SH "\n\t"                                    \
  "v_fmac_f32_dpp %1, %5, %11 " SH
#define NSE_A_MUL "v_mul_f32 %0, %6, %2"
#define NSE_A_FMA "v_fmac_f32 %0, %6, %2"
#define NSE_M_MUL "v_mul_f32 %1, %9, %2"
#define NSE_M_FMA "v_fmac_f32 %1, %9, %2"
#define NSE_PAIR_IN                                                                    \
  "v"(pP), "v"(mP), "v"(dp), "v"(dm), "v"(cP), "v"(ncP), "v"(cM), "v"(sM), "v"(sP), \
      "v"(nsP)

template <int DX, bool AF, bool MF>
__device__ __forceinline__ void nse_pair_sh(float &a, float &m, float pP, float mP, float dp,
                                            float dm, float cP, float ncP, float cM, float sM,
                                            float sP, float nsP) {
  static_assert(DX == -1 || DX == 1, "lane shift by one");
  if constexpr (DX < 0) {
    if constexpr (AF && MF)
      asm(NSE_PAIR_ASM(NSE_A_MUL, NSE_M_MUL, NSE_DPP_L) : "=&v"(a), "=&v"(m) : NSE_PAIR_IN);
    else if constexpr (AF)
      asm(NSE_PAIR_ASM(NSE_A_MUL, NSE_M_FMA, NSE_DPP_L) : "=&v"(a), "+v"(m) : NSE_PAIR_IN);
    else if constexpr (MF)
      asm(NSE_PAIR_ASM(NSE_A_FMA, NSE_M_MUL, NSE_DPP_L) : "+v"(a), "=&v"(m) : NSE_PAIR_IN);
    else
      asm(NSE_PAIR_ASM(NSE_A_FMA, NSE_M_FMA, NSE_DPP_L) : "+v"(a), "+v"(m) : NSE_PAIR_IN);
  } else {
    if constexpr (AF && MF)
      asm(NSE_PAIR_ASM(NSE_A_MUL, NSE_M_MUL, NSE_DPP_R) : "=&v"(a), "=&v"(m) : NSE_PAIR_IN);
    else if constexpr (AF)
      asm(NSE_PAIR_ASM(NSE_A_MUL, NSE_M_FMA, NSE_DPP_R) : "=&v"(a), "+v"(m) : NSE_PAIR_IN);
    else if constexpr (MF)
      asm(NSE_PAIR_ASM(NSE_A_FMA, NSE_M_MUL, NSE_DPP_R) : "+v"(a), "=&v"(m) : NSE_PAIR_IN);
    else
      asm(NSE_PAIR_ASM(NSE_A_FMA, NSE_M_FMA, NSE_DPP_R) : "+v"(a), "+v"(m) : NSE_PAIR_IN);
  }
}
#undef NSE_PAIR_IN
#undef NSE_M_FMA
#undef NSE_M_MUL
#undef NSE_A_FMA
#undef NSE_A_MUL
#undef NSE_PAIR_ASM
#undef NSE_DPP_R
#undef NSE_DPP_L

// nse32_node in the register window.  Each node holds the differences to
// its +e_p neighbours (dc: this row; dp: the row before), and its difference
// to x - e_p is minus that neighbour's (exactly: d and -d round alike).  The
// sign goes into the constants, c * (-d) = (-c) * d exactly, so every term
// keeps its value and its place in the sums of nse32_node, and the results
// agree with it bit for bit; the terms that read the lane beside take the
// shift inside their multiply-add (nse_pair_sh).  vc: nse32_node's per-pair
// constants, with the negated ones, in VGPRs.
struct NseLaneC {
  float cP[4], ncP[4], cM[4], sMp[4], sPp[4], nsPp[4];
};

template <class L>
__device__ __forceinline__ NseLaneC nse_lane_consts(const KC<float> &kc) {
  static_assert(L::P <= 4, "2D pair lattices");
  NseLaneC v;
  static_for<L::P>([&](auto PI) {
    constexpr int P = decltype(PI)::value;
    constexpr int J = L::PR[P];
    const float cP = kc.nw[P][0], cM = kc.nw[P][1], bP = kc.nw[P][2], bM = kc.nw[P][3];
    float sP = bP, sM = bM;
    if constexpr (nse32_ncomp<L, P>() == 1) {
      constexpr int a = L::E[J][0] != 0 ? 0 : 1;
      if constexpr (L::E[J][a] < 0) {
        sP = -bP;
        sM = -bM;
      }
    }
    v.cP[P] = cP;
    v.ncP[P] = -cP;
    v.cM[P] = cM;
    v.sMp[P] = sM;
    v.sPp[P] = sP;
    v.nsPp[P] = -sP;
  });
  // keep them in VGPRs: a DPP multiply-add takes no scalar operand
  float *f = &v.cP[0];
#pragma unroll
  for (int i = 0; i < 6 * 4; ++i) asm volatile("" : "+v"(f[i]));
  return v;
}

template <class L, bool THREE>
__device__ __forceinline__ void nse32_node_lane(const float *dc, const float *dp,
                                                const float *cur_c, const float *prev_c,
                                                float *out_c, const KC<float> &kc,
                                                const NseLaneC &vc) {
  constexpr int D = L::D;
  float acc = 0.f, mo[D];
#pragma unroll
  for (int a = 0; a < D; ++a) mo[a] = 0.f;
  static_for<L::P>([&](auto PI) {
    constexpr int P = decltype(PI)::value;
    constexpr int J = L::PR[P];
    constexpr int ex = L::E[J][0], ey = L::E[J][1];
    constexpr bool single = nse32_ncomp<L, P>() == 1;
    constexpr int sa = ex != 0 ? 0 : 1;  // the component of a single-component pair
    const float pP = dc[2 * P], mP = dc[2 * P + 1];
    // the neighbour x - e_p's differences (negated through the constants)
    const float *dn = ey == 1 ? dp : dc;
    const float dpP = dn[2 * P], dmP = dn[2 * P + 1];
    float b;  // the momentum sum of a pair with two components
    if constexpr (ex != 0) {
      constexpr bool mf = !single || nse32_first_pair<L>(sa) == P;
      nse_pair_sh<-ex, P == 0, mf>(acc, single ? mo[sa] : b, pP, mP, dpP, dmP, vc.cP[P],
                                   vc.ncP[P], vc.cM[P], vc.sMp[P], vc.sPp[P], vc.nsPp[P]);
    } else {
      // rho: cP pP + cP pM + cM mP - cM mM, pM = -dpP, mM = -dmP
      if constexpr (P == 0) acc = vc.cP[P] * pP;
      else acc = __builtin_fmaf(vc.cP[P], pP, acc);
      acc = __builtin_fmaf(vc.ncP[P], dpP, acc);
      acc = __builtin_fmaf(vc.cM[P], mP, acc);
      acc = __builtin_fmaf(vc.cM[P], dmP, acc);
      float &m = single ? mo[sa] : b;
      if constexpr (!single || nse32_first_pair<L>(sa) == P) m = vc.sMp[P] * pP;
      else m = __builtin_fmaf(vc.sMp[P], pP, m);
      m = __builtin_fmaf(vc.sMp[P], dpP, m);
      m = __builtin_fmaf(vc.sPp[P], mP, m);
      m = __builtin_fmaf(vc.nsPp[P], dmP, m);
    }
    if constexpr (!single) {
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
      const float t = __builtin_fmaf(f == 0 ? -kc.Ah0t : -kc.Abh0t, c - prev_c[f], d);
      out_c[f] = c + t;
    } else {
      out_c[f] = __builtin_fmaf(f == 0 ? kc.A0t : kc.Ab0t, c, d);
    }
  }
}

__device__ __forceinline__ int xcd_remap_nse(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}
}  // namespace

// Window with origin (x0, y0): load, TBS steps, store of the interior that
// starts TBW nodes in.  WRAP_ANY: grids of any size; otherwise nx >= W and
// ny >= H (one conditional wrap).
template <class L, bool THREE, int W, int RG, int R, bool WRAP_ANY, typename T>
__device__ __forceinline__ void nse_window(const T *__restrict__ cur, const T *__restrict__ prev,
                                           T *__restrict__ out_cur, T *__restrict__ out_prev,
                                           int nx, int ny, int TBW, int TBS, int x0, int y0,
                                           const KC<T> &kc, T *pf) {
  using Rc = Rec<L, kNSE>;
  constexpr int NR = Rc::NR, NF = Rc::NF, NPF = 2 * L::P;
  constexpr int H = R * RG;
  const int64_t N = (int64_t)nx * ny;
  const int xx = threadIdx.x % W, rg = threadIdx.x / W;
  const int yr = rg * R;  // first row of this thread
  auto wrap = [&](int i, int n) {
    if constexpr (WRAP_ANY) return wrapi(i, n);
    else return i < 0 ? i + n : (i >= n ? i - n : i);
  };

  // binary32: the unweighted pair form of nse32_parts / nse32_node; each
  // thread keeps its own nodes' parts of the step in registers
  constexpr bool F32 = std::is_same<T, float>::value;
  T cm[R][NF], pm[R][NF];
  T own[F32 ? R : 1][NPF];
  {
    const int gx = wrap(x0 + xx, nx);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int gy = wrap(y0 + yr + r, ny);
      const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        cm[r][q] = cur[q * N + gi];
        pm[r][q] = THREE ? prev[q * N + gi] : T(0);
      }
    }
  }
#pragma unroll 1
  for (int t = 1; t <= TBS; ++t) {
    // A: pair parts on the region t - 1 nodes in
    if (xx >= t - 1 && xx < W - t + 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = yr + r;
        if (y >= t - 1 && y < H - t + 1) {
          T f[NPF];
          if constexpr (F32) {
            nse32_parts<L>(cm[r], f, kc);
#pragma unroll
            for (int q = 0; q < NPF; ++q) own[r][q] = f[q];
          } else {
            T rec[NR];
            make_record<L, kNSE>(cm[r], rec, kc);
            pair_parts<L, kNSE>(rec, f, kc);
          }
#pragma unroll
          for (int q = 0; q < NPF; ++q) pf[(q * H + y) * W + xx] = f[q];
        }
      }
    }
    __syncthreads();
    // B: node updates on the region t nodes in
    if (xx >= t && xx < W - t) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = yr + r;
        if (y >= t && y < H - t) {
          T oc[NF];
          if constexpr (F32) {
            auto at = [&](int q, int, int dy, int dx) { return pf[(q * H + y + dy) * W + xx + dx]; };
            nse32_node<L, THREE>(at, own[r], cm[r], pm[r], oc, kc);
          } else {
            auto at = [&](int q, int, int dy, int dx) { return pf[(q * H + y + dy) * W + xx + dx]; };
            auto ath = [&](int, int, int, int) { return T(0); };
            mmfd_node<L, kNSE, THREE, false, T, false, true>(at, ath, cm[r], pm[r], oc, kc);
          }
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            pm[r][q] = cm[r][q];
            cm[r][q] = oc[q];
          }
        }
      }
    }
    __syncthreads();
  }
  // store the interior of the last level (and the one before it)
  if (xx >= TBW && xx < W - TBW) {
    const int gx = x0 + xx;
    if (gx < nx) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = yr + r;
        const int gy = y0 + y;
        if (y >= TBW && y < H - TBW && gy < ny) {
          const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            out_cur[q * N + gi] = cm[r][q];
            if constexpr (THREE) out_prev[q * N + gi] = pm[r][q];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- binary32
// The binary32 window with the parts kept in registers: a thread owns one
// column (its lane) and kNseRR consecutive rows, whose moments at t and
// t - dt stay in its registers across the launch's steps.  A step forms the
// pair parts (nse32_parts) of each of the thread's rows as the update slides
// down them; the node update (nse32_node) reads the parts of the columns
// beside from the lanes beside (DPP) and those of the rows above and below
// from the thread's own registers, except for the row above its first row
// and the row below its last, which the neighbouring wavefronts own: the
// parts of every wavefront's first and last rows pass through LDS (two slots
// by step parity, so one barrier a step suffices).  Lanes at the wavefront's
// edges read 0 for their missing neighbour; like every node outside the
// step's region their values are not used by any node of the region.
// Each node forms its differences to its +e_p neighbours once; the node
// beside (same row, or the next row for pairs with a y component) takes them
// negated as its differences to x - e_p (nse32_node_lane).  The new level
// is written over the registers of the oldest one, and two steps per loop
// turn swap the roles of the two register sets, so nothing is copied.
template <class L, bool THREE, int RG, bool WRAP_ANY>
__device__ __forceinline__ void nse_window_reg(const float *__restrict__ cur,
                                               const float *__restrict__ prev,
                                               float *__restrict__ out_cur,
                                               float *__restrict__ out_prev, int nx, int ny,
                                               int TBW, int TBS, int x0, int y0,
                                               const KC<float> &kc, float *bnd) {
  constexpr int NF = 1 + L::D, NPF = 2 * L::P, R = kNseRR, W = 64;
  constexpr int H = R * RG;
  constexpr int SLOT = RG * 2 * NPF * W;  // one parity's slots
  const int64_t N = (int64_t)nx * ny;
  const int lane = threadIdx.x & 63;
  const int rg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int yr = rg * R;
  auto wrap = [&](int i, int n) {
    if constexpr (WRAP_ANY) return wrapi(i, n);
    else return i < 0 ? i + n : (i >= n ? i - n : i);
  };
  float cm[R][NF], pm[R][NF];
  {
    const int gx = wrap(x0 + lane, nx);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int gy = wrap(y0 + yr + r, ny);
      const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        cm[r][q] = cur[q * N + gi];
        pm[r][q] = THREE ? prev[q * N + gi] : 0.f;
      }
    }
  }
  // slot (parity, wavefront, 0 = first row / 1 = last row, part, lane)
  auto sl = [&](int par, int g, int end, int q) -> float & {
    return bnd[par * SLOT + ((g * 2 + end) * NPF + q) * W + lane];
  };
  const int ga = rg > 0 ? rg - 1 : rg, gb = rg < RG - 1 ? rg + 1 : rg;
  const NseLaneC vc = nse_lane_consts<L>(kc);
  // One step: c holds the moments at t - dt, p those at t - 2 dt; the new
  // level is written over p (the update reads each node's p before), so
  // the two roles swap from step to step and no register is copied.
  auto step = [&](int t, float (&c)[R][NF], float (&p)[R][NF]) {
    const int par = t & 1;
    {
      float f[NPF];
      nse32_parts<L>(c[0], f, kc);
#pragma unroll
      for (int q = 0; q < NPF; ++q) sl(par, rg, 0, q) = f[q];
      nse32_parts<L>(c[R - 1], f, kc);
#pragma unroll
      for (int q = 0; q < NPF; ++q) sl(par, rg, 1, q) = f[q];
    }
    __syncthreads();
    // parts of the rows r - 1, r, r + 1 of the slide
    float pa[NPF], pb[NPF], pc[NPF];
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      pa[q] = sl(par, ga, 1, q);  // the last row of the wavefront above
      pb[q] = sl(par, rg, 0, q);  // this thread's first row
    }
    // Each node forms the differences to its +e_p neighbour only,
    // d(x) = G(x + e_p) - G(x); its difference to x - e_p is -d(x - e_p),
    // exactly, taken from the lane beside (pairs in the row) or from the
    // previous row's registers (pairs with a y component, which all have
    // e_y = 1 as representatives).
    auto shx = [](float v, int dx) {
      return dx < 0 ? nse_from_left(v) : (dx > 0 ? nse_from_right(v) : v);
    };
    float dprev[NPF], dcur[NPF];
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      constexpr int ex = L::E[J][0], ey = L::E[J][1];
      static_assert(ey == 0 || ey == 1, "pair representatives point up or along x");
      if constexpr (ey == 1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) dprev[2 * P + h] = shx(pb[2 * P + h], ex) - pa[2 * P + h];
      }
    });
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r + 1 < R - 1) {
        nse32_parts<L>(c[r + 1], pc, kc);
      } else {
#pragma unroll
        for (int q = 0; q < NPF; ++q) pc[q] = r + 1 == R - 1 ? sl(par, rg, 1, q) : sl(par, gb, 0, q);
      }
      static_for<L::P>([&](auto PI) {
        constexpr int P = decltype(PI)::value;
        constexpr int J = L::PR[P];
        constexpr int ex = L::E[J][0], ey = L::E[J][1];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          dcur[2 * P + h] = shx(ey == 1 ? pc[2 * P + h] : pb[2 * P + h], ex) - pb[2 * P + h];
          // formed here, before the row's branch, so that the lane shift
          // stays fused into the subtraction
          asm("" : "+v"(dcur[2 * P + h]));
        }
      });
      const int y = yr + r;
      if (y >= t && y < H - t) {
        float oc[NF];
        nse32_node_lane<L, THREE>(dcur, dprev, c[r], p[r], oc, kc, vc);
#pragma unroll
        for (int q = 0; q < NF; ++q) p[r][q] = oc[q];
      }
#pragma unroll
      for (int q = 0; q < NPF; ++q) {
        pa[q] = pb[q];
        pb[q] = pc[q];
        dprev[q] = dcur[q];
      }
    }
  };
  int t = 1;
#pragma unroll 1
  for (; t + 1 <= TBS; t += 2) {
    step(t, cm, pm);
    step(t + 1, pm, cm);
  }
  if (t <= TBS) {
    step(t, cm, pm);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const float v = pm[r][q];
        pm[r][q] = cm[r][q];
        cm[r][q] = v;
      }
    }
  }
  // store the interior of the last level (and the one before it)
  if (lane >= TBW && lane < W - TBW) {
    const int gx = x0 + lane;
    if (gx < nx) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = yr + r;
        const int gy = y0 + y;
        if (y >= TBW && y < H - TBW && gy < ny) {
          const int64_t gi = (int64_t)gy * nx + gx;
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            out_cur[q * N + gi] = cm[r][q];
            if constexpr (THREE) out_prev[q * N + gi] = pm[r][q];
          }
        }
      }
    }
  }
}

template <class L, bool THREE, int RG>
__global__ __launch_bounds__(64 * RG) void k_nse_tb_reg(const float *__restrict__ cur,
                                                       const float *__restrict__ prev,
                                                       float *__restrict__ out_cur,
                                                       float *__restrict__ out_prev, int nx, int ny,
                                                       int TB, int tiles_x, int ntiles,
                                                       KC<float> kc) {
  extern __shared__ float smem_nse_reg[];
  constexpr int H = kNseRR * RG;
  const int TX = 64 - 2 * TB, TY = H - 2 * TB;
  const int tile = xcd_remap_nse(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  nse_window_reg<L, THREE, RG, false>(cur, prev, out_cur, out_prev, nx, ny, TB, TB, x0, y0, kc,
                                      smem_nse_reg);
}

template <class L, bool THREE, int RG>
__global__ __launch_bounds__(64 * RG) void k_batch_nse_tb_reg(const BatchInst<float> *__restrict__ inst,
                                                             const int *__restrict__ tile_inst,
                                                             int ntiles, int64_t launch, int TB) {
  extern __shared__ float smem_bnse_reg[];
  constexpr int H = kNseRR * RG;
  const int t = xcd_remap_nse(blockIdx.x, ntiles);
  const BatchInst<float> &I = inst[tile_inst[t]];
  const int64_t left = I.nsteps - launch * TB;
  const int TBS = left < TB ? (int)left : TB;
  const int TX = 64 - 2 * TB, TY = H - 2 * TB;
  const int lt = t - I.tile0;
  const int x0 = (lt % I.tiles_x) * TX - TB, y0 = (lt / I.tiles_x) * TY - TB;
  const int64_t r = I.c0 + launch;
  const float *cur, *prev;
  float *oc, *op;
  if constexpr (THREE) {
    const int a = (int)(r & 1) * 2, b = 2 - a;
    cur = I.ring[a];
    prev = I.ring[a + 1];
    oc = I.ring[b];
    op = I.ring[b + 1];
  } else {
    cur = I.ring[r & 1];
    prev = nullptr;
    oc = I.ring[(r + 1) & 1];
    op = nullptr;
  }
  nse_window_reg<L, THREE, RG, true>(cur, prev, oc, op, I.nx, I.ny, TB, TBS, x0, y0, I.kc,
                                     smem_bnse_reg);
}

template <class L, bool THREE, int W, int RG, int R, typename T>
__global__ __launch_bounds__(W *RG) void k_nse_tb(const T *__restrict__ cur,
                                                 const T *__restrict__ prev,
                                                 T *__restrict__ out_cur, T *__restrict__ out_prev,
                                                 int nx, int ny, int TB, int tiles_x, int ntiles,
                                                 KC<T> kc) {
  extern __shared__ unsigned char smem_nse[];
  constexpr int H = R * RG;
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int tile = xcd_remap_nse(blockIdx.x, ntiles);
  const int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  nse_window<L, THREE, W, RG, R, false, T>(cur, prev, out_cur, out_prev, nx, ny, TB, TB, x0, y0, kc,
                                           reinterpret_cast<T *>(smem_nse));
}

// Batched: launch `launch` of a run whose launches advance TB steps; the
// ring holds (t, t - dt) in ring[0..1] and the other pair in ring[2..3]
// (three-level), or t and the spare level in ring[0..1] (two-level).
template <class L, bool THREE, int W, int RG, int R, typename T>
__global__ __launch_bounds__(W *RG) void k_batch_nse_tb(const BatchInst<T> *__restrict__ inst,
                                                       const int *__restrict__ tile_inst,
                                                       int ntiles, int64_t launch, int TB) {
  extern __shared__ unsigned char smem_bnse[];
  constexpr int H = R * RG;
  const int t = xcd_remap_nse(blockIdx.x, ntiles);
  const BatchInst<T> &I = inst[tile_inst[t]];
  const int64_t left = I.nsteps - launch * TB;
  const int TBS = left < TB ? (int)left : TB;
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int lt = t - I.tile0;
  const int x0 = (lt % I.tiles_x) * TX - TB, y0 = (lt / I.tiles_x) * TY - TB;
  const int64_t r = I.c0 + launch;
  const T *cur, *prev;
  T *oc, *op;
  if constexpr (THREE) {
    const int a = (int)(r & 1) * 2, b = 2 - a;
    cur = I.ring[a];
    prev = I.ring[a + 1];
    oc = I.ring[b];
    op = I.ring[b + 1];
  } else {
    cur = I.ring[r & 1];
    prev = nullptr;
    oc = I.ring[(r + 1) & 1];
    op = nullptr;
  }
  nse_window<L, THREE, W, RG, R, true, T>(cur, prev, oc, op, I.nx, I.ny, TB, TBS, x0, y0, I.kc,
                                          reinterpret_cast<T *>(smem_bnse));
}

// ------------------------------------------------------------ host side
// binary32 64 x 64 and 64 x 128 windows run the register window
// (kNseRR rows per thread); the others the LDS window
static bool nse_reg_plan(const TbPlan &pl, int elem) {
  return elem == 4 && (pl.h == 64 || pl.h == 128);
}
static size_t nse_reg_lds(int h, int npair) {
  return (size_t)2 * (h / kNseRR) * 2 * (2 * npair) * kNseW * sizeof(float);
}

bool nse_tb_plan_valid(const TbPlan &pl, int npair, int elem) {
  // 64 x 32 (2 rows per thread) or 64 x 64 windows (4 rows per thread);
  // binary32: 64 x 64 or 64 x 128 (8 rows per thread, register window)
  if (pl.w != kNseW) return false;
  if (pl.h != 32 && pl.h != 64 && !nse_reg_plan(pl, elem)) return false;
  if (pl.tb < 1 || pl.h - 2 * pl.tb < 8 || pl.w - 2 * pl.tb < 8) return false;
  if (nse_reg_plan(pl, elem)) return nse_reg_lds(pl.h, npair) <= 160 * 1024;
  return (size_t)2 * npair * pl.h * pl.w * elem <= 160 * 1024;
}

namespace {

template <class L, bool THREE, int RG, typename T, int R = kNseR>
hipError_t nse_tb_cfg(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                      const T *prev, T *oc, T *op, hipStream_t st) {
  const KC<T> kc = make_kc<T>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  constexpr int H = R * RG;
  const int TX = kNseW - 2 * pl.tb, TY = H - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)2 * L::P * H * kNseW * sizeof(T);  // the pair parts
  auto fn = k_nse_tb<L, THREE, kNseW, RG, R, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(kNseW * RG), lds, st, cur, prev, oc, op, nx, ny,
                     pl.tb, tx, tx * ty, kc);
  return hipGetLastError();
}

template <class L, bool THREE, int RG>
hipError_t nse_reg_cfg(const Consts &c, const Grid &g, const TbPlan &pl, const float *cur,
                       const float *prev, float *oc, float *op, hipStream_t st) {
  const KC<float> kc = make_kc<float>(c);
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  constexpr int H = kNseRR * RG;
  const int TX = kNseW - 2 * pl.tb, TY = H - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = nse_reg_lds(H, L::P);
  auto fn = k_nse_tb_reg<L, THREE, RG>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(64 * RG), lds, st, cur, prev, oc, op, nx, ny, pl.tb,
                     tx, tx * ty, kc);
  return hipGetLastError();
}

template <class L, typename T>
hipError_t nse_tb_l(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, const T *prev,
                    T *oc, T *op, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (nse_reg_plan(pl, 4)) {
      if (pl.h == 64) {
        if (c.three) return nse_reg_cfg<L, true, 8>(c, g, pl, cur, prev, oc, op, st);
        return nse_reg_cfg<L, false, 8>(c, g, pl, cur, prev, oc, op, st);
      }
      if (c.three) return nse_reg_cfg<L, true, 16>(c, g, pl, cur, prev, oc, op, st);
      return nse_reg_cfg<L, false, 16>(c, g, pl, cur, prev, oc, op, st);
    }
  }
  if (pl.h == 32) {
    if (c.three) return nse_tb_cfg<L, true, 16, T, 2>(c, g, pl, cur, prev, oc, op, st);
    return nse_tb_cfg<L, false, 16, T, 2>(c, g, pl, cur, prev, oc, op, st);
  }
  if (c.three) return nse_tb_cfg<L, true, 16, T>(c, g, pl, cur, prev, oc, op, st);
  return nse_tb_cfg<L, false, 16, T>(c, g, pl, cur, prev, oc, op, st);
}

template <class L, bool THREE, int RG, typename T, int R = kNseR>
hipError_t bnse_cfg(const BatchInst<T> *inst, const int *tile_inst, int ntiles, int64_t launch,
                    const TbPlan &pl, hipStream_t st) {
  constexpr int H = R * RG;
  const size_t lds = (size_t)2 * L::P * H * kNseW * sizeof(T);
  auto fn = k_batch_nse_tb<L, THREE, kNseW, RG, R, T>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(ntiles), dim3(kNseW * RG), lds, st, inst, tile_inst, ntiles, launch,
                     pl.tb);
  return hipGetLastError();
}

template <class L, bool THREE, int RG>
hipError_t bnse_reg_cfg(const BatchInst<float> *inst, const int *tile_inst, int ntiles,
                        int64_t launch, const TbPlan &pl, hipStream_t st) {
  const size_t lds = nse_reg_lds(kNseRR * RG, L::P);
  auto fn = k_batch_nse_tb_reg<L, THREE, RG>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(ntiles), dim3(64 * RG), lds, st, inst, tile_inst, ntiles, launch,
                     pl.tb);
  return hipGetLastError();
}

template <class L, typename T>
hipError_t bnse_l(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst, int ntiles,
                  int64_t launch, const TbPlan &pl, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (nse_reg_plan(pl, 4)) {
      if (pl.h == 64) {
        if (k.three) return bnse_reg_cfg<L, true, 8>(inst, tile_inst, ntiles, launch, pl, st);
        return bnse_reg_cfg<L, false, 8>(inst, tile_inst, ntiles, launch, pl, st);
      }
      if (k.three) return bnse_reg_cfg<L, true, 16>(inst, tile_inst, ntiles, launch, pl, st);
      return bnse_reg_cfg<L, false, 16>(inst, tile_inst, ntiles, launch, pl, st);
    }
  }
  if (pl.h == 32) {
    if (k.three) return bnse_cfg<L, true, 16, T, 2>(inst, tile_inst, ntiles, launch, pl, st);
    return bnse_cfg<L, false, 16, T, 2>(inst, tile_inst, ntiles, launch, pl, st);
  }
  if (k.three) return bnse_cfg<L, true, 16, T>(inst, tile_inst, ntiles, launch, pl, st);
  return bnse_cfg<L, false, 16, T>(inst, tile_inst, ntiles, launch, pl, st);
}

}  // namespace

template <typename T>
hipError_t launch_nse_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                         const T *prev, T *out_cur, T *out_prev, hipStream_t st) {
  if (c.three_stencil) return hipErrorInvalidValue;
  if (c.lattice == 3) return nse_tb_l<LatD2Q9, T>(c, g, pl, cur, prev, out_cur, out_prev, st);
  if (c.lattice == 2) return nse_tb_l<LatD2Q5, T>(c, g, pl, cur, prev, out_cur, out_prev, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batch_nse_tb(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst,
                               int ntiles, int64_t launch, const TbPlan &pl, hipStream_t st) {
  if (k.three_st || k.eq != kNSE) return hipErrorInvalidValue;
  if (k.lattice == 3) return bnse_l<LatD2Q9, T>(k, inst, tile_inst, ntiles, launch, pl, st);
  if (k.lattice == 2) return bnse_l<LatD2Q5, T>(k, inst, tile_inst, ntiles, launch, pl, st);
  return hipErrorInvalidValue;
}

#define MFD_INST(T)                                                                               \
  template hipError_t launch_nse_tb<T>(const Consts &, const Grid &, const TbPlan &, const T *,  \
                                       const T *, T *, T *, hipStream_t);                         \
  template hipError_t launch_batch_nse_tb<T>(const BatchKey &, const BatchInst<T> *, const int *, \
                                             int, int64_t, const TbPlan &, hipStream_t);
MFD_INST(float)
MFD_INST(double)
#undef MFD_INST

}  // namespace mfd
