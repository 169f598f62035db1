// Temporally blocked binary32 MMFD steps of the two-level linear CDE and of
// Burgers' equation (beta = 1) on D2Q5 / D2Q9: one launch advances TB time
// steps of a 128-column window updated in place, with neighbour values
// shared across the lanes of a wavefront instead of formed again or read
// again from LDS.  Results equal the single-step kernel's value for value.
//
// Linear CDE (Eq. (LMMFD-3)): the binary32 pair form of the single-step
// kernel (mmfd_node): acc = sum over pairs p of A+_p (phi(x + e_p) - phi(x))
// and A-_p (phi(x - e_p) - phi(x)), in pair order, then phi' = A0 phi + acc.
// Each difference phi(x - e_p) - phi(x) is the negative of a difference
// phi(y + e_p) - phi(y) that the node y = x - e_p forms for its own first
// term, so every node forms one difference per pair (4 on D2Q9) and takes
// the other from where it was formed: from the lane to its left or right by
// a DPP lane shift fused into the subtraction or multiply-add, from the
// lane's other column, or for the row below from its own registers of the
// previous row.  Negation is exact.
//
// Burgers' equation (Eq. (2-2-1) with the EDF of Eq. (3-4)): each node forms
// its pair parts F+-_p once and shares them the same way (see BurgSeg).
#include <cstring>
#include <map>
#include <type_traits>
#include <mutex>
#include <tuple>

#include "../../include/mfd.h"
#include "batch_kernels.h"
#include "edf.h"
#include "mesofd_node.h"
#include "mfd_internal.h"
#include "mmfd_node.h"

namespace mfd {

namespace {

struct LinC {
  float ap[4], nam[4];  // A+_p and -A-_p
  float a0;
};

__device__ __forceinline__ int xcd_remap_l(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// value of the lane one above (lane + 1) / one below (lane - 1) in the
// wavefront; lanes without a source read 0
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// acc + x[lane - 1] * c and acc + x[lane + 1] * c, one fused multiply-add with
// the lane shift on its first source.  The two wait states before it let a
// value written by the instruction just before be read through the shift.
__device__ __forceinline__ float fmac_from_left(float acc, float x, float c) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(x), "v"(c));
  return acc;
}
__device__ __forceinline__ float fmac_from_right(float acc, float x, float c) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(x), "v"(c));
  return acc;
}

// LDS-only barrier: waits for this wavefront's LDS operations, not for its
// global loads (the next window's loads stay in flight across the steps)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// the two-column value of a lane's row, in the precision T
template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
  using type = float2;
};
template <>
struct Pair2<double> {
  using type = double2;
};
template <typename T>
using V2 = typename Pair2<T>::type;
template <typename T>
__device__ __forceinline__ V2<T> mk2(T a, T b) {
  V2<T> v;
  v.x = a;
  v.y = b;
  return v;
}

// binary64 lane shifts: the two halves moved by DPP (lanes without a
// source read 0)
template <int CTRL>
__device__ __forceinline__ double shift64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double v) { return shift64<0x130>(v); }
__device__ __forceinline__ double from_left(double v) { return shift64<0x138>(v); }

}  // namespace

// Lane l owns columns 2l and 2l + 1 of a 128-column window (one wavefront
// spans it; its first and last columns, whose neighbours lie outside the
// wavefront, are never updated: every step updates a region one node smaller
// than the last), and the window lives in one LDS buffer updated in place.
// Wavefront g owns a segment of rows; it reads each row before it overwrites
// the row above it, and its two boundary rows (the row above its segment and
// the one below, which the neighbouring segments overwrite) are read into
// registers before a barrier at the start of every step.  Every lane computes
// its columns in every step; values outside the step's region are not used
// by any later update of the region.  The last step writes the tile's
// interior straight to global memory.
//
// Workgroups are persistent: workgroup b takes the tiles of the virtual
// blocks b, b + G, b + 2G, ... (G = gridDim.x; a multiple of 8 when there are
// more tiles than workgroups, so that every virtual block of a workgroup maps
// to tiles of its own XCD, else one workgroup per tile).  While a tile's
// steps run, the next tile's window is loaded into registers, and it goes to
// the buffer after the last step.
template <int P>
struct PairNode {
  // rc: row y, rn: row y + 1 of this lane's two columns; d*: the differences
  // of row y - 1 (e: column 2l, o: column 2l + 1); returns the new values
  // and leaves the differences of row y in d*.
  float ap[4], nam[4], a0;
  __device__ __forceinline__ float2 operator()(float2 rc, float2 rn, float &dye, float &dyo,
                                               float &dde, float &ddo, float &dae,
                                               float &dao) const {
    // x differences: phi(x+1, y) - phi(x, y)
    const float dxe = rc.y - rc.x;
    const float dxo = from_right(rc.x) - rc.y;
    const float nye = rn.x - rc.x, nyo = rn.y - rc.y;
    // column 2l: left neighbour's x difference from lane l - 1
    float ae = __builtin_fmaf(ap[0], dxe, 0.0f);
    ae = fmac_from_left(ae, dxo, nam[0]);
    ae = __builtin_fmaf(ap[1], nye, ae);
    ae = __builtin_fmaf(nam[1], dye, ae);
    // column 2l + 1: its left neighbour is column 2l of this lane
    float ao = __builtin_fmaf(ap[0], dxo, 0.0f);
    ao = __builtin_fmaf(nam[0], dxe, ao);
    ao = __builtin_fmaf(ap[1], nyo, ao);
    ao = __builtin_fmaf(nam[1], dyo, ao);
    dye = nye;
    dyo = nyo;
    if constexpr (P == 4) {
      // (1, 1): phi(x+1, y+1) - phi(x, y); (-1, 1): phi(x-1, y+1) - phi(x, y)
      const float nde = rn.y - rc.x, ndo = from_right(rn.x) - rc.y;
      const float nae = from_left(rn.y) - rc.x, nao = rn.x - rc.y;
      ae = __builtin_fmaf(ap[2], nde, ae);
      ae = fmac_from_left(ae, ddo, nam[2]);  // (2l-1, y-1): lane l - 1
      ae = __builtin_fmaf(ap[3], nae, ae);
      ae = __builtin_fmaf(nam[3], dao, ae);  // (2l+1, y-1): this lane
      ao = __builtin_fmaf(ap[2], ndo, ao);
      ao = __builtin_fmaf(nam[2], dde, ao);  // (2l, y-1): this lane
      ao = __builtin_fmaf(ap[3], nao, ao);
      ao = fmac_from_right(ao, dae, nam[3]);  // (2l+2, y-1): lane l + 1
      dde = nde;
      ddo = ndo;
      dae = nae;
      dao = nao;
    }
    return make_float2(__builtin_fmaf(a0, rc.x, ae), __builtin_fmaf(a0, rc.y, ao));
  }
};

// Row segment of the linear CDE: rows [ya, yb) of the window, `top` the row
// above, `bot` the row below (both read before the step's first barrier).
template <int P>
struct LinSeg {
  using Params = LinC;
  using T = float;
  static constexpr int kRG = 8, kNPF = 32;  // 8 wavefronts, 16 rows each
  static constexpr int kQ = 0;              // no populations
  PairNode<P> node;
  __device__ __forceinline__ explicit LinSeg(const LinC &kc) {
    node.a0 = kc.a0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      node.ap[p] = kc.ap[p];
      node.nam[p] = kc.nam[p];
      // in vector registers, so that the lane shifts fuse into the
      // multiply-adds
      asm("" : "+v"(node.ap[p]));
      asm("" : "+v"(node.nam[p]));
    }
  }
  template <class Emit>
  __device__ __forceinline__ void operator()(const float2 *lds, int lane, int ya, int yb,
                                             float2 top, float2 bot, const Emit &emit) const {
    float2 rc = lds[ya * 64 + lane];
    // differences of row ya - 1
    float dye = rc.x - top.x, dyo = rc.y - top.y;
    float dde = rc.y - top.x, ddo = from_right(rc.x) - top.y;
    float dae = from_left(rc.y) - top.x, dao = rc.x - top.y;
    int y = ya;
    // two rows per pass: both rows are read before either is written
    for (; y + 2 < yb; y += 2) {
      const float2 r1 = lds[(y + 1) * 64 + lane];
      const float2 r2 = lds[(y + 2) * 64 + lane];
      const float2 o1 = node(rc, r1, dye, dyo, dde, ddo, dae, dao);
      const float2 o2 = node(r1, r2, dye, dyo, dde, ddo, dae, dao);
      emit(y, o1);
      emit(y + 1, o2);
      rc = r2;
    }
    if (y + 1 < yb) {
      const float2 r1 = lds[(y + 1) * 64 + lane];
      const float2 o1 = node(rc, r1, dye, dyo, dde, ddo, dae, dao);
      const float2 o2 = node(r1, bot, dye, dyo, dde, ddo, dae, dao);
      emit(y, o1);
      emit(y + 1, o2);
    } else {
      emit(y, node(rc, bot, dye, dyo, dde, ddo, dae, dao));
    }
  }
};

// Burgers' equation with beta = 1 (D2Q9 or D2Q5), binary32: the node update
// of the single-step kernel (mmfd_node with the records phi and
// s = phi^2 dt / (2 dx)), whose pair parts are F+_p = w_p phi and
// F-_p = w1_p (e_p . (s, s)).  By the lattice symmetry they take four values
// per node: fa = w_a phi (axis pairs), fd = w_d phi (diagonal pairs),
// ga = w1_a s (axis pairs), gd = w1_d (s + s) (the (1, 1) pair; the (-1, 1)
// pair's is 0).  Each node forms its four once, when its row enters, and its
// neighbours take them from its lane (DPP) or from their own registers of
// the rows above and below, instead of forming them again from records.
struct BurgC {
  float wa, wd, w1a, w1d, bh, cpl, cmi, a0;
};

struct PP {  // pair parts of a lane's two columns
  float fae, fao, fde, fdo, gae, gao, gde, gdo;
};

template <int P>
struct BurgSeg {
  using Params = BurgC;
  using T = float;
  static constexpr int kRG = 16, kNPF = 16;  // 16 wavefronts, 8 rows each
  static constexpr int kQ = 0;               // no populations
  BurgC k;
  __device__ __forceinline__ explicit BurgSeg(const BurgC &kc) : k(kc) {}
  __device__ __forceinline__ PP parts(float2 r) const {
    PP q;
    const float se = (r.x * r.x) * k.bh, so = (r.y * r.y) * k.bh;
    q.fae = k.wa * r.x;
    q.fao = k.wa * r.y;
    q.gae = k.w1a * se;
    q.gao = k.w1a * so;
    if constexpr (P == 4) {
      q.fde = k.wd * r.x;
      q.fdo = k.wd * r.y;
      q.gde = k.w1d * (se + se);
      q.gdo = k.w1d * (so + so);
    } else {
      q.fde = q.fdo = q.gde = q.gdo = 0.0f;
    }
    return q;
  }
  // node update of row y: c, n, p the pair parts of rows y, y + 1, y - 1
  __device__ __forceinline__ float2 node(float2 rc, const PP &c, const PP &n,
                                         const PP &p) const {
    const float two = 2.0f;
    // column 2l: x - 1 is lane l - 1's column 2l - 1
    const float t2ae = two * c.fae;
    float ae = __builtin_fmaf(k.cpl, (c.fao - t2ae) + from_left(c.fao), 0.0f);
    ae = __builtin_fmaf(k.cmi, c.gao - from_left(c.gao), ae);
    ae = __builtin_fmaf(k.cpl, (n.fae - t2ae) + p.fae, ae);
    ae = __builtin_fmaf(k.cmi, n.gae - p.gae, ae);
    // column 2l + 1: x + 1 is lane l + 1's column 2l + 2
    const float t2ao = two * c.fao;
    float ao = __builtin_fmaf(k.cpl, (from_right(c.fae) - t2ao) + c.fae, 0.0f);
    ao = __builtin_fmaf(k.cmi, from_right(c.gae) - c.gae, ao);
    ao = __builtin_fmaf(k.cpl, (n.fao - t2ao) + p.fao, ao);
    ao = __builtin_fmaf(k.cmi, n.gao - p.gao, ao);
    if constexpr (P == 4) {
      // (1, 1): x + e = (x+1, y+1), x - e = (x-1, y-1)
      const float t2de = two * c.fde;
      ae = __builtin_fmaf(k.cpl, (n.fdo - t2de) + from_left(p.fdo), ae);
      ae = __builtin_fmaf(k.cmi, n.gdo - from_left(p.gdo), ae);
      // (-1, 1): x + e = (x-1, y+1), x - e = (x+1, y-1); its F- is 0
      ae = __builtin_fmaf(k.cpl, (from_left(n.fdo) - t2de) + p.fdo, ae);
      ae = __builtin_fmaf(k.cmi, 0.0f, ae);
      const float t2do = two * c.fdo;
      ao = __builtin_fmaf(k.cpl, (from_right(n.fde) - t2do) + p.fde, ao);
      ao = __builtin_fmaf(k.cmi, from_right(n.gde) - p.gde, ao);
      ao = __builtin_fmaf(k.cpl, (n.fde - t2do) + from_right(p.fde), ao);
      ao = __builtin_fmaf(k.cmi, 0.0f, ao);
    }
    return make_float2(__builtin_fmaf(k.a0, rc.x, ae), __builtin_fmaf(k.a0, rc.y, ao));
  }
  template <class Emit>
  __device__ __forceinline__ void operator()(const float2 *lds, int lane, int ya, int yb,
                                             float2 top, float2 bot, const Emit &emit) const {
    // three rows per pass: the pair parts of rows y - 1, y (pa, pb) and the
    // incoming row rotate through three register sets, so that none is copied
    float2 rc = lds[ya * 64 + lane];
    PP pa = parts(top), pb = parts(rc);
    int y = ya;
    for (; y + 3 < yb; y += 3) {
      const float2 r1 = lds[(y + 1) * 64 + lane];
      const float2 r2 = lds[(y + 2) * 64 + lane];
      const float2 r3 = lds[(y + 3) * 64 + lane];
      const PP p1 = parts(r1);
      const float2 o1 = node(rc, pb, p1, pa);
      const PP p2 = parts(r2);
      const float2 o2 = node(r1, p1, p2, pb);
      const PP p3 = parts(r3);
      const float2 o3 = node(r2, p2, p3, p1);
      emit(y, o1);
      emit(y + 1, o2);
      emit(y + 2, o3);
      rc = r3;
      pa = p2;
      pb = p3;
    }
    // the last one to three rows; the row below the segment is `bot`
    const int left = yb - y;
    const float2 r1 = left > 1 ? lds[(y + 1) * 64 + lane] : bot;
    const PP p1 = parts(r1);
    emit(y, node(rc, pb, p1, pa));
    if (left > 1) {
      const float2 r2 = left > 2 ? lds[(y + 2) * 64 + lane] : bot;
      const PP p2 = parts(r2);
      emit(y + 1, node(r1, p1, p2, pb));
      if (left > 2) emit(y + 2, node(r2, p2, parts(bot), p1));
    }
  }
};

// MesoFD form of the two-level linear CDE (Eq. (2-1), the moments by
// Eq. (2-1-1)): the node function of the single-step kernel (mesofd_pops,
// moments_of), whose EDF values are g_J(y) = ubar_J phi(y) for the moving
// directions and, at rest, g_0 = ubar_0 phi (binary64) or phi - sum_J g_J
// (binary32, so that a node's populations sum to phi).  Each node forms its
// products ubar_J phi once, when its row enters, and the populations
// f_J(x) = sum_k a_k g_J(x + k e_J) take their neighbours' from the lanes
// beside (DPP) or the rows' registers.  The populations of the launch's last
// step go to memory with the moment (when the launch is given a population
// buffer).  binary32 accumulates with fused
// multiply-adds, binary64 with a rounded product and sum, as the single-step
// kernel does.
template <typename T>
struct MesoC {
  T ub[9];  // ubar_J, J = 0 .. Q-1
  T a[3];   // a_k, k = -1, 0, +1
};

// AM: bit k + 1 set when a_k is not zero (the terms the scheme has)
template <class L, int AM, typename TT>
struct MesoSeg {
  using T = TT;
  using Params = MesoC<TT>;
  static constexpr bool F32 = std::is_same<TT, float>::value;
  // binary64 values take two registers: 8 wavefronts, 16 prefetch rows each
  static constexpr int kRG = F32 ? 16 : 8, kNPF = 256 / kRG;
  static constexpr int kQ = L::Q;
  static constexpr int QM = L::Q - 1;  // moving directions
  static constexpr bool ak[3] = {(AM & 1) != 0, (AM & 2) != 0, (AM & 4) != 0};
  T ub0, ub[QM], a[3];
  __device__ __forceinline__ explicit MesoSeg(const MesoC<TT> &kc) {
    ub0 = kc.ub[0];
#pragma unroll
    for (int j = 0; j < QM; ++j) ub[j] = kc.ub[j + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = kc.a[k];
      asm("" : "+v"(a[k]));  // a VGPR operand of the lane-shifted multiply-adds
    }
  }
  struct Row {  // a row's two columns: the products ubar_J phi and g_0
    T ue[QM], uo[QM], g0e, g0o;
  };
  __device__ __forceinline__ Row parts(V2<T> r) const {
    Row q;
    T se = T(0), so = T(0);
#pragma unroll
    for (int j = 0; j < QM; ++j) {
      q.ue[j] = ub[j] * r.x;
      q.uo[j] = ub[j] * r.y;
      se = se + q.ue[j];
      so = so + q.uo[j];
    }
    if constexpr (F32) {
      q.g0e = r.x - se;
      q.g0o = r.y - so;
    } else {
      q.g0e = ub0 * r.x;
      q.g0o = ub0 * r.y;
    }
    return q;
  }
  // f + c g in the single-step kernel's rounding
  __device__ __forceinline__ static T mac(T c, T g, T f) {
    if constexpr (F32) return __builtin_fmaf(c, g, f);
    else return c * g + f;
  }
  // f += a_k g, with g the product of direction J at column offset dx (-1,
  // 0, +1) from column 2l (ODD = 0) or 2l + 1 (ODD = 1) in row R
  template <int J, bool ODD>
  __device__ __forceinline__ T term(T f, int k, int dx, const Row &R) const {
    const int j = J - 1;
    if constexpr (!ODD) {
      if (dx < 0) {
        if constexpr (F32) return fmac_from_left(f, R.uo[j], a[k]);
        else return mac(a[k], from_left(R.uo[j]), f);
      }
      return mac(a[k], dx == 0 ? R.ue[j] : R.uo[j], f);
    } else {
      if (dx > 0) {
        if constexpr (F32) return fmac_from_right(f, R.ue[j], a[k]);
        else return mac(a[k], from_right(R.ue[j]), f);
      }
      return mac(a[k], dx == 0 ? R.uo[j] : R.ue[j], f);
    }
  }
  // the populations and the moment of row y (rows y - 1, y, y + 1: p, c, n)
  template <bool ODD>
  __device__ __forceinline__ T node(const Row &p, const Row &c, const Row &n,
                                    T (&fo)[L::Q]) const {
    // rest direction: g_0 at x for every k
    {
      T f = T(0);
      const T g = ODD ? c.g0o : c.g0e;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (ak[k]) f = mac(a[k], g, f);
      fo[0] = f;
    }
    static_for<L::Q - 1>([&](auto JI) {
      constexpr int J = decltype(JI)::value + 1;
      constexpr int ex = L::E[J][0], ey = L::E[J][1];
      T f = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (ak[k]) {
          const int dy = (k - 1) * ey, dx = (k - 1) * ex;
          const Row &R = dy < 0 ? p : (dy > 0 ? n : c);
          f = term<J, ODD>(f, k, dx, R);
        }
      }
      fo[J] = f;
    });
    T m = T(0);
#pragma unroll
    for (int j = 0; j < L::Q; ++j) m = m + fo[j];
    return m;
  }
  template <class Emit>
  __device__ __forceinline__ void operator()(const V2<T> *lds, int lane, int ya, int yb,
                                             V2<T> top, V2<T> bot, const Emit &emit) const {
    auto row = [&](int y, const Row &p, const Row &c, const Row &n) {
      T fe[L::Q], fo[L::Q];
      const T me = node<false>(p, c, n, fe);
      const T mo = node<true>(p, c, n, fo);
      emit(y, mk2<T>(me, mo), fe, fo);
    };
    Row pa = parts(top), pb = parts(lds[ya * 64 + lane]);
    int y = ya;
    // three rows per pass; each row's parts are formed just before the row
    // that needs them, so that at most four rows' are live
    for (; y + 3 < yb; y += 3) {
      const V2<T> r1 = lds[(y + 1) * 64 + lane];
      const V2<T> r2 = lds[(y + 2) * 64 + lane];
      const V2<T> r3 = lds[(y + 3) * 64 + lane];
      const Row p1 = parts(r1);
      row(y, pa, pb, p1);
      const Row p2 = parts(r2);
      row(y + 1, pb, p1, p2);
      const Row p3 = parts(r3);
      row(y + 2, p1, p2, p3);
      pa = p2;
      pb = p3;
    }
    const int left = yb - y;
    const Row p1 = parts(left > 1 ? lds[(y + 1) * 64 + lane] : bot);
    row(y, pa, pb, p1);
    if (left > 1) {
      const Row p2 = parts(left > 2 ? lds[(y + 2) * 64 + lane] : bot);
      row(y + 1, pb, p1, p2);
      if (left > 2) row(y + 2, p1, p2, parts(bot));
    }
  }
};

// Any two-level linear CDE or Burgers step, MMFD or MesoFD form, binary32
// or binary64, through the single-step kernels' node functions (mmfd_node;
// mesofd_pops and moments_of), which read the nine values around a node from
// an accessor: here the lane's two columns and their neighbours in the lanes
// beside (DPP, taken once per row) for the rows y - 1, y, y + 1 held in
// registers (Burgers' second record field, phi^2 dt / (2 dx), is formed from
// them where read).  The segment for the cases without a specialized one.
template <class L, int EQ, bool B1, bool MESO, typename TT>
struct AccSeg {
  using T = TT;
  using Params = KC<TT>;
  // binary32: 16 wavefronts, 8 prefetch rows each; binary64 (twice the
  // registers a value): 8 wavefronts, 16 rows each
  static constexpr int kRG = sizeof(TT) == 8 ? 8 : 16, kNPF = 256 / kRG;
  static constexpr int kQ = MESO ? L::Q : 0;
  const KC<TT> &kc;
  __device__ __forceinline__ explicit AccSeg(const KC<TT> &k) : kc(k) {}
  struct Row {  // this lane's columns 2l, 2l + 1 and the columns 2l - 1, 2l + 2
    T e, o, l, r;
  };
  __device__ __forceinline__ Row row(V2<T> v) const {
    Row q;
    q.e = v.x;
    q.o = v.y;
    q.l = from_left(v.y);
    q.r = from_right(v.x);
    return q;
  }
  // the new moment (and, MesoFD, populations) of column 2l (ODD = 0) or 2l + 1
  template <bool ODD>
  __device__ __forceinline__ T node(const Row &p, const Row &c, const Row &n,
                                    T (&fo)[MESO ? L::Q : 1]) const {
    auto val = [&](int dy, int dx) {
      const Row &R = dy < 0 ? p : (dy > 0 ? n : c);
      if constexpr (ODD) return dx < 0 ? R.e : (dx == 0 ? R.o : R.r);
      else return dx < 0 ? R.l : (dx == 0 ? R.e : R.o);
    };
    auto at = [&](int q, int, int dy, int dx) {
      const T v = val(dy, dx);
      if constexpr (EQ == kBurgers) return q == 0 ? v : (v * v) * kc.bh;
      else return v;
    };
    auto ath = [&](int, int, int, int) { return T(0); };
    if constexpr (MESO) {
      T m[1];
      mesofd_pops<L, EQ, false, B1>(at, ath, (const T *)nullptr, false, fo, kc);
      moments_of<L, EQ>(fo, m);
      return m[0];
    } else {
      T cc[1] = {ODD ? c.o : c.e}, pc[1] = {T(0)}, oc[1];
      mmfd_node<L, EQ, false, false, T, B1>(at, ath, cc, pc, oc, kc);
      return oc[0];
    }
  }
  template <class Emit>
  __device__ __forceinline__ void operator()(const V2<T> *lds, int lane, int ya, int yb,
                                             V2<T> top, V2<T> bot, const Emit &emit) const {
    auto one = [&](int y, const Row &p, const Row &c, const Row &n) {
      T fe[MESO ? L::Q : 1], fo[MESO ? L::Q : 1];
      const T me = node<false>(p, c, n, fe);
      const T mo = node<true>(p, c, n, fo);
      if constexpr (MESO) emit(y, mk2<T>(me, mo), fe, fo);
      else emit(y, mk2<T>(me, mo));
    };
    Row pa = row(top), pb = row(lds[ya * 64 + lane]);
    int y = ya;
    for (; y + 3 < yb; y += 3) {
      const Row p1 = row(lds[(y + 1) * 64 + lane]);
      const Row p2 = row(lds[(y + 2) * 64 + lane]);
      const Row p3 = row(lds[(y + 3) * 64 + lane]);
      one(y, pa, pb, p1);
      one(y + 1, pb, p1, p2);
      one(y + 2, p1, p2, p3);
      pa = p2;
      pb = p3;
    }
    const int left = yb - y;
    const Row p1 = row(left > 1 ? lds[(y + 1) * 64 + lane] : bot);
    one(y, pa, pb, p1);
    if (left > 1) {
      const Row p2 = row(left > 2 ? lds[(y + 2) * 64 + lane] : bot);
      one(y + 1, pb, p1, p2);
      if (left > 2) one(y + 2, p1, p2, row(bot));
    }
  }
};

// The steps of one window: TBS steps (TBS <= TBW) of the window in LDS whose
// origin is (x0, y0); the last one writes the tile, the interior that starts
// TBW nodes in, to `out` (an nx x ny grid).  Every wavefront of the
// workgroup calls it; it ends with a barrier.
template <class Seg, int RG>
__device__ __forceinline__ void window_steps(V2<typename Seg::T> *lds, int lane, int rg, int H,
                                             int TBS, int TBW, int x0, int y0, int nx, int ny,
                                             typename Seg::T *__restrict__ out,
                                             typename Seg::T *__restrict__ pop,
                                             const Seg &seg_run) {
  using T = typename Seg::T;
  constexpr int W = 128;
  // this lane's columns inside the tile (last step's stores)
  const int c0 = 2 * lane;
  const bool se = c0 >= TBW && c0 < W - TBW && x0 + c0 < nx;
  const bool so = c0 + 1 >= TBW && c0 + 1 < W - TBW && x0 + c0 + 1 < nx;
#pragma unroll 1
  for (int t = 1; t <= TBS; ++t) {
    const int Hr = H - 2 * t;
    const int seg = (Hr + RG - 1) / RG;
    const int ya = t + rg * seg, yb = min(ya + seg, H - t);
    const bool act = ya < yb;  // uniform across the wavefront
    V2<T> top = mk2<T>(T(0), T(0)), bot = top;
    if (act) {
      top = lds[(ya - 1) * 64 + lane];
      bot = lds[yb * 64 + lane];
    }
    lds_barrier();
    if (act) {
      if (t < TBS) {
        seg_run(lds, lane, ya, yb, top, bot,
                [&](int y, V2<T> o, const auto &...) { lds[y * 64 + lane] = o; });
      } else {
        // the tile: moments, and the populations of segments that form them
        seg_run(lds, lane, ya, yb, top, bot, [&](int y, V2<T> o, const auto &...pops) {
          const int gy = y0 + y;
          if (y >= TBW && y < H - TBW && gy < ny) {
            const int64_t gi = (int64_t)gy * nx + x0 + c0;
            if (se) out[gi] = o.x;
            if (so) out[gi + 1] = o.y;
            if constexpr (sizeof...(pops) == 2) {
              if (pop == nullptr) return;  // moments only
              const int64_t N = (int64_t)nx * ny;
              auto store = [&](const T *fe, const T *fo) {
#pragma unroll
                for (int j = 0; j < Seg::kQ; ++j) {
                  if (se) pop[j * N + gi] = fe[j];
                  if (so) pop[j * N + gi + 1] = fo[j];
                }
              };
              store(pops...);
            }
          }
        });
      }
    }
    lds_barrier();
  }
}

// The W x H window of an nx x ny grid whose origin is (x0, y0): rows rg,
// rg + RG, ... (NPF / 2 of them) of this lane's two columns, into registers.
// ANY: modular wrap (grids smaller than the window); else one conditional
// wrap (nx >= W, ny >= H).
template <int RG, int NPF, bool ANY, typename T>
__device__ __forceinline__ void window_fetch(const T *__restrict__ cur, int nx, int ny, int H,
                                             int x0, int y0, int lane, int rg, T (&pf)[NPF]) {
  auto wrap = [&](int i, int n) {
    if constexpr (ANY) {
      i %= n;
      return i < 0 ? i + n : i;
    } else {
      return i < 0 ? i + n : (i >= n ? i - n : i);
    }
  };
  const int ge = wrap(x0 + 2 * lane, nx), go = wrap(x0 + 2 * lane + 1, nx);
  // byte offsets within a row (a row is far below 4 GiB): each load is a row
  // base in scalar registers plus one of these two offsets
  const uint32_t be = (uint32_t)ge * (uint32_t)sizeof(T), bo = (uint32_t)go * (uint32_t)sizeof(T);
#pragma unroll
  for (int j = 0; j < NPF / 2; ++j) {
    const int r = min(rg + RG * j, H - 1);
    const int y = wrap(y0 + r, ny);
    const char *row = reinterpret_cast<const char *>(cur + (int64_t)y * nx);
    pf[2 * j] = *reinterpret_cast<const T *>(row + be);
    pf[2 * j + 1] = *reinterpret_cast<const T *>(row + bo);
  }
}

template <int RG, int NPF, typename T>
__device__ __forceinline__ void window_put(V2<T> *lds, int H, int lane, int rg,
                                           const T (&pf)[NPF]) {
#pragma unroll
  for (int j = 0; j < NPF / 2; ++j) {
    const int r = rg + RG * j;
    if (r < H) lds[r * 64 + lane] = mk2<T>(pf[2 * j], pf[2 * j + 1]);
  }
}

// One kernel for every lane-shared segment type Seg; RG wavefronts of row
// segments; NPF prefetch values per thread (NPF / 2 rows of the next window).
template <class Seg, int RG, int NPF, typename T = typename Seg::T>
__global__ __launch_bounds__(64 * RG) void k_lane_tb(const T *__restrict__ cur,
                                                    T *__restrict__ out, T *__restrict__ pop,
                                                    int nx, int ny, int H, int TB, int tiles_x,
                                                    int ntiles, typename Seg::Params kc) {
  constexpr int W = 128;
  extern __shared__ unsigned char smem_lane[];
  V2<T> *lds = reinterpret_cast<V2<T> *>(smem_lane);  // [H][64]
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int G = gridDim.x;
  if ((int)blockIdx.x >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int rg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Seg seg_run(kc);

  T pf[NPF];
  int v = blockIdx.x;
  int tile = xcd_remap_l(v, ntiles);
  int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  window_fetch<RG, NPF, false>(cur, nx, ny, H, x0, y0, lane, rg, pf);
  window_put<RG, NPF>(lds, H, lane, rg, pf);
  lds_barrier();
  while (true) {
    // the next tile of this workgroup, its window in flight during the steps
    const int vn = v + G;
    const bool more = vn < ntiles;
    int xn = 0, yn = 0;
    if (more) {
      const int tn = xcd_remap_l(vn, ntiles);
      xn = (tn % tiles_x) * TX - TB;
      yn = (tn / tiles_x) * TY - TB;
      window_fetch<RG, NPF, false>(cur, nx, ny, H, xn, yn, lane, rg, pf);
    }
    window_steps<Seg, RG>(lds, lane, rg, H, TB, TB, x0, y0, nx, ny, out, pop, seg_run);
    if (!more) break;
    window_put<RG, NPF>(lds, H, lane, rg, pf);
    lds_barrier();
    v = vn;
    x0 = xn;
    y0 = yn;
  }
}

// One instance of a batch group run by the lane-shared window: its two
// level buffers (launch l reads ring[(c0 + l) & 1]), size, tiles and steps.
template <class Prm>
struct LaneInst {
  float *ring[2];
  int nx, ny, tiles_x, tile0;
  int64_t nsteps, c0;
  Prm prm;
};

// Batched launch `launch` of a run whose launches advance up to TB steps: the
// tiles of the instances with steps left are the prefix [0, ntiles) of the
// table; each advances min(TB, its remaining steps) in a window sized for
// TB.  Persistent workgroups as in k_lane_tb; grids of any size (modular
// wrap).
template <class Seg, int RG, int NPF>
__global__ __launch_bounds__(64 * RG) void k_batch_lane_tb(
    const LaneInst<typename Seg::Params> *__restrict__ inst, const int *__restrict__ tile_inst,
    int ntiles, int64_t launch, int H, int TB) {
  constexpr int W = 128;
  extern __shared__ unsigned char smem_blane[];
  float2 *lds = reinterpret_cast<float2 *>(smem_blane);  // [H][64]
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int G = gridDim.x;
  if ((int)blockIdx.x >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int rg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  struct Where {
    int i, x0, y0;
  };
  auto locate = [&](int v) {
    const int t = xcd_remap_l(v, ntiles);
    Where w;
    w.i = tile_inst[t];
    const int lt = t - inst[w.i].tile0, tx = inst[w.i].tiles_x;
    w.x0 = (lt % tx) * TX - TB;
    w.y0 = (lt / tx) * TY - TB;
    return w;
  };
  auto cur_of = [&](int i) { return inst[i].ring[(inst[i].c0 + launch) & 1]; };

  float pf[NPF];
  int v = blockIdx.x;
  Where w = locate(v);
  window_fetch<RG, NPF, true>(cur_of(w.i), inst[w.i].nx, inst[w.i].ny, H, w.x0, w.y0, lane, rg,
                              pf);
  window_put<RG, NPF>(lds, H, lane, rg, pf);
  lds_barrier();
  while (true) {
    const int vn = v + G;
    const bool more = vn < ntiles;
    Where wn{0, 0, 0};
    if (more) {
      wn = locate(vn);
      window_fetch<RG, NPF, true>(cur_of(wn.i), inst[wn.i].nx, inst[wn.i].ny, H, wn.x0, wn.y0,
                                  lane, rg, pf);
    }
    const LaneInst<typename Seg::Params> &I = inst[w.i];
    const int64_t left = I.nsteps - launch * TB;
    const int TBS = left < TB ? (int)left : TB;
    const Seg seg_run(I.prm);
    window_steps<Seg, RG>(lds, lane, rg, H, TBS, TB, w.x0, w.y0, I.nx, I.ny,
                          I.ring[(I.c0 + launch + 1) & 1], nullptr, seg_run);
    if (!more) break;
    window_put<RG, NPF>(lds, H, lane, rg, pf);
    lds_barrier();
    v = vn;
    w = wn;
  }
}

// ------------------------------------------------------------ host side
namespace {
// Burgers' pair parts take one value per weight class only when the
// directions of a class carry equal weights in binary32
bool burgers_weights_symmetric(const KC<float> &k, int lattice) {
  if (k.w[1] != k.w[2] || k.w1[1] != k.w1[2]) return false;
  return lattice != 3 || k.w[5] == k.w[6];
}
}  // namespace

bool lane_tb_applies(const Consts &c, int elem) {
  if ((elem != 4 && elem != 8) || c.three || c.dim != 2) return false;
  return (c.lattice == 2 || c.lattice == 3) && (c.eq == kLCDE || c.eq == kBurgers);
}

bool lane_shared_fp32(const Consts &c) {
  if (!lane_tb_applies(c, 4)) return false;
  if (c.eq == kLCDE) return true;
  return c.beta_one && burgers_weights_symmetric(make_kc<float>(c), c.lattice);
}

bool lane_tb_window_fits(const TbPlan &pl) {
  return pl.w == 128 && pl.h <= 128;  // RG NPF / 2 = 128 rows of prefetch
}

namespace {
// resident workgroups per CU and CUs of the current device (cached)
int lane_slots(const void *fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void *, size_t>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_tuple(dev, fn, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int slots = (per_cu < 1 ? 1 : per_cu) * cus;
  cache[key] = slots;
  return slots;
}

// 128-column window in place: RG wavefronts, NPF / 2 rows of the next
// window each (RG NPF / 2 = 128 rows)
template <class Seg>
hipError_t lane_cfg(const Grid &g, const TbPlan &pl, const typename Seg::T *cur,
                    typename Seg::T *out, typename Seg::T *pop, const typename Seg::Params &prm,
                    hipStream_t st) {
  using T = typename Seg::T;
  constexpr int RG = Seg::kRG, NPF = Seg::kNPF, W = 128;
  if (pl.h > RG * NPF / 2) return hipErrorInvalidValue;
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int TX = W - 2 * pl.tb, TY = pl.h - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)pl.h * W * sizeof(T);
  auto fn = k_lane_tb<Seg, RG, NPF>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  // persistent grid: the resident workgroups (a multiple of 8, the XCDs),
  // or one workgroup per tile when the tiles fit in one round
  const int ntiles = tx * ty;
  int grid = lane_slots((const void *)fn, 64 * RG, lds);
  if (grid <= 0) return hipErrorInvalidValue;
  if (ntiles <= grid) grid = ntiles;  // one tile per workgroup: no walk
  else if (grid >= 8) grid &= ~7;     // the walk v, v + G, ... stays on one XCD
  hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * RG), lds, st, cur, out, pop, nx, ny, pl.h, pl.tb,
                     tx, ntiles, prm);
  return hipGetLastError();
}

LinC lin_params(const KC<float> &k, int npair) {
  LinC lc{};
  for (int p = 0; p < npair; ++p) {
    lc.ap[p] = k.Ap[p];
    lc.nam[p] = -k.Am[p];
  }
  lc.a0 = k.A0t;
  return lc;
}

BurgC burg_params(const KC<float> &k, int npair) {
  BurgC bc{};
  bc.wa = k.w[1];
  bc.wd = npair == 4 ? k.w[5] : 0.0f;
  bc.w1a = k.w1[1];
  bc.w1d = npair == 4 ? k.w1[5] : 0.0f;
  bc.bh = k.bh;
  bc.cpl = k.ap;
  bc.cmi = k.am;
  bc.a0 = k.A0t;
  return bc;
}

// the node-function segment for every case without a specialized one
template <class L, int EQ, bool MESO, typename T>
hipError_t acc_eq(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *out, T *pop,
                  hipStream_t st) {
  const KC<T> k = make_kc<T>(c);
  if constexpr (EQ == kBurgers) {
    if (c.beta_one) return lane_cfg<AccSeg<L, EQ, true, MESO, T>>(g, pl, cur, out, pop, k, st);
  }
  return lane_cfg<AccSeg<L, EQ, false, MESO, T>>(g, pl, cur, out, pop, k, st);
}

template <class L, typename T>
hipError_t lane_eq(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *out,
                   hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (lane_shared_fp32(c)) {
      const KC<float> k = make_kc<float>(c);
      if (c.eq == kLCDE)
        return lane_cfg<LinSeg<L::P>>(g, pl, cur, out, nullptr, lin_params(k, L::P), st);
      return lane_cfg<BurgSeg<L::P>>(g, pl, cur, out, nullptr, burg_params(k, L::P), st);
    }
  }
  if (c.eq == kLCDE) return acc_eq<L, kLCDE, false, T>(c, g, pl, cur, out, nullptr, st);
  return acc_eq<L, kBurgers, false, T>(c, g, pl, cur, out, nullptr, st);
}

template <class L, typename T>
hipError_t meso_eq(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *mom_out,
                   T *pop_out, hipStream_t st) {
  if (c.eq != kLCDE) return acc_eq<L, kBurgers, true, T>(c, g, pl, cur, mom_out, pop_out, st);
  const KC<T> k = make_kc<T>(c);
  MesoC<T> mc{};
  for (int j = 0; j < L::Q; ++j) mc.ub[j] = k.ubar[j];
  int am = 0;
  for (int q = 0; q < 3; ++q) {
    mc.a[q] = k.a[q];
    if (k.a[q] != T(0)) am |= 1 << q;
  }
  switch (am) {
    case 0: return lane_cfg<MesoSeg<L, 0, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    case 1: return lane_cfg<MesoSeg<L, 1, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    case 2: return lane_cfg<MesoSeg<L, 2, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    case 3: return lane_cfg<MesoSeg<L, 3, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    case 4: return lane_cfg<MesoSeg<L, 4, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    case 5: return lane_cfg<MesoSeg<L, 5, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    case 6: return lane_cfg<MesoSeg<L, 6, T>>(g, pl, cur, mom_out, pop_out, mc, st);
    default: return lane_cfg<MesoSeg<L, 7, T>>(g, pl, cur, mom_out, pop_out, mc, st);
  }
}

template <class Seg>
hipError_t batch_lane_cfg(const void *inst, const int *tile_inst, int ntiles, int64_t launch,
                          const TbPlan &pl, hipStream_t st) {
  constexpr int RG = Seg::kRG, NPF = Seg::kNPF, W = 128;
  if (pl.h > RG * NPF / 2) return hipErrorInvalidValue;
  const size_t lds = (size_t)pl.h * W * sizeof(float);
  auto fn = k_batch_lane_tb<Seg, RG, NPF>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  int grid = lane_slots((const void *)fn, 64 * RG, lds);
  if (grid <= 0) return hipErrorInvalidValue;
  if (ntiles <= grid) grid = ntiles;  // one tile per workgroup: no walk
  else if (grid >= 8) grid &= ~7;     // the walk v, v + G, ... stays on one XCD
  hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * RG), lds, st,
                     (const LaneInst<typename Seg::Params> *)inst, tile_inst, ntiles, launch, pl.h,
                     pl.tb);
  return hipGetLastError();
}
}  // namespace

bool lane_batch_applies(const BatchKey &k) {
  return k.precision == MFD_FP32 && !k.three && (k.lattice == MFD_D2Q5 || k.lattice == MFD_D2Q9) &&
         (k.eq == kLCDE || (k.eq == kBurgers && k.b1));
}

size_t lane_inst_bytes(const BatchKey &k) {
  return k.eq == kLCDE ? sizeof(LaneInst<LinC>) : sizeof(LaneInst<BurgC>);
}

bool lane_inst_fill(const BatchKey &k, const Consts &c, float *cur, float *other, int nx, int ny,
                    int tiles_x, int tile0, int64_t nsteps, void *dst) {
  if (!lane_shared_fp32(c)) return false;
  const KC<float> kc = make_kc<float>(c);
  const int np = c.npair;
  if (k.eq == kLCDE) {
    LaneInst<LinC> li{{cur, other}, nx, ny, tiles_x, tile0, nsteps, 0, lin_params(kc, np)};
    std::memcpy(dst, &li, sizeof(li));
  } else {
    LaneInst<BurgC> li{{cur, other}, nx, ny, tiles_x, tile0, nsteps, 0, burg_params(kc, np)};
    std::memcpy(dst, &li, sizeof(li));
  }
  return true;
}

hipError_t launch_batch_lane_tb(const BatchKey &k, const void *inst, const int *tile_inst,
                                int ntiles, int64_t launch, const TbPlan &pl, hipStream_t st) {
  if (!lane_batch_applies(k) || pl.w != 128) return hipErrorInvalidValue;
  if (k.lattice == MFD_D2Q9) {
    if (k.eq == kLCDE) return batch_lane_cfg<LinSeg<4>>(inst, tile_inst, ntiles, launch, pl, st);
    return batch_lane_cfg<BurgSeg<4>>(inst, tile_inst, ntiles, launch, pl, st);
  }
  if (k.eq == kLCDE) return batch_lane_cfg<LinSeg<2>>(inst, tile_inst, ntiles, launch, pl, st);
  return batch_lane_cfg<BurgSeg<2>>(inst, tile_inst, ntiles, launch, pl, st);
}

bool lane_meso_applies(const Consts &c, int elem) { return lane_tb_applies(c, elem); }

template <typename T>
hipError_t launch_lane_mesofd_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur,
                                 T *mom_out, T *pop_out, hipStream_t st) {
  if (!lane_meso_applies(c, sizeof(T)) || pl.w != 128) return hipErrorInvalidValue;
  if (c.lattice == 3) return meso_eq<LatD2Q9, T>(c, g, pl, cur, mom_out, pop_out, st);
  return meso_eq<LatD2Q5, T>(c, g, pl, cur, mom_out, pop_out, st);
}

template <typename T>
hipError_t launch_lane_tb(const Consts &c, const Grid &g, const TbPlan &pl, const T *cur, T *out,
                          hipStream_t st) {
  if (!lane_tb_applies(c, sizeof(T)) || pl.w != 128) return hipErrorInvalidValue;
  if (c.lattice == 3) return lane_eq<LatD2Q9, T>(c, g, pl, cur, out, st);
  return lane_eq<LatD2Q5, T>(c, g, pl, cur, out, st);
}

#define MFD_LANE_INST(T)                                                                     \
  template hipError_t launch_lane_mesofd_tb<T>(const Consts &, const Grid &, const TbPlan &, \
                                               const T *, T *, T *, hipStream_t);            \
  template hipError_t launch_lane_tb<T>(const Consts &, const Grid &, const TbPlan &,        \
                                        const T *, T *, hipStream_t);
MFD_LANE_INST(float)
MFD_LANE_INST(double)
#undef MFD_LANE_INST

}  // namespace mfd
