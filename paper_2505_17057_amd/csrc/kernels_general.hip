// The general MMFD step of Eq. (2-2-1) for a linear EDF (the linear CDE), and
// (k_general_nl, at the end) for Burgers' equation and the NSE:
// any stencil reach m and number of levels n, any lattice (rD3Q27 included),
// periodic wrap.  Each thread updates one node:
//   out = sum_l A_l phi_l + sum_l sum_p sum_{k=1..m} [Cp_lkp D2_{p,k} phi_l
//                                                  + Cm_lkp D1_{p,k} phi_l],
//   D2_{p,k} g = (g(x + k e_p) - g(x)) + (g(x - k e_p) - g(x)),
//   D1_{p,k} g = g(x + k e_p) - g(x - k e_p),
// accumulated level by level, pairs in lattice order, then k, each product
// and sum rounded on its own (no fused multiply-add), then the base terms
// level by level and their sum with the accumulator.  The constants are read
// from device memory (uniform loads: the rD3Q27 tables exceed what the
// kernel argument block comfortably holds); the neighbours come through the
// caches (one load per neighbour and level).  The reach m is a template
// parameter: each thread forms the wrapped coordinates x + j, y + j, z + j
// (|j| <= m) once, so a neighbour's index is three table entries added (no
// integer division per neighbour).
#include "general.h"
#include "edf.h"

namespace mfd {

namespace {

// offsets of the wrapped coordinates c + j, j = -M..M, on an axis of extent
// n, times the axis stride; the branch on n is uniform over the launch
template <int M>
__device__ __forceinline__ void wrap_axis(int c, int n, int64_t stride, int64_t (&o)[2 * M + 1]) {
  if (n >= M) {
#pragma unroll
    for (int j = -M; j <= M; ++j) {
      int i = c + j;
      i = i < 0 ? i + n : (i >= n ? i - n : i);
      o[j + M] = (int64_t)i * stride;
    }
  } else {
#pragma unroll
    for (int j = -M; j <= M; ++j) {
      const int i = (c + j) % n;
      o[j + M] = (int64_t)(i < 0 ? i + n : i) * stride;
    }
  }
}

template <int M>
struct GenIdx {
  int64_t xo[2 * M + 1], yo[2 * M + 1], zo[2 * M + 1];
  __device__ __forceinline__ GenIdx(int x, int y, int z, int nx, int ny, int nz) {
    wrap_axis<M>(x, nx, 1, xo);
    wrap_axis<M>(y, ny, nx, yo);
    wrap_axis<M>(z, nz, (int64_t)nx * ny, zo);
  }
  // the node x + sk e (sk = +-k)
  template <int EX, int EY, int EZ>
  __device__ __forceinline__ int64_t at(int sk) const {
    return zo[M + sk * EZ] + yo[M + sk * EY] + xo[M + sk * EX];
  }
  __device__ __forceinline__ int64_t centre() const { return zo[M] + yo[M] + xo[M]; }
};

template <class L, int M, typename T>
__global__ __launch_bounds__(256) void k_general_step(GenLevels<T> lev, T *__restrict__ out, int nx,
                                                      int ny, int nz,
                                                      const GenC<T> *__restrict__ gc) {
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int nl = gc->nl;
  const GenIdx<M> ix(x, y, z, nx, ny, nz);
  const int64_t i0 = ix.centre();
  T acc = 0;
  for (int l = 0; l < nl; ++l) {
    const T *__restrict__ g = lev.p[l];
    const T g0 = g[i0];
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
#pragma unroll
      for (int k = 1; k <= M; ++k) {
        const T gp = g[ix.template at<ex, ey, ez>(k)], gm = g[ix.template at<ex, ey, ez>(-k)];
        const T d2 = (gp - g0) + (gm - g0);
        const T d1 = gp - gm;
        acc = acc + gc->Cp[l][k - 1][P] * d2;
        acc = acc + gc->Cm[l][k - 1][P] * d1;
      }
    });
  }
  T base = gc->A[0] * lev.p[0][i0];
  for (int l = 1; l < nl; ++l) base = base + gc->A[l] * lev.p[l][i0];
  out[i0] = base + acc;
}

// Burgers' equation / the NSE: the pair parts of each neighbour formed from
// its moments; the sums in the order of the oracle's pair-part form:
//   density / scalar: acc over (level, pair, k) of a+ D2 F+ and a- D1 F-,
//   momentum j_a: over (level, pair with e_pa != 0, k) of +-(ab+ D2 F- and
//   ab- D1 F+), then the base terms level by level.
template <class L, int EQ, int M, typename T>
__global__ __launch_bounds__(256) void k_general_nl(GenLevels<T> lev, T *__restrict__ out, int nx,
                                                    int ny, int nz, KC<T> kc,
                                                    const GenNL<T> *__restrict__ g) {
  using R = Rec<L, EQ>;
  constexpr int NF = R::NF, NR = R::NR, D = L::D;
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int nl = g->nl;
  const int64_t N = (int64_t)nx * ny * nz;
  const GenIdx<M> ix(x, y, z, nx, ny, nz);
  const int64_t i0 = ix.centre();
  T acc = 0, mo[D > 0 ? D : 1];
#pragma unroll
  for (int a = 0; a < D; ++a) mo[a] = 0;
  auto rec_at = [&](const T *f, int64_t i, T *r) {
    T mm[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) mm[q] = f[q * N + i];
    make_record<L, EQ>(mm, r, kc);
  };
  for (int l = 0; l < nl; ++l) {
    const T *__restrict__ f = lev.p[l];
    T r0[NR];
    rec_at(f, i0, r0);
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
      const T p0 = fplus<L, EQ, J>(r0, kc), q0 = fminus<L, EQ, J>(r0, kc);
#pragma unroll
      for (int k = 1; k <= M; ++k) {
        T rp[NR], rm[NR];
        rec_at(f, ix.template at<ex, ey, ez>(k), rp);
        rec_at(f, ix.template at<ex, ey, ez>(-k), rm);
        const T pP = fplus<L, EQ, J>(rp, kc), pM = fplus<L, EQ, J>(rm, kc);
        const T qP = fminus<L, EQ, J>(rp, kc), qM = fminus<L, EQ, J>(rm, kc);
        acc = acc + g->ap[l][k - 1] * ((pP - p0) + (pM - p0));
        acc = acc + g->am[l][k - 1] * (qP - qM);
        if constexpr (EQ == kNSE) {
          const T t1 = g->abp[l][k - 1] * ((qP - q0) + (qM - q0));
          const T t2 = g->abm[l][k - 1] * (pP - pM);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (L::E[J][a] == 0) continue;
            if (L::E[J][a] > 0) {
              mo[a] = mo[a] + t1;
              mo[a] = mo[a] + t2;
            } else {
              mo[a] = mo[a] - t1;
              mo[a] = mo[a] - t2;
            }
          }
        }
      }
    });
  }
  T base = g->A[0] * lev.p[0][i0];
  for (int l = 1; l < nl; ++l) base = base + g->A[l] * lev.p[l][i0];
  out[i0] = base + acc;
  if constexpr (EQ == kNSE) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int64_t fi = (int64_t)(a + 1) * N + i0;
      T bj = g->Ab[0] * lev.p[0][fi];
      for (int l = 1; l < nl; ++l) bj = bj + g->Ab[l] * lev.p[l][fi];
      out[fi] = bj + mo[a];
    }
  }
}

#define MFD_GEN_LAUNCH(KERNEL, ...)                                                          \
  switch (m) {                                                                             \
    case 1: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 1, T>), grid, block, 0, st, ARGS); break; \
    case 2: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 2, T>), grid, block, 0, st, ARGS); break; \
    case 3: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 3, T>), grid, block, 0, st, ARGS); break; \
    default: return hipErrorInvalidValue;                                                  \
  }

template <class L, int EQ, typename T>
hipError_t gnl(const Consts &c, int m, GenLevels<T> lev, T *out, const int64_t n[3],
               const GenNL<T> *g, hipStream_t st) {
  const int nx = (int)n[0], ny = (int)n[1], nz = (int)n[2];
  const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz), block(64, 4);
  const KC<T> kc = make_kc<T>(c);
#define ARGS lev, out, nx, ny, nz, kc, g
  MFD_GEN_LAUNCH(k_general_nl, L, EQ)
#undef ARGS
  return hipGetLastError();
}

template <class L, typename T>
hipError_t gnl_eq(const Consts &c, int m, GenLevels<T> lev, T *out, const int64_t n[3],
                  const GenNL<T> *g, hipStream_t st) {
  if (c.eq == kBurgers) return gnl<L, kBurgers, T>(c, m, lev, out, n, g, st);
  if constexpr (L::D >= 2) {
    if (c.eq == kNSE) return gnl<L, kNSE, T>(c, m, lev, out, n, g, st);
  }
  return hipErrorInvalidValue;
}

template <class L, typename T>
hipError_t gl(int m, GenLevels<T> lev, T *out, const int64_t n[3], const GenC<T> *gc,
              hipStream_t st) {
  const int nx = (int)n[0], ny = (int)n[1], nz = (int)n[2];
  const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz), block(64, 4);
#define ARGS lev, out, nx, ny, nz, gc
  MFD_GEN_LAUNCH(k_general_step, L)
#undef ARGS
  return hipGetLastError();
}

#undef MFD_GEN_LAUNCH

}  // namespace

template <typename T>
hipError_t launch_general_step(int lattice, int m, GenLevels<T> lev, T *out, const int64_t n[3],
                               const GenC<T> *gc, hipStream_t st) {
  if (n[2] > 65535) return hipErrorInvalidValue;
  switch (lattice) {
    case 1: return gl<LatD1Q3, T>(m, lev, out, n, gc, st);
    case 2: return gl<LatD2Q5, T>(m, lev, out, n, gc, st);
    case 3: return gl<LatD2Q9, T>(m, lev, out, n, gc, st);
    case 4: return gl<LatD3Q19, T>(m, lev, out, n, gc, st);
    case 5: return gl<LatD2Q5II, T>(m, lev, out, n, gc, st);
    case 6: return gl<LatD3Q7, T>(m, lev, out, n, gc, st);
    case 7: return gl<LatD3Q9, T>(m, lev, out, n, gc, st);
    case 8: return gl<LatD3Q27, T>(m, lev, out, n, gc, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_general_nl_step(const Consts &c, int m, GenLevels<T> lev, T *out,
                                  const int64_t n[3], const GenNL<T> *g, hipStream_t st) {
  if (n[2] > 65535) return hipErrorInvalidValue;
  switch (c.lattice) {
    case 1: return gnl_eq<LatD1Q3, T>(c, m, lev, out, n, g, st);
    case 2: return gnl_eq<LatD2Q5, T>(c, m, lev, out, n, g, st);
    case 3: return gnl_eq<LatD2Q9, T>(c, m, lev, out, n, g, st);
    case 4: return gnl_eq<LatD3Q19, T>(c, m, lev, out, n, g, st);
    case 5: return gnl_eq<LatD2Q5II, T>(c, m, lev, out, n, g, st);
    case 6: return gnl_eq<LatD3Q7, T>(c, m, lev, out, n, g, st);
    case 7: return gnl_eq<LatD3Q9, T>(c, m, lev, out, n, g, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_general_nl_step<float>(const Consts &, int, GenLevels<float>, float *,
                                                  const int64_t *, const GenNL<float> *,
                                                  hipStream_t);
template hipError_t launch_general_nl_step<double>(const Consts &, int, GenLevels<double>, double *,
                                                   const int64_t *, const GenNL<double> *,
                                                   hipStream_t);
template hipError_t launch_general_step<float>(int, int, GenLevels<float>, float *, const int64_t *,
                                               const GenC<float> *, hipStream_t);
template hipError_t launch_general_step<double>(int, int, GenLevels<double>, double *, const int64_t *,
                                                const GenC<double> *, hipStream_t);

}  // namespace mfd
