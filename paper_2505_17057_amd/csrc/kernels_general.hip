// The general MMFD step of Eq. (2-2-1) for a linear EDF (the linear CDE), and
// (k_general_nl, at the end) for Burgers' equation and the NSE:
// any stencil reach m and number of levels n, any lattice (rD3Q27 included),
// periodic wrap.  Each thread updates one node:
//   out = sum_l A_l phi_l + sum_l sum_p sum_{k=1..m} [Cp_lkp D2_{p,k} phi_l
//                                                  + Cm_lkp D1_{p,k} phi_l],
//   D2_{p,k} g = (g(x + k e_p) - g(x)) + (g(x - k e_p) - g(x)),
//   D1_{p,k} g = g(x + k e_p) - g(x - k e_p),
// accumulated level by level, pairs in lattice order, then k, then the base
// terms level by level and their sum with the accumulator; in binary64 each
// product and sum is rounded on its own (the oracle's operations, so the
// results agree bit for bit), in binary32 the linear CDE's multiply-adds are
// fused.  The constants are read
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

// acc + c d: binary64 rounds the product and the sum on their own (the
// oracle's operations); binary32 fuses them (one rounding, one instruction)
template <typename T>
__device__ __forceinline__ T gmac(T acc, T c, T d) {
  if constexpr (std::is_same<T, float>::value) return __builtin_fmaf(c, d, acc);
  else return acc + c * d;
}

// fourth word of a raw buffer resource on gfx9-family parts (32-bit data
// format, no stride, no swizzle)
constexpr int kBufWord3 = 0x00020000;

// offsets of the wrapped coordinates c + j, j = -M..M, on an axis of extent
// n, times the axis stride; the branch on n is uniform over the launch
template <int M, typename I>
__device__ __forceinline__ void wrap_axis(int c, int n, int64_t stride, I (&o)[2 * M + 1]) {
  if (n >= M) {
#pragma unroll
    for (int j = -M; j <= M; ++j) {
      int i = c + j;
      i = i < 0 ? i + n : (i >= n ? i - n : i);
      o[j + M] = (I)(i * stride);
    }
  } else {
#pragma unroll
    for (int j = -M; j <= M; ++j) {
      const int i = (c + j) % n;
      o[j + M] = (I)((i < 0 ? i + n : i) * stride);
    }
  }
}

// Byte offsets of a node's neighbours within one field: 32-bit (I =
// uint32_t) when a field spans less than 4 GiB, so a load is a uniform base
// plus one 32-bit register offset; 64-bit otherwise.
template <int M, typename T, typename I>
struct GenIdx {
  I xo[2 * M + 1], yo[2 * M + 1], zo[2 * M + 1];
  __device__ __forceinline__ GenIdx(int x, int y, int z, int nx, int ny, int nz) {
    wrap_axis<M>(x, nx, (int64_t)sizeof(T), xo);
    wrap_axis<M>(y, ny, (int64_t)nx * sizeof(T), yo);
    wrap_axis<M>(z, nz, (int64_t)nx * ny * sizeof(T), zo);
  }
  // the node x + sk e (sk = +-k)
  template <int EX, int EY, int EZ>
  __device__ __forceinline__ I at(int sk) const {
    return zo[M + sk * EZ] + yo[M + sk * EY] + xo[M + sk * EX];
  }
  __device__ __forceinline__ I centre() const { return zo[M] + yo[M] + xo[M]; }
};

// load of the element at byte offset off of a field starting at base: a
// buffer load (resource over the field's nb bytes, 32-bit offset) when I is
// uint32_t, a global load otherwise
template <typename T, typename I>
__device__ __forceinline__ T ld(const T *base, uint32_t nb, I off) {
  if constexpr (std::is_same<I, uint32_t>::value) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)nb, kBufWord3);
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  } else {
    (void)nb;
    return *(const T *)((const char *)base + off);
  }
}

template <class L, int M, typename T, typename I>
__global__ __launch_bounds__(256) void k_general_step(GenLevels<T> lev, T *__restrict__ out, int nx,
                                                      int ny, int nz,
                                                      const GenC<T> *__restrict__ gc) {
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int nl = gc->nl;
  const GenIdx<M, T, I> ix(x, y, z, nx, ny, nz);
  const I i0 = ix.centre();
  const uint32_t nb = (uint32_t)((int64_t)nx * ny * nz * (int64_t)sizeof(T));
  T acc = 0;
  for (int l = 0; l < nl; ++l) {
    const T *__restrict__ g = lev.p[l];
    const T g0 = ld(g, nb, i0);
    static_for<L::P>([&](auto PI) {
      constexpr int P = decltype(PI)::value;
      constexpr int J = L::PR[P];
      constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
#pragma unroll
      for (int k = 1; k <= M; ++k) {
        const T gp = ld(g, nb, ix.template at<ex, ey, ez>(k));
        const T gm = ld(g, nb, ix.template at<ex, ey, ez>(-k));
        const T d2 = (gp - g0) + (gm - g0);
        const T d1 = gp - gm;
        acc = gmac(acc, gc->Cp[l][k - 1][P], d2);
        acc = gmac(acc, gc->Cm[l][k - 1][P], d1);
      }
    });
  }
  T base = gc->A[0] * ld(lev.p[0], nb, i0);
  for (int l = 1; l < nl; ++l) base = gmac(base, gc->A[l], ld(lev.p[l], nb, i0));
  *(T *)((char *)out + i0) = base + acc;
}

// The linear CDE on 2D and 3D grids with R nodes per thread along the column
// axis (y in 2D, z in 3D): a level's values at the thread's nodes and all
// their neighbours (a (2m+1) x (R+2m) box in 2D, (2m+1)^2 x (R+2m) in 3D)
// are loaded once per thread and level, so a value that several of the
// thread's nodes use is loaded once.  Each node's sums are formed exactly as
// k_general_step forms them (same terms, same order), so the results are the
// same bit for bit.
template <int LO, int CNT, typename I>
__device__ __forceinline__ void wrap_range(int c, int n, int64_t stride, bool fast, I (&o)[CNT]) {
#pragma unroll
  for (int j = 0; j < CNT; ++j) {
    int i = c + LO + j;
    if (fast) {
      i = i < 0 ? i + n : (i >= n ? i - n : i);
    } else {
      i %= n;
      i = i < 0 ? i + n : i;
    }
    o[j] = (I)(i * stride);
  }
}

template <class L, int M, int R, typename T, typename I>
__global__ __launch_bounds__(256) void k_general_col(GenLevels<T> lev, T *__restrict__ out, int nx,
                                                     int ny, int nz,
                                                     const GenC<T> *__restrict__ gc) {
  constexpr int D = L::D;
  static_assert(D == 2 || D == 3, "column kernel: 2D and 3D lattices");
  constexpr int S = 2 * M + 1, W = R + 2 * M;  // stencil width, column window
  constexpr int BY = D == 2 ? W : S, BZ = D == 3 ? W : 1;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = D == 2 ? (blockIdx.y * 4 + threadIdx.y) * R : blockIdx.y * 4 + threadIdx.y;
  const int z = D == 3 ? blockIdx.z * R : 0;
  if (x >= nx || y >= ny) return;
  const int nw = D == 2 ? ny : nz, w0 = D == 2 ? y : z;
  // one conditional add or subtract wraps c + j (-M <= j < R + M) when the
  // axis has at least M + R nodes; else the remainder
  const bool fast = nx >= M + R && ny >= M + R && (D == 2 || nz >= M + R);
  I xo[S], yo[BY], zo[BZ];
  wrap_range<-M, S>(x, nx, (int64_t)sizeof(T), fast, xo);
  if constexpr (D == 2) {
    wrap_range<-M, W>(y, ny, (int64_t)nx * sizeof(T), fast, yo);
    zo[0] = 0;
  } else {
    wrap_range<-M, S>(y, ny, (int64_t)nx * sizeof(T), fast, yo);
    wrap_range<-M, W>(z, nz, (int64_t)nx * ny * sizeof(T), fast, zo);
  }
  const uint32_t nb = (uint32_t)((int64_t)nx * ny * nz * (int64_t)sizeof(T));
  const int nl = gc->nl;
  T acc[R], base[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0;
  for (int l = 0; l < nl; ++l) {
    const T *__restrict__ g = lev.p[l];
    T v[S][BY][BZ];
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < BY; ++b)
#pragma unroll
        for (int c = 0; c < BZ; ++c) v[a][b][c] = ld(g, nb, (I)(zo[c] + yo[b] + xo[a]));
    // value at the offset (dx, dy, dz) from the thread's node r
    auto at = [&](int r, int dx, int dy, int dz) -> T {
      if constexpr (D == 2) return v[M + dx][M + r + dy][0];
      else return v[M + dx][M + dy][M + r + dz];
    };
    const T Al = gc->A[l];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T g0 = at(r, 0, 0, 0);
      T a_r = acc[r];
      static_for<L::P>([&](auto PI) {
        constexpr int P = decltype(PI)::value;
        constexpr int J = L::PR[P];
        constexpr int ex = L::E[J][0], ey = L::E[J][1], ez = L::E[J][2];
#pragma unroll
        for (int k = 1; k <= M; ++k) {
          const T gp = at(r, k * ex, k * ey, k * ez), gm = at(r, -k * ex, -k * ey, -k * ez);
          const T d2 = (gp - g0) + (gm - g0);
          const T d1 = gp - gm;
          a_r = gmac(a_r, gc->Cp[l][k - 1][P], d2);
          a_r = gmac(a_r, gc->Cm[l][k - 1][P], d1);
        }
      });
      acc[r] = a_r;
      base[r] = l == 0 ? Al * g0 : gmac(base[r], Al, g0);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (w0 + r < nw) {
      const I o = D == 2 ? (I)(yo[M + r] + xo[M]) : (I)(zo[M + r] + yo[M] + xo[M]);
      *(T *)((char *)out + o) = base[r] + acc[r];
    }
  }
}

// Burgers' equation / the NSE: the pair parts of each neighbour formed from
// its moments; the sums in the order of the oracle's pair-part form:
//   density / scalar: acc over (level, pair, k) of a+ D2 F+ and a- D1 F-,
//   momentum j_a: over (level, pair with e_pa != 0, k) of +-(ab+ D2 F- and
//   ab- D1 F+), then the base terms level by level.
template <class L, int EQ, int M, typename T, typename I>
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
  const GenIdx<M, T, I> ix(x, y, z, nx, ny, nz);
  const I i0 = ix.centre();
  const uint32_t nb = (uint32_t)(N * (int64_t)sizeof(T));
  T acc = 0, mo[D > 0 ? D : 1];
#pragma unroll
  for (int a = 0; a < D; ++a) mo[a] = 0;
  auto rec_at = [&](const T *f, I i, T *r) {
    T mm[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) mm[q] = ld(f + q * N, nb, i);
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
  T base = g->A[0] * ld(lev.p[0], nb, i0);
  for (int l = 1; l < nl; ++l) base = base + g->A[l] * ld(lev.p[l], nb, i0);
  *(T *)((char *)out + i0) = base + acc;
  if constexpr (EQ == kNSE) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int64_t fo = (int64_t)(a + 1) * N;
      T bj = g->Ab[0] * ld(lev.p[0] + fo, nb, i0);
      for (int l = 1; l < nl; ++l) bj = bj + g->Ab[l] * ld(lev.p[l] + fo, nb, i0);
      *(T *)((char *)(out + fo) + i0) = bj + mo[a];
    }
  }
}

// Burgers' equation / the NSE on 2D grids: a TX x TY tile per workgroup; per
// level, every node of the tile and its m-wide halo forms its record and its
// pair parts F+-_p once into LDS (one evaluation per node instead of one per
// neighbour that uses it), then each node of the tile adds its terms reading
// the parts from LDS.  The terms and their order are k_general_nl's, and the
// parts are the same function of the same moments, so the results are the
// same bit for bit.
template <class L, int EQ, int M, typename T>
__global__ __launch_bounds__(256) void k_general_nl_tile(GenLevels<T> lev, T *__restrict__ out,
                                                         int nx, int ny, int tiles_x, KC<T> kc,
                                                         const GenNL<T> *__restrict__ g) {
  using R = Rec<L, EQ>;
  constexpr int NF = R::NF, NR = R::NR, D = L::D, P = L::P;
  constexpr int TX = 64, TY = 8, HX = TX + 2 * M, HY = TY + 2 * M;
  constexpr int KI = TX * TY / 256;  // tile nodes per thread
  static_assert(D == 2, "2D lattices");
  __shared__ T pf[2 * P][HY][HX];
  const int x0 = (blockIdx.x % tiles_x) * TX, y0 = (blockIdx.x / tiles_x) * TY;
  const int64_t N = (int64_t)nx * ny;
  const int nl = g->nl;
  T acc[KI], mo[KI][D];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    acc[i] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) mo[i][a] = 0;
  }
  for (int l = 0; l < nl; ++l) {
    const T *__restrict__ f = lev.p[l];
    if (l > 0) __syncthreads();  // the previous level's parts are read
    for (int i = threadIdx.x; i < HX * HY; i += 256) {
      const int lx = i % HX, ly = i / HX;
      int gx = (x0 - M + lx) % nx, gy = (y0 - M + ly) % ny;
      gx = gx < 0 ? gx + nx : gx;
      gy = gy < 0 ? gy + ny : gy;
      const int64_t gi = (int64_t)gy * nx + gx;
      T mm[NF], r[NR];
#pragma unroll
      for (int q = 0; q < NF; ++q) mm[q] = f[q * N + gi];
      make_record<L, EQ>(mm, r, kc);
      static_for<P>([&](auto PI) {
        constexpr int PP = decltype(PI)::value;
        constexpr int J = L::PR[PP];
        pf[2 * PP][ly][lx] = fplus<L, EQ, J>(r, kc);
        pf[2 * PP + 1][ly][lx] = fminus<L, EQ, J>(r, kc);
      });
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KI; ++i) {
      const int t = threadIdx.x + 256 * i;
      const int cx = t % TX + M, cy = t / TX + M;
      static_for<P>([&](auto PI) {
        constexpr int PP = decltype(PI)::value;
        constexpr int J = L::PR[PP];
        constexpr int ex = L::E[J][0], ey = L::E[J][1];
        const T p0 = pf[2 * PP][cy][cx], q0 = pf[2 * PP + 1][cy][cx];
#pragma unroll
        for (int k = 1; k <= M; ++k) {
          const T pP = pf[2 * PP][cy + k * ey][cx + k * ex];
          const T pM = pf[2 * PP][cy - k * ey][cx - k * ex];
          const T qP = pf[2 * PP + 1][cy + k * ey][cx + k * ex];
          const T qM = pf[2 * PP + 1][cy - k * ey][cx - k * ex];
          acc[i] = acc[i] + g->ap[l][k - 1] * ((pP - p0) + (pM - p0));
          acc[i] = acc[i] + g->am[l][k - 1] * (qP - qM);
          if constexpr (EQ == kNSE) {
            const T t1 = g->abp[l][k - 1] * ((qP - q0) + (qM - q0));
            const T t2 = g->abm[l][k - 1] * (pP - pM);
#pragma unroll
            for (int a = 0; a < D; ++a) {
              if (L::E[J][a] == 0) continue;
              if (L::E[J][a] > 0) {
                mo[i][a] = mo[i][a] + t1;
                mo[i][a] = mo[i][a] + t2;
              } else {
                mo[i][a] = mo[i][a] - t1;
                mo[i][a] = mo[i][a] - t2;
              }
            }
          }
        }
      });
    }
  }
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int t = threadIdx.x + 256 * i;
    const int gx = x0 + t % TX, gy = y0 + t / TX;
    if (gx >= nx || gy >= ny) continue;
    const int64_t i0 = (int64_t)gy * nx + gx;
    T base = g->A[0] * lev.p[0][i0];
    for (int l = 1; l < nl; ++l) base = base + g->A[l] * lev.p[l][i0];
    out[i0] = base + acc[i];
    if constexpr (EQ == kNSE) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int64_t fi = (int64_t)(a + 1) * N + i0;
        T bj = g->Ab[0] * lev.p[0][fi];
        for (int l = 1; l < nl; ++l) bj = bj + g->Ab[l] * lev.p[l][fi];
        out[fi] = bj + mo[i][a];
      }
    }
  }
}

// the reach m and the offset width (32-bit when a field spans < 4 GiB) as
// template arguments
#define MFD_GEN_LAUNCH(KERNEL, ...)                                                          \
  const bool small = (int64_t)nx * ny * nz * (int64_t)sizeof(T) < ((int64_t)1 << 32);        \
  switch (m * 2 + (small ? 1 : 0)) {                                                       \
    case 2: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 1, T, int64_t>), grid, block, 0, st, ARGS); break; \
    case 3: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 1, T, uint32_t>), grid, block, 0, st, ARGS); break; \
    case 4: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 2, T, int64_t>), grid, block, 0, st, ARGS); break; \
    case 5: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 2, T, uint32_t>), grid, block, 0, st, ARGS); break; \
    case 6: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 3, T, int64_t>), grid, block, 0, st, ARGS); break; \
    case 7: hipLaunchKernelGGL((KERNEL<__VA_ARGS__, 3, T, uint32_t>), grid, block, 0, st, ARGS); break; \
    default: return hipErrorInvalidValue;                                                  \
  }

template <class L, int EQ, typename T>
hipError_t gnl(const Consts &c, int m, GenLevels<T> lev, T *out, const int64_t n[3],
               const GenNL<T> *g, hipStream_t st) {
  const int nx = (int)n[0], ny = (int)n[1], nz = (int)n[2];
  if constexpr (L::D == 2) {  // the LDS tile of pair parts
    const int tiles_x = (nx + 63) / 64, nt = tiles_x * ((ny + 7) / 8);
    const KC<T> kc = make_kc<T>(c);
    switch (m) {
      case 1: hipLaunchKernelGGL((k_general_nl_tile<L, EQ, 1, T>), dim3(nt), dim3(256), 0, st, lev, out, nx, ny, tiles_x, kc, g); break;
      case 2: hipLaunchKernelGGL((k_general_nl_tile<L, EQ, 2, T>), dim3(nt), dim3(256), 0, st, lev, out, nx, ny, tiles_x, kc, g); break;
      case 3: hipLaunchKernelGGL((k_general_nl_tile<L, EQ, 3, T>), dim3(nt), dim3(256), 0, st, lev, out, nx, ny, tiles_x, kc, g); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
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

// nodes per thread of the column kernel (1: the one-node kernel)
template <class L>
constexpr int col_nodes(int m) {
  return L::D == 2 ? (m == 1 ? 8 : m == 2 ? 4 : 2) : L::D == 3 && m == 1 ? 4 : 1;
}

template <class L, int M, int R, typename T>
hipError_t gcol(GenLevels<T> lev, T *out, int nx, int ny, int nz, const GenC<T> *gc,
                hipStream_t st) {
  const dim3 block(64, 4);
  const dim3 grid((nx + 63) / 64, L::D == 2 ? (ny + 4 * R - 1) / (4 * R) : (ny + 3) / 4,
                  L::D == 3 ? (nz + R - 1) / R : 1);
  const bool small = (int64_t)nx * ny * nz * (int64_t)sizeof(T) < ((int64_t)1 << 32);
  if (small)
    hipLaunchKernelGGL((k_general_col<L, M, R, T, uint32_t>), grid, block, 0, st, lev, out, nx, ny,
                       nz, gc);
  else
    hipLaunchKernelGGL((k_general_col<L, M, R, T, int64_t>), grid, block, 0, st, lev, out, nx, ny,
                       nz, gc);
  return hipGetLastError();
}

template <class L, int M, typename T>
hipError_t gl_m(GenLevels<T> lev, T *out, int nx, int ny, int nz, const GenC<T> *gc,
                hipStream_t st) {
  constexpr int R = col_nodes<L>(M);
  if constexpr (R > 1) {
    return gcol<L, M, R, T>(lev, out, nx, ny, nz, gc, st);
  } else {
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz), block(64, 4);
    const bool small = (int64_t)nx * ny * nz * (int64_t)sizeof(T) < ((int64_t)1 << 32);
    if (small)
      hipLaunchKernelGGL((k_general_step<L, M, T, uint32_t>), grid, block, 0, st, lev, out, nx,
                         ny, nz, gc);
    else
      hipLaunchKernelGGL((k_general_step<L, M, T, int64_t>), grid, block, 0, st, lev, out, nx, ny,
                         nz, gc);
    return hipGetLastError();
  }
}

template <class L, typename T>
hipError_t gl(int m, GenLevels<T> lev, T *out, const int64_t n[3], const GenC<T> *gc,
              hipStream_t st) {
  const int nx = (int)n[0], ny = (int)n[1], nz = (int)n[2];
  switch (m) {
    case 1: return gl_m<L, 1, T>(lev, out, nx, ny, nz, gc, st);
    case 2: return gl_m<L, 2, T>(lev, out, nx, ny, nz, gc, st);
    case 3: return gl_m<L, 3, T>(lev, out, nx, ny, nz, gc, st);
    default: return hipErrorInvalidValue;
  }
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
