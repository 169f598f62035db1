// Temporally blocked binary32 MMFD step of the two-level linear CDE on D2Q5 /
// D2Q9 (Eq. (LMMFD-3)), with neighbour values shared across the lanes of a
// wavefront instead of read again from LDS.
//
// The node update is the binary32 pair form of the single-step kernel
// (mmfd_node): acc = sum over pairs p of A+_p (phi(x + e_p) - phi(x)) and
// A-_p (phi(x - e_p) - phi(x)), in pair order, then phi' = A0 phi + acc.
// Each difference phi(x - e_p) - phi(x) is the negative of a difference
// phi(y + e_p) - phi(y) that the node y = x - e_p forms for its own first
// term, so every node forms one difference per pair (4 on D2Q9) and takes
// the other from the lane that formed it: from the lane to its left or right
// by a DPP lane shift fused into the multiply-add, and for the row below from
// its own registers of the previous row.  Negation is exact, so results equal
// the single-step kernel's value for value.
//
// A lane owns one column and slides down its row segment, reading one LDS
// word per node (its own column of the next row) and taking the columns
// beside it from the neighbouring lanes.  The first and last lanes of a
// wavefront have a neighbour in another wavefront, so their results are not
// used: wavefront k covers columns 62 k .. 62 k + 63 of a window of 62 NW + 2
// columns and writes 62 of them; the window's own first and last columns are
// never updated anyway (every step updates a region one node smaller than the
// last).
#include <map>
#include <mutex>
#include <tuple>

#include "mfd_internal.h"

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

// The W x H window of level t whose origin is (x0, y0), by rows: wavefront
// w of the NW RG loads rows w, w + NW RG, ..., each as NW chunks of 64
// columns, NPF values per thread (NPF / NW rows).  Rows past the window and
// columns past W repeat the last one, so that the loads issue back to back
// without branches between them.  One conditional wrap per coordinate
// (nx >= W, ny >= H).
template <int NW, int RG, int NPF>
__device__ __forceinline__ void window_fetch(const float *__restrict__ cur, int nx, int ny, int H,
                                             int x0, int y0, int wave, float (&v)[NPF]) {
  constexpr int W = 62 * NW + 2, WAVES = NW * RG, ROWS = NPF / NW;
  const int lane = threadIdx.x & 63;
  int gx[NW];
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    const int c = min(lane + 64 * m, W - 1);
    const int x = x0 + c;
    gx[m] = x < 0 ? x + nx : (x >= nx ? x - nx : x);
  }
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const int r = min(wave + WAVES * j, H - 1);
    int y = y0 + r;
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    const float *row = cur + (int64_t)y * nx;
#pragma unroll
    for (int m = 0; m < NW; ++m) v[j * NW + m] = row[gx[m]];
  }
}

template <int NW, int RG, int NPF>
__device__ __forceinline__ void window_put(float *lds, int H, int wave, const float (&v)[NPF]) {
  constexpr int W = 62 * NW + 2, WP = 64 * NW, WAVES = NW * RG, ROWS = NPF / NW;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const int r = wave + WAVES * j;
    if (r < H) {
#pragma unroll
      for (int m = 0; m < NW; ++m)
        if (lane + 64 * m < W) lds[r * WP + lane + 64 * m] = v[j * NW + m];
    }
  }
}

}  // namespace

// Persistent workgroups: workgroup b takes the tiles of the virtual blocks
// b, b + G, b + 2G, ... (G = gridDim.x, a multiple of 8, so that every virtual
// block of a workgroup maps to the tiles of its own XCD).  While a tile's
// steps run, the next tile's window is loaded into registers; it goes to the
// LDS buffer the last step did not write.
// NW wavefronts across (window W = 62 NW + 2 columns, LDS pitch 64 NW),
// RG row groups; TB steps; tile (W - 2 TB) x (H - 2 TB); H <= NW RG NPF / NW.
template <int P, int NW, int RG, int NPF>
__global__ __launch_bounds__(64 * NW *RG) void k_lcde_tb(const float *__restrict__ cur,
                                                        float *__restrict__ out, int nx, int ny,
                                                        int H, int TB, int tiles_x, int ntiles,
                                                        LinC kc) {
  constexpr int W = 62 * NW + 2, WP = 64 * NW, NT = 64 * NW * RG;
  extern __shared__ unsigned char smem_lcde[];
  float *lds = reinterpret_cast<float *>(smem_lcde);  // [2][H][WP]
  const int TX = W - 2 * TB, TY = H - 2 * TB;
  const int WH = WP * H;
  const int G = gridDim.x;
  if ((int)blockIdx.x >= ntiles) return;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wx = wave % NW, rg = wave / NW;
  const int col = 62 * wx + lane;
  // LDS column this lane writes: its own, except the two lanes a wavefront
  // shares with its neighbour, which write to the spare columns W + 1, W of
  // the pitch (never read; the same LDS banks as their own columns).  Lanes
  // outside the step's region write values no later update of the region
  // reads.
  const int wcol = (lane == 63 && wx < NW - 1) ? W + 1 : ((lane == 0 && wx > 0) ? W : col);
  float ap[4], nam[4], a0 = kc.a0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    ap[p] = kc.ap[p];
    nam[p] = kc.nam[p];
    // in vector registers, so that the lane shifts fuse into the multiply-adds
    asm("" : "+v"(ap[p]));
    asm("" : "+v"(nam[p]));
  }

  int v = blockIdx.x;
  int tile = xcd_remap_l(v, ntiles);
  int x0 = (tile % tiles_x) * TX - TB, y0 = (tile / tiles_x) * TY - TB;
  float pf[NPF];
  window_fetch<NW, RG, NPF>(cur, nx, ny, H, x0, y0, wave, pf);
  window_put<NW, RG, NPF>(lds, H, wave, pf);
  __syncthreads();
  int ic = 0;
  while (true) {
    // the next tile of this workgroup, its window in flight during the steps
    const int vn = v + G;
    const bool more = vn < ntiles;
    int xn = 0, yn = 0;
    if (more) {
      const int tn = xcd_remap_l(vn, ntiles);
      xn = (tn % tiles_x) * TX - TB;
      yn = (tn / tiles_x) * TY - TB;
      window_fetch<NW, RG, NPF>(cur, nx, ny, H, xn, yn, wave, pf);
    }
#pragma unroll 1
    for (int t = 1; t <= TB; ++t) {
      const float *A = lds + ic * WH;
      float *O = lds + (1 - ic) * WH;
      const int Hr = H - 2 * t;
      const int seg = (Hr + RG - 1) / RG;
      const int ya = t + rg * seg, yb = min(ya + seg, H - t);
      if (ya < yb) {  // uniform across the wavefront
        // node (x, y): rc = phi(x, y), rn = phi(x, y + 1); *p: the differences
        // the node (x, y - 1) formed; *o: this node's, for the row below
        auto node = [&](float rc, float rn, float dyp, float ddp, float dap, float &dyo,
                        float &ddo, float &dao) {
          const float dx = from_right(rc) - rc;  // phi(x+1, y) - phi(x, y)
          const float dy = rn - rc;              // phi(x, y+1) - phi(x, y)
          float acc = __builtin_fmaf(ap[0], dx, 0.0f);
          acc = fmac_from_left(acc, dx, nam[0]);  // phi(x-1, y) - phi(x, y), negated
          acc = __builtin_fmaf(ap[1], dy, acc);
          acc = __builtin_fmaf(nam[1], dyp, acc);
          dyo = dy;
          if constexpr (P == 4) {
            const float dd = from_right(rn) - rc;  // phi(x+1, y+1) - phi(x, y)
            const float da = from_left(rn) - rc;   // phi(x-1, y+1) - phi(x, y)
            acc = __builtin_fmaf(ap[2], dd, acc);
            acc = fmac_from_left(acc, ddp, nam[2]);
            acc = __builtin_fmaf(ap[3], da, acc);
            acc = fmac_from_right(acc, dap, nam[3]);
            ddo = dd;
            dao = da;
          }
          return __builtin_fmaf(a0, rc, acc);
        };
        // differences of the row above the segment's first row
        float r0 = A[(ya - 1) * WP + col];
        const float ra = A[ya * WP + col];
        float dy0 = ra - r0, dd0 = from_right(ra) - r0, da0 = from_left(ra) - r0;
        float dy1 = 0.f, dd1 = 0.f, da1 = 0.f;
        r0 = ra;
        const float *ar = A + (ya + 1) * WP + col;
        float *ow = O + ya * WP + wcol;
        int y = ya;
        // two rows per pass, the carried differences alternating between two
        // register sets
        for (; y + 1 < yb; y += 2) {
          const float r1 = ar[0];
          const float r2 = ar[WP];
          ow[0] = node(r0, r1, dy0, dd0, da0, dy1, dd1, da1);
          ow[WP] = node(r1, r2, dy1, dd1, da1, dy0, dd0, da0);
          r0 = r2;
          ar += 2 * WP;
          ow += 2 * WP;
        }
        if (y < yb) ow[0] = node(r0, ar[0], dy0, dd0, da0, dy1, dd1, da1);
      }
      lds_barrier();
      ic = 1 - ic;
    }

    // ---- the tile: the interior of the last level.  The next window goes to
    // the buffer the last step did not write, before the tile's stores, so
    // that its wait is for the loads alone.
    const float *C = lds + ic * WH;
    auto store = [&]() {
      for (int i = threadIdx.x; i < TX * TY; i += NT) {
        const int lx = i % TX, ly = i / TX;
        const int gx = x0 + TB + lx, gy = y0 + TB + ly;
        if (gx < nx && gy < ny) out[(int64_t)gy * nx + gx] = C[(TB + ly) * WP + TB + lx];
      }
    };
    if (!more) {
      store();
      break;
    }
    window_put<NW, RG, NPF>(lds + (1 - ic) * WH, H, wave, pf);
    asm volatile("" ::: "memory");
    store();
    ic = 1 - ic;
    lds_barrier();
    v = vn;
    x0 = xn;
    y0 = yn;
  }
}

// ------------------------------------------------------------ host side
bool lcde_tb_applies(const Consts &c, int elem) {
  return elem == 4 && c.eq == kLCDE && !c.three && c.dim == 2 && (c.lattice == 2 || c.lattice == 3);
}

namespace {
constexpr int kLcdeNpf = 16;  // window values per thread (512 threads)

}  // namespace

bool lcde_tb_window_fits(const TbPlan &pl) {
  // 8 wavefronts; NPF / NW rows each
  const int nw = pl.w == 64 ? 1 : 2;
  return pl.h <= 8 * (kLcdeNpf / nw);
}

namespace {
// resident workgroups per CU and CUs of the current device (cached)
int lcde_slots(const void *fn, int threads, size_t lds) {
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

template <int P, int NW>
hipError_t lcde_cfg(const Consts &c, const Grid &g, const TbPlan &pl, const float *cur, float *out,
                    hipStream_t st) {
  constexpr int RG = NW == 1 ? 8 : 4;
  constexpr int W = 62 * NW + 2;
  const KC<float> k = make_kc<float>(c);
  LinC lc{};
  for (int p = 0; p < P; ++p) {
    lc.ap[p] = k.Ap[p];
    lc.nam[p] = -k.Am[p];
  }
  lc.a0 = k.A0t;
  const int nx = (int)g.n[0], ny = (int)g.n[1];
  const int TX = W - 2 * pl.tb, TY = pl.h - 2 * pl.tb;
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const size_t lds = (size_t)2 * pl.h * 64 * NW * sizeof(float);
  if (pl.h > NW * RG * (kLcdeNpf / NW)) return hipErrorInvalidValue;
  auto fn = k_lcde_tb<P, NW, RG, kLcdeNpf>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  // persistent grid: the resident workgroups, a multiple of 8 (XCDs)
  const int ntiles = tx * ty;
  int grid = lcde_slots((const void *)fn, 64 * NW * RG, lds);
  if (grid <= 0) return hipErrorInvalidValue;
  grid = grid < ntiles ? grid : ntiles;
  if (grid >= 8) grid &= ~7;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * NW * RG), lds, st, cur, out, nx, ny, pl.h, pl.tb,
                     tx, ntiles, lc);
  return hipGetLastError();
}

template <int P>
hipError_t lcde_w(const Consts &c, const Grid &g, const TbPlan &pl, const float *cur, float *out,
                  hipStream_t st) {
  if (pl.w == 126) return lcde_cfg<P, 2>(c, g, pl, cur, out, st);
  if (pl.w == 64) return lcde_cfg<P, 1>(c, g, pl, cur, out, st);
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_lcde_tb(const Consts &c, const Grid &g, const TbPlan &pl, const float *cur,
                          float *out, hipStream_t st) {
  if (c.lattice == 3) return lcde_w<4>(c, g, pl, cur, out, st);
  if (c.lattice == 2) return lcde_w<2>(c, g, pl, cur, out, st);
  return hipErrorInvalidValue;
}

}  // namespace mfd
