// Batched MMFD step over many independent periodic 2D grids.
//
// One launch advances every active instance of a group (same lattice,
// equation, levels and precision; any grid sizes and coefficients) by one
// time step.  The tile table is instance-major and instances are ordered by
// decreasing step count, so the instances still running at step s own a
// prefix of the table and the launch covers exactly that prefix.  Each
// workgroup reads its instance descriptor (sizes, level ring, constants) with
// uniform loads and runs the same tile body as the single-grid kernel, so a
// batched run equals the instance run alone value for value.  Small binary32
// instances can instead run all of their steps LDS-resident (below).
#include "../../include/mfd.h"
#include "batch_kernels.h"
#include "mmfd_node.h"

namespace mfd {

template <class L, int EQ, bool THREE, bool THREE_ST, int TX, int TY, typename T>
__global__ __launch_bounds__(256) void k_batch_step(const BatchInst<T> *__restrict__ inst,
                                                    const int *__restrict__ tile_inst,
                                                    int ntiles, int64_t s) {
  const int t = xcd_remap(blockIdx.x, ntiles);
  const BatchInst<T> &I = inst[tile_inst[t]];
  const int lt = t - I.tile0;
  const int x0 = (lt % I.tiles_x) * TX, y0 = (lt / I.tiles_x) * TY;
  const int64_t r = I.c0 + s;
  const T *cur = I.ring[r % I.ring_len];
  T *out = I.ring[(r + 1) % I.ring_len];
  const T *prev = THREE ? I.ring[(r + 2) % 3] : nullptr;
  mmfd_plane_tile<L, EQ, THREE, THREE_ST, TX, TY, T>(cur, prev, out, I.nx, I.ny, x0, y0, I.kc);
}

namespace {

template <class L, int EQ, bool THREE, bool THREE_ST, typename T>
hipError_t bcfg(const BatchInst<T> *inst, const int *tile_inst, int ntiles, int64_t s,
                hipStream_t st) {
  constexpr int TX = kBatchTX, TY = EQ == kNSE ? kBatchTYNse : kBatchTY;
  hipLaunchKernelGGL((k_batch_step<L, EQ, THREE, THREE_ST, TX, TY, T>), dim3(ntiles), dim3(256), 0,
                     st, inst, tile_inst, ntiles, s);
  return hipGetLastError();
}

template <class L, int EQ, typename T>
hipError_t blev(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst, int ntiles,
                int64_t s, hipStream_t st) {
  if (!k.three) return bcfg<L, EQ, false, false, T>(inst, tile_inst, ntiles, s, st);
  if (!k.three_st) return bcfg<L, EQ, true, false, T>(inst, tile_inst, ntiles, s, st);
  return bcfg<L, EQ, true, true, T>(inst, tile_inst, ntiles, s, st);
}

template <class L, typename T>
hipError_t beq(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst, int ntiles,
               int64_t s, hipStream_t st) {
  switch (k.eq) {
    case kLCDE: return blev<L, kLCDE, T>(k, inst, tile_inst, ntiles, s, st);
    case kBurgers: return blev<L, kBurgers, T>(k, inst, tile_inst, ntiles, s, st);
    case kNSE: return blev<L, kNSE, T>(k, inst, tile_inst, ntiles, s, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename T>
hipError_t launch_batch_step(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst,
                             int ntiles, int64_t s, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (k.lattice == 3) return beq<LatD2Q9, T>(k, inst, tile_inst, ntiles, s, st);
  if (k.lattice == 2) return beq<LatD2Q5, T>(k, inst, tile_inst, ntiles, s, st);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ LDS-resident
// One workgroup per instance: the instance's level t goes to LDS, every step
// updates all nodes from one LDS level into the other (periodic neighbours
// by index wrap) with the single-step kernel's node function (mmfd_node; the
// Burgers record phi^2 dt / (2 dx) formed where read, as make_record forms
// it), so results equal a run of single steps value for value; the last two
// levels are stored.
namespace {
template <class L, int EQ, bool B1>
__global__ __launch_bounds__(1024) void k_batch_resident(const ResInst *__restrict__ inst) {
  extern __shared__ float smem_res[];
  const ResInst &I = inst[blockIdx.x];
  const int nx = I.nx, ny = I.ny, N = nx * ny;
  const int64_t n = I.nsteps;
  float *A = smem_res, *B = smem_res + N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) A[i] = I.lv[0][i];
  // a thread's nodes i = tid + k T: their coordinates advance by (T mod nx,
  // T / nx) with a carry, so no division inside the steps
  const int T = blockDim.x;
  const int dyT = T / nx, dxT = T - dyT * nx;
  const int y0 = (int)threadIdx.x / nx, x0 = (int)threadIdx.x - y0 * nx;
  __syncthreads();
  for (int64_t s = 0; s < n; ++s) {
    const float *src = (s & 1) ? B : A;
    float *dst = (s & 1) ? A : B;
    int x = x0, y = y0;
    for (int i = threadIdx.x; i < N; i += T) {
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      auto at = [&](int q, int, int dy, int dx) {
        const int yy = dy < 0 ? ym : (dy > 0 ? yp : y);
        const int xx = dx < 0 ? xm : (dx > 0 ? xp : x);
        const float v = src[yy * nx + xx];
        if constexpr (EQ == kBurgers) return q == 0 ? v : (v * v) * I.kc.bh;
        else return v;
      };
      auto ath = [](int, int, int, int) { return 0.f; };
      float cc[1] = {src[i]}, pc[1] = {0.f}, oc[1];
      mmfd_node<L, EQ, false, false, float, B1>(at, ath, cc, pc, oc, I.kc);
      dst[i] = oc[0];
      x += dxT;
      y += dyT;
      if (x >= nx) {
        x -= nx;
        ++y;
      }
    }
    __syncthreads();
  }
  const float *fin = (n & 1) ? B : A, *pre = (n & 1) ? A : B;
  float *ofin = I.lv[n & 1], *opre = I.lv[(n + 1) & 1];
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    ofin[i] = fin[i];
    if (n > 0) opre[i] = pre[i];
  }
}

// LDS for the largest instance's two levels; about 4 nodes a thread
// (64 .. 1024 threads): a run of steps is bound by the latency of each step
template <class L, int EQ, bool B1>
hipError_t res_cfg(const ResInst *inst, int count, int nmax, hipStream_t st) {
  const size_t lds = (size_t)2 * nmax * sizeof(float);
  int threads = ((nmax + 4 * 64 - 1) / (4 * 64)) * 64;
  threads = threads < 64 ? 64 : (threads > 1024 ? 1024 : threads);
  auto fn = k_batch_resident<L, EQ, B1>;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(count), dim3(threads), lds, st, inst);
  return hipGetLastError();
}

template <class L>
hipError_t res_l(const BatchKey &k, const ResInst *inst, int count, int nmax, hipStream_t st) {
  if (k.eq == kLCDE) return res_cfg<L, kLCDE, false>(inst, count, nmax, st);
  if (k.b1) return res_cfg<L, kBurgers, true>(inst, count, nmax, st);
  return res_cfg<L, kBurgers, false>(inst, count, nmax, st);
}
}  // namespace

bool resident_applies(const BatchKey &k, int64_t nx, int64_t ny) {
  if (k.precision != MFD_FP32 || k.three || k.three_st) return false;
  if (k.lattice != MFD_D2Q5 && k.lattice != MFD_D2Q9) return false;
  if (k.eq != kLCDE && k.eq != kBurgers) return false;
  return nx >= 3 && ny >= 3 && nx * ny <= kResMaxNodes;
}

hipError_t launch_batch_resident(const BatchKey &k, const ResInst *inst, int count, int nmax,
                                 hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (nmax < 1 || nmax > kResMaxNodes) return hipErrorInvalidValue;
  if (k.lattice == MFD_D2Q9) return res_l<LatD2Q9>(k, inst, count, nmax, st);
  if (k.lattice == MFD_D2Q5) return res_l<LatD2Q5>(k, inst, count, nmax, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_batch_step<float>(const BatchKey &, const BatchInst<float> *,
                                             const int *, int, int64_t, hipStream_t);
template hipError_t launch_batch_step<double>(const BatchKey &, const BatchInst<double> *,
                                              const int *, int, int64_t, hipStream_t);

}  // namespace mfd
