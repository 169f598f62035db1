// Batched MMFD step over many independent periodic 2D grids.
//
// One launch advances every active instance of a group (same lattice,
// equation, levels and precision; any grid sizes and coefficients) by one
// time step.  The tile table is instance-major and instances are ordered by
// decreasing step count, so the instances still running at step s own a
// prefix of the table and the launch covers exactly that prefix.  Each
// workgroup reads its instance descriptor (sizes, level ring, constants) with
// uniform loads and runs the same tile body as the single-grid kernel, so a
// batched run equals the instance run alone value for value.
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

template hipError_t launch_batch_step<float>(const BatchKey &, const BatchInst<float> *,
                                             const int *, int, int64_t, hipStream_t);
template hipError_t launch_batch_step<double>(const BatchKey &, const BatchInst<double> *,
                                              const int *, int, int64_t, hipStream_t);

}  // namespace mfd
