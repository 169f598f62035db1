// Device descriptors of the batched step (see kernels_batch.hip).
#pragma once

#include "mfd_internal.h"

namespace mfd {

constexpr int kBatchTX = 64, kBatchTY = 16, kBatchTYNse = 8;

// one instance of a batch group, as the kernel reads it
template <typename T>
struct BatchInst {
  T *ring[4];     // level buffers: two-level ring[0..1]; three-level ring[0..2], or
                  // (t, t - dt) pairs ring[0..1] / ring[2..3] under a blocked plan
  int nx, ny;
  int ring_len;   // 2 or 3
  int c0;         // ring index of level t at the first step of the run
  int tiles_x;
  int tile0;      // first tile of this instance in the group's tile table
  int64_t nsteps; // steps of this instance in the run
  KC<T> kc;       // the instance's step constants
};

// what selects the kernel of a group
struct BatchKey {
  int lattice, eq, three, three_st, precision;
  int b1;  // Burgers with beta = 1 (no quadratic EDF term)
  bool operator<(const BatchKey &o) const {
    if (b1 != o.b1) return b1 < o.b1;
    if (lattice != o.lattice) return lattice < o.lattice;
    if (eq != o.eq) return eq < o.eq;
    if (three != o.three) return three < o.three;
    if (three_st != o.three_st) return three_st < o.three_st;
    return precision < o.precision;
  }
};

template <typename T>
hipError_t launch_batch_step(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst,
                             int ntiles, int64_t s, hipStream_t st);

// temporally blocked batched launch `launch` (two-level LCDE / Burgers groups;
// NSE groups: launch_batch_nse_tb)
template <typename T>
hipError_t launch_batch_tb(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst,
                           int ntiles, int64_t launch, const TbPlan &pl, hipStream_t st);
template <typename T>
hipError_t launch_batch_nse_tb(const BatchKey &k, const BatchInst<T> *inst, const int *tile_inst,
                               int ntiles, int64_t launch, const TbPlan &pl, hipStream_t st);

// LDS-resident batched run (kernels_batch.hip): binary32 two-level linear CDE
// and Burgers MMFD instances whose two levels fit in LDS; one workgroup per
// instance runs all of its steps.  lv[0] holds level t at the start; after
// nsteps steps level t + nsteps is in lv[nsteps % 2] and the level before it
// in the other (the roles a run of single steps leaves).
struct ResInst {
  float *lv[2];
  int nx, ny;
  int64_t nsteps;
  KC<float> kc;
};
constexpr int kResMaxNodes = 20480;  // two binary32 levels in 160 KiB of LDS
bool resident_applies(const BatchKey &k, int64_t nx, int64_t ny);
// nmax: the largest instance's node count (sizes the LDS and the workgroup)
hipError_t launch_batch_resident(const BatchKey &k, const ResInst *inst, int count, int nmax,
                                 hipStream_t st);

// lane-shared batched launch (kernels_lane_tb.hip): binary32 two-level LCDE and
// Burgers (beta = 1) groups under 128-column plans, with an instance table of
// their own (lane_inst_bytes per instance, filled by lane_inst_fill; false:
// this solver's constants do not suit the kernel)
bool lane_batch_applies(const BatchKey &k);
size_t lane_inst_bytes(const BatchKey &k);
bool lane_inst_fill(const BatchKey &k, const Consts &c, float *cur, float *other, int nx, int ny,
                    int tiles_x, int tile0, int64_t nsteps, void *dst);
hipError_t launch_batch_lane_tb(const BatchKey &k, const void *inst, const int *tile_inst,
                                int ntiles, int64_t launch, const TbPlan &pl, hipStream_t st);

}  // namespace mfd
