// The batch object behind the opaque mfd_batch handle.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "batch_kernels.h"
#include "solver.h"

namespace mfd {

struct BatchEntry {
  Solver *s;
  int64_t nsteps;
  int tb = 1;  // steps per launch of its group in the last run
};

struct Group {
  BatchKey key{};
  bool tb_ok = false;           // two-level LCDE / Burgers: blocked kernel usable
  TbPlan plan{1, 0};            // tb = 1: one launch per step (k_batch_step)
  std::vector<int> order;       // entry indices, decreasing step count
  std::vector<int> tile0;       // first tile of each instance (sorted order)
  std::vector<int> tiles_x;
  std::vector<int64_t> steps;   // step count of each instance (sorted order)
  int ntiles = 0, tile_cap = 0;
  void *d_inst = nullptr;       // BatchInst<T>[instances]
  int *d_tile_inst = nullptr;   // instance slot of every tile (capacity tile_cap)
  size_t inst_bytes = 0;
  std::vector<unsigned char> h_inst;
  void *d_lane = nullptr;       // instance table of the lane-shared kernel (128-column plans)
  size_t lane_bytes = 0;
  std::vector<unsigned char> h_lane;
};

// instances run by the LDS-resident kernel (one launch per kind)
struct ResGroup {
  BatchKey key{};
  std::vector<int> order;  // entry indices
  ResInst *d = nullptr;
  std::vector<ResInst> h;
};

// group kind of a solver, and whether such groups can be temporally blocked
BatchKey batch_key_of(const Solver *s);
bool batch_blockable(const BatchKey &k);

struct Batch {
  std::vector<BatchEntry> entries;
  std::vector<Group> groups;
  std::vector<ResGroup> res;            // LDS-resident instances
  int resident_max = 4096;              // binary32 instances of at most this many nodes run LDS-resident
  hipStream_t stream = nullptr, own_stream = nullptr;
  hipStream_t side = nullptr;           // the resident launches' branch of a run
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true, dirty = true, sticky = false;
  TbPlan req{0, 0};                     // plan set by the caller (tb = 0: automatic)
  std::map<BatchKey, TbPlan> tuned;     // plans chosen by autotune()
  int64_t max_steps = 0, launches_per_run = 0, lups_per_run = 0;
  std::string err;

  int fail(int code, const char *fmt, ...);
  int hip(hipError_t e, const char *what);
  void free_graph();
  void free_groups();
  int build();
  int make_tables(Group &g);
  int upload_instances();
  int enqueue_steps();
  int enqueue_group_steps();
  hipError_t launch_group_tb(const Group &g, int nt, int64_t l);
  int run();
  int autotune();
};

}  // namespace mfd
