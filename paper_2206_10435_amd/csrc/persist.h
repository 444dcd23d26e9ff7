// Stage instances, tasks and arguments of the persistent batch kernel
// (batch_persist.hip).
#pragma once
#include <vector>

#include "plan.h"

namespace gjk {

enum PKind : int32_t {
  PK_FILL_Q = 0,  // join size 0 and status GJ_OK of query t
  PK_FILL_DG,     // downward messages of table t set to 0
  PK_FILL_DIDX,   // dense group index of table t set to -1
  PK_PACK,
  PK_UP,
  PK_DSCAN,
  PK_DN,
  PK_RCOUNT,
  PK_RSCAN,
  PK_RWRITE,
  PK_GIDX,
  PK_UPAGG,
  PK_SEGT,
  PK_UPSCAN,
  PK_DOWN,
  PK_CCOUNT,
  PK_CSCAN,
  PK_CWRITE,
  PK_GRECS,
  PK_CLINKS,
};

struct PStage {
  int32_t kind, t, pass;
  int32_t units;     // tiles, digits, fill chunks or 1
  int32_t per_task;  // units per task
  int32_t ntasks;
  int32_t dep_off, ndep;
};

struct PTask {
  int32_t stage, unit0;
};

struct PArgs {
  const PTask* tasks;
  const PStage* stages;
  const int32_t* deps;
  int32_t* done;  // per stage instance: tasks completed
  int32_t* ctl;   // [0] next task, [1] blocks finished, [2] a wait timed out
  int32_t ntasks, nstages, nq;
  int64_t spin_limit;
  const TDesc* D;
  FPtrs F;
  SPtrs S;
};

// The stage instances, their dependencies and the task list of a plan.
void build_persistent_plan(const gjh::Plan& P, int task_rows, std::vector<PStage>& stages,
                           std::vector<int32_t>& deps, std::vector<PTask>& tasks);
// Dynamic LDS of the persistent kernel, its grid, its launch.
size_t persistent_lds(int sort_items64);
int persistent_grid(int sort_items64, int ntasks, int device);
void launch_persistent(hipStream_t s, int sort_items64, int grid, const PArgs& a);
void zero_i32(hipStream_t s, int32_t* p, int64_t n);

}  // namespace gjk
