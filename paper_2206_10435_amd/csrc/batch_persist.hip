// Persistent batch kernel: the factor build and the summary of every query of
// a batch in ONE kernel launch.
//
// The host turns the batch into stage instances -- one per (table, stage) and,
// for the radix sort, per pass -- in the order the one-launch-per-stage path
// launches them, and splits every stage instance into tasks of a few tiles.
// Blocks of the persistent grid take tasks in that order from a device counter.
// A task first waits until every stage instance it depends on has completed
// all its tasks (per-instance completion counters), runs its tiles with the
// same stage bodies as the per-stage kernels (stages.h), and then counts
// itself complete.  Dependencies are per table, never global: a small query
// moves on to its summary while a large one is still sorting, and no stage
// waits for a whole-grid barrier.
//
// Progress.  A block takes a task only while it runs, and every task's
// dependencies come earlier in the task order; so the earliest unfinished
// task always has all its dependencies complete, and the grid drains whatever
// the residency.  Every wait is still bounded: a wait that exceeds its limit
// skips the task's work, flags the launch, and the last block marks every
// query GJ_E_DEVICE instead of leaving a wrong result unflagged.
//
// Memory ordering.  Each XCD has its own L2, so a task's writes are released
// at agent scope by every wave before the completion count, and a waiting
// task acquires at agent scope before it reads.  The last block to leave
// resets the counters, so a recorded graph of this one kernel can be replayed.
#include <algorithm>
#include <vector>

#include "kernels.h"
#include "persist.h"
#include "stages.h"


namespace {

using gjk::PArgs;
using gjk::PStage;

constexpr int FILL_CHUNK = GJ_TILE;

template <int I0>
__device__ __forceinline__ void run_unit(const PArgs& a, const PStage& st, int u, unsigned char* lds) {
  const WorkItem w{st.t, u};
  const TDesc* D = a.D;
  const FPtrs& F = a.F;
  const SPtrs& S = a.S;
  switch (st.kind) {
    case gjk::PK_FILL_Q:
      if (threadIdx.x == 0) {
        S.qsize[st.t] = 0;
        S.qstatus[st.t] = GJ_OK;
      }
      break;
    case gjk::PK_FILL_DG: {
      const TDesc& d = D[st.t];
      const int64_t end = d.off + max((int64_t)1, d.n);
      for (int64_t i = d.off + (int64_t)u * FILL_CHUNK + threadIdx.x; i < min(end, d.off + (int64_t)(u + 1) * FILL_CHUNK);
           i += GJ_BLOCK)
        S.Dg[i] = 0;
      break;
    }
    case gjk::PK_FILL_DIDX: {
      const TDesc& d = D[st.t];
      const int64_t end = d.didx_off + d.drange;
      for (int64_t i = d.didx_off + (int64_t)u * FILL_CHUNK + threadIdx.x;
           i < min(end, d.didx_off + (int64_t)(u + 1) * FILL_CHUNK); i += GJ_BLOCK)
        F.didx[i] = -1;
      break;
    }
    case gjk::PK_PACK:
      if (D[st.t].wide)
        pack_body<1>(w, D, F.words[0], F.hist, lds);
      else
        pack_body<0>(w, D, F.words[0], F.hist, lds);
      break;
    case gjk::PK_UP:
      if (D[st.t].wide)
        upsweep_body<1, 8>(w, D, F.words[0], F.words[1], F.hist, st.pass, lds);
      else
        upsweep_body<0, I0>(w, D, F.words[0], F.words[1], F.hist, st.pass, lds);
      break;
    case gjk::PK_DSCAN:
      digit_scan_body(st.t, u, D, F.hist, F.dtot, lds);
      break;
    case gjk::PK_DN:
      if (D[st.t].wide)
        downsweep_body<1, 8>(w, D, F.words[0], F.words[1], F.hist, F.dtot, st.pass, lds);
      else
        downsweep_body<0, I0>(w, D, F.words[0], F.words[1], F.hist, F.dtot, st.pass, lds);
      break;
    case gjk::PK_RCOUNT:
      if (D[st.t].wide)
        runs_count_body<1>(w, D, F.words[0], F.words[1], F.agg, lds);
      else
        runs_count_body<0>(w, D, F.words[0], F.words[1], F.agg, lds);
      break;
    case gjk::PK_RSCAN:
      tile_scan_pair_body(st.t, D, F.agg, F.cnt, CNT_M, CNT_G, lds);
      break;
    case gjk::PK_RWRITE:
      if (D[st.t].wide)
        runs_write_body<1>(w, D, F.words[0], F.words[1], F.agg, F, lds);
      else
        runs_write_body<0>(w, D, F.words[0], F.words[1], F.agg, F, lds);
      break;
    case gjk::PK_GIDX:
      group_index_body(w, D, F);
      break;
    case gjk::PK_UPAGG:
      up_agg_body(w, D, F, S, lds);
      break;
    case gjk::PK_SEGT:
      seg_tiles_body(st.t, D, F, lds);
      break;
    case gjk::PK_UPSCAN:
      up_scan_body(w, D, F, S, lds);
      break;
    case gjk::PK_DOWN:
      down_body(w, D, F, S, lds);
      break;
    case gjk::PK_CCOUNT:
      compact_count_body(w, D, F, S, lds);
      break;
    case gjk::PK_CSCAN:
      tile_scan_pair_body(st.t, D, F.agg, F.cnt, CNT_MC, CNT_GC, lds);
      break;
    case gjk::PK_CWRITE:
      compact_write_body(w, D, F, S, lds);
      break;
    case gjk::PK_GRECS:
      group_recs_body(w, D, F, S);
      break;
    case gjk::PK_CLINKS:
      compact_links_body(w, D, F, S);
      break;
    default:
      break;
  }
}

template <int I0>
__global__ void __launch_bounds__(GJ_BLOCK) k_batch_persistent(PArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int32_t s_task;
  __shared__ int32_t s_skip;
  __shared__ int32_t s_last;
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(&a.ctl[0], 1);
    __syncthreads();
    const int32_t ti = s_task;
    if (ti >= a.ntasks) break;
    const gjk::PTask tk = a.tasks[ti];
    const PStage st = a.stages[tk.stage];
    if (threadIdx.x == 0) {
      int skip = 0;
      for (int k = 0; k < st.ndep && !skip; ++k) {
        const int32_t ds = a.deps[st.dep_off + k];
        const int32_t need = a.stages[ds].ntasks;
        int64_t spins = 0;
        while (__hip_atomic_load(&a.done[ds], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          // once any wait has timed out, every other wait gives up at once,
          // so a launch that went wrong ends within one wait's bound
          if (++spins > a.spin_limit ||
              __hip_atomic_load(&a.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            skip = 1;
            __hip_atomic_store(&a.ctl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      s_skip = skip;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (!s_skip) {
      const int u1 = min(st.units, tk.unit0 + st.per_task);
      for (int u = tk.unit0; u < u1; ++u) {
        run_unit<I0>(a, st, u, lds);
        __syncthreads();  // the next unit reuses the LDS
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&a.done[tk.stage], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // the last block to leave flags a timed-out launch and resets the counters
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    s_last = __hip_atomic_fetch_add(&a.ctl[1], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool failed = __hip_atomic_load(&a.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    for (int i = threadIdx.x; i < a.nstages; i += GJ_BLOCK) a.done[i] = 0;
    if (failed)
      for (int q = threadIdx.x; q < a.nq; q += GJ_BLOCK) a.S.qstatus[q] = GJ_E_DEVICE;
    __syncthreads();
    if (threadIdx.x == 0) {
      a.ctl[0] = 0;
      a.ctl[1] = 0;
      a.ctl[2] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace

namespace gjk {

size_t persistent_lds(int sort_items64) {
  size_t m = std::max<size_t>(LDS_DOWN, LDS_SEG);
  m = std::max<size_t>(m, LDS_UPSWEEP);
  m = std::max<size_t>(m, LDS_PACK);
  m = std::max<size_t>(m, lds_downsweep<1, 8>());
  m = std::max<size_t>(m, sort_items64 == 16 ? lds_downsweep<0, 16>() : lds_downsweep<0, 8>());
  return m;
}

// Host side: the stage instances, their dependencies and the task list of a
// plan, in the order the per-stage path launches them.
struct PPlan {
  std::vector<PStage> stages;
  std::vector<int32_t> deps;
  std::vector<PTask> tasks;
  int per_task_rows = 16384;

  int add(int kind, int t, int pass, int64_t units, int unit_rows, const std::vector<int>& dep) {
    PStage s{};
    s.kind = kind;
    s.t = t;
    s.pass = pass;
    s.units = (int32_t)units;
    s.per_task = std::max(1, per_task_rows / std::max(1, unit_rows));
    s.ntasks = (int32_t)((units + s.per_task - 1) / s.per_task);
    s.dep_off = (int32_t)deps.size();
    s.ndep = 0;
    for (int d : dep)
      if (d >= 0) {
        deps.push_back(d);
        ++s.ndep;
      }
    stages.push_back(s);
    return (int)stages.size() - 1;
  }
};

void build_persistent_plan(const gjh::Plan& P, int task_rows, std::vector<PStage>& stages, std::vector<int32_t>& deps,
                           std::vector<PTask>& tasks) {
  PPlan pp;
  pp.per_task_rows = task_rows > 0 ? task_rows : 16384;
  const int nt = P.nt;
  std::vector<int> fillq(P.nq, -1), filldg(nt, -1), filldidx(nt, -1), pack(nt, -1), last(nt, -1), rcount(nt, -1),
      rscan(nt, -1), rwrite(nt, -1), gidx(nt, -1), upagg(nt, -1), segt(nt, -1), upscan(nt, -1), down(nt, -1),
      ccount(nt, -1), cscan(nt, -1), cwrite(nt, -1), grecs(nt, -1), clinks(nt, -1);
  auto tiles = [&](int t) { return (int64_t)P.td[t].ntiles; };
  // fills
  for (int q = 0; q < P.nq; ++q) fillq[q] = pp.add(PK_FILL_Q, q, 0, 1, 1, {});
  for (int t = 0; t < nt; ++t) {
    const TDesc& d = P.td[t];
    if (d.parent >= 0) filldg[t] = pp.add(PK_FILL_DG, t, 0, (std::max<int64_t>(d.n, 1) + FILL_CHUNK - 1) / FILL_CHUNK,
                                          FILL_CHUNK, {});
    if (d.didx_off >= 0)
      filldidx[t] = pp.add(PK_FILL_DIDX, t, 0, (d.drange + FILL_CHUNK - 1) / FILL_CHUNK, FILL_CHUNK, {});
  }
  // factor build
  for (int t = 0; t < nt; ++t) pack[t] = pp.add(PK_PACK, t, 0, tiles(t), GJ_TILE, {});
  for (int t = 0; t < nt; ++t) last[t] = pack[t];
  for (int p = 0; p < P.max_passes; ++p) {
    std::vector<int> up(nt, -1), ds(nt, -1);
    for (int t = 0; t < nt; ++t)
      if (P.td[t].npasses > p) up[t] = pp.add(PK_UP, t, p, P.td[t].ntiles_sort, P.td[t].sort_tile, {last[t]});
    for (int t = 0; t < nt; ++t)
      if (P.td[t].npasses > p) ds[t] = pp.add(PK_DSCAN, t, p, 1 << P.td[t].dbits, 1024, {up[t]});
    for (int t = 0; t < nt; ++t)
      if (P.td[t].npasses > p) last[t] = pp.add(PK_DN, t, p, P.td[t].ntiles_sort, P.td[t].sort_tile, {ds[t]});
  }
  for (int t = 0; t < nt; ++t) rcount[t] = pp.add(PK_RCOUNT, t, 0, tiles(t), GJ_TILE, {last[t]});
  for (int t = 0; t < nt; ++t) rscan[t] = pp.add(PK_RSCAN, t, 0, 1, 1, {rcount[t]});
  for (int t = 0; t < nt; ++t) rwrite[t] = pp.add(PK_RWRITE, t, 0, tiles(t), GJ_TILE, {rscan[t]});
  for (int t = 0; t < nt; ++t)
    if (P.td[t].didx_off >= 0) gidx[t] = pp.add(PK_GIDX, t, 0, tiles(t), GJ_TILE, {rwrite[t], filldidx[t]});
  // upward pass, leaves first
  for (int h = 0; h <= P.max_height; ++h) {
    for (int t = 0; t < nt; ++t) {
      if (P.ht[t].height != h) continue;
      std::vector<int> dep{rwrite[t]};
      for (int ch : P.ht[t].children) {
        dep.push_back(upscan[ch]);
        dep.push_back(gidx[ch]);
      }
      upagg[t] = pp.add(PK_UPAGG, t, 0, tiles(t), GJ_TILE, dep);
    }
    for (int t = 0; t < nt; ++t)
      if (P.ht[t].height == h) segt[t] = pp.add(PK_SEGT, t, 0, 1, 1, {upagg[t]});
    for (int t = 0; t < nt; ++t)
      if (P.ht[t].height == h)
        upscan[t] = pp.add(PK_UPSCAN, t, 0, tiles(t), GJ_TILE,
                           {segt[t], P.td[t].is_root ? fillq[P.ht[t].query] : -1});
  }
  // downward pass, root first
  for (int dd = 1; dd <= P.max_depth; ++dd)
    for (int t = 0; t < nt; ++t) {
      if (P.ht[t].depth != dd - 1 || P.ht[t].children.empty()) continue;
      std::vector<int> dep{upscan[t]};
      if (P.ht[t].parent >= 0) dep.push_back(down[P.ht[t].parent]);
      for (int ch : P.ht[t].children) dep.push_back(filldg[ch]);
      down[t] = pp.add(PK_DOWN, t, 0, tiles(t), GJ_TILE, dep);
    }
  // compaction
  for (int t = 0; t < nt; ++t)
    ccount[t] = pp.add(PK_CCOUNT, t, 0, tiles(t), GJ_TILE,
                       {upscan[t], P.ht[t].parent >= 0 ? down[P.ht[t].parent] : -1});
  for (int t = 0; t < nt; ++t) cscan[t] = pp.add(PK_CSCAN, t, 0, 1, 1, {ccount[t]});
  for (int t = 0; t < nt; ++t) cwrite[t] = pp.add(PK_CWRITE, t, 0, tiles(t), GJ_TILE, {cscan[t]});
  for (int t = 0; t < nt; ++t)
    if (P.ht[t].parent >= 0) grecs[t] = pp.add(PK_GRECS, t, 0, tiles(t), GJ_TILE, {cwrite[t]});
  for (int t = 0; t < nt; ++t) {
    if (P.ht[t].children.empty()) continue;
    std::vector<int> dep{cwrite[t]};
    for (int ch : P.ht[t].children) dep.push_back(grecs[ch]);
    clinks[t] = pp.add(PK_CLINKS, t, 0, tiles(t), GJ_TILE, dep);
  }
  // tasks in stage order
  tasks.clear();
  for (size_t s = 0; s < pp.stages.size(); ++s) {
    const PStage& st = pp.stages[s];
    for (int k = 0; k < st.ntasks; ++k) tasks.push_back(PTask{(int32_t)s, k * st.per_task});
  }
  stages = std::move(pp.stages);
  deps = std::move(pp.deps);
}

void zero_i32(hipStream_t s, int32_t* p, int64_t n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 1024);
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks), dim3(GJ_BLOCK), 0, s, p, n);
}

// Grid of the persistent kernel: as many blocks as fit on the device at once
// (a whole number per XCD), at most one per task.
int persistent_grid(int sort_items64, int ntasks, int device) {
  const size_t lds = persistent_lds(sort_items64);
  int per_cu = 1;
  if (sort_items64 == 16)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<16>, GJ_BLOCK, lds);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<8>, GJ_BLOCK, lds);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
  int64_t g = (int64_t)std::max(1, per_cu) * cus;
  g = std::min<int64_t>(g, std::max(1, ntasks));
  if (g >= 8) g = g / 8 * 8;
  return (int)std::max<int64_t>(g, 1);
}

void launch_persistent(hipStream_t s, int sort_items64, int grid, const PArgs& a) {
  const size_t lds = persistent_lds(sort_items64);
  if (sort_items64 == 16)
    hipLaunchKernelGGL(k_batch_persistent<16>, dim3(grid), dim3(GJ_BLOCK), lds, s, a);
  else
    hipLaunchKernelGGL(k_batch_persistent<8>, dim3(grid), dim3(GJ_BLOCK), lds, s, a);
}

}  // namespace gjk
