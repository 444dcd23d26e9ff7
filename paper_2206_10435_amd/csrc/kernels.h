// Host-side launchers of the device kernels (one namespace, defined in the
// .hip translation units).  All launches are asynchronous on stream `s`.
#pragma once
#include "gj_internal.h"

namespace gjk {

// factor.hip
void fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v0, int32_t v1);
// per-column ranges: per-tile partials into mmt (agg_slots x MAXK x 2), reduced per table into mm
void minmax(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
            int32_t* mmt, int32_t* mm);
void pack(hipStream_t s, int wide, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& P);
// rank[perm[i]] = entry of position i of a one-column factor (m entries, n rows).
void rank_rows(hipStream_t s, const int32_t* perm, const int32_t* estart, int64_t m, int64_t n, int32_t* rank);
// one LSD pass; upsweep = false when the digit counts are already in P.hist
// (the pack writes the first pass's)
void radix_pass(hipStream_t s, int wide, int items, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab,
                const TDesc* D, const FPtrs& P, int pass, bool upsweep = true);
// sort_local.hip: the buckets of tables with `local` set, sorted in LDS
// (words[0] -> words[1]); lflag[t] = 1 where a bucket is too long
void local_sort(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F);
void runs(hipStream_t s, int wide, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
          const FPtrs& P);
void runs_scan(hipStream_t s, const int32_t* tabs, int ntab, const TDesc* D, const FPtrs& P);
void runs_write(hipStream_t s, int wide, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& P);
void tile_scan_pair(hipStream_t s, const int32_t* tabs, int ntab, const TDesc* D, uint64_t* agg, int64_t* cnt, int ca,
                    int cb);

// separator value -> group for tables with a dense index (after the runs)
void group_index(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F);
// out[entry slot] = the entry's frequency (given count, or its row count)
void entry_counts(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, int64_t* out);

// summary.hip
void fill_i64(hipStream_t s, int64_t* p, int64_t n, int64_t v);
void up_pass(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
             const FPtrs& F, const SPtrs& S);
// One level of the downward pass: wl/nwl the parents' tiles, rwl/nrwl the
// (child, bucket and tile range) items of the bucket sums; bucketed / scattered:
// a child of the level takes the bucket sums / the atomic scatter.
void down_pass(hipStream_t s, const WorkItem* wl, int nwl, const WorkItem* rwl, int nrwl, bool bucketed,
               bool scattered, const TDesc* D, const FPtrs& F, const SPtrs& S);
void compact(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
             const FPtrs& F, const SPtrs& S);
// copies one query's join size and status (device) to caller arrays
void export_status(hipStream_t s, const int64_t* qsize, const int32_t* qstatus, int64_t* out_size,
                   int32_t* out_status);

// desum.hip
struct DesumArgs;
// Launch shape of the expansion kernel (host only): staging round KS, tuples
// per lane, grid, LDS allocated per block and used by the actual columns,
// bytes a lane stages per round.  ok = 0 if the arguments or the shape are
// outside what the kernel supports.
struct DesumPlan {
  int ok;
  int stage, tuples_per_lane, kernel_tables, seg_bytes;
  int64_t blocks, lds_bytes, lds_used;
};
DesumPlan desum_plan(int n_tables, int rowid_bytes, int n_cols, int64_t n_rows, int rounds_per_lane, int stage);
// returns -1 if the launch does not fit one grid
int desummarize(hipStream_t s, const DesumArgs& a, int rowid_bytes, int n_tables, int rounds_per_lane, int stage);
// Expansion of a summary whose middle tables hold one entry per group
// (desum_unit.hip): row ids (a.n_cols = 0) or a.n_cols int32 value columns
// (rowid_bytes 4); 0 on success, -1 for unsupported arguments.  tl_single:
// the innermost table holds one entry per group too.  With `rec` (int32,
// desum_unit_record_bytes of `cap` entries, cap from
// desum_unit_record_entries) and `range` (2 int64) the root entries' records
// are written by a pass of their own first; rec = nullptr decodes them in place.
int desummarize_unit(hipStream_t s, const DesumArgs& a, int rowid_bytes, int n_tables, bool tl_single, int64_t* range,
                     int32_t* rec, int64_t cap);
int64_t desum_unit_blocks(int64_t n_rows);
int64_t desum_unit_record_entries(int64_t n_root, int64_t n_rows, int n_tables, bool tl_single, int n_cols,
                                  int tuple_bytes);
int64_t desum_unit_record_bytes(int64_t cap, int n_tables, bool tl_single, int n_cols);
// value columns (desum_values.hip): tuples per staging round, and the launch
int value_round(int n_tables, int n_cols);
void launch_values(hipStream_t s, const DesumArgs& a, int blocks);
// run expansion of a projected summary (desum_runs.hip); -1 if it does not fit one launch
struct RunArgs;
int expand_runs(hipStream_t s, const RunArgs& a, int rounds_per_lane);
// projections (project.hip): per kept table of the full factors, the frequency
// each full entry carries into the projection (its row count times the
// completions of its deleted children); then per projected entry, the sum
// over the full entries it groups
struct ProjArgs {
  uint32_t kept;                // bit t: table t is kept
  uint32_t del[GJ_MAX_TABLES];  // bit i: child i of table t is deleted
  int64_t full_off[GJ_MAX_TABLES];  // projected table -> slot offset of its table in the full plan
};
void proj_weights(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, const SPtrs& S,
                  const ProjArgs& pa, int64_t* w);
// (zeroes F.ecnt's `slots` first)
void proj_counts(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, const int64_t* w,
                 const ProjArgs& pa, int64_t slots);
// out[i] = data[perm[i]] for i < n: a row-order column in grouped row order
void gather_rows(hipStream_t s, const int32_t* perm, const int32_t* data, int64_t n, int32_t* out);

}  // namespace gjk
