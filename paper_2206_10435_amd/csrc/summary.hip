// Stage 2 -- summary.  Integer sum-product message passing over the join tree.
//
// Upward (Sec. 3.3, Algorithm 2; variable elimination Eq. 4 from the leaves):
// for every entry e of table t, U_t(e) = product over t's children ch of the
// child's message at e's value of the joining column (1 at a leaf); the
// message of t is M_t(s) = sum of c_t(e) * U_t(e) over t's entries with
// separator value s, and the root's sum is the join size (Eq. 3's Z).
//   k_up_agg    U per entry (looking each child value up in the child's
//               sorted separator values, which also records the entry ->
//               child-group link), tile aggregates of a segmented scan of c*U
//   k_seg_tiles carry-in of every tile
//   k_up_scan   exclusive prefix of c*U inside each separator group (the block
//               offsets used by desummarization) and the group totals M
// Downward (Sec. 3.5, Algorithms 3-4 condition each level on the levels
// above): D_t(s) = sum over parent entries e' with value s in the joining
// column of c_p(e') * D_p(e') * product of the other children's messages
// (that product is recorded per entry and child by the upward pass).  Per
// level, for children of at most DOWN_MAX_GROUPS groups:
//   k_down_tile     a parent tile's items (group, term) ordered by bucket of
//                   2^sh child groups in LDS, written in that order
//   k_down_reduce   one bucket over a range of tiles summed per group in LDS,
//                   written to D (or added, for buckets of several ranges)
// and for larger children k_down scatters the terms with 64-bit atomics after
// merging a tile's repeats in LDS.  Integer sums: exact in any order (every
// partial sum is bounded by the join size once the upward pass has not
// overflowed).
// Compaction keeps entries with F = c*U*D > 0 and groups with M*D > 0 (Sec.
// 3.3: entries of frequency below 1 are excluded) and re-links them.
#include "gj_internal.h"
#include "kernels.h"
#include "stages.h"

namespace {

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One launch per stage: every block runs one unit of the work list (the
// bodies are in stages.h).
__global__ void __launch_bounds__(GJ_BLOCK) k_up_agg(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                     FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_SEG];
  up_agg_body(wl[blockIdx.x], D, F, S, lds);
}

// One block per table.
__global__ void __launch_bounds__(GJ_BLOCK) k_seg_tiles(const int32_t* __restrict__ tabs, const TDesc* __restrict__ D,
                                                        FPtrs F) {
  __shared__ __align__(16) unsigned char lds[LDS_SEG];
  seg_tiles_body(tabs[blockIdx.x], D, F, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_up_scan(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                      FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_SEG];
  up_scan_body(wl[blockIdx.x], D, F, S, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_down(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                   FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_DOWN];
  down_body<true>(wl[blockIdx.x], D, F, S, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_down_tile(const WorkItem* __restrict__ wl,
                                                        const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_DTILE];
  down_tile_body(wl[blockIdx.x], D, F, S, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_down_reduce(const WorkItem* __restrict__ wl,
                                                          const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_DRED];
  down_reduce_body(wl[blockIdx.x], D, F, S, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_compact_count(const WorkItem* __restrict__ wl,
                                                            const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_SCAN64];
  compact_count_body(wl[blockIdx.x], D, F, S, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_compact_write(const WorkItem* __restrict__ wl,
                                                            const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  __shared__ __align__(16) unsigned char lds[LDS_SCAN64];
  compact_write_body(wl[blockIdx.x], D, F, S, lds);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_group_recs(const WorkItem* __restrict__ wl,
                                                         const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  group_recs_body(wl[blockIdx.x], D, F, S);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_compact_links(const WorkItem* __restrict__ wl,
                                                            const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  compact_links_body(wl[blockIdx.x], D, F, S);
}

__global__ void k_export_status(const int64_t* __restrict__ qsize, const int32_t* __restrict__ qstatus,
                                int64_t* __restrict__ out_size, int32_t* __restrict__ out_status) {
  if (threadIdx.x == 0) {
    *out_size = *qsize;
    *out_status = *qstatus;
  }
}

}  // namespace

namespace gjk {

void export_status(hipStream_t s, const int64_t* qsize, const int32_t* qstatus, int64_t* out_size,
                   int32_t* out_status) {
  hipLaunchKernelGGL(k_export_status, dim3(1), dim3(64), 0, s, qsize, qstatus, out_size, out_status);
}

void fill_i64(hipStream_t s, int64_t* p, int64_t n, int64_t v) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 4096);
  hipLaunchKernelGGL(k_fill_i64, dim3(blocks), dim3(GJ_BLOCK), 0, s, p, n, v);
}

void up_pass(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
             const FPtrs& F, const SPtrs& S) {
  if (nwl <= 0) return;
  hipLaunchKernelGGL(k_up_agg, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  hipLaunchKernelGGL(k_seg_tiles, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, F);
  hipLaunchKernelGGL(k_up_scan, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
}

void down_pass(hipStream_t s, const WorkItem* wl, int nwl, const WorkItem* rwl, int nrwl, bool bucketed,
               bool scattered, const TDesc* D, const FPtrs& F, const SPtrs& S) {
  if (nwl <= 0) return;
  if (bucketed) {
    hipLaunchKernelGGL(k_down_tile, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
    if (nrwl > 0) hipLaunchKernelGGL(k_down_reduce, dim3(nrwl), dim3(GJ_BLOCK), 0, s, rwl, D, F, S);
  }
  if (scattered) hipLaunchKernelGGL(k_down, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
}

void compact(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
             const FPtrs& F, const SPtrs& S) {
  if (nwl <= 0) return;
  hipLaunchKernelGGL(k_compact_count, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  tile_scan_pair(s, tabs, ntab, D, F.agg, F.cnt, CNT_MC, CNT_GC);
  hipLaunchKernelGGL(k_compact_write, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  hipLaunchKernelGGL(k_group_recs, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  hipLaunchKernelGGL(k_compact_links, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
}

}  // namespace gjk
