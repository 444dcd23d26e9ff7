// Stage 1 -- factors (Sec. 3.2, quantitative learning): one group-by count per
// table.  A table's factor is every distinct key tuple with its frequency; the
// GPU form is a sort of the rows by key tuple followed by run detection:
//
//   minmax   per-column range of every table (host picks field widths)
//   pack     one sort word per row: key fields (separator field most
//            significant for non-root tables) above the row id
//   radix    LSD radix sort over the key bits only; each pass is an upsweep
//            (per-tile digit counts), a digit scan and a downsweep that ranks
//            keys inside the tile with wavefront ballots, stages the tile in
//            LDS in digit order and writes contiguous digit runs.  LSD is
//            stable and the words start in row order, so rows inside an entry
//            come out ascending by row id.
//   runs     entry / separator-group boundaries, their exclusive scan, and the
//            entry arrays (keys, row range, group) plus the grouped row ids.
#include "gj_internal.h"
#include "kernels.h"
#include "stages.h"

namespace {

// ---------------------------------------------------------------------------
// Per-tile column ranges (no atomics: every tile writes its own slot), then
// one block per table reduces its tiles.
__global__ void __launch_bounds__(GJ_BLOCK) k_minmax(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                     int32_t* __restrict__ mmt) {
  __shared__ int32_t sh[2][GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int c = 0; c < d.k; ++c) {
    const int32_t* col = d.col[c];
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      int64_t i = base + r * GJ_BLOCK + threadIdx.x;
      if (i < d.n) {
        int32_t v = col[i];
        lo = min(lo, v);
        hi = max(hi, v);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane_id() == 0) {
      sh[0][wave_id()] = lo;
      sh[1][wave_id()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = 1; v < GJ_WAVES; ++v) {
        lo = min(lo, sh[0][v]);
        hi = max(hi, sh[1][v]);
      }
      mmt[((d.agg_off + w.tile) * MAXK + c) * 2 + 0] = lo;
      mmt[((d.agg_off + w.tile) * MAXK + c) * 2 + 1] = hi;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(GJ_BLOCK) k_minmax_reduce(const int32_t* __restrict__ tabs,
                                                            const TDesc* __restrict__ D,
                                                            const int32_t* __restrict__ mmt, int32_t* __restrict__ mm) {
  __shared__ int32_t sh[2][GJ_WAVES];
  const int t = tabs[blockIdx.x];
  const TDesc& d = D[t];
  for (int c = 0; c < d.k; ++c) {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int64_t i = threadIdx.x; i < d.ntiles; i += GJ_BLOCK) {
      lo = min(lo, mmt[((d.agg_off + i) * MAXK + c) * 2 + 0]);
      hi = max(hi, mmt[((d.agg_off + i) * MAXK + c) * 2 + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane_id() == 0) {
      sh[0][wave_id()] = lo;
      sh[1][wave_id()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = 1; v < GJ_WAVES; ++v) {
        lo = min(lo, sh[0][v]);
        hi = max(hi, sh[1][v]);
      }
      mm[(t * MAXK + c) * 2 + 0] = lo;
      mm[(t * MAXK + c) * 2 + 1] = hi;
    }
    __syncthreads();
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v0, int32_t v1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (i & 1) ? v1 : v0;
}

// ---------------------------------------------------------------------------
// One launch per stage: every block runs one unit of the work list (the
// bodies are in stages.h).
// ---------------------------------------------------------------------------
template <int WIDE>
__global__ void __launch_bounds__(GJ_BLOCK) k_pack(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                   uint64_t* __restrict__ words0, uint32_t* __restrict__ hist) {
  __shared__ __align__(16) unsigned char lds[LDS_PACK];
  pack_body<WIDE>(wl[blockIdx.x], D, words0, hist, lds);
}

template <int WIDE, int ITEMS>
__global__ void __launch_bounds__(GJ_BLOCK) k_upsweep(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                      uint64_t* words0, uint64_t* words1, uint32_t* __restrict__ hist,
                                                      int pass) {
  __shared__ __align__(16) unsigned char lds[LDS_UPSWEEP];
  upsweep_body<WIDE, ITEMS>(wl[blockIdx.x], D, words0, words1, hist, pass, lds);
}

// One block per (table, digit).
__global__ void __launch_bounds__(GJ_BLOCK) k_digit_scan(const int32_t* __restrict__ tabs,
                                                         const TDesc* __restrict__ D, uint32_t* __restrict__ hist,
                                                         uint32_t* __restrict__ dtot) {
  __shared__ __align__(16) unsigned char lds[LDS_SCAN32];
  digit_scan_body(tabs[blockIdx.x >> 8], blockIdx.x & 255, D, hist, dtot, lds);
}

template <int WIDE, int ITEMS>
__global__ void __launch_bounds__(GJ_BLOCK) k_downsweep(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                        uint64_t* words0, uint64_t* words1,
                                                        const uint32_t* __restrict__ hist,
                                                        const uint32_t* __restrict__ dtot, int pass) {
  __shared__ __align__(16) unsigned char lds[lds_downsweep<WIDE, ITEMS>()];
  downsweep_body<WIDE, ITEMS>(wl[blockIdx.x], D, words0, words1, hist, dtot, pass, lds);
}

template <int WIDE>
__global__ void __launch_bounds__(GJ_BLOCK) k_runs_count(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                         uint64_t* words0, uint64_t* words1,
                                                         uint64_t* __restrict__ agg) {
  __shared__ __align__(16) unsigned char lds[LDS_SCAN64];
  runs_count_body<WIDE>(wl[blockIdx.x], D, words0, words1, agg, lds);
}

template <int WIDE>
__global__ void __launch_bounds__(GJ_BLOCK) k_runs_write(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                         uint64_t* words0, uint64_t* words1,
                                                         const uint64_t* __restrict__ agg, FPtrs P) {
  __shared__ __align__(16) unsigned char lds[LDS_SCAN64];
  runs_write_body<WIDE>(wl[blockIdx.x], D, words0, words1, agg, P, lds);
}

}  // namespace

// Dense separator index (see group_index_body).
__global__ void __launch_bounds__(GJ_BLOCK) k_group_index(const WorkItem* __restrict__ wl,
                                                          const TDesc* __restrict__ D, FPtrs F) {
  group_index_body(wl[blockIdx.x], D, F);
}

// Entry frequencies as int64 (the factor view's count column).
__global__ void __launch_bounds__(GJ_BLOCK) k_entry_counts(const WorkItem* __restrict__ wl,
                                                           const TDesc* __restrict__ D, FPtrs F,
                                                           int64_t* __restrict__ out) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    if (e >= M) break;
    const int64_t se = d.off + e;
    out[se] = F.ecnt ? F.ecnt[se] : (int64_t)(F.eend[se] - F.estart[se]);
  }
}

// rank[row] = the entry of the row's position, for the rows of a one-column
// factor (entry e holds positions [estart[e], estart[e+1]) of perm).
__global__ void k_rank_rows(const int32_t* __restrict__ perm, const int32_t* __restrict__ estart, int64_t m,
                            int64_t n, int32_t* __restrict__ rank) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = m;  // the last entry starting at or before i
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (estart[mid] <= i)
        lo = mid;
      else
        hi = mid;
    }
    rank[perm[i]] = (int32_t)lo;
  }
}

// One block per table (see tile_scan_pair_body).
__global__ void __launch_bounds__(GJ_BLOCK) k_tile_scan_pair(const int32_t* __restrict__ tabs,
                                                             const TDesc* __restrict__ D, uint64_t* __restrict__ agg,
                                                             int64_t* __restrict__ cnt, int ca, int cb) {
  __shared__ __align__(16) unsigned char lds[LDS_SCAN64];
  tile_scan_pair_body(tabs[blockIdx.x], D, agg, cnt, ca, cb, lds);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace gjk {

void fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v0, int32_t v1) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(GJ_BLOCK), 0, s, p, n, v0, v1);
}

void minmax(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
            int32_t* mmt, int32_t* mm) {
  if (nwl > 0) hipLaunchKernelGGL(k_minmax, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, mmt);
  if (ntab > 0) hipLaunchKernelGGL(k_minmax_reduce, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, mmt, mm);
}

void pack(hipStream_t s, int wide, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& P) {
  if (nwl <= 0) return;
  if (wide)
    hipLaunchKernelGGL(k_pack<1>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.hist);
  else
    hipLaunchKernelGGL(k_pack<0>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.hist);
}

void radix_pass(hipStream_t s, int wide, int items, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab,
                const TDesc* D, const FPtrs& P, int pass, bool upsweep) {
  if (nwl <= 0) return;
#define GJ_RADIX_CASE(W, I)                                                                                        \
  if (wide == W && items == I) {                                                                                   \
    if (upsweep)                                                                                                   \
      hipLaunchKernelGGL((k_upsweep<W, I>), dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1],      \
                         P.hist, pass);                                                                            \
    hipLaunchKernelGGL(k_digit_scan, dim3(ntab * 256), dim3(GJ_BLOCK), 0, s, tabs, D, P.hist, P.dtot);            \
    hipLaunchKernelGGL((k_downsweep<W, I>), dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1],       \
                       P.hist, P.dtot, pass);                                                                      \
    return;                                                                                                        \
  }
  GJ_RADIX_CASE(0, 8)
  GJ_RADIX_CASE(0, 16)
  GJ_RADIX_CASE(1, 8)
#undef GJ_RADIX_CASE
}

void runs(hipStream_t s, int wide, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
          const FPtrs& P) {
  if (nwl <= 0) return;
  if (wide)
    hipLaunchKernelGGL(k_runs_count<1>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg);
  else
    hipLaunchKernelGGL(k_runs_count<0>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg);
}

void runs_scan(hipStream_t s, const int32_t* tabs, int ntab, const TDesc* D, const FPtrs& P) {
  if (ntab > 0)
    hipLaunchKernelGGL(k_tile_scan_pair, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, P.agg, P.cnt, CNT_M, CNT_G);
}

void runs_write(hipStream_t s, int wide, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& P) {
  if (nwl <= 0) return;
  if (wide)
    hipLaunchKernelGGL(k_runs_write<1>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg, P);
  else
    hipLaunchKernelGGL(k_runs_write<0>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg, P);
}

void rank_rows(hipStream_t s, const int32_t* perm, const int32_t* estart, int64_t m, int64_t n, int32_t* rank) {
  if (n <= 0 || m <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 8192);
  hipLaunchKernelGGL(k_rank_rows, dim3(blocks), dim3(GJ_BLOCK), 0, s, perm, estart, m, n, rank);
}

void group_index(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F) {
  if (nwl > 0) hipLaunchKernelGGL(k_group_index, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F);
}

void entry_counts(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, int64_t* out) {
  if (nwl > 0) hipLaunchKernelGGL(k_entry_counts, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, out);
}

void tile_scan_pair(hipStream_t s, const int32_t* tabs, int ntab, const TDesc* D, uint64_t* agg, int64_t* cnt, int ca,
                    int cb) {
  if (ntab > 0) hipLaunchKernelGGL(k_tile_scan_pair, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, agg, cnt, ca, cb);
}

}  // namespace gjk
