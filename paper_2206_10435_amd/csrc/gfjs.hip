// The paper-literal GFJS of a row range (Sec. 1.2 Definition 1; the runs
// Algorithms 3-4 emit, one per distinct value prefix): for every result
// column i, the runs of equal (v_0..v_i) among consecutive result rows, as
// (value of column i, run length) pairs.
//
//   1. the range is expanded into row-id tuples (the desummarization kernel);
//   2. every surviving entry scatters its index to its rows (row -> entry), so
//      a row id gives its key values;
//   3. per result column, a row starts a run if it starts one at the previous
//      column or its value differs from the previous row's; the run heads are
//      compacted by an exclusive scan and the lengths are differences of
//      consecutive heads.
#include <vector>

#include "desum.h"
#include "kernels.h"
#include "plan.h"

using namespace gjh;

namespace {

constexpr int TILE = GJ_TILE;

// row -> surviving entry: one thread per grouped position p (an entry of many
// rows is spread over many threads); its entry is the last surviving one
// starting at or before p, if p lies inside it (rows of pruned entries are
// never looked up)
__global__ void k_rmap(const int32_t* __restrict__ perm, const int2* __restrict__ ccs, int64_t nent, int64_t n,
                       int32_t* __restrict__ rmap) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    if (ccs[0].y > p) continue;
    int64_t lo = 0, hi = nent;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (ccs[mid].y <= p)
        lo = mid;
      else
        hi = mid;
    }
    const int2 cs = ccs[lo];
    if (p < (int64_t)cs.y + cs.x) rmap[perm[p]] = (int32_t)lo;
  }
}

// value of result column (table t, column c) for row j of the range
__device__ __forceinline__ int32_t colval(const int32_t* __restrict__ rid, int n, int t,
                                          const int32_t* __restrict__ rmap, const int32_t* __restrict__ keys,
                                          int64_t j) {
  return keys[rmap[rid[j * n + t]]];
}

// head flags of one column (flags hold the previous column's heads on entry),
// plus per-tile head counts
__global__ void __launch_bounds__(GJ_BLOCK) k_heads(const int32_t* __restrict__ rid, int n, int t,
                                                    const int32_t* __restrict__ rmap,
                                                    const int32_t* __restrict__ keys, int64_t rows,
                                                    uint8_t* __restrict__ flags, uint32_t* __restrict__ tcnt) {
  __shared__ uint32_t sh[GJ_WAVES];
  const int64_t base = (int64_t)blockIdx.x * TILE;
  uint32_t cnt = 0;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t j = base + r * GJ_BLOCK + threadIdx.x;
    if (j < rows) {
      bool h = j == 0 || flags[j] != 0;
      if (!h) h = colval(rid, n, t, rmap, keys, j) != colval(rid, n, t, rmap, keys, j - 1);
      flags[j] = h ? 1 : 0;
      cnt += h ? 1u : 0u;
    }
  }
  uint32_t tot;
  block_excl_sum(cnt, sh, tot);
  if (threadIdx.x == 0) tcnt[blockIdx.x] = tot;
}

// exclusive scan of the tile counts (one block); total into *nruns
__global__ void __launch_bounds__(GJ_BLOCK) k_scan_tiles(uint32_t* __restrict__ tcnt, int64_t ntiles,
                                                         int64_t* __restrict__ nruns) {
  __shared__ uint32_t sh[GJ_WAVES];
  uint32_t carry = 0;
  for (int64_t i0 = 0; i0 < ntiles; i0 += GJ_BLOCK) {
    const int64_t i = i0 + threadIdx.x;
    const uint32_t v = i < ntiles ? tcnt[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_sum(v, sh, tot);
    if (i < ntiles) tcnt[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *nruns = carry;
}

__global__ void __launch_bounds__(GJ_BLOCK) k_runs_out(const int32_t* __restrict__ rid, int n, int t,
                                                       const int32_t* __restrict__ rmap,
                                                       const int32_t* __restrict__ keys, int64_t rows,
                                                       const uint8_t* __restrict__ flags,
                                                       const uint32_t* __restrict__ tcnt, int32_t* __restrict__ vout,
                                                       int64_t* __restrict__ start) {
  __shared__ uint32_t sh[GJ_WAVES];
  const int64_t base = (int64_t)blockIdx.x * TILE;
  uint32_t carry = tcnt[blockIdx.x];
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t j = base + r * GJ_BLOCK + threadIdx.x;
    const uint32_t h = (j < rows && flags[j]) ? 1u : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_sum(h, sh, tot) + carry;
    carry += tot;
    if (h) {
      vout[ex] = colval(rid, n, t, rmap, keys, j);
      start[ex] = j;
    }
  }
}

// run lengths from consecutive run heads
__global__ void k_lengths(const int64_t* __restrict__ heads, int64_t* __restrict__ len,
                          const int64_t* __restrict__ nruns, int64_t rows) {
  const int64_t k = *nruns;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x)
    len[i] = ((i + 1 < k) ? heads[i + 1] : rows) - heads[i];
}

}  // namespace

extern "C" gj_status gj_unroll_gfjs(gj_ctx* ctx, const gj_summary* s, int64_t first_row, int64_t n_rows,
                                    int32_t* const* values, int64_t* const* freqs, int64_t* n_runs) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || !values || !freqs || !n_runs || first_row < 0 || n_rows < 0) {
    set_error("gj_unroll_gfjs: bad argument");
    return GJ_E_INVALID;
  }
  if (s->projected || !s->f->F.perm) {
    set_error("gj_unroll_gfjs: the summary has no row ids (projected, or loaded without rows)");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  if (first_row > s->join_size) {
    set_error("first_row beyond the join size");
    return GJ_E_RANGE;
  }
  const int64_t rows = std::min(n_rows, s->join_size - first_row);
  const Plan& P = s->f->plan;
  const int base = P.qfirst[s->query];
  const int n = P.qfirst[s->query + 1] - base;
  // result columns: (table, column) in result order
  std::vector<std::pair<int, int>> cols;
  for (int t = 0; t < n; ++t) {
    const TDesc& d = P.td[base + t];
    for (int c = 0; c < d.k; ++c)
      if (d.is_root || c != d.sep) cols.push_back({t, c});
  }
  for (size_t i = 0; i < cols.size(); ++i) n_runs[i] = 0;
  if (rows == 0) return GJ_OK;
  for (size_t i = 0; i < cols.size(); ++i)
    if (!values[i] || !freqs[i]) {
      set_error("gj_unroll_gfjs: null output for column %zu", i);
      return GJ_E_INVALID;
    }
  hipStream_t st = ctx->stream;
  Arena A(ctx);
  int32_t* rid = A.get_n<int32_t>(rows * n);
  int64_t total_rows = 0;
  for (int t = 0; t < n; ++t) total_rows += std::max<int64_t>(P.td[base + t].n, 1);
  int32_t* rmap = A.get_n<int32_t>(total_rows);
  uint8_t* flags = A.get_n<uint8_t>(rows);
  const int64_t ntiles = (rows + TILE - 1) / TILE;
  uint32_t* tcnt = A.get_n<uint32_t>(ntiles);
  int64_t* nr = A.get_n<int64_t>((int64_t)cols.size());
  if (!rid || !rmap || !flags || !tcnt || !nr) return GJ_E_OOM;
  int64_t nw = 0;
  gj_status r = gj_desummarize(ctx, s, first_row, rows, 4, rid, &nw);
  if (r) return r;
  // row -> surviving entry, per table
  std::vector<int64_t> roff(n, 0);
  for (int t = 1; t < n; ++t) roff[t] = roff[t - 1] + std::max<int64_t>(P.td[base + t - 1].n, 1);
  for (int t = 0; t < n; ++t) {
    const TDesc& d = P.td[base + t];
    const int64_t nent = s->cnt_host[(base + t) * CNT_STRIDE + CNT_MC];
    if (nent > 0)
      hipLaunchKernelGGL(k_rmap, dim3((unsigned)std::min<int64_t>((d.n + 255) / 256, 4096)), dim3(256), 0, st,
                         s->f->F.perm + d.off, s->S.ccs + d.off, nent, d.n, rmap + roff[t]);
  }
  if ((r = check(hipMemsetAsync(flags, 0, rows, st), "gfjs flags"))) return r;
  for (size_t i = 0; i < cols.size(); ++i) {
    const int t = cols[i].first, c = cols[i].second;
    const TDesc& d = P.td[base + t];
    const int32_t* keys = s->S.ckey + d.key_off + (int64_t)c * d.n;
    // the rid columns are strided by n; rid + t points at table t's ids
    hipLaunchKernelGGL(k_heads, dim3((unsigned)ntiles), dim3(GJ_BLOCK), 0, st, rid, n, t, rmap + roff[t], keys, rows,
                       flags, tcnt);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(GJ_BLOCK), 0, st, tcnt, ntiles, nr + i);
    hipLaunchKernelGGL(k_runs_out, dim3((unsigned)ntiles), dim3(GJ_BLOCK), 0, st, rid, n, t, rmap + roff[t], keys,
                       rows, flags, tcnt, values[i], freqs[i]);
  }
  if ((r = check(hipGetLastError(), "gfjs kernels"))) return r;
  std::vector<int64_t> h(cols.size());
  if ((r = check(hipMemcpyAsync(h.data(), nr, 8 * cols.size(), hipMemcpyDeviceToHost, st), "gfjs")) ||
      (r = check(hipStreamSynchronize(st), "gfjs")))
    return r;
  // lengths: consecutive differences of the run heads (read from a copy)
  for (size_t i = 0; i < cols.size(); ++i) {
    if (h[i] == 0) continue;
    int64_t* heads = A.get_n<int64_t>(h[i]);
    if (!heads) return GJ_E_OOM;
    if ((r = check(hipMemcpyAsync(heads, freqs[i], 8 * h[i], hipMemcpyDeviceToDevice, st), "gfjs"))) return r;
    hipLaunchKernelGGL(k_lengths, dim3((unsigned)std::min<int64_t>((h[i] + 255) / 256, 4096)), dim3(256), 0, st,
                       heads, freqs[i], nr + i, rows);
  }
  if ((r = check(hipStreamSynchronize(st), "gfjs"))) return r;
  for (size_t i = 0; i < cols.size(); ++i) n_runs[i] = h[i];
  return GJ_OK;
}
