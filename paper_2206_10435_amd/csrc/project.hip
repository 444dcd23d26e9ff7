// Early projections (Sec. 3.7).  Attributes that are not in the output are
// removed from the generator before it is built: a table whose attributes are
// all summed out (its separator aside) is deleted -- its subtree's
// completions still count, as a factor carried by its parent -- and the kept
// tables' entries are grouped by their output attributes only.
//
// On the device this is the hot path run twice:
//   1. the upward pass over the full factors gives every deleted child's
//      message; each entry of a kept table carries the frequency
//      w(e) = c(e) * prod over its deleted children of M_ch(e's value)
//      (k_proj_weights);
//   2. the kept tables' entry keys, restricted to the output columns, are
//      built into factors again (the same group-by, with full entries in place
//      of rows), and a projected entry's frequency is the sum of w over the
//      full entries it groups (k_proj_counts);
//   3. the summary kernels run on those factors with the frequencies in place
//      of row counts.
// The projected result is materialized by run expansion (desum_runs.hip).
#include <algorithm>
#include <cstring>
#include <vector>

#include "desum.h"
#include "kernels.h"
#include "plan.h"

using namespace gjh;

namespace {

__global__ void __launch_bounds__(GJ_BLOCK) k_proj_weights(const WorkItem* __restrict__ wl,
                                                           const TDesc* __restrict__ D, FPtrs F, SPtrs S,
                                                           gjk::ProjArgs pa, int64_t* __restrict__ w) {
  const WorkItem it = wl[blockIdx.x];
  if (!((pa.kept >> it.t) & 1u)) return;
  const TDesc& d = D[it.t];
  const int64_t M = F.cnt[it.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)it.tile * GJ_TILE;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    if (e >= M) break;
    const int64_t se = d.off + e;
    uint64_t v = (uint64_t)(F.eend[se] - F.estart[se]);
    for (int i = 0; i < d.nchild; ++i) {
      if ((pa.del[it.t] >> i) & 1u) {
        const TDesc& dc = D[d.child[i]];
        const int32_t j = S.link[dc.link_off + e];
        v = smul(v, j >= 0 ? (uint64_t)S.Mg[dc.off + j] : 0ULL);
      }
    }
    w[se] = (int64_t)v;
  }
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int off) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, off);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), off);
  return ((uint64_t)hi << 32) | lo;
}

// A projected entry's frequency: the saturating sum of w over the full
// entries it groups (F.ecnt zeroed beforehand).  One thread per grouped
// position, so a projected entry that groups many full entries (a heavy
// value of the kept columns) is summed by many threads: the position's entry
// is a binary search over the entries' starts, each wave sums its runs of
// equal entries, and the run's last lane adds the sum with a saturating
// compare-and-swap.
__global__ void __launch_bounds__(GJ_BLOCK) k_proj_counts(const WorkItem* __restrict__ wl,
                                                          const TDesc* __restrict__ D, FPtrs F,
                                                          const int64_t* __restrict__ w, gjk::ProjArgs pa) {
  const WorkItem it = wl[blockIdx.x];
  const TDesc& d = D[it.t];
  const int64_t M = F.cnt[it.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)it.tile * GJ_TILE;
  const int64_t* wt = w + pa.full_off[it.t];
  const int32_t* estart = F.estart + d.off;
  const int ln = lane_id();
  const int64_t wave0 = base + (threadIdx.x - ln);
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    if (wave0 + r * GJ_BLOCK >= d.n) break;  // wave-uniform
    const int64_t x = base + r * GJ_BLOCK + threadIdx.x;
    int32_t e = -1;
    uint64_t v = 0;
    if (x < d.n) {
      int64_t lo = 0, hi = M;  // the last entry starting at or before x
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (estart[mid] <= x)
          lo = mid;
        else
          hi = mid;
      }
      e = (int32_t)lo;
      v = (uint64_t)wt[F.perm[d.off + x]];
    }
    const int32_t eprev = __shfl_up(e, 1);
    const bool head = ln == 0 || eprev != e;
    const uint64_t heads = __ballot(head);
    const int sst = 63 - __clzll(heads & (ln == 63 ? ~0ull : ((2ull << ln) - 1)));
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t u = shfl_up_u64(v, off);
      if (ln - off >= sst) v = sadd(v, u);
    }
    const int32_t enext = __shfl_down(e, 1);
    const bool tail = ln == 63 || enext != e;
    if (tail && e >= 0) {
      unsigned long long* dst = reinterpret_cast<unsigned long long*>(F.ecnt + d.off + e);
      unsigned long long old = *dst;
      while (true) {
        const unsigned long long nv = sadd((uint64_t)old, v);
        const unsigned long long prev = atomicCAS(dst, old, nv);
        if (prev == old) break;
        old = prev;
      }
    }
  }
}

}  // namespace

namespace gjk {

void proj_weights(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, const SPtrs& S,
                  const ProjArgs& pa, int64_t* w) {
  if (nwl > 0) hipLaunchKernelGGL(k_proj_weights, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S, pa, w);
}

void proj_counts(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, const int64_t* w,
                 const ProjArgs& pa, int64_t slots) {
  fill_i64(s, F.ecnt, slots, 0);
  if (nwl > 0) hipLaunchKernelGGL(k_proj_counts, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, w, pa);
}

}  // namespace gjk

extern "C" {

gj_status gj_summarize_projected(gj_ctx* ctx, const gj_factors* fc, const uint32_t* out_cols, gj_summary** out,
                                 int64_t* join_size) {
  GJ_SCOPE(ctx);
  if (!ctx || !fc || !out_cols || !out) {
    set_error("gj_summarize_projected: null argument");
    return GJ_E_INVALID;
  }
  gj_factors* f = const_cast<gj_factors*>(fc);
  const Plan& P = f->plan;
  if (P.nq != 1) {
    set_error("gj_summarize_projected: factors of a single query are needed");
    return GJ_E_INVALID;
  }
  const int n = P.nt;
  // output attributes; a join attribute marked on one side is marked on both
  std::vector<uint32_t> m(out_cols, out_cols + n);
  for (int t = 0; t < n; ++t) {
    if (P.td[t].k < 32 && (m[t] >> P.td[t].k) != 0) {
      set_error("gj_summarize_projected: table %d has %d key columns; mask 0x%x", t, P.td[t].k, m[t]);
      return GJ_E_INVALID;
    }
  }
  for (int t = 1; t < n; ++t) {
    const TDesc& d = P.td[t];
    if (((m[t] >> d.sep) & 1u) || ((m[d.parent] >> d.pcol) & 1u)) {
      m[t] |= 1u << d.sep;
      m[d.parent] |= 1u << d.pcol;
    }
  }
  // kept: an output attribute besides the separator (the root: any), or a kept child
  std::vector<int> kept(n, 0);
  for (int t = n - 1; t >= 0; --t) {
    const TDesc& d = P.td[t];
    const uint32_t own = t == 0 ? m[t] : (m[t] & ~(1u << d.sep));
    kept[t] = own != 0;
    for (int i = 0; i < d.nchild; ++i) kept[t] |= kept[d.child[i]];
  }
  if (!kept[0]) {
    set_error("gj_summarize_projected: no output attribute");
    return GJ_E_INVALID;
  }
  for (int t = 1; t < n; ++t) {
    if (kept[t] && !((m[t] >> P.td[t].sep) & 1u)) {
      set_error("gj_summarize_projected: table %d holds output attributes but its separator is summed out "
                "(that needs a fill-in edge; root the query at a table holding the output attributes)", t);
      return GJ_E_GRAPH;
    }
  }
  if (m[0] == 0) {
    set_error("gj_summarize_projected: the root holds no output attribute");
    return GJ_E_GRAPH;
  }
  // the projected query: kept tables in order, keys = their output columns
  std::vector<int> idx(n, -1), src;
  for (int t = 0; t < n; ++t)
    if (kept[t]) {
      idx[t] = (int)src.size();
      src.push_back(t);
    }
  const int np = (int)src.size();
  int ncols_out = 0;
  std::vector<std::vector<int>> ocols(n);
  for (int t : src) {
    for (int c = 0; c < P.td[t].k; ++c)
      if ((m[t] >> c) & 1u) ocols[t].push_back(c);
    ncols_out += t == 0 ? (int)ocols[t].size() : (int)ocols[t].size() - 1;
  }
  if (ncols_out > GJ_MAX_OUT_COLS) {
    set_error("gj_summarize_projected: %d output columns (at most %d)", ncols_out, GJ_MAX_OUT_COLS);
    return GJ_E_INVALID;
  }

  // 1. full summary: messages of the deleted children
  gj_summary* full = nullptr;
  int64_t Q = 0;
  gj_status st = gj_summarize(ctx, f, &full, &Q);
  if (st) return st;
  hipStream_t hs = ctx->stream;
  Arena tmp(ctx);
  int64_t* w = tmp.get_n<int64_t>(P.S);
  if (!w) {
    gj_free_summary(full);
    return GJ_E_OOM;
  }
  gjk::ProjArgs pa{};
  for (int t = 0; t < n; ++t) {
    if (!kept[t]) continue;
    pa.kept |= 1u << t;
    for (int i = 0; i < P.td[t].nchild; ++i)
      if (!kept[P.td[t].child[i]]) pa.del[t] |= 1u << i;
  }
  gjk::proj_weights(hs, P.d_wl + P.all.off, P.all.n, P.d_desc, f->F, full->S, pa, w);

  // 2. factors of the projected query over the full entries' keys
  std::vector<std::vector<const int32_t*>> cols(np);
  std::vector<gj_table> tabs(np);
  std::vector<int32_t> par(np), sep(np), pcol(np);
  for (int i = 0; i < np; ++i) {
    const int t = src[i];
    const TDesc& d = P.td[t];
    for (int c : ocols[t]) cols[i].push_back(f->F.ekey + d.key_off + (int64_t)c * d.n);
    tabs[i].n_rows = full->cnt_host[t * CNT_STRIDE + CNT_M];
    tabs[i].n_keys = (int32_t)cols[i].size();
    tabs[i].keys = cols[i].data();
    par[i] = t == 0 ? -1 : idx[d.parent];
    sep[i] = t == 0 ? 0 : (int32_t)(std::find(ocols[t].begin(), ocols[t].end(), d.sep) - ocols[t].begin());
    pcol[i] = t == 0 ? 0
                     : (int32_t)(std::find(ocols[d.parent].begin(), ocols[d.parent].end(), d.pcol) -
                                 ocols[d.parent].begin());
    pa.full_off[i] = d.off;
  }
  gj_join_graph g{np, par.data(), sep.data(), pcol.data()};
  gj_factors* pf = new gj_factors(ctx);
  pf->plan.ctx = ctx;
  int qoff[2] = {0, np};
  if ((st = plan_tables(pf->plan, 1, qoff, tabs.data(), &g)) || (st = plan_device(pf->plan, pf->arena, pf->F))) {
    delete pf;
    gj_free_summary(full);
    return st;
  }
  pf->F.ecnt = pf->arena.get_n<int64_t>(pf->plan.S);
  if (!pf->F.ecnt) {
    delete pf;
    gj_free_summary(full);
    return GJ_E_OOM;
  }
  launch_factors(pf->plan, pf->F, hs);
  const Plan& PP = pf->plan;
  gjk::proj_counts(hs, PP.d_wl + PP.all.off, PP.all.n, PP.d_desc, pf->F, w, pa, PP.S);

  // 3. the summary of the projected factors
  gj_summary* s = new gj_summary(ctx);
  s->f = pf;  // owns the projected factors (one reference)
  s->projected = true;
  int64_t q = 0;
  int32_t qs = 0;
  if ((st = alloc_summary(PP, s->arena, s->S)) == GJ_OK) {
    launch_summary(PP, pf->F, s->S, hs);
    if (!(st = check(hipGetLastError(), "projection kernels")) &&
        !(st = check(hipMemcpyAsync(&q, s->S.qsize, 8, hipMemcpyDeviceToHost, hs), "join size")) &&
        !(st = check(hipMemcpyAsync(&qs, s->S.qstatus, 4, hipMemcpyDeviceToHost, hs), "join size")))
      st = read_counters(PP, pf->F, hs, s->cnt_host);
  }
  gj_free_summary(full);
  if (st) {
    gj_free_summary(s);
    return st;
  }
  pf->cnt_host = s->cnt_host;
  if (qs == GJ_E_OVERFLOW || q != Q) {
    set_error(qs == GJ_E_OVERFLOW ? "join size does not fit below 2^63-1"
                                  : "projected join size %lld differs from the join size %lld",
              (long long)q, (long long)Q);
    gj_free_summary(s);
    return qs == GJ_E_OVERFLOW ? GJ_E_OVERFLOW : GJ_E_DEVICE;
  }
  s->join_size = q;
  if (join_size) *join_size = q;
  *out = s;
  return GJ_OK;
}

int32_t gj_summary_n_tables(const gj_summary* s) {
  if (!s) return 0;
  return s->f->plan.qfirst[s->query + 1] - s->f->plan.qfirst[s->query];
}

gj_status gj_desummarize_projected(gj_ctx* ctx, const gj_summary* s, int64_t first_row, int64_t n_rows, int32_t* out,
                                   int64_t* n_written) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || n_rows < 0 || first_row < 0) {
    set_error("gj_desummarize_projected: bad argument");
    return GJ_E_INVALID;
  }
  if (first_row > s->join_size) {
    set_error("first_row %lld beyond the join size %lld", (long long)first_row, (long long)s->join_size);
    return GJ_E_RANGE;
  }
  const int64_t nw = std::min(n_rows, s->join_size - first_row);
  if (nw > 0 && (!out || ((uintptr_t)out & 15) != 0)) {
    set_error("gj_desummarize_projected: output must be a non-null, 16-byte aligned device buffer");
    return GJ_E_INVALID;
  }
  const Plan& P = s->f->plan;
  const int base = P.qfirst[s->query];
  const int n = P.qfirst[s->query + 1] - base;
  gjk::RunArgs a{};
  int nc = 0;
  for (int t = 0; t < n; ++t) {
    const TDesc& d = P.td[base + t];
    gjk::RunTab& T = a.tab[t];
    T.cpre = s->S.cpre + d.off;
    T.cc = s->S.cc + d.off;
    T.cU = s->S.cU + d.off;
    T.crec = d.parent >= 0 ? s->S.crec + d.link_off : nullptr;
    T.parent = d.parent >= 0 ? d.parent - base : -1;
  }
  std::vector<std::pair<int, int>> cols = s->result_cols;
  if (cols.empty())
    for (int t = 0; t < n; ++t) {
      const TDesc& d = P.td[base + t];
      for (int c = 0; c < d.k; ++c)
        if (d.is_root || c != d.sep) cols.push_back({t, c});
    }
  if ((int)cols.size() > GJ_MAX_OUT_COLS) {
    set_error("gj_desummarize_projected: %d result columns (at most %d)", (int)cols.size(), GJ_MAX_OUT_COLS);
    return GJ_E_INVALID;
  }
  for (auto& tc : cols) {
    const TDesc& d = P.td[base + tc.first];
    a.col_tab[nc] = tc.first;
    a.col_key[nc] = s->S.ckey + d.key_off + (int64_t)tc.second * d.n;
    ++nc;
  }
  a.first = first_row;
  a.n_rows = nw;
  a.n_root = s->cnt_host[base * CNT_STRIDE + CNT_MC];
  a.out = out;
  a.n_tables = n;
  a.n_cols = nc;
  if (nw > 0 && nc > 0) {
    if (gjk::expand_runs(ctx->stream, a, ctx->tune.desum_rounds) != 0) {
      set_error("gj_desummarize_projected: chunk too large for one launch");
      return GJ_E_INVALID;
    }
    gj_status st = check(hipGetLastError(), "run expansion kernel");
    if (st) return st;
  }
  if (n_written) *n_written = nc > 0 ? nw : 0;
  return GJ_OK;
}

}  // extern "C"
