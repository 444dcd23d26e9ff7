// Host runtime and C ABI of libgj: validation, planning, buffer management and
// the ordering of the kernel launches.  No join arithmetic happens here; every
// step of the path runs in the device kernels.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "desum.h"
#include "kernels.h"
#include "plan.h"

namespace gjh {

static thread_local std::string g_err;
static thread_local gj_ctx* g_cur = nullptr;

CtxScope::CtxScope(const gj_ctx* c) : prev(g_cur) { g_cur = const_cast<gj_ctx*>(c); }
CtxScope::~CtxScope() { g_cur = prev; }

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  if (g_cur) g_cur->err = buf;
}

gj_status check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return GJ_E_DEVICE;
  }
  return GJ_OK;
}

void* Arena::get(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = nullptr;
  if (ctx->alloc) {
    p = ctx->alloc(bytes, ctx->user);
  } else if (hipMallocAsync(&p, bytes, ctx->stream) != hipSuccess) {
    p = nullptr;
  }
  if (!p) {
    set_error("device allocation of %zu bytes failed", bytes);
    return nullptr;
  }
  bufs.push_back({p, bytes});
  return p;
}

void Arena::release() {
  for (auto& b : bufs) {
    if (ctx->free_fn)
      ctx->free_fn(b.p, ctx->user);
    else
      (void)hipFreeAsync(b.p, ctx->stream);
  }
  bufs.clear();
}

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
static int bitwidth32(uint32_t v) { return v == 0 ? 0 : 32 - __builtin_clz(v); }
static int bitwidth64(uint64_t v) { return v == 0 ? 0 : 64 - __builtin_clzll(v); }

WL Plan::add_list(const std::vector<int>& tables, int tile, bool sort_tiles) {
  WL l;
  l.off = (int)wl_host.size();
  l.toff = (int)tabs_host.size();
  for (int t : tables) {
    int64_t nt_ = sort_tiles ? td[t].ntiles_sort : (ht[t].n + tile - 1) / tile;
    for (int64_t i = 0; i < nt_; ++i) wl_host.push_back(WorkItem{t, (int32_t)i});
    tabs_host.push_back(t);
  }
  l.n = (int)wl_host.size() - l.off;
  l.tn = (int)tabs_host.size() - l.toff;
  return l;
}

gj_status validate_one(const gj_table* tables, const gj_join_graph* g) {
  if (!tables || !g) {
    set_error("null tables or graph");
    return GJ_E_INVALID;
  }
  const int n = g->n_tables;
  if (n < 1 || n > GJ_MAX_TABLES) {
    set_error("n_tables = %d outside [1, %d]", n, GJ_MAX_TABLES);
    return GJ_E_INVALID;
  }
  if (n > 1 && (!g->parent || !g->sep_col || !g->parent_col)) {
    set_error("null join-graph arrays");
    return GJ_E_INVALID;
  }
  for (int t = 0; t < n; ++t) {
    const gj_table& tb = tables[t];
    if (tb.n_keys < 1 || tb.n_keys > GJ_MAX_KEYS) {
      set_error("table %d: n_keys = %d outside [1, %d]", t, tb.n_keys, GJ_MAX_KEYS);
      return GJ_E_INVALID;
    }
    if (tb.n_rows < 0 || tb.n_rows > INT32_MAX) {
      set_error("table %d: n_rows = %lld outside [0, 2^31-1]", t, (long long)tb.n_rows);
      return GJ_E_INVALID;
    }
    if (tb.n_rows > 0) {
      if (!tb.keys) {
        set_error("table %d: null key array", t);
        return GJ_E_INVALID;
      }
      for (int c = 0; c < tb.n_keys; ++c)
        if (!tb.keys[c]) {
          set_error("table %d: null key column %d", t, c);
          return GJ_E_INVALID;
        }
    }
  }
  if (g->parent && g->parent[0] != -1) {
    set_error("parent[0] must be -1 (table 0 is the root)");
    return GJ_E_GRAPH;
  }
  std::vector<int> nch(n, 0);
  for (int t = 1; t < n; ++t) {
    int p = g->parent[t];
    if (p < 0 || p >= t) {
      set_error("table %d: parent %d is not an earlier table (cycle or forest)", t, p);
      return GJ_E_GRAPH;
    }
    if (g->sep_col[t] < 0 || g->sep_col[t] >= tables[t].n_keys) {
      set_error("table %d: separator column %d out of range", t, g->sep_col[t]);
      return GJ_E_GRAPH;
    }
    if (g->parent_col[t] < 0 || g->parent_col[t] >= tables[p].n_keys) {
      set_error("table %d: parent column %d out of range for table %d", t, g->parent_col[t], p);
      return GJ_E_GRAPH;
    }
    if (++nch[p] > GJ_MAX_CHILDREN) {
      set_error("table %d has more than %d children", p, GJ_MAX_CHILDREN);
      return GJ_E_GRAPH;
    }
  }
  return GJ_OK;
}

gj_status plan_tables(Plan& P, int nq, const int* q_off, const gj_table* tables, const gj_join_graph* graphs) {
  P.nq = nq;
  P.qfirst.assign(nq + 1, 0);
  P.ht.clear();
  for (int q = 0; q < nq; ++q) {
    const gj_join_graph& g = graphs[q];
    if (q_off[q + 1] - q_off[q] != g.n_tables) {
      set_error("query %d: %d tables given, graph has %d", q, q_off[q + 1] - q_off[q], g.n_tables);
      return GJ_E_INVALID;
    }
    gj_status st = validate_one(tables + q_off[q], &g);
    if (st != GJ_OK) return st;
    const int base = (int)P.ht.size();
    P.qfirst[q] = base;
    for (int t = 0; t < g.n_tables; ++t) {
      const gj_table& tb = tables[q_off[q] + t];
      HTable h;
      h.n = tb.n_rows;
      h.k = tb.n_keys;
      for (int c = 0; c < h.k; ++c) h.cols[c] = tb.n_rows > 0 ? tb.keys[c] : nullptr;
      h.parent = t == 0 ? -1 : base + g.parent[t];
      h.sep = t == 0 ? 0 : g.sep_col[t];
      h.pcol = t == 0 ? 0 : g.parent_col[t];
      h.query = q;
      h.local = t;
      P.ht.push_back(h);
    }
    for (int t = 1; t < g.n_tables; ++t) P.ht[base + g.parent[t]].children.push_back(base + t);
  }
  P.qfirst[nq] = (int)P.ht.size();
  P.nt = (int)P.ht.size();
  P.max_depth = 0;
  P.max_height = 0;
  for (int t = 0; t < P.nt; ++t) {
    HTable& h = P.ht[t];
    h.depth = h.parent < 0 ? 0 : P.ht[h.parent].depth + 1;
    P.max_depth = std::max(P.max_depth, h.depth);
  }
  for (int t = P.nt - 1; t >= 0; --t) {
    HTable& h = P.ht[t];
    h.height = 0;
    for (int ch : h.children) h.height = std::max(h.height, P.ht[ch].height + 1);
    P.max_height = std::max(P.max_height, h.height);
  }
  return GJ_OK;
}

static void fill_desc_static(Plan& P) {
  P.td.assign(P.nt, TDesc{});
  int64_t off = 0, koff = 0, loff = 0, aoff = 0;
  for (int t = 0; t < P.nt; ++t) {
    const HTable& h = P.ht[t];
    TDesc& d = P.td[t];
    for (int c = 0; c < h.k; ++c) d.col[c] = h.cols[c];
    d.n = h.n;
    d.k = h.k;
    d.off = off;
    off = align_up(off + std::max<int64_t>(h.n, 1), 64);
    d.key_off = koff;
    koff = align_up(koff + (int64_t)h.k * std::max<int64_t>(h.n, 1), 64);
    d.sep = h.sep;
    d.parent = h.parent;
    d.pcol = h.pcol;
    d.is_root = h.parent < 0;
    d.query = h.query;
    d.depth = h.depth;
    d.height = h.height;
    d.nchild = (int)h.children.size();
    for (int i = 0; i < d.nchild; ++i) {
      d.child[i] = h.children[i];
      d.child_col[i] = P.ht[h.children[i]].pcol;
    }
    d.ntiles = (int32_t)((h.n + GJ_TILE - 1) / GJ_TILE);
    d.agg_off = aoff;
    aoff += std::max(d.ntiles, 1);
  }
  // link regions: table t >= 1 gets one slot per entry of its parent; its
  // bucket counts one row of parent tiles per bucket
  int64_t hoff = 0;
  for (int t = 0; t < P.nt; ++t) {
    TDesc& d = P.td[t];
    if (d.parent >= 0) {
      d.link_off = loff;
      const int64_t np = P.ht[d.parent].n;
      loff = align_up(loff + std::max<int64_t>(np, 1), 64);
      const int64_t nc = P.ht[t].n;
      d.dbucketed = nc <= DOWN_MAX_GROUPS && np >= (int64_t)DOWN_PARENT_RATIO * std::max<int64_t>(nc, 1);
      const int64_t pt = std::max(P.td[d.parent].ntiles, 1);
      d.dhist_off = hoff;
      if (d.dbucketed) hoff += (int64_t)(DOWN_BUCKETS + 1) * pt;
      // reduce blocks take a bucket over up to 2048 parent tiles (about 8 ranges
      // of tiles for the largest parents)
      d.dslice = (int32_t)std::min<int64_t>(2048, std::max<int64_t>(GJ_BLOCK, (pt + 7) / 8));
    }
  }
  P.dhist_slots = std::max<int64_t>(hoff, 64);
  P.S = std::max<int64_t>(off, 64);
  P.key_slots = std::max<int64_t>(koff, 64);
  P.link_slots = std::max<int64_t>(loff, 64);
  P.agg_slots = std::max<int64_t>(aoff, 64);
}

// Sort-word layout of table t from its column ranges: fields in entry order
// (separator first for non-root tables), most significant first, above
// ceil(log2 n) row-id bits.
static gj_status pack_layout(Plan& P, int t, const int32_t* mm) {
  const HTable& h = P.ht[t];
  TDesc& d = P.td[t];
  std::vector<int> order;
  if (h.parent >= 0) order.push_back(h.sep);
  for (int c = 0; c < h.k; ++c)
    if (h.parent < 0 || c != h.sep) order.push_back(c);
  int bits[MAXK] = {};
  int total = 0;
  for (int c = 0; c < h.k; ++c) {
    if (h.n == 0) {
      d.kmin[c] = 0;
      bits[c] = 0;
      continue;
    }
    int32_t lo = mm[(t * MAXK + c) * 2], hi = mm[(t * MAXK + c) * 2 + 1];
    d.kmin[c] = (uint32_t)lo;
    bits[c] = bitwidth32((uint32_t)hi - (uint32_t)lo);
    total += bits[c];
  }
  int pos = total;
  for (int c : order) {
    pos -= bits[c];
    d.fshift[c] = pos;
    d.fbits[c] = bits[c];
  }
  d.keybits = total;
  d.rb = h.n <= 1 ? 0 : bitwidth64((uint64_t)(h.n - 1));
  d.sepshift = h.parent >= 0 ? d.fshift[h.sep] : total;
  const int width = d.rb + d.keybits;
  if (width > 128) {
    set_error("table %d: %d key bits + %d row-id bits do not fit a 128-bit sort word", t, d.keybits, d.rb);
    return GJ_E_INVALID;
  }
  d.wide = width > 64;
  const int rbits = std::max(1, std::min(8, P.radix_bits));
  d.npasses = total == 0 ? 0 : (total + rbits - 1) / rbits;
  d.dbits = d.npasses == 0 ? 1 : (total + d.npasses - 1) / d.npasses;
  d.sort_tile = GJ_BLOCK * P.sort_items[d.wide];
  d.ntiles_sort = (int32_t)((h.n + d.sort_tile - 1) / d.sort_tile);
  d.final_buf = d.npasses & 1;
  d.sh0 = d.rb;
  d.npasses_full = d.npasses;
  d.local = 0;
  // Large 128-bit-word tables: global passes over the top two digits only
  // (buckets of about n / 2^(2 dbits) rows when the keys spread), then every
  // bucket sorted in LDS (sort_local.hip) into words[1].  A block takes
  // buckets of up to 1216 rows wherever they start: tables whose buckets
  // would average over 1000 rows keep the per-digit passes.
  if (P.local_rows > 0 && d.wide && h.n >= P.local_rows && d.npasses >= 3 &&
      h.n <= ((int64_t)1000 << (2 * d.dbits))) {
    d.local = 1;
    d.sh0 = d.rb + d.keybits - 2 * d.dbits;
    d.npasses = 2;
    d.final_buf = 1;
  }
  return GJ_OK;
}

// Tables whose key fields and row ids exceed a 128-bit sort word: their
// widest columns are replaced by each row's rank among the column's distinct
// values (ascending, so the order of key tuples is kept), found by the same
// group-by run on that one column, until the key fits; the run writer maps
// ranks back to values.  mm is updated to the ranks' range.
static gj_status compress_wide_columns(Plan& P, Arena& A, std::vector<int32_t>& mm) {
  hipStream_t s = P.ctx->stream;
  for (int t = 0; t < P.nt; ++t) {
    HTable& h = P.ht[t];
    TDesc& d = P.td[t];
    for (int c = 0; c < MAXK; ++c) d.vmap[c] = nullptr;
    if (h.n <= 1) continue;
    const int rb = bitwidth64((uint64_t)(h.n - 1));
    int bits[MAXK] = {};
    int total = 0;
    for (int c = 0; c < h.k; ++c) {
      bits[c] = bitwidth32((uint32_t)mm[(t * MAXK + c) * 2 + 1] - (uint32_t)mm[(t * MAXK + c) * 2]);
      total += bits[c];
    }
    if (rb + total <= 128) continue;
    std::vector<int> order(h.k), pick;
    for (int c = 0; c < h.k; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return bits[a] > bits[b]; });
    for (int c : order) {
      if (rb + total <= 128) break;
      if (bits[c] > rb) {  // a rank is below n, so it needs at most rb bits
        total -= bits[c] - rb;
        pick.push_back(c);
      }
    }
    if (rb + total > 128) continue;  // pack_layout refuses the table
    for (int c : pick) {
      gj_factors sub(P.ctx);
      sub.plan.ctx = P.ctx;
      const int32_t* col = h.cols[c];
      const gj_table tab{h.n, 1, &col};
      const int32_t zero = 0, none = -1;
      const gj_join_graph g{1, &none, &zero, &zero};
      const int qoff[2] = {0, 1};
      gj_status st;
      if ((st = plan_tables(sub.plan, 1, qoff, &tab, &g)) || (st = plan_device(sub.plan, sub.arena, sub.F))) return st;
      launch_factors(sub.plan, sub.F, s);
      std::vector<int64_t> cnt;
      if ((st = read_counters(sub.plan, sub.F, s, cnt))) return st;
      const int64_t M = cnt[CNT_M];
      int32_t* rank = A.get_n<int32_t>(h.n);
      int32_t* vals = A.get_n<int32_t>(M);
      if (!rank || !vals) return GJ_E_OOM;
      const TDesc& sd = sub.plan.td[0];
      if ((st = check(hipMemcpyAsync(vals, sub.F.ekey + sd.key_off, (size_t)M * 4, hipMemcpyDeviceToDevice, s),
                      "column ranks")))
        return st;
      gjk::rank_rows(s, sub.F.perm + sd.off, sub.F.estart + sd.off, M, h.n, rank);
      if ((st = check(hipGetLastError(), "column ranks")) || (st = check(hipStreamSynchronize(s), "column ranks")))
        return st;
      h.cols[c] = rank;
      d.col[c] = rank;
      d.vmap[c] = vals;
      mm[(t * MAXK + c) * 2] = 0;
      mm[(t * MAXK + c) * 2 + 1] = (int32_t)(M - 1);
    }
  }
  return GJ_OK;
}

gj_status plan_device(Plan& P, Arena& A, FPtrs& F) {
  gj_ctx* ctx = P.ctx;
  hipStream_t s = ctx->stream;
  P.radix_bits = ctx->tune.radix_bits;
  P.local_rows = P.allow_local ? ctx->tune.sort_local_rows : 0;
  P.sort_items[0] = ctx->tune.sort_items == 8 ? 8 : 16;
  P.sort_items[1] = 8;  // 128-bit words: 8 per thread (measured best of 4, 8, 16)
  fill_desc_static(P);
  std::vector<int> all;
  for (int t = 0; t < P.nt; ++t) all.push_back(t);
  P.wl_host.clear();
  P.tabs_host.clear();
  P.all = P.add_list(all, GJ_TILE, false);
  // key ranges (one synchronization)
  int32_t* d_mm = A.get_n<int32_t>((int64_t)P.nt * MAXK * 2);
  int32_t* d_mmt = A.get_n<int32_t>(P.agg_slots * MAXK * 2);
  TDesc* d_desc = A.get_n<TDesc>(P.nt);
  WorkItem* d_wl0 = A.get_n<WorkItem>(std::max(1, P.all.n));
  int32_t* d_tabs0 = A.get_n<int32_t>(std::max(1, P.all.tn));
  if (!d_mm || !d_mmt || !d_desc || !d_wl0 || !d_tabs0) return GJ_E_OOM;
  gj_status st;
  if ((st = check(hipMemcpyAsync(d_desc, P.td.data(), sizeof(TDesc) * P.nt, hipMemcpyHostToDevice, s), "upload")))
    return st;
  if ((st = check(hipMemcpyAsync(d_wl0, P.wl_host.data(), sizeof(WorkItem) * std::max(1, P.all.n),
                                 hipMemcpyHostToDevice, s),
                  "upload")))
    return st;
  if ((st = check(hipMemcpyAsync(d_tabs0, P.tabs_host.data(), sizeof(int32_t) * std::max(1, P.all.tn),
                                 hipMemcpyHostToDevice, s),
                  "upload")))
    return st;
  gjk::fill_i32(s, d_mm, (int64_t)P.nt * MAXK * 2, INT32_MAX, INT32_MIN);
  gjk::minmax(s, d_wl0, P.all.n, d_tabs0, P.all.tn, d_desc, d_mmt, d_mm);
  std::vector<int32_t> mm((size_t)P.nt * MAXK * 2);
  if ((st = check(hipMemcpyAsync(mm.data(), d_mm, mm.size() * 4, hipMemcpyDeviceToHost, s), "key ranges"))) return st;
  if ((st = check(hipStreamSynchronize(s), "key ranges"))) return st;
  const std::vector<int32_t> mm_values = mm;  // the columns' own ranges (separator indexes use them)
  if ((st = compress_wide_columns(P, A, mm))) return st;
  // layout of the sort words
  int64_t woff = 0, hoff = 0;
  P.max_passes = 0;
  for (int t = 0; t < P.nt; ++t) {
    if ((st = pack_layout(P, t, mm.data()))) return st;
    TDesc& d = P.td[t];
    d.word_off = woff;
    woff = align_up(woff + std::max<int64_t>(d.n, 1) * (d.wide ? 2 : 1), 32);
    d.hist_off = hoff;
    hoff += (int64_t)(1 << d.dbits) * std::max(d.ntiles_sort, 1);
    P.max_passes = std::max(P.max_passes, d.npasses);
  }
  P.word_units = std::max<int64_t>(woff, 64);
  P.hist_slots = std::max<int64_t>(hoff, 64);
  // dense separator indexes: a direct value -> group table where the
  // separator's value range is at most a few times the table's rows
  P.didx_slots = 0;
  for (int t = 0; t < P.nt; ++t) {
    TDesc& d = P.td[t];
    d.didx_off = -1;
    d.drange = 0;
    d.dmin = 0;
    if (d.parent < 0 || d.n == 0) continue;
    const int32_t lo = mm_values[(t * MAXK + d.sep) * 2], hi = mm_values[(t * MAXK + d.sep) * 2 + 1];
    const int64_t range = (int64_t)hi - (int64_t)lo + 1;
    if (range > 0 && range <= 4 * d.n + 4096 && range <= (1LL << 30)) {
      d.didx_off = P.didx_slots;
      d.drange = range;
      d.dmin = lo;
      P.didx_slots += range;
    }
  }
  // work lists
  P.wl_host.clear();
  P.tabs_host.clear();
  P.all = P.add_list(all, GJ_TILE, false);
  for (int w = 0; w < 2; ++w) {
    std::vector<int> tw;
    for (int t = 0; t < P.nt; ++t)
      if (P.td[t].wide == w) tw.push_back(t);
    P.allw[w] = P.add_list(tw, GJ_TILE, false);
    P.sort[w].clear();
    for (int p = 0; p < P.max_passes; ++p) {
      std::vector<int> tp;
      for (int t : tw)
        if (P.td[t].npasses > p) tp.push_back(t);
      P.sort[w].push_back(P.add_list(tp, 0, true));
    }
  }
  {
    std::vector<int> lt;
    for (int t = 0; t < P.nt; ++t)
      if (P.td[t].local) lt.push_back(t);
    P.local = P.add_list(lt, GJ_LOCAL_TILE, false);
    P.local_full.clear();
    for (int t : lt) P.local_full.push_back(P.add_list({t}, 0, true));
    P.sort_kind.assign(P.nt, 0);
    for (int t : lt) P.sort_kind[t] = 1;
  }
  P.up.clear();
  for (int h = 0; h <= P.max_height; ++h) {
    std::vector<int> th;
    for (int t = 0; t < P.nt; ++t)
      if (P.ht[t].height == h) th.push_back(t);
    P.up.push_back(P.add_list(th, GJ_TILE, false));
  }
  P.down.assign(1, WL{});
  for (int dd = 1; dd <= P.max_depth; ++dd) {
    std::vector<int> tp;
    for (int t = 0; t < P.nt; ++t)
      if (P.ht[t].depth == dd - 1 && !P.ht[t].children.empty()) tp.push_back(t);
    P.down.push_back(P.add_list(tp, GJ_TILE, false));
  }
  // bucket sums of each level: items (child, x) for every bucket of the
  // child and every range of dslice parent tiles
  P.dred.assign(1, WL{});
  P.dfall.assign(1, 0);
  P.dbuck.assign(1, 0);
  for (int dd = 1; dd <= P.max_depth; ++dd) {
    WL l;
    l.off = (int)P.wl_host.size();
    l.toff = (int)P.tabs_host.size();
    char fall = 0, buck = 0;
    for (int t = 0; t < P.nt; ++t) {
      if (P.ht[t].depth != dd) continue;
      const TDesc& d = P.td[t];
      const int64_t ns =
          d.dbucketed ? (int64_t)DOWN_BUCKETS * ((std::max(P.td[d.parent].ntiles, 1) + d.dslice - 1) / d.dslice) : 0;
      for (int64_t i = 0; i < ns; ++i) P.wl_host.push_back(WorkItem{t, (int32_t)i});
      P.tabs_host.push_back(t);
      if (d.dbucketed)
        buck = 1;
      else
        fall = 1;
    }
    l.n = (int)P.wl_host.size() - l.off;
    l.tn = (int)P.tabs_host.size() - l.toff;
    P.dred.push_back(l);
    P.dfall.push_back(fall);
    P.dbuck.push_back(buck);
  }
  // factor buffers
  F.words[0] = A.get_n<uint64_t>(P.word_units);
  F.words[1] = A.get_n<uint64_t>(P.word_units);
  F.perm = A.get_n<int32_t>(P.S);
  F.ekey = A.get_n<int32_t>(P.key_slots);
  F.estart = A.get_n<int32_t>(P.S);
  F.eend = A.get_n<int32_t>(P.S);
  F.egrp = A.get_n<int32_t>(P.S);
  F.gval = A.get_n<int32_t>(P.S);
  F.glo = A.get_n<int32_t>(P.S);
  F.ghi = A.get_n<int32_t>(P.S);
  F.cnt = A.get_n<int64_t>((int64_t)P.nt * CNT_STRIDE);
  F.hist = A.get_n<uint32_t>(P.hist_slots);
  F.dtot = A.get_n<uint32_t>((int64_t)P.nt * 256);
  F.mm = d_mm;
  F.agg = A.get_n<uint64_t>(P.agg_slots);
  F.agg2 = A.get_n<uint64_t>(P.agg_slots);
  F.didx = A.get_n<int32_t>(P.didx_slots);
  F.lflag = A.get_n<int32_t>(P.nt);
  P.d_wl = A.get_n<WorkItem>(std::max<int64_t>((int64_t)P.wl_host.size(), 1));
  P.d_tabs = A.get_n<int32_t>(std::max<int64_t>((int64_t)P.tabs_host.size(), 1));
  P.d_desc = d_desc;
  if (!F.words[0] || !F.words[1] || !F.perm || !F.ekey || !F.estart || !F.eend || !F.egrp || !F.gval || !F.glo ||
      !F.ghi || !F.cnt || !F.hist || !F.dtot || !F.agg || !F.agg2 || !F.didx || !F.lflag || !P.d_wl || !P.d_tabs)
    return GJ_E_OOM;
  if ((st = check(hipMemcpyAsync(d_desc, P.td.data(), sizeof(TDesc) * P.nt, hipMemcpyHostToDevice, s), "upload")))
    return st;
  if (!P.wl_host.empty() &&
      (st = check(hipMemcpyAsync(P.d_wl, P.wl_host.data(), sizeof(WorkItem) * P.wl_host.size(),
                                 hipMemcpyHostToDevice, s),
                  "upload")))
    return st;
  if (!P.tabs_host.empty() &&
      (st = check(hipMemcpyAsync(P.d_tabs, P.tabs_host.data(), sizeof(int32_t) * P.tabs_host.size(),
                                 hipMemcpyHostToDevice, s),
                  "upload")))
    return st;
  // the host copies of the lists must outlive the asynchronous uploads
  return check(hipStreamSynchronize(s), "upload");
}

// Pack and sort the words of every table (the radix passes; for tables with
// `local` set, the top-digit passes and the in-LDS bucket sort).
static void launch_sort(const Plan& P, const FPtrs& F, hipStream_t s) {
  for (int w = 0; w < 2; ++w) gjk::pack(s, w, P.d_wl + P.allw[w].off, P.allw[w].n, P.d_desc, F);
  for (int p = 0; p < P.max_passes; ++p)
    for (int w = 0; w < 2; ++w) {
      const WL& l = P.sort[w][p];
      // the pack counted the first pass's digits
      gjk::radix_pass(s, w, P.sort_items[w], P.d_wl + l.off, l.n, P.d_tabs + l.toff, l.tn, P.d_desc, F, p, p > 0);
    }
  if (P.local.n > 0) {
    gjk::fill_i32(s, F.lflag, P.nt, 0, 0);
    gjk::local_sort(s, P.d_wl + P.local.off, P.local.n, P.d_desc, F);
  }
}

// Tables whose in-LDS bucket sort met a bucket longer than a block holds
// (heavily repeated top bits): sorted again in full by the plain passes,
// which take the bucket order (words[0]) as their input.  Waits for the host.
static gj_status local_fallback(Plan& P, const FPtrs& F, hipStream_t s) {
  std::vector<int32_t> fl(P.nt, 0);
  gj_status st;
  if ((st = check(hipMemcpyAsync(fl.data(), F.lflag, sizeof(int32_t) * P.nt, hipMemcpyDeviceToHost, s),
                  "bucket sort")) ||
      (st = check(hipStreamSynchronize(s), "bucket sort")))
    return st;
  int k = 0;
  for (int t = 0; t < P.nt; ++t) {
    TDesc& d = P.td[t];
    if (!d.local) continue;
    const WL& l = P.local_full[k++];
    if (!fl[t]) continue;
    d.local = 0;
    P.sort_kind[t] = 2;
    d.sh0 = d.rb;
    d.npasses = d.npasses_full;
    d.final_buf = d.npasses & 1;
    if ((st = check(hipMemcpyAsync(P.d_desc + t, &d, sizeof(TDesc), hipMemcpyHostToDevice, s), "upload"))) return st;
    for (int p = 0; p < d.npasses; ++p)
      gjk::radix_pass(s, 1, P.sort_items[1], P.d_wl + l.off, l.n, P.d_tabs + l.toff, l.tn, P.d_desc, F, p);
  }
  return check(hipGetLastError(), "bucket sort");
}

// Entries and groups from the sorted words.
static void launch_runs(const Plan& P, const FPtrs& F, hipStream_t s) {
  for (int w = 0; w < 2; ++w)
    gjk::runs(s, w, P.d_wl + P.allw[w].off, P.allw[w].n, nullptr, 0, P.d_desc, F);
  gjk::runs_scan(s, P.d_tabs + P.all.toff, P.all.tn, P.d_desc, F);
  for (int w = 0; w < 2; ++w) gjk::runs_write(s, w, P.d_wl + P.allw[w].off, P.allw[w].n, P.d_desc, F);
  if (P.didx_slots > 0) {
    gjk::fill_i32(s, F.didx, P.didx_slots, -1, -1);
    gjk::group_index(s, P.d_wl + P.all.off, P.all.n, P.d_desc, F);
  }
}

void launch_factors(const Plan& P, const FPtrs& F, hipStream_t s) {
  launch_sort(P, F, s);
  launch_runs(P, F, s);
}

gj_status alloc_summary(const Plan& P, Arena& A, SPtrs& S) {
  S.U = A.get_n<int64_t>(P.S);
  S.pre = A.get_n<int64_t>(P.S);
  S.Mg = A.get_n<int64_t>(P.S);
  S.Dg = A.get_n<int64_t>(P.S);
  S.link = A.get_n<int32_t>(P.link_slots);
  S.e2c = A.get_n<int32_t>(P.S);
  S.g2c = A.get_n<int32_t>(P.S);
  S.ckey = A.get_n<int32_t>(P.key_slots);
  S.cc = A.get_n<int64_t>(P.S);
  S.cU = A.get_n<int64_t>(P.S);
  S.cD = A.get_n<int64_t>(P.S);
  S.cF = A.get_n<int64_t>(P.S);
  S.cpre = A.get_n<int64_t>(P.S);
  S.cstart = A.get_n<int32_t>(P.S);
  S.cgval = A.get_n<int32_t>(P.S);
  S.cgM = A.get_n<int64_t>(P.S);
  S.cgD = A.get_n<int64_t>(P.S);
  S.ccs = A.get_n<int2>(P.S);
  S.crec = A.get_n<ChildRec>(P.link_slots);
  S.grec = A.get_n<ChildRec>(P.S);
  S.xprod = A.get_n<int64_t>(P.link_slots);
  S.dkey = A.get_n<int32_t>(P.link_slots);
  S.dval = A.get_n<int64_t>(P.link_slots);
  S.dhist = A.get_n<uint32_t>(P.dhist_slots);
  S.qsize = A.get_n<int64_t>(P.nq);
  S.qstatus = A.get_n<int32_t>(P.nq);
  void* all[] = {S.U,  S.pre,    S.Mg,    S.Dg,  S.link, S.e2c,  S.g2c,  S.ckey,  S.cc,    S.cU,   S.cD,
                 S.cF, S.cpre,   S.cstart, S.cgval, S.cgM, S.cgD,  S.qsize, S.qstatus, S.ccs, S.crec, S.grec,
                 S.xprod, S.dkey, S.dval, S.dhist};
  for (void* p : all)
    if (!p) return GJ_E_OOM;
  return GJ_OK;
}

void launch_summary(const Plan& P, const FPtrs& F, const SPtrs& S, hipStream_t s) {
  gjk::fill_i64(s, S.qsize, P.nq, 0);
  gjk::fill_i32(s, S.qstatus, P.nq, GJ_OK, GJ_OK);
  for (int h = 0; h <= P.max_height; ++h) {
    const WL& l = P.up[h];
    gjk::up_pass(s, P.d_wl + l.off, l.n, P.d_tabs + l.toff, l.tn, P.d_desc, F, S);
  }
  gjk::fill_i64(s, S.Dg, P.S, 0);
  for (int dd = 1; dd <= P.max_depth; ++dd) {
    const WL& l = P.down[dd];
    const WL& r = P.dred[dd];
    gjk::down_pass(s, P.d_wl + l.off, l.n, P.d_wl + r.off, r.n, P.dbuck[dd] != 0, P.dfall[dd] != 0, P.d_desc, F,
                   S);
  }
  gjk::compact(s, P.d_wl + P.all.off, P.all.n, P.d_tabs + P.all.toff, P.all.tn, P.d_desc, F, S);
}

gj_status read_counters(const Plan& P, const FPtrs& F, hipStream_t s, std::vector<int64_t>& out) {
  out.assign((size_t)P.nt * CNT_STRIDE, 0);
  gj_status st = check(hipMemcpyAsync(out.data(), F.cnt, out.size() * 8, hipMemcpyDeviceToHost, s), "counters");
  if (st) return st;
  return check(hipStreamSynchronize(s), "counters");
}

gj_status summary_host(const gj_summary* sc) {
  gj_summary* s = const_cast<gj_summary*>(sc);
  if (s->host_stale) {
    hipStream_t hs = s->ctx->stream;
    int64_t q = 0;
    int32_t qs = 0;
    gj_status st;
    if ((st = check(hipMemcpyAsync(&q, s->S.qsize + s->query, 8, hipMemcpyDeviceToHost, hs), "join size")) ||
        (st = check(hipMemcpyAsync(&qs, s->S.qstatus + s->query, 4, hipMemcpyDeviceToHost, hs), "join size")) ||
        (st = read_counters(s->f->plan, s->f->F, hs, s->cnt_host)))
      return st;
    s->join_size = q;
    s->status = qs;
    s->host_stale = false;
  }
  if (s->status == GJ_E_OVERFLOW) {
    set_error("join size does not fit below 2^63-1");
    return GJ_E_OVERFLOW;
  }
  return GJ_OK;
}

}  // namespace gjh

using namespace gjh;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* gj_last_error(const gj_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

gj_status gj_ctx_create(int device, void* hip_stream, gj_alloc_fn alloc, gj_free_fn free_fn, void* user,
                        gj_ctx** out) {
  if (!out || ((alloc == nullptr) != (free_fn == nullptr))) {
    set_error("gj_ctx_create: need an output pointer and both or neither allocator callbacks");
    return GJ_E_INVALID;
  }
  gj_status st = check(hipSetDevice(device), "hipSetDevice");
  if (st) return st;
  gj_ctx* c = new gj_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  c->tune.sort_items = 8;
  c->tune.radix_bits = 8;
  c->tune.desum_rounds = 0;
  c->tune.desum_stage = 4;
  c->tune.batch_task_rows = 0;
  c->tune.desum_general = 0;
  c->tune.sort_local_rows = 1 << 20;
  *out = c;
  return GJ_OK;
}

void gj_ctx_destroy(gj_ctx* ctx) { delete ctx; }

gj_status gj_ctx_set_tune(gj_ctx* ctx, const gj_tune* tune) {
  GJ_SCOPE(ctx);
  if (!ctx || !tune) {
    set_error("gj_ctx_set_tune: null argument");
    return GJ_E_INVALID;
  }
  const int stg = tune->desum_stage;
  const int btr = tune->batch_task_rows;
  if ((tune->sort_items != 8 && tune->sort_items != 16) || tune->radix_bits < 4 || tune->radix_bits > 8 ||
      tune->desum_rounds < 0 || tune->desum_rounds > 1024 || !(stg == 2 || stg == 4 || stg == 8) ||
      !(btr == 0 || (btr >= 256 && btr <= (1 << 24))) || (tune->desum_general != 0 && tune->desum_general != 1) ||
      tune->sort_local_rows < 0) {
    set_error("gj_ctx_set_tune: sort_items in {8,16}, radix_bits in [4,8], desum_rounds in [0,1024], "
              "desum_stage in {2,4,8}, batch_task_rows 0 or in [256, 2^24], desum_general 0 or 1, "
              "sort_local_rows >= 0");
    return GJ_E_INVALID;
  }
  ctx->tune = *tune;
  return GJ_OK;
}

gj_status gj_validate(const gj_table* tables, const gj_join_graph* graph) { return validate_one(tables, graph); }

gj_status gj_build_factors(gj_ctx* ctx, const gj_table* tables, const gj_join_graph* graph, gj_factors** out) {
  GJ_SCOPE(ctx);
  if (!ctx || !out) {
    set_error("gj_build_factors: null argument");
    return GJ_E_INVALID;
  }
  gj_status st = validate_one(tables, graph);
  if (st) return st;
  gj_factors* f = new gj_factors(ctx);
  f->plan.ctx = ctx;
  f->plan.allow_local = true;
  int qoff[2] = {0, graph->n_tables};
  if ((st = plan_tables(f->plan, 1, qoff, tables, graph)) || (st = plan_device(f->plan, f->arena, f->F))) {
    delete f;
    return st;
  }
  launch_sort(f->plan, f->F, ctx->stream);
  if (f->plan.local.n > 0 && (st = local_fallback(f->plan, f->F, ctx->stream))) {
    delete f;
    return st;
  }
  launch_runs(f->plan, f->F, ctx->stream);
  if ((st = check(hipGetLastError(), "factor kernels"))) {
    delete f;
    return st;
  }
  *out = f;
  return GJ_OK;
}

gj_status gj_factor_sort(const gj_factors* f, int32_t t, int32_t* kind) {
  GJ_SCOPE(f ? f->ctx : nullptr);
  if (!f || !kind || t < 0 || t >= f->plan.nt || (int)f->plan.sort_kind.size() != f->plan.nt) {
    set_error("gj_factor_sort: bad argument");
    return GJ_E_INVALID;
  }
  *kind = f->plan.sort_kind[t];
  return GJ_OK;
}

static gj_status ensure_counters(const gj_factors* f) {
  gj_factors* m = const_cast<gj_factors*>(f);
  if (!m->cnt_host.empty()) return GJ_OK;
  return read_counters(m->plan, m->F, m->ctx->stream, m->cnt_host);
}

gj_status gj_factor_table(const gj_factors* f, int32_t t, gj_factor_view* v) {
  GJ_SCOPE(f ? f->ctx : nullptr);
  if (!f || !v || t < 0 || t >= f->plan.nt) {
    set_error("gj_factor_table: bad argument");
    return GJ_E_INVALID;
  }
  gj_status st = ensure_counters(f);
  if (st) return st;
  if (!f->ecount) {
    gj_factors* m = const_cast<gj_factors*>(f);
    int64_t* ec = m->arena.get_n<int64_t>(m->plan.S);
    if (!ec) return GJ_E_OOM;
    gjk::entry_counts(m->ctx->stream, m->plan.d_wl + m->plan.all.off, m->plan.all.n, m->plan.d_desc, m->F, ec);
    if ((st = check(hipGetLastError(), "entry counts"))) return st;
    m->ecount = ec;
  }
  const TDesc& d = f->plan.td[t];
  gj_factor_view r{};
  r.n_entries = f->cnt_host[t * CNT_STRIDE + CNT_M];
  r.count = f->ecount + d.off;
  r.n_rows = d.n;
  r.n_keys = d.k;
  for (int c = 0; c < d.k; ++c) r.keys[c] = f->F.ekey + d.key_off + (int64_t)c * d.n;
  r.start = f->F.estart + d.off;
  r.end = f->F.eend + d.off;
  r.perm = f->F.perm + d.off;
  *v = r;
  return GJ_OK;
}

void gj_free_factors(gj_factors* f) {
  if (!f) return;
  if (--f->refs == 0) delete f;
}

gj_status gj_summarize(gj_ctx* ctx, const gj_factors* fc, gj_summary** out, int64_t* join_size) {
  GJ_SCOPE(ctx);
  if (!ctx || !fc || !out) {
    set_error("gj_summarize: null argument");
    return GJ_E_INVALID;
  }
  gj_factors* f = const_cast<gj_factors*>(fc);
  gj_summary* s = new gj_summary(ctx);
  s->f = f;
  f->refs++;
  gj_status st = alloc_summary(f->plan, s->arena, s->S);
  if (st) {
    gj_free_summary(s);
    return st;
  }
  launch_summary(f->plan, f->F, s->S, ctx->stream);
  if ((st = check(hipGetLastError(), "summary kernels"))) {
    gj_free_summary(s);
    return st;
  }
  int64_t q = 0;
  int32_t qs = 0;
  hipStream_t hs = ctx->stream;
  if ((st = check(hipMemcpyAsync(&q, s->S.qsize, 8, hipMemcpyDeviceToHost, hs), "join size")) ||
      (st = check(hipMemcpyAsync(&qs, s->S.qstatus, 4, hipMemcpyDeviceToHost, hs), "join size")) ||
      (st = read_counters(f->plan, f->F, hs, s->cnt_host))) {
    gj_free_summary(s);
    return st;
  }
  if (f->cnt_host.empty()) f->cnt_host = s->cnt_host;
  if (qs == GJ_E_OVERFLOW) {
    set_error("join size does not fit below 2^63-1");
    gj_free_summary(s);
    return GJ_E_OVERFLOW;
  }
  s->join_size = q;
  if (join_size) *join_size = q;
  *out = s;
  return GJ_OK;
}

gj_status gj_summarize_batch(gj_ctx* ctx, const gj_factors* const* factors, int32_t n_queries, gj_summary** outs,
                             int64_t* d_join_sizes, int32_t* d_status) {
  GJ_SCOPE(ctx);
  if (!ctx || n_queries < 0 || (n_queries > 0 && (!factors || !outs || !d_join_sizes || !d_status))) {
    set_error("gj_summarize_batch: bad argument");
    return GJ_E_INVALID;
  }
  // validate everything before launching anything
  for (int32_t i = 0; i < n_queries; ++i) {
    const gj_factors* f = factors[i];
    if (!f || f->ctx != ctx || f->plan.nq != 1) {
      set_error("gj_summarize_batch: factors %d are null, from another context, or not one query's", i);
      return GJ_E_INVALID;
    }
    for (int32_t j = 0; j < i; ++j)
      if (factors[j] == f) {
        set_error("gj_summarize_batch: factors %d and %d are the same set", j, i);
        return GJ_E_INVALID;
      }
    const gj_summary* o = outs[i];
    if (o && (o->f != f || o->borrowed || o->projected || o->query != 0)) {
      set_error("gj_summarize_batch: summary %d was not made for factors %d", i, i);
      return GJ_E_INVALID;
    }
  }
  // summaries to allocate (only when the caller passed none)
  std::vector<gj_summary*> fresh(n_queries, nullptr);
  for (int32_t i = 0; i < n_queries; ++i) {
    if (outs[i]) continue;
    gj_factors* f = const_cast<gj_factors*>(factors[i]);
    gj_summary* s = new gj_summary(ctx);
    s->f = f;
    f->refs++;
    fresh[i] = s;
    if (gj_status st = alloc_summary(f->plan, s->arena, s->S)) {
      for (gj_summary* x : fresh) gj_free_summary(x);
      return st;
    }
  }
  hipStream_t hs = ctx->stream;
  for (int32_t i = 0; i < n_queries; ++i) {
    gj_summary* s = outs[i] ? outs[i] : fresh[i];
    launch_summary(s->f->plan, s->f->F, s->S, hs);
    gjk::export_status(hs, s->S.qsize, s->S.qstatus, d_join_sizes + i, d_status + i);
    s->host_stale = true;
  }
  if (gj_status st = check(hipGetLastError(), "summary kernels")) {
    for (gj_summary* x : fresh) gj_free_summary(x);
    return st;
  }
  for (int32_t i = 0; i < n_queries; ++i)
    if (fresh[i]) outs[i] = fresh[i];
  return GJ_OK;
}

static const TDesc* summary_table_desc(const gj_summary* s, int32_t t) {
  const Plan& P = s->f->plan;
  int base = P.qfirst[s->query];
  int n = P.qfirst[s->query + 1] - base;
  if (t < 0 || t >= n) return nullptr;
  return &P.td[base + t];
}

gj_status gj_summary_table(const gj_summary* s, int32_t t, gj_summary_view* v) {
  GJ_SCOPE(s ? s->ctx : nullptr);
  const TDesc* d = s && v ? summary_table_desc(s, t) : nullptr;
  if (!d) {
    set_error("gj_summary_table: bad argument");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  const int gt = (int)(d - s->f->plan.td.data());
  gj_summary_view r{};
  r.n_entries = s->cnt_host[gt * CNT_STRIDE + CNT_MC];
  r.n_keys = d->k;
  for (int c = 0; c < d->k; ++c) r.keys[c] = s->S.ckey + d->key_off + (int64_t)c * d->n;
  r.c = s->S.cc + d->off;
  r.U = s->S.cU + d->off;
  r.D = s->S.cD + d->off;
  r.F = s->S.cF + d->off;
  r.pre = s->S.cpre + d->off;
  *v = r;
  return GJ_OK;
}

gj_status gj_summary_edge(const gj_summary* s, int32_t t, gj_edge_view* v) {
  GJ_SCOPE(s ? s->ctx : nullptr);
  const TDesc* d = s && v && t >= 1 ? summary_table_desc(s, t) : nullptr;
  if (!d) {
    set_error("gj_summary_edge: bad argument (edges exist for tables >= 1)");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  const int gt = (int)(d - s->f->plan.td.data());
  gj_edge_view r{};
  r.n = s->cnt_host[gt * CNT_STRIDE + CNT_GC];
  r.s = s->S.cgval + d->off;
  r.M = s->S.cgM + d->off;
  r.D = s->S.cgD + d->off;
  *v = r;
  return GJ_OK;
}

gj_status gj_download(gj_ctx* ctx, void* host_dst, const void* dev_src, size_t bytes) {
  GJ_SCOPE(ctx);
  if (!ctx || (bytes && (!host_dst || !dev_src))) {
    set_error("gj_download: null argument");
    return GJ_E_INVALID;
  }
  if (!bytes) return GJ_OK;
  gj_status st = check(hipMemcpyAsync(host_dst, dev_src, bytes, hipMemcpyDeviceToHost, ctx->stream), "download");
  if (st) return st;
  return check(hipStreamSynchronize(ctx->stream), "download");
}

int64_t gj_summary_join_size(const gj_summary* s) {
  if (!s) return -1;
  GJ_SCOPE(s->ctx);
  return summary_host(s) == GJ_OK ? s->join_size : -1;
}

void gj_free_summary(gj_summary* s) {
  if (!s || s->borrowed) return;
  gj_factors* f = s->f;
  delete s;
  gj_free_factors(f);
}

int32_t gj_result_columns(const gj_summary* s) {
  if (!s) return 0;
  if (!s->result_cols.empty()) return (int32_t)s->result_cols.size();
  const Plan& P = s->f->plan;
  int32_t L = 0;
  for (int t = P.qfirst[s->query]; t < P.qfirst[s->query + 1]; ++t) L += P.td[t].is_root ? P.td[t].k : P.td[t].k - 1;
  return L;
}

}  // extern "C"

// Expansion-kernel arguments for rows [first_row, first_row + nw) of summary s.
static void desum_args(const gj_summary* s, int64_t first_row, int64_t nw, void* out, gjk::DesumArgs& a, int& n) {
  const Plan& P = s->f->plan;
  const int base = P.qfirst[s->query];
  n = P.qfirst[s->query + 1] - base;
  for (int t = 0; t < n; ++t) {
    const TDesc& d = P.td[base + t];
    gjk::DTab& T = a.tab[t];
    T.perm = s->f->F.perm + d.off;
    T.cpre = s->S.cpre + d.off;
    T.ccs = s->S.ccs + d.off;
    T.cU = s->S.cU + d.off;
    T.crec = d.parent >= 0 ? s->S.crec + d.link_off : nullptr;
    T.parent = d.parent >= 0 ? d.parent - base : -1;
  }
  a.first = first_row;
  a.n_rows = nw;
  a.n_root = s->cnt_host[base * CNT_STRIDE + CNT_MC];
  a.out = out;
}

// The keyed-lookup expansion applies when every table strictly between the
// root and the innermost one has one surviving entry per surviving group: a
// surviving group has at least one surviving entry (its message is positive
// and the entries' groups survive with it), so equal counts mean exactly one.
static bool unit_expansion(const gj_ctx* ctx, const gj_summary* s) {
  if (ctx->tune.desum_general || s->projected || !s->f->F.perm) return false;
  const Plan& P = s->f->plan;
  const int base = P.qfirst[s->query];
  const int n = P.qfirst[s->query + 1] - base;
  if (n < 2) return false;
  for (int t = 1; t < n - 1; ++t) {
    const int64_t* c = &s->cnt_host[(size_t)(base + t) * CNT_STRIDE];
    if (c[CNT_MC] != c[CNT_GC]) return false;
  }
  return true;
}

// The keyed-lookup expansion of a (row ids, or a.n_cols value columns): the
// root entries' records first when they are small against the output
// (stream-ordered scratch, released on return), else decoded in place.
static int run_unit_expansion(gj_ctx* ctx, const gj_summary* s, const gjk::DesumArgs& a, int n, int rowid_bytes) {
  Arena A(ctx);
  // the innermost table with one entry per group as well: no entry range per record
  const int64_t* ct = &s->cnt_host[(size_t)(s->f->plan.qfirst[s->query] + n - 1) * CNT_STRIDE];
  const bool tl_single = ct[CNT_MC] == ct[CNT_GC];
  const int tuple_bytes = a.n_cols > 0 ? a.n_cols * 4 : n * rowid_bytes;
  int64_t cap = gjk::desum_unit_record_entries(a.n_root, a.n_rows, n, tl_single, a.n_cols, tuple_bytes);
  int64_t* range = nullptr;
  int32_t* rec = nullptr;
  if (cap > 0) {
    range = A.get_n<int64_t>(2);
    rec = range ? reinterpret_cast<int32_t*>(A.get(gjk::desum_unit_record_bytes(cap, n, tl_single, a.n_cols)))
                : nullptr;
    if (!rec) {
      // no room for the records: they are decoded in place (and the failed
      // allocation is not reported as the launch's error)
      (void)hipGetLastError();
      set_error("%s", "");
      range = nullptr;
      cap = 0;
    }
  }
  return gjk::desummarize_unit(ctx->stream, a, rowid_bytes, n, tl_single, range, rec, cap);
}

extern "C" {

gj_status gj_desum_kernel(gj_ctx* ctx, const gj_summary* s, int32_t* kind) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || !kind) {
    set_error("gj_desum_kernel: null argument");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  *kind = unit_expansion(ctx, s) ? 1 : 0;
  return GJ_OK;
}

gj_status gj_desummarize(gj_ctx* ctx, const gj_summary* s, int64_t first_row, int64_t n_rows, int32_t rowid_bytes,
                         void* out, int64_t* n_written) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || (rowid_bytes != 4 && rowid_bytes != 8) || n_rows < 0 || first_row < 0) {
    set_error("gj_desummarize: bad argument");
    return GJ_E_INVALID;
  }
  if (s->projected || !s->f->F.perm) {
    set_error("gj_desummarize: the summary has no row ids (projected, or loaded without rows): "
              "use gj_desummarize_projected");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  if (first_row > s->join_size) {
    set_error("first_row %lld beyond the join size %lld", (long long)first_row, (long long)s->join_size);
    return GJ_E_RANGE;
  }
  const int64_t nw = std::min(n_rows, s->join_size - first_row);
  if (nw > 0 && (!out || ((uintptr_t)out & 15) != 0)) {
    set_error("gj_desummarize: output must be a non-null, 16-byte aligned device buffer");
    return GJ_E_INVALID;
  }
  int n = 0;
  gjk::DesumArgs a{};
  desum_args(s, first_row, nw, out, a, n);
  if (nw > 0) {
    int rc;
    if (unit_expansion(ctx, s)) {
      rc = run_unit_expansion(ctx, s, a, n, rowid_bytes);
    } else {
      rc = gjk::desummarize(ctx->stream, a, rowid_bytes, n, ctx->tune.desum_rounds, ctx->tune.desum_stage);
    }
    if (rc != 0) {
      set_error("gj_desummarize: chunk too large for one launch");
      return GJ_E_INVALID;
    }
    gj_status st = check(hipGetLastError(), "expansion kernel");
    if (st) return st;
  }
  if (n_written) *n_written = nw;
  return GJ_OK;
}

gj_status gj_colset_create(gj_ctx* ctx, const gj_summary* s, int32_t n_cols, const int32_t* tab,
                           const int32_t* const* data, gj_colset** out) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || !out || n_cols < 1 || n_cols > GJ_MAX_OUT_COLS || !tab || !data) {
    set_error("gj_colset_create: bad argument (1 <= n_cols <= %d)", GJ_MAX_OUT_COLS);
    return GJ_E_INVALID;
  }
  if (s->projected || !s->f->F.perm) {
    set_error("gj_colset_create: the summary has no row ids (projected, or loaded without rows)");
    return GJ_E_INVALID;
  }
  const Plan& P = s->f->plan;
  const int base = P.qfirst[s->query];
  const int n = P.qfirst[s->query + 1] - base;
  for (int j = 0; j < n_cols; ++j) {
    if (tab[j] < 0 || tab[j] >= n) {
      set_error("gj_colset_create: column %d names table %d of a %d-table query", j, tab[j], n);
      return GJ_E_INVALID;
    }
    if (!data[j] && P.td[base + tab[j]].n > 0) {
      set_error("gj_colset_create: null column %d", j);
      return GJ_E_INVALID;
    }
  }
  gj_colset* c = new gj_colset(ctx);
  c->f = s->f;
  c->f->refs++;
  c->query = s->query;
  c->n_cols = n_cols;
  for (int j = 0; j < n_cols; ++j) {
    const TDesc& d = P.td[base + tab[j]];
    c->tab[j] = tab[j];
    c->col[j] = c->arena.get_n<int32_t>(d.n);
    if (!c->col[j]) {
      gj_free_colset(c);
      return GJ_E_OOM;
    }
    gjk::gather_rows(ctx->stream, s->f->F.perm + d.off, data[j], d.n, c->col[j]);
  }
  gj_status st = check(hipGetLastError(), "column layout kernel");
  if (st) {
    gj_free_colset(c);
    return st;
  }
  *out = c;
  return GJ_OK;
}

void gj_free_colset(gj_colset* c) {
  if (!c) return;
  c->arena.release();
  gj_free_factors(c->f);
  delete c;
}

gj_status gj_desummarize_values(gj_ctx* ctx, const gj_summary* s, const gj_colset* cs, int64_t first_row,
                                int64_t n_rows, int32_t* out, int64_t* n_written) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || !cs || n_rows < 0 || first_row < 0) {
    set_error("gj_desummarize_values: bad argument");
    return GJ_E_INVALID;
  }
  if (s->projected || cs->f != s->f || cs->query != s->query) {
    set_error("gj_desummarize_values: the column set was made for another summary's factors");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  if (first_row > s->join_size) {
    set_error("first_row %lld beyond the join size %lld", (long long)first_row, (long long)s->join_size);
    return GJ_E_RANGE;
  }
  const int64_t nw = std::min(n_rows, s->join_size - first_row);
  if (nw > 0 && (!out || ((uintptr_t)out & 15) != 0)) {
    set_error("gj_desummarize_values: output must be a non-null, 16-byte aligned device buffer");
    return GJ_E_INVALID;
  }
  int n = 0;
  gjk::DesumArgs a{};
  desum_args(s, first_row, nw, out, a, n);
  a.n_cols = cs->n_cols;
  for (int j = 0; j < cs->n_cols; ++j) {
    a.col_tab[j] = cs->tab[j];
    a.col_src[j] = cs->col[j];
  }
  if (nw > 0) {
    const int rc = unit_expansion(ctx, s)
                       ? run_unit_expansion(ctx, s, a, n, 4)
                       : gjk::desummarize(ctx->stream, a, 4, n, ctx->tune.desum_rounds, ctx->tune.desum_stage);
    if (rc != 0) {
      set_error("gj_desummarize_values: chunk too large for one launch");
      return GJ_E_INVALID;
    }
    gj_status st = check(hipGetLastError(), "expansion kernel");
    if (st) return st;
  }
  if (n_written) *n_written = nw;
  return GJ_OK;
}

}  // extern "C"
