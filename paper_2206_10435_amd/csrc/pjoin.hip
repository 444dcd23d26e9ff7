// POTENTIAL-JOIN (Sec. 3.2.1, Algorithm 1): the joint potential of several
// frequency tables over the variables of one maxclique -- every combination
// of values on which all the tables agree, with the product of the matching
// entries' frequencies.  Like Algorithm 1 this binds one variable at a time
// and only ever extends value prefixes that every table containing the
// variable shares (a worst-case optimal join over the factors, not the rows).
//
// On the GPU the recursion is unrolled into levels.  Each table's factor is
// sorted by its variables in the clique's variable order, so the entries that
// agree with a bound prefix form a contiguous range and, inside it, the next
// variable's values are sorted.  A frontier item is one bound prefix, held as
// one entry range per table.  Binding variable v: every item's driver is the
// smallest range among the tables containing v; the driver range is cut into
// slices of at most PJ_SLICE entries at value boundaries (so a heavy value
// never serializes one thread and every value lies in one slice); each slice
// walks its distinct values of v and keeps a value if each of the other tables
// holds it too (binary searches).  Per level: slice counts, a scan, slice
// listing, a count pass, a scan and a write pass that emits the child items
// with the tables' ranges narrowed to the value, in order.  After the last
// variable every range is one entry; its frequency is the product of the
// tables' entry counts and its values are read from the entries.
#include <algorithm>
#include <vector>

#include "kernels.h"
#include "plan.h"

using namespace gjh;

namespace {

constexpr int PJ_MAX = GJ_MAX_CLIQUE_TABLES;
constexpr int32_t PJ_SLICE = 32;  // driver entries per work unit (measured: 8, 16, 32, 64, 256)

struct PJTab {
  const int32_t* key[GJ_MAX_KEYS];  // entry key columns, in clique-variable order
  const int32_t* start;             // entry row ranges: count = end - start
  const int32_t* end;
  int32_t nvar;
  int32_t var[GJ_MAX_KEYS];  // clique variable of each column (ascending)
};

struct PJArgs {
  PJTab tab[PJ_MAX];
  int32_t n_tabs;
  uint32_t ind;             // bit j: table j only filters (its frequency is counted elsewhere)
  uint32_t has;             // bit j: table j holds the variable being bound
  int32_t col[PJ_MAX];      // its column in table j
  int64_t n_items;          // frontier items
  const int32_t* lo;        // [n_tabs][cap] ranges of the current frontier
  const int32_t* hi;
  int64_t cap;              // frontier capacity (stride of lo/hi)
};

__device__ __forceinline__ int32_t lower_in(const int32_t* __restrict__ a, int32_t l, int32_t h, int32_t x) {
  while (l < h) {
    const int32_t m = l + ((h - l) >> 1);
    if (a[m] < x)
      l = m + 1;
    else
      h = m;
  }
  return l;
}
__device__ __forceinline__ int32_t upper_in(const int32_t* __restrict__ a, int32_t l, int32_t h, int32_t x) {
  while (l < h) {
    const int32_t m = l + ((h - l) >> 1);
    if (a[m] <= x)
      l = m + 1;
    else
      h = m;
  }
  return l;
}

// Driver of item f: the table with the smallest range among those holding
// the variable.
__device__ __forceinline__ int driver_of(const PJArgs& a, int64_t f) {
  int d = -1;
  int32_t best = 0x7fffffff;
  for (int j = 0; j < a.n_tabs; ++j) {
    if (!((a.has >> j) & 1u)) continue;
    const int32_t w = a.hi[j * a.cap + f] - a.lo[j * a.cap + f];
    if (w < best) {
      best = w;
      d = j;
    }
  }
  return d;
}

// Slices per item (at least one) and each item's driver.
__global__ void k_pj_plan(PJArgs a, int32_t* __restrict__ drv, int64_t* __restrict__ nsl) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= a.n_items) return;
  const int d = driver_of(a, f);
  drv[f] = d;
  const int32_t w = a.hi[d * a.cap + f] - a.lo[d * a.cap + f];
  nsl[f] = w <= 0 ? 1 : (w + PJ_SLICE - 1) / PJ_SLICE;
}

// Work units: (item, slice) for every slice of every item, in order.
__global__ void k_pj_units(int64_t n_items, const int64_t* __restrict__ uoff, int64_t n_units,
                           int32_t* __restrict__ uitem, int32_t* __restrict__ uslice) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_items) return;
  const int64_t b = uoff[f], e = f + 1 < n_items ? uoff[f + 1] : n_units;
  for (int64_t u = b; u < e; ++u) {
    uitem[u] = (int32_t)f;
    uslice[u] = (int32_t)(u - b);
  }
}

// Walks the values of one work unit shared by every table holding the
// variable; calls emit(value, k) for the k-th.  Returns the number of values.
template <typename F>
__device__ __forceinline__ int64_t shared_values(const PJArgs& a, int64_t f, int d, int32_t slice, F emit) {
  const int32_t* dk = a.tab[d].key[a.col[d]];
  const int32_t lo = a.lo[d * a.cap + f], hi = a.hi[d * a.cap + f];
  // slice boundaries moved back to where the value starts
  auto cut = [&](int64_t p) -> int32_t { return p >= hi ? hi : lower_in(dk, lo, hi, dk[p]); };
  int32_t p = cut((int64_t)lo + (int64_t)slice * PJ_SLICE);
  const int32_t ph = cut((int64_t)lo + (int64_t)(slice + 1) * PJ_SLICE);
  int64_t k = 0;
  while (p < ph) {
    const int32_t x = dk[p];
    const int32_t q = upper_in(dk, p, ph, x);
    bool ok = true;
    for (int j = 0; j < a.n_tabs && ok; ++j) {
      if (j == d || !((a.has >> j) & 1u)) continue;
      const int32_t* jk = a.tab[j].key[a.col[j]];
      const int32_t l = a.lo[j * a.cap + f], h = a.hi[j * a.cap + f];
      const int32_t i = lower_in(jk, l, h, x);
      ok = i < h && jk[i] == x;
    }
    if (ok) emit(x, k++);
    p = q;
  }
  return k;
}

__global__ void k_pj_count(PJArgs a, int64_t n_units, const int32_t* __restrict__ uitem,
                           const int32_t* __restrict__ uslice, const int32_t* __restrict__ drv,
                           int64_t* __restrict__ cnt) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_units) return;
  const int32_t f = uitem[u];
  cnt[u] = shared_values(a, f, drv[f], uslice[u], [](int32_t, int64_t) {});
}

__global__ void k_pj_write(PJArgs a, int64_t n_units, const int32_t* __restrict__ uitem,
                           const int32_t* __restrict__ uslice, const int32_t* __restrict__ drv,
                           const int64_t* __restrict__ off, int32_t* __restrict__ nlo, int32_t* __restrict__ nhi,
                           int64_t ncap) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_units) return;
  const int32_t f = uitem[u];
  const int64_t o = off[u];
  shared_values(a, f, drv[f], uslice[u], [&](int32_t x, int64_t k) {
    for (int j = 0; j < a.n_tabs; ++j) {
      int32_t l = a.lo[j * a.cap + f], h = a.hi[j * a.cap + f];
      if ((a.has >> j) & 1u) {
        const int32_t* jk = a.tab[j].key[a.col[j]];
        const int32_t nl = lower_in(jk, l, h, x);
        h = upper_in(jk, nl, h, x);
        l = nl;
      }
      nlo[j * ncap + o + k] = l;
      nhi[j * ncap + o + k] = h;
    }
  });
}

// Final items: every range is one entry.  Values of each clique variable from
// a table holding it, frequency = product of the entries' counts (saturating).
__global__ void k_pj_emit(PJArgs a, int32_t nv, const int32_t* __restrict__ vtab, const int32_t* __restrict__ vcol,
                          int32_t* __restrict__ keys, int64_t kstride, int64_t* __restrict__ freq) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= a.n_items) return;
  uint64_t p = 1;
  for (int j = 0; j < a.n_tabs; ++j) {
    if ((a.ind >> j) & 1u) continue;
    const int32_t e = a.lo[j * a.cap + f];
    p = smul(p, (uint64_t)(a.tab[j].end[e] - a.tab[j].start[e]));
  }
  freq[f] = (int64_t)p;
  for (int v = 0; v < nv; ++v) {
    const int j = vtab[v];
    keys[v * kstride + f] = a.tab[j].key[vcol[v]][a.lo[j * a.cap + f]];
  }
}

// Exclusive scan of n int64 counts (in place) and their total.
__global__ void k_scan_tiles(int64_t* __restrict__ x, int64_t n, int64_t* __restrict__ tile_sum) {
  __shared__ int64_t sh[GJ_WAVES];
  const int64_t base = (int64_t)blockIdx.x * GJ_TILE;
  int64_t acc = 0;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    int64_t tot;
    const int64_t v = i < n ? x[i] : 0;
    const int64_t ex = block_excl_sum(v, sh, tot);
    if (i < n) x[i] = acc + ex;
    acc += tot;
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = acc;
}
__global__ void k_scan_top(int64_t* __restrict__ tile_sum, int64_t ntiles, int64_t* __restrict__ total) {
  __shared__ int64_t sh[GJ_WAVES];
  int64_t carry = 0;
  for (int64_t i0 = 0; i0 < ntiles; i0 += GJ_BLOCK) {
    const int64_t i = i0 + threadIdx.x;
    int64_t tot;
    const int64_t v = i < ntiles ? tile_sum[i] : 0;
    const int64_t ex = block_excl_sum(v, sh, tot);
    if (i < ntiles) tile_sum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}
__global__ void k_scan_add(int64_t* __restrict__ x, int64_t n, const int64_t* __restrict__ tile_sum) {
  const int64_t base = (int64_t)blockIdx.x * GJ_TILE;
  const int64_t add = tile_sum[blockIdx.x];
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    if (i < n) x[i] += add;
  }
}

// The first frontier: one item holding every table's whole range.
__global__ void k_pj_init(int32_t* lo, int32_t* hi, int n_tabs, const int64_t* __restrict__ cnt,
                          const int32_t* __restrict__ tidx) {
  const int j = threadIdx.x;
  if (j < n_tabs) {
    lo[j] = 0;
    hi[j] = (int32_t)cnt[tidx[j] * CNT_STRIDE + CNT_M];
  }
}

}  // namespace

namespace gjh {

// Joint potential of the tables `tabs` (indices into the factors `f`, one
// single-table query each, columns already in clique-variable order;
// tvar[j][c] = clique variable of column c).  nv clique variables, each held
// by at least one table.  Writes the entries into arena `A`.
gj_status potential_join(gj_ctx* ctx, const gj_factors* f, const std::vector<int>& tabs,
                         const std::vector<std::vector<int>>& tvar, int nv, Arena& A, PotentialOut& out,
                         uint32_t indicator) {
  hipStream_t s = ctx->stream;
  const Plan& P = f->plan;
  const int k = (int)tabs.size();
  if (k < 1 || k > PJ_MAX) {
    set_error("potential join: %d tables in one clique (1..%d)", k, PJ_MAX);
    return GJ_E_GRAPH;
  }
  PJArgs a{};
  a.n_tabs = k;
  a.ind = indicator;
  std::vector<int32_t> vtab(nv, -1), vcol(nv, -1);
  for (int j = 0; j < k; ++j) {
    const TDesc& d = P.td[tabs[j]];
    PJTab& T = a.tab[j];
    T.nvar = (int32_t)tvar[j].size();
    for (int c = 0; c < T.nvar; ++c) {
      T.key[c] = f->F.ekey + d.key_off + (int64_t)c * d.n;
      T.var[c] = tvar[j][c];
      if (vtab[tvar[j][c]] < 0) {
        vtab[tvar[j][c]] = j;
        vcol[tvar[j][c]] = c;
      }
    }
    T.start = f->F.estart + d.off;
    T.end = f->F.eend + d.off;
  }
  for (int v = 0; v < nv; ++v)
    if (vtab[v] < 0) {
      set_error("potential join: variable %d is held by none of the tables", v);
      return GJ_E_GRAPH;
    }
  // frontiers of consecutive levels alternate between two arenas
  Arena tmp(ctx), lvl0(ctx), lvl1(ctx);
  Arena* lvl[2] = {&lvl0, &lvl1};
  int64_t cap = 1;
  int32_t* lo = tmp.get_n<int32_t>(k);
  int32_t* hi = tmp.get_n<int32_t>(k);
  int32_t* d_tidx = tmp.get_n<int32_t>(k);
  int64_t* d_total = tmp.get_n<int64_t>(1);
  if (!lo || !hi || !d_tidx || !d_total) return GJ_E_OOM;
  std::vector<int32_t> tidx(tabs.begin(), tabs.end());
  gj_status st = check(hipMemcpyAsync(d_tidx, tidx.data(), k * 4, hipMemcpyHostToDevice, s), "potential join");
  if (st) return st;
  hipLaunchKernelGGL(k_pj_init, dim3(1), dim3(64), 0, s, lo, hi, k, f->F.cnt, d_tidx);
  // exclusive scan of x[0..n) in place; returns the total (synchronizes)
  auto scan = [&](Arena& L, int64_t* x, int64_t n, int64_t& total) -> gj_status {
    const int64_t ntiles = (n + GJ_TILE - 1) / GJ_TILE;
    int64_t* tsum = L.get_n<int64_t>(ntiles);
    if (!tsum) return GJ_E_OOM;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(GJ_BLOCK), 0, s, x, n, tsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(GJ_BLOCK), 0, s, tsum, ntiles, d_total);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntiles), dim3(GJ_BLOCK), 0, s, x, n, tsum);
    gj_status e = check(hipMemcpyAsync(&total, d_total, 8, hipMemcpyDeviceToHost, s), "potential join");
    if (!e) e = check(hipStreamSynchronize(s), "potential join");
    return e;
  };
  auto grid = [](int64_t n) { return dim3((unsigned)((n + GJ_BLOCK - 1) / GJ_BLOCK)); };
  int64_t n_items = 1;
  for (int v = 0; v < nv && n_items > 0; ++v) {
    a.has = 0;
    for (int j = 0; j < k; ++j) {
      a.col[j] = -1;
      for (int c = 0; c < a.tab[j].nvar; ++c)
        if (a.tab[j].var[c] == v) {
          a.has |= 1u << j;
          a.col[j] = c;
        }
    }
    a.n_items = n_items;
    a.lo = lo;
    a.hi = hi;
    a.cap = cap;
    Arena& L = *lvl[v & 1];  // held level v-2's frontier, no longer read
    L.release();
    // work units: slices of every item's driver range
    int32_t* drv = L.get_n<int32_t>(n_items);
    int64_t* uoff = L.get_n<int64_t>(n_items);
    if (!drv || !uoff) return GJ_E_OOM;
    hipLaunchKernelGGL(k_pj_plan, grid(n_items), dim3(GJ_BLOCK), 0, s, a, drv, uoff);
    int64_t n_units = 0;
    if ((st = scan(L, uoff, n_items, n_units))) return st;
    if (n_units > INT32_MAX) {
      set_error("potential join: too many work units");
      return GJ_E_INVALID;
    }
    int32_t* uitem = L.get_n<int32_t>(n_units);
    int32_t* uslice = L.get_n<int32_t>(n_units);
    int64_t* cnt = L.get_n<int64_t>(n_units);
    if (!uitem || !uslice || !cnt) return GJ_E_OOM;
    hipLaunchKernelGGL(k_pj_units, grid(n_items), dim3(GJ_BLOCK), 0, s, n_items, uoff, n_units, uitem, uslice);
    hipLaunchKernelGGL(k_pj_count, grid(n_units), dim3(GJ_BLOCK), 0, s, a, n_units, uitem, uslice, drv, cnt);
    int64_t total = 0;
    if ((st = scan(L, cnt, n_units, total))) return st;
    if (total > INT32_MAX) {
      set_error("potential join: %lld joint entries (at most 2^31-1)", (long long)total);
      return GJ_E_INVALID;
    }
    const int64_t ncap = std::max<int64_t>(total, 1);
    int32_t* nlo = L.get_n<int32_t>(k * ncap);
    int32_t* nhi = L.get_n<int32_t>(k * ncap);
    if (!nlo || !nhi) return GJ_E_OOM;
    if (total > 0)
      hipLaunchKernelGGL(k_pj_write, grid(n_units), dim3(GJ_BLOCK), 0, s, a, n_units, uitem, uslice, drv, cnt, nlo,
                         nhi, ncap);
    lo = nlo;
    hi = nhi;
    cap = ncap;
    n_items = total;
  }
  out.n = n_items;
  out.nv = nv;
  out.stride = std::max<int64_t>(n_items, 1);
  out.keys = A.get_n<int32_t>((int64_t)nv * out.stride);
  out.freq = A.get_n<int64_t>(out.stride);
  int32_t* d_v = tmp.get_n<int32_t>(2 * nv);
  if (!out.keys || !out.freq || !d_v) return GJ_E_OOM;
  std::vector<int32_t> vv(vtab);
  vv.insert(vv.end(), vcol.begin(), vcol.end());
  if ((st = check(hipMemcpyAsync(d_v, vv.data(), 2 * nv * 4, hipMemcpyHostToDevice, s), "potential join")))
    return st;
  if (n_items > 0) {
    a.n_items = n_items;
    a.lo = lo;
    a.hi = hi;
    a.cap = cap;
    hipLaunchKernelGGL(k_pj_emit, dim3((unsigned)((n_items + GJ_BLOCK - 1) / GJ_BLOCK)), dim3(GJ_BLOCK), 0, s, a,
                       nv, d_v, d_v + nv, out.keys, out.stride, out.freq);
  }
  st = check(hipGetLastError(), "potential join kernels");
  if (!st) st = check(hipStreamSynchronize(s), "potential join");  // tmp is released on return
  return st;
}

}  // namespace gjh

struct gj_potential {
  gj_ctx* ctx = nullptr;
  gjh::Arena arena;
  gjh::PotentialOut pot;
  std::vector<int32_t> attr;
  explicit gj_potential(gj_ctx* c) : ctx(c), arena(c) {}
};

namespace gjh {

// Factors of `n` tables built as single-table queries with their columns
// reordered by attribute id (ascending): the order a potential join needs.
// vars: the distinct attribute ids (ascending); tvar[t][c]: variable index of
// the reordered column c of table t.
gj_status sorted_factors(gj_ctx* ctx, int n, const gj_table* tables, const gj_natural_query* q,
                         std::vector<int32_t>& vars, std::vector<std::vector<int>>& tvar, gj_factors** out) {
  vars.clear();
  tvar.assign(n, {});
  for (int t = 0; t < n; ++t) {
    if (q->n_keys[t] != tables[t].n_keys) {
      set_error("table %d: %d key columns but %d attributes", t, tables[t].n_keys, q->n_keys[t]);
      return GJ_E_INVALID;
    }
    for (int c = 0; c < q->n_keys[t]; ++c) {
      const int32_t a = q->attr[t * GJ_MAX_KEYS + c];
      for (int c2 = 0; c2 < c; ++c2)
        if (q->attr[t * GJ_MAX_KEYS + c2] == a) {
          set_error("table %d names attribute %d twice", t, a);
          return GJ_E_GRAPH;
        }
      if (a < 0) {
        set_error("negative attribute id");
        return GJ_E_INVALID;
      }
      vars.push_back(a);
    }
  }
  std::sort(vars.begin(), vars.end());
  vars.erase(std::unique(vars.begin(), vars.end()), vars.end());
  if ((int)vars.size() > GJ_MAX_ATTRS) {
    set_error("%d attributes (at most %d)", (int)vars.size(), GJ_MAX_ATTRS);
    return GJ_E_INVALID;
  }
  std::vector<std::vector<const int32_t*>> cols(n);
  std::vector<gj_table> tabs(n);
  std::vector<gj_join_graph> graphs(n);
  std::vector<int32_t> qoff(n + 1), zero(1, 0), root(1, -1);
  for (int t = 0; t < n; ++t) {
    std::vector<std::pair<int, int>> vc;  // (variable, column)
    for (int c = 0; c < q->n_keys[t]; ++c) {
      const int v = (int)(std::lower_bound(vars.begin(), vars.end(), q->attr[t * GJ_MAX_KEYS + c]) - vars.begin());
      vc.push_back({v, c});
    }
    std::sort(vc.begin(), vc.end());
    for (auto& p : vc) {
      tvar[t].push_back(p.first);
      cols[t].push_back(tables[t].n_rows > 0 ? tables[t].keys[p.second] : nullptr);
    }
    tabs[t].n_rows = tables[t].n_rows;
    tabs[t].n_keys = tables[t].n_keys;
    tabs[t].keys = cols[t].data();
    graphs[t] = gj_join_graph{1, root.data(), zero.data(), zero.data()};
    qoff[t] = t;
  }
  qoff[n] = n;
  gj_factors* f = new gj_factors(ctx);
  f->plan.ctx = ctx;
  gj_status st;
  if ((st = plan_tables(f->plan, n, qoff.data(), tabs.data(), graphs.data())) ||
      (st = plan_device(f->plan, f->arena, f->F))) {
    delete f;
    return st;
  }
  launch_factors(f->plan, f->F, ctx->stream);
  if ((st = check(hipGetLastError(), "factor kernels"))) {
    delete f;
    return st;
  }
  *out = f;
  return GJ_OK;
}

}  // namespace gjh

extern "C" {

gj_status gj_potential_join(gj_ctx* ctx, const gj_table* tables, const gj_natural_query* q, gj_potential** out) {
  GJ_SCOPE(ctx);
  if (!ctx || !tables || !q || !out || !q->n_keys || !q->attr || q->n_tables < 1 ||
      q->n_tables > GJ_MAX_CLIQUE_TABLES) {
    set_error("gj_potential_join: bad argument (1..%d tables)", GJ_MAX_CLIQUE_TABLES);
    return GJ_E_INVALID;
  }
  const int n = q->n_tables;
  std::vector<int32_t> vars;
  std::vector<std::vector<int>> tvar;
  gj_factors* f = nullptr;
  gj_status st = sorted_factors(ctx, n, tables, q, vars, tvar, &f);
  if (st) return st;
  gj_potential* p = new gj_potential(ctx);
  p->attr = vars;
  std::vector<int> tabs(n);
  for (int t = 0; t < n; ++t) tabs[t] = t;
  st = potential_join(ctx, f, tabs, tvar, (int)vars.size(), p->arena, p->pot);
  gj_free_factors(f);
  if (st) {
    delete p;
    return st;
  }
  *out = p;
  return GJ_OK;
}

gj_status gj_potential_table(const gj_potential* p, gj_potential_view* v) {
  GJ_SCOPE(p ? p->ctx : nullptr);
  if (!p || !v) {
    set_error("gj_potential_table: null argument");
    return GJ_E_INVALID;
  }
  gj_potential_view r{};
  r.n_entries = p->pot.n;
  r.n_vars = p->pot.nv;
  for (int i = 0; i < p->pot.nv; ++i) {
    r.attr[i] = p->attr[i];
    r.keys[i] = p->pot.keys + (int64_t)i * p->pot.stride;
  }
  r.freq = p->pot.freq;
  *v = r;
  return GJ_OK;
}

void gj_free_potential(gj_potential* p) { delete p; }

}  // extern "C"
