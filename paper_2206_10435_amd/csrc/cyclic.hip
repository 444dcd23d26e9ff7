// Cyclic queries (Sec. 3.2.1 joining potentials in maxcliques, Sec. 3.4
// inference on a junction tree).  The query's attribute graph is turned into
// a junction tree of maxcliques (jtree.hip); each maxclique gets one potential,
// the POTENTIAL-JOIN of the tables assigned to it (pjoin.hip); and the tree of
// clique potentials is summarized by the same kernels as an acyclic query.
//
//   - A clique variable that no assigned table holds (a clique grown by
//     fill-in) is restricted by the distinct projection of another table that
//     holds it: a filter only, its frequency is counted in its own clique.
//   - A clique's potential becomes a table whose rows are the potential's
//     entries and whose rows carry the entries' frequencies (the counts of the
//     summary are sums of these, as for projected factors).
//   - A separator of several attributes (a composite separator) becomes one
//     column on both sides: the index of the value combination among the
//     combinations either side holds (one group-by over both sides).
//   - The result has no row ids; its columns are every attribute once: the
//     root clique's attributes, then each further clique's attributes outside
//     its separator (the running intersection property places every other
//     attribute in an earlier clique).
#include <algorithm>
#include <vector>

#include "kernels.h"
#include "plan.h"

using namespace gjh;

namespace {

// row -> index of its entry, for every entry of a one-table factor: one
// thread per grouped position (an entry of many rows is spread over many
// threads); the entry of position x is the last one starting at or before x
__global__ void k_entry_ids(const int32_t* __restrict__ estart, int64_t n, const int32_t* __restrict__ perm,
                            const int64_t* __restrict__ cnt, int32_t* __restrict__ id) {
  const int64_t M = cnt[CNT_M];
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = M;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (estart[mid] <= x)
        lo = mid;
      else
        hi = mid;
    }
    id[perm[x]] = (int32_t)lo;
  }
}

int popc(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace

extern "C" {

gj_status gj_summarize_cyclic(gj_ctx* ctx, const gj_table* tables, const gj_natural_query* q, gj_summary** out,
                              int64_t* join_size) {
  GJ_SCOPE(ctx);
  if (!ctx || !tables || !q || !out) {
    set_error("gj_summarize_cyclic: null argument");
    return GJ_E_INVALID;
  }
  gj_junction_tree jt;
  gj_status st = gj_junction_tree_build(q, &jt);
  if (st) return st;
  const int n = q->n_tables;
  const int k = jt.n_cliques;
  if (k > GJ_MAX_TABLES) {
    set_error("gj_summarize_cyclic: %d maxcliques (at most %d)", k, GJ_MAX_TABLES);
    return GJ_E_GRAPH;
  }
  hipStream_t hs = ctx->stream;
  // clique variables (attribute indices, ascending)
  std::vector<std::vector<int>> cv(k);
  for (int i = 0; i < k; ++i)
    for (int a = 0; a < jt.n_attrs; ++a)
      if ((jt.clique[i] >> a) & 1) cv[i].push_back(a);
  // factors: every table in full, plus, for a clique variable no assigned
  // table holds, the distinct projection of a table holding it onto the clique
  std::vector<gj_table> ftab;
  std::vector<std::vector<int32_t>> fattr;           // attribute ids per factor table
  std::vector<std::vector<const int32_t*>> fcols;
  std::vector<std::vector<int>> members(k);          // factor tables per clique
  std::vector<uint32_t> filt(k, 0);                  // bit j of clique i: member j only filters
  auto attr_of = [&](int t, int c) { return q->attr[t * GJ_MAX_KEYS + c]; };
  auto idx_of = [&](int32_t a) {
    return (int)(std::find(jt.attr_id, jt.attr_id + jt.n_attrs, a) - jt.attr_id);
  };
  for (int t = 0; t < n; ++t) {
    ftab.push_back(tables[t]);
    fattr.push_back(std::vector<int32_t>(q->attr + t * GJ_MAX_KEYS, q->attr + t * GJ_MAX_KEYS + q->n_keys[t]));
    fcols.push_back({});
    members[jt.table_clique[t]].push_back(t);
  }
  for (int i = 0; i < k; ++i) {
    uint64_t held = 0;
    for (int t : members[i])
      for (int c = 0; c < q->n_keys[t]; ++c) held |= 1ull << idx_of(attr_of(t, c));
    for (int v : cv[i]) {
      if ((held >> v) & 1) continue;
      int best = -1, best_cov = 0;  // the table covering most of the missing variables
      for (int t = 0; t < n; ++t) {
        uint64_t tm = 0;
        for (int c = 0; c < q->n_keys[t]; ++c) tm |= 1ull << idx_of(attr_of(t, c));
        if (!((tm >> v) & 1)) continue;
        const int cov = popc(tm & jt.clique[i] & ~held);
        if (cov > best_cov) {
          best_cov = cov;
          best = t;
        }
      }
      std::vector<const int32_t*> cols;
      std::vector<int32_t> at;
      for (int c = 0; c < q->n_keys[best]; ++c) {
        const int a = idx_of(attr_of(best, c));
        if ((jt.clique[i] >> a) & 1) {
          cols.push_back(tables[best].n_rows > 0 ? tables[best].keys[c] : nullptr);
          at.push_back(attr_of(best, c));
          held |= 1ull << a;
        }
      }
      fcols.push_back(cols);
      fattr.push_back(at);
      ftab.push_back(gj_table{tables[best].n_rows, (int32_t)cols.size(), nullptr});
      filt[i] |= 1u << members[i].size();
      members[i].push_back((int)ftab.size() - 1);
    }
  }
  for (size_t j = n; j < ftab.size(); ++j) ftab[j].keys = fcols[j].data();
  const int nf = (int)ftab.size();
  std::vector<int32_t> fnk(nf), fat((size_t)nf * GJ_MAX_KEYS, -1);
  for (int j = 0; j < nf; ++j) {
    fnk[j] = (int32_t)fattr[j].size();
    for (size_t c = 0; c < fattr[j].size(); ++c) fat[(size_t)j * GJ_MAX_KEYS + c] = fattr[j][c];
  }
  if (nf > GJ_MAX_TABLES) {
    set_error("gj_summarize_cyclic: %d tables and filters (at most %d)", nf, GJ_MAX_TABLES);
    return GJ_E_GRAPH;
  }
  gj_natural_query fq{nf, fnk.data(), fat.data()};
  std::vector<int32_t> vars;
  std::vector<std::vector<int>> tvar;
  gj_factors* f = nullptr;
  if ((st = sorted_factors(ctx, nf, ftab.data(), &fq, vars, tvar, &f))) return st;

  // 1. one potential per clique (variables renumbered 0.. within the clique)
  Arena pots(ctx);
  std::vector<PotentialOut> pot(k);
  for (int i = 0; i < k && !st; ++i) {
    std::vector<std::vector<int>> tv;
    for (int j : members[i]) {
      std::vector<int> v;
      for (int g : tvar[j]) v.push_back((int)(std::find(cv[i].begin(), cv[i].end(), idx_of(vars[g])) - cv[i].begin()));
      tv.push_back(v);
    }
    st = potential_join(ctx, f, members[i], tv, (int)cv[i].size(), pots, pot[i], filt[i]);
  }
  gj_free_factors(f);
  if (st) return st;

  // 2. separators: one column per edge (the attribute itself, or the index of
  //    a composite separator's value combination)
  std::vector<std::vector<const int32_t*>> vcols(k);
  for (int i = 0; i < k; ++i)
    for (size_t v = 0; v < cv[i].size(); ++v) vcols[i].push_back(pot[i].keys + (int64_t)v * pot[i].stride);
  std::vector<int32_t> par(k), sep(k, 0), pcol(k, 0);
  Arena ids(ctx);
  for (int i = 0; i < k && !st; ++i) {
    par[i] = jt.parent[i];
    if (i == 0) continue;
    const int p = par[i];
    const uint64_t S = jt.clique[i] & jt.clique[p];
    std::vector<int> sv;
    for (int a = 0; a < jt.n_attrs; ++a)
      if ((S >> a) & 1) sv.push_back(a);
    auto pos = [&](int c, int a) { return (int)(std::find(cv[c].begin(), cv[c].end(), a) - cv[c].begin()); };
    if (sv.size() == 1) {
      sep[i] = pos(i, sv[0]);
      pcol[i] = pos(p, sv[0]);
      continue;
    }
    // both sides' combinations, grouped together
    const int64_t np_ = pot[p].n, ni = pot[i].n, tot = np_ + ni;
    std::vector<const int32_t*> cc;
    std::vector<int32_t> at;
    for (int a : sv) {
      int32_t* buf = ids.get_n<int32_t>(tot);
      if (!buf) return GJ_E_OOM;
      if (np_ > 0 && (st = check(hipMemcpyAsync(buf, vcols[p][pos(p, a)], np_ * 4, hipMemcpyDeviceToDevice, hs),
                                 "separator")))
        return st;
      if (ni > 0 && (st = check(hipMemcpyAsync(buf + np_, vcols[i][pos(i, a)], ni * 4, hipMemcpyDeviceToDevice, hs),
                                "separator")))
        return st;
      cc.push_back(buf);
      at.push_back(jt.attr_id[a]);
    }
    gj_table st1{tot, (int32_t)cc.size(), cc.data()};
    int32_t nk1 = (int32_t)cc.size();
    std::vector<int32_t> at1(GJ_MAX_KEYS, -1);
    std::copy(at.begin(), at.end(), at1.begin());
    gj_natural_query q1{1, &nk1, at1.data()};
    std::vector<int32_t> v1;
    std::vector<std::vector<int>> tv1;
    gj_factors* g = nullptr;
    if ((st = sorted_factors(ctx, 1, &st1, &q1, v1, tv1, &g))) return st;
    int32_t* id = ids.get_n<int32_t>(tot);
    if (!id) {
      gj_free_factors(g);
      return GJ_E_OOM;
    }
    const TDesc& d = g->plan.td[0];
    if (tot > 0)
      hipLaunchKernelGGL(k_entry_ids, dim3((unsigned)std::min<int64_t>((tot + GJ_BLOCK - 1) / GJ_BLOCK, 4096)),
                         dim3(GJ_BLOCK), 0, hs, g->F.estart + d.off, tot, g->F.perm + d.off, g->F.cnt, id);
    st = check(hipStreamSynchronize(hs), "separator ids");
    gj_free_factors(g);
    if (st) return st;
    if ((int)vcols[p].size() >= GJ_MAX_KEYS || (int)vcols[i].size() >= GJ_MAX_KEYS) {
      set_error("gj_summarize_cyclic: a clique needs more than %d columns", GJ_MAX_KEYS);
      return GJ_E_GRAPH;
    }
    pcol[i] = (int)vcols[p].size();
    vcols[p].push_back(id);
    sep[i] = (int)vcols[i].size();
    vcols[i].push_back(id + np_);
  }
  if (st) return st;

  // 3. the tree of clique potentials: factors whose rows carry frequencies
  std::vector<gj_table> vt(k);
  int64_t wtot = 0;
  std::vector<int64_t> woff(k);
  for (int i = 0; i < k; ++i) {
    vt[i] = gj_table{pot[i].n, (int32_t)vcols[i].size(), vcols[i].data()};
    woff[i] = wtot;
    wtot += std::max<int64_t>(pot[i].n, 1);
  }
  int64_t* w = ids.get_n<int64_t>(wtot);
  if (!w) return GJ_E_OOM;
  for (int i = 0; i < k; ++i)
    if (pot[i].n > 0 &&
        (st = check(hipMemcpyAsync(w + woff[i], pot[i].freq, pot[i].n * 8, hipMemcpyDeviceToDevice, hs), "frequencies")))
      return st;
  gj_join_graph g{k, par.data(), sep.data(), pcol.data()};
  gj_factors* pf = new gj_factors(ctx);
  pf->plan.ctx = ctx;
  int qoff[2] = {0, k};
  if ((st = plan_tables(pf->plan, 1, qoff, vt.data(), &g)) || (st = plan_device(pf->plan, pf->arena, pf->F))) {
    delete pf;
    return st;
  }
  pf->F.ecnt = pf->arena.get_n<int64_t>(pf->plan.S);
  if (!pf->F.ecnt) {
    delete pf;
    return GJ_E_OOM;
  }
  launch_factors(pf->plan, pf->F, hs);
  const Plan& PP = pf->plan;
  gjk::ProjArgs pa{};
  for (int i = 0; i < k; ++i) pa.full_off[i] = woff[i];
  gjk::proj_counts(hs, PP.d_wl + PP.all.off, PP.all.n, PP.d_desc, pf->F, w, pa, PP.S);

  gj_summary* s = new gj_summary(ctx);
  s->f = pf;
  s->projected = true;
  for (int i = 0; i < k; ++i) {
    const uint64_t S = i == 0 ? 0 : (jt.clique[i] & jt.clique[par[i]]);
    for (size_t v = 0; v < cv[i].size(); ++v)
      if (!((S >> cv[i][v]) & 1)) {
        s->result_cols.push_back({i, (int)v});
        s->result_attr.push_back(jt.attr_id[cv[i][v]]);
      }
  }
  int64_t qv = 0;
  int32_t qs = 0;
  if ((st = alloc_summary(PP, s->arena, s->S)) == GJ_OK) {
    launch_summary(PP, pf->F, s->S, hs);
    if (!(st = check(hipGetLastError(), "cyclic summary kernels")) &&
        !(st = check(hipMemcpyAsync(&qv, s->S.qsize, 8, hipMemcpyDeviceToHost, hs), "join size")) &&
        !(st = check(hipMemcpyAsync(&qs, s->S.qstatus, 4, hipMemcpyDeviceToHost, hs), "join size")))
      st = read_counters(PP, pf->F, hs, s->cnt_host);
  }
  if (st) {
    gj_free_summary(s);
    return st;
  }
  pf->cnt_host = s->cnt_host;
  if (qs == GJ_E_OVERFLOW) {
    set_error("join size does not fit below 2^63-1");
    gj_free_summary(s);
    return GJ_E_OVERFLOW;
  }
  s->join_size = qv;
  if (join_size) *join_size = qv;
  *out = s;
  return GJ_OK;
}

int32_t gj_result_attribute(const gj_summary* s, int32_t j) {
  if (!s || j < 0 || j >= (int32_t)s->result_attr.size()) return -1;
  return s->result_attr[j];
}

}  // extern "C"
