// Junction tree of a natural-join query (Sec. 2.2.1, background: JT of
// maxcliques; Sec. 3.2 qualitative learning; Sec. 3.4 inference on graphs).
// Host code only.
//
// The query graph has one node per attribute and a clique per table (all
// attributes of a table are pairwise connected).  The min fill-in heuristic
// eliminates, one at a time, the attribute whose remaining neighbours miss
// the fewest edges among themselves, adds those fill-in edges, and records the
// attribute with its remaining neighbours as a clique; the maximal ones are
// the maxcliques of the triangulated graph.  Maxcliques are joined by a
// maximal spanning tree over separator sizes (Prim's algorithm from the
// clique that holds table 0's attributes), which has the running intersection
// property on a triangulated graph.  Ties break towards the smallest index so
// the plan is deterministic.  Every table is assigned to the first clique (in
// tree order) that holds all of its attributes.
#include <algorithm>
#include <map>
#include <vector>

#include "plan.h"

using namespace gjh;

namespace {

int popc(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace

extern "C" {

gj_status gj_junction_tree_build(const gj_natural_query* q, gj_junction_tree* out) {
  if (!q || !out || !q->n_keys || !q->attr || q->n_tables < 1 || q->n_tables > GJ_MAX_TABLES) {
    set_error("gj_junction_tree_build: bad argument (1..%d tables)", GJ_MAX_TABLES);
    return GJ_E_INVALID;
  }
  const int n = q->n_tables;
  std::map<int32_t, int> idx;
  for (int t = 0; t < n; ++t) {
    if (q->n_keys[t] < 1 || q->n_keys[t] > GJ_MAX_KEYS) {
      set_error("gj_junction_tree_build: table %d has %d key columns", t, q->n_keys[t]);
      return GJ_E_INVALID;
    }
    for (int c = 0; c < q->n_keys[t]; ++c) {
      const int32_t a = q->attr[t * GJ_MAX_KEYS + c];
      if (a < 0) {
        set_error("gj_junction_tree_build: negative attribute id");
        return GJ_E_INVALID;
      }
      idx.emplace(a, 0);
    }
  }
  if ((int)idx.size() > GJ_MAX_ATTRS) {
    set_error("gj_junction_tree_build: %d attributes (at most %d)", (int)idx.size(), GJ_MAX_ATTRS);
    return GJ_E_INVALID;
  }
  gj_junction_tree r{};
  r.n_attrs = 0;
  for (auto& kv : idx) {
    kv.second = r.n_attrs;
    r.attr_id[r.n_attrs++] = kv.first;
  }
  const int m = r.n_attrs;
  std::vector<uint64_t> tab(n, 0), adj(m, 0);
  for (int t = 0; t < n; ++t) {
    for (int c = 0; c < q->n_keys[t]; ++c) tab[t] |= 1ull << idx[q->attr[t * GJ_MAX_KEYS + c]];
    for (int i = 0; i < m; ++i)
      if ((tab[t] >> i) & 1) adj[i] |= tab[t] & ~(1ull << i);
  }
  // min fill-in elimination
  uint64_t left = m == 64 ? ~0ull : ((1ull << m) - 1);
  std::vector<uint64_t> cliques;
  for (int step = 0; step < m; ++step) {
    int best = -1, best_fill = 1 << 30;
    for (int v = 0; v < m; ++v) {
      if (!((left >> v) & 1)) continue;
      const uint64_t nb = adj[v] & left;
      int fill = 0;
      for (int u = 0; u < m; ++u)
        if ((nb >> u) & 1) fill += popc(nb & ~adj[u] & ~(1ull << u));
      fill /= 2;
      if (fill < best_fill) {
        best_fill = fill;
        best = v;
      }
    }
    const uint64_t nb = adj[best] & left;
    for (int u = 0; u < m; ++u)
      if ((nb >> u) & 1) adj[u] |= nb & ~(1ull << u);
    r.elim_order[step] = best;
    r.n_fill += best_fill;
    cliques.push_back(nb | (1ull << best));
    left &= ~(1ull << best);
  }
  // maxcliques: drop cliques contained in another (and duplicates)
  std::vector<uint64_t> mc;
  for (size_t i = 0; i < cliques.size(); ++i) {
    bool sub = false;
    for (size_t j = 0; j < cliques.size() && !sub; ++j)
      if (j != i && (cliques[i] & ~cliques[j]) == 0 && (cliques[i] != cliques[j] || j < i)) sub = true;
    if (!sub) mc.push_back(cliques[i]);
  }
  const int k = (int)mc.size();
  // root: the clique holding table 0's attributes
  int root = 0;
  for (int i = 0; i < k; ++i)
    if ((tab[0] & ~mc[i]) == 0) {
      root = i;
      break;
    }
  // maximal spanning tree (Prim), separator sizes as weights
  std::vector<int> order{root}, par(k, -2);
  par[root] = -1;
  std::vector<char> in(k, 0);
  in[root] = 1;
  for (int step = 1; step < k; ++step) {
    int bi = -1, bj = -1, bw = 0;
    for (int i : order)
      for (int j = 0; j < k; ++j) {
        if (in[j]) continue;
        const int w = popc(mc[i] & mc[j]);
        if (w > bw) {
          bw = w;
          bi = i;
          bj = j;
        }
      }
    if (bj < 0) {
      set_error("gj_junction_tree_build: the query is not connected (a cross product)");
      return GJ_E_GRAPH;
    }
    par[bj] = bi;
    in[bj] = 1;
    order.push_back(bj);
  }
  // renumber in tree order (parents first)
  std::vector<int> pos(k);
  for (int i = 0; i < k; ++i) pos[order[i]] = i;
  r.n_cliques = k;
  for (int i = 0; i < k; ++i) {
    r.clique[i] = mc[order[i]];
    r.parent[i] = par[order[i]] < 0 ? -1 : pos[par[order[i]]];
  }
  for (int t = 0; t < n; ++t) {
    r.table_clique[t] = -1;
    for (int i = 0; i < k && r.table_clique[t] < 0; ++i)
      if ((tab[t] & ~r.clique[i]) == 0) r.table_clique[t] = i;
  }
  *out = r;
  return GJ_OK;
}

}  // extern "C"
