// Graphical Join -- CPU ORACLE.  TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct CPU implementation of what the Graphical
// Join hot path computes.  Only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark may load it; the product library never does.
// It shares no code, header or table with the HIP path.
//
// Everything here follows the definitions, not the paper's algorithms:
//   * the join result is the natural equi-join of the tables (Sec. 1.1); here
//     it is enumerated by a hash-join DFS (materialize) or, for tiny inputs, by
//     an all-combinations nested loop (brute_force);
//   * the GFJS of Definition 1 (Sec. 1.2) is "sort the result by all columns,
//     then run-length encode each column"; sorting is a comparator over the
//     attribute values, ties broken by the row ids (r_0, .., r_{n-1}), table 0
//     most significant (the paper orders values only; a join over row
//     identifiers has to order tuples with equal values somehow);
//   * the join size is the partition function Z of Eq. 3 (Sec. 2.2): the number
//     of row combinations that agree on every join edge.  It is counted at the
//     level of individual rows: down(t,r) = number of ways to complete the
//     subtree below row r, up(t,r) = number of ways to complete everything
//     outside that subtree; fan-out(r) = down*up is the number of result tuples
//     that use row r.
//   * the factor ("potential", Sec. 3.2) of a table is every distinct key tuple
//     with its frequency, computed with std::map (group-by count).
//   * the weighted join size W = sum over result tuples of the product of the
//     tuple's row weights, with its gradient and central finite differences, in
//     __float128.
//
// Counts are __int128 saturated at 2^120, far above the int64 range in which
// the GPU path reports results; "overflow" means the join size is >= 2^63-1.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

typedef __int128 i128;
typedef __float128 f128;

namespace {

const i128 CAP = ((i128)1) << 120;
const i128 I64MAX = (i128)INT64_MAX;

i128 sadd(i128 a, i128 b) {
  i128 s = a + b;
  return s > CAP ? CAP : s;
}
i128 smul(i128 a, i128 b) {
  if (a == 0 || b == 0) return 0;
  if (a > CAP / b) return CAP;
  i128 p = a * b;
  return p > CAP ? CAP : p;
}
int64_t to64(i128 v) { return v >= I64MAX ? INT64_MAX : (int64_t)v; }

const int MAXK = 8;

}  // namespace

extern "C" {

// Query description handed over from Python (all host memory, borrowed).
struct orc_query {
  int32_t n;                   // number of tables
  const int64_t* n_rows;       // [n]
  const int32_t* n_keys;       // [n]
  const int32_t* const* cols;  // cols[t*8 + c]: int32 column c of table t
  const int32_t* parent;       // [n]; parent[0] = -1, parent[t] < t
  const int32_t* sep_col;      // [n]; column of t equal to ...
  const int32_t* parent_col;   // [n]; ... this column of parent[t]
};

}  // extern "C"

namespace {

struct State {
  int n = 0;
  std::vector<int64_t> N;
  std::vector<int> K, par, sep, pcol;
  std::vector<std::vector<const int32_t*>> col;
  std::vector<std::vector<int>> children;
  // row lists of table t (t >= 1) by separator value, rows ascending
  std::vector<std::unordered_map<int32_t, std::vector<int32_t>>> by_sep;
  // row-level counts
  std::vector<std::vector<i128>> down, up;
  std::vector<std::unordered_map<int32_t, i128>> sumdown, upval;
  i128 Q = 0;
  // the root's group-by, computed once on first use by rank/unrank
  std::map<std::vector<int32_t>, std::vector<int32_t>> root_groups;
  bool root_grouped = false;

  int32_t key(int t, int c, int64_t r) const { return col[t][c][r]; }

  // Key columns of t in the order its factor entries are sorted: the root in
  // declared order; any other table by its separator first, then the rest in
  // declared order.
  std::vector<int> canon_cols(int t) const {
    std::vector<int> v;
    if (t > 0) v.push_back(sep[t]);
    for (int c = 0; c < K[t]; ++c)
      if (t == 0 || c != sep[t]) v.push_back(c);
    return v;
  }
  // Columns of t that contribute attribute values to the sort order of the
  // result: all of the root's, and for any other table all but its separator
  // (whose value equals a column already listed for its parent).
  std::vector<int> sigma_cols(int t) const {
    std::vector<int> v;
    for (int c = 0; c < K[t]; ++c)
      if (t == 0 || c != sep[t]) v.push_back(c);
    return v;
  }
  std::vector<int32_t> canon_key(int t, int64_t r) const {
    std::vector<int32_t> k;
    for (int c : canon_cols(t)) k.push_back(key(t, c, r));
    return k;
  }
};

void load(State& s, const orc_query* q) {
  s.n = q->n;
  s.N.assign(q->n_rows, q->n_rows + q->n);
  s.K.assign(q->n_keys, q->n_keys + q->n);
  s.par.assign(q->parent, q->parent + q->n);
  s.sep.assign(q->sep_col, q->sep_col + q->n);
  s.pcol.assign(q->parent_col, q->parent_col + q->n);
  s.col.resize(s.n);
  s.children.assign(s.n, {});
  for (int t = 0; t < s.n; ++t) {
    for (int c = 0; c < s.K[t]; ++c) s.col[t].push_back(q->cols[t * MAXK + c]);
    if (t > 0) s.children[s.par[t]].push_back(t);
  }
  s.by_sep.assign(s.n, {});
  for (int t = 1; t < s.n; ++t)
    for (int64_t r = 0; r < s.N[t]; ++r) s.by_sep[t][s.key(t, s.sep[t], r)].push_back((int32_t)r);
}

// Row-level counting (definition of the join size as the number of agreeing
// row combinations, Eq. 3).  down(t,r): completions of the subtree of t given
// row r.  up(t,r): completions of the rest of the tree given row r of t.
void count(State& s) {
  int n = s.n;
  s.down.assign(n, {});
  s.up.assign(n, {});
  s.sumdown.assign(n, {});
  s.upval.assign(n, {});
  for (int t = n - 1; t >= 0; --t) {
    s.down[t].assign(s.N[t], 0);
    for (int64_t r = 0; r < s.N[t]; ++r) {
      i128 d = 1;
      for (int ch : s.children[t]) {
        auto it = s.sumdown[ch].find(s.key(t, s.pcol[ch], r));
        d = smul(d, it == s.sumdown[ch].end() ? 0 : it->second);
      }
      s.down[t][r] = d;
    }
    if (t > 0)
      for (int64_t r = 0; r < s.N[t]; ++r) {
        i128& acc = s.sumdown[t][s.key(t, s.sep[t], r)];
        acc = sadd(acc, s.down[t][r]);
      }
  }
  s.Q = 0;
  for (int64_t r = 0; r < s.N[0]; ++r) s.Q = sadd(s.Q, s.down[0][r]);
  s.up[0].assign(s.N[0], 1);
  for (int t = 1; t < n; ++t) {
    int p = s.par[t];
    for (int64_t r = 0; r < s.N[p]; ++r) {
      i128 term = s.up[p][r];
      for (int sib : s.children[p]) {
        if (sib == t) continue;
        auto it = s.sumdown[sib].find(s.key(p, s.pcol[sib], r));
        term = smul(term, it == s.sumdown[sib].end() ? 0 : it->second);
      }
      i128& acc = s.upval[t][s.key(p, s.pcol[t], r)];
      acc = sadd(acc, term);
    }
    s.up[t].assign(s.N[t], 0);
    for (int64_t r = 0; r < s.N[t]; ++r) {
      auto it = s.upval[t].find(s.key(t, s.sep[t], r));
      s.up[t][r] = it == s.upval[t].end() ? 0 : it->second;
    }
  }
}

i128 lookup(const std::unordered_map<int32_t, i128>& m, int32_t v) {
  auto it = m.find(v);
  return it == m.end() ? 0 : it->second;
}

// Group-by count of table t: distinct key tuples (in canonical column order)
// -> ascending row list.  std::map orders the tuples lexicographically as
// signed int32.
std::map<std::vector<int32_t>, std::vector<int32_t>> group_by(const State& s, int t) {
  std::map<std::vector<int32_t>, std::vector<int32_t>> g;
  for (int64_t r = 0; r < s.N[t]; ++r) g[s.canon_key(t, r)].push_back((int32_t)r);
  return g;
}

// The same group-by as a sorted row list: the rows of t sorted by (key tuple
// in canonical column order, row id), split where the key tuple changes.
// Group g is rows[start[g] .. start[g+1]); its key is that of any of its rows.
struct SortedGroups {
  std::vector<int32_t> rows;
  std::vector<int64_t> start;  // groups + 1
};
SortedGroups sorted_groups(const State& s, int t) {
  SortedGroups g;
  const std::vector<int> cc = s.canon_cols(t);
  auto less_key = [&](int32_t a, int32_t b) {
    for (int c : cc) {
      const int32_t x = s.key(t, c, a), y = s.key(t, c, b);
      if (x != y) return x < y;
    }
    return false;
  };
  g.rows.resize(s.N[t]);
  std::iota(g.rows.begin(), g.rows.end(), 0);
  std::sort(g.rows.begin(), g.rows.end(), [&](int32_t a, int32_t b) { return less_key(a, b) || (!less_key(b, a) && a < b); });
  for (int64_t i = 0; i < s.N[t]; ++i)
    if (i == 0 || less_key(g.rows[i - 1], g.rows[i])) g.start.push_back(i);
  g.start.push_back(s.N[t]);
  return g;
}

// Sort key of a result tuple: attribute values in result-column order, then
// the row ids in table order.
std::vector<int64_t> tuple_sort_key(const State& s, const int32_t* rows) {
  std::vector<int64_t> k;
  for (int t = 0; t < s.n; ++t)
    for (int c : s.sigma_cols(t)) k.push_back(s.key(t, c, rows[t]));
  for (int t = 0; t < s.n; ++t) k.push_back(rows[t]);
  return k;
}

struct Emitter {
  int32_t* out;
  int64_t limit, count = 0;
  int n;
  bool emit(const std::vector<int32_t>& rows) {
    if (count >= limit) return false;
    if (out)
      for (int t = 0; t < n; ++t) out[count * n + t] = rows[t];
    ++count;
    return count < limit;
  }
};

// Hash-join DFS in table order: the rows of t that agree with the chosen row of
// its parent on the separator.
bool dfs(const State& s, int t, std::vector<int32_t>& rows, Emitter& em) {
  if (t == s.n) return em.emit(rows);
  if (t == 0) {
    for (int64_t r = 0; r < s.N[0]; ++r) {
      rows[0] = (int32_t)r;
      if (!dfs(s, 1, rows, em)) return false;
    }
    return true;
  }
  auto it = s.by_sep[t].find(s.key(s.par[t], s.pcol[t], rows[s.par[t]]));
  if (it == s.by_sep[t].end()) return true;
  for (int32_t r : it->second) {
    rows[t] = r;
    if (!dfs(s, t + 1, rows, em)) return false;
  }
  return true;
}

// Candidate entries of table t below the chosen prefix: rows whose separator
// matches the parent's chosen row, grouped by key tuple (canonical order).
// For the root these are all its rows; that grouping is kept in the state.
typedef std::map<std::vector<int32_t>, std::vector<int32_t>> Groups;
const Groups& candidates(State& s, int t, const std::vector<int32_t>& rep, Groups& scratch) {
  if (t == 0) {
    if (!s.root_grouped) {
      const SortedGroups g = sorted_groups(s, 0);
      for (size_t x = 0; x + 1 < g.start.size(); ++x)
        s.root_groups.emplace_hint(s.root_groups.end(), s.canon_key(0, g.rows[g.start[x]]),
                                   std::vector<int32_t>(g.rows.begin() + g.start[x], g.rows.begin() + g.start[x + 1]));
      s.root_grouped = true;
    }
    return s.root_groups;
  }
  scratch.clear();
  auto it = s.by_sep[t].find(s.key(s.par[t], s.pcol[t], rep[s.par[t]]));
  if (it == s.by_sep[t].end()) return scratch;
  for (int32_t r : it->second) scratch[s.canon_key(t, r)].push_back(r);
  return scratch;
}

// Number of result tuples whose value groups for tables 0..t are fixed to
// `groups` (rep[i] is any row of group i): the product of the group sizes,
// times the completions of every subtree hanging below the fixed tables.
i128 prefix_count(const State& s, int t, const std::vector<int64_t>& gsize, const std::vector<int32_t>& rep) {
  i128 c = 1;
  for (int i = 0; i <= t; ++i) c = smul(c, gsize[i]);
  c = smul(c, s.down[t][rep[t]]);  // children of t
  for (int j = t + 1; j < s.n; ++j) {
    int p = s.par[j];
    if (p < t) c = smul(c, lookup(s.sumdown[j], s.key(p, s.pcol[j], rep[p])));
  }
  return c;
}

}  // namespace

extern "C" {

void* orc_open(const orc_query* q) {
  State* s = new State();
  load(*s, q);
  count(*s);
  return s;
}
void orc_close(void* h) { delete (State*)h; }

// Join size; returns 0, or 3 when it does not fit below 2^63-1 (overflow).
int orc_join_size(void* h, int64_t* out) {
  State& s = *(State*)h;
  *out = to64(s.Q);
  return s.Q >= I64MAX ? 3 : 0;
}

// Factor (potential) of table t: distinct key tuples in canonical entry order,
// keys written in *declared* column order (row-major, M x K[t]), their counts,
// first position in the grouped row list, and the grouped row list itself.
int64_t orc_factor(void* h, int t, int32_t* keys, int64_t* cnt, int64_t* start, int32_t* perm) {
  State& s = *(State*)h;
  const SortedGroups g = sorted_groups(s, t);
  const int64_t M = (int64_t)g.start.size() - 1;
  for (int64_t e = 0; e < M; ++e) {
    const int32_t r0 = g.rows[g.start[e]];
    if (keys)
      for (int c = 0; c < s.K[t]; ++c) keys[e * s.K[t] + c] = s.key(t, c, r0);
    if (cnt) cnt[e] = g.start[e + 1] - g.start[e];
    if (start) start[e] = g.start[e];
  }
  if (perm) std::copy(g.rows.begin(), g.rows.end(), perm);
  return M;
}

// Surviving entries of table t (frequency in the result F > 0) with
// c = rows in the group, U = completions below (down of any of its rows),
// D = completions outside (up), F = sum of the rows' fan-outs.
int64_t orc_summary_table(void* h, int t, int32_t* keys, int64_t* c, int64_t* U, int64_t* D, int64_t* F) {
  State& s = *(State*)h;
  const SortedGroups g = sorted_groups(s, t);
  const int64_t M = (int64_t)g.start.size() - 1;
  int64_t e = 0;
  for (int64_t x = 0; x < M; ++x) {
    i128 f = 0;
    for (int64_t i = g.start[x]; i < g.start[x + 1]; ++i) f = sadd(f, smul(s.down[t][g.rows[i]], s.up[t][g.rows[i]]));
    if (f == 0) continue;
    const int32_t r0 = g.rows[g.start[x]];
    if (keys)
      for (int cc = 0; cc < s.K[t]; ++cc) keys[e * s.K[t] + cc] = s.key(t, cc, r0);
    if (c) c[e] = g.start[x + 1] - g.start[x];
    if (U) U[e] = to64(s.down[t][r0]);
    if (D) D[e] = to64(s.up[t][r0]);
    if (F) F[e] = to64(f);
    ++e;
  }
  return e;
}

// Edge into table t >= 1: every separator value s with M(s) = completions of
// t's subtree over rows carrying s, and D(s) = completions outside it; only
// values with M*D > 0, ascending.
int64_t orc_summary_edge(void* h, int t, int32_t* sv, int64_t* M, int64_t* D) {
  State& s = *(State*)h;
  std::map<int32_t, std::pair<i128, i128>> m;
  for (auto& kv : s.sumdown[t]) {
    i128 d = lookup(s.upval[t], kv.first);
    if (kv.second > 0 && d > 0) m[kv.first] = {kv.second, d};
  }
  int64_t e = 0;
  for (auto& kv : m) {
    if (sv) sv[e] = kv.first;
    if (M) M[e] = to64(kv.second.first);
    if (D) D[e] = to64(kv.second.second);
    ++e;
  }
  return e;
}

// Per-row fan-out of table t: number of result tuples that contain row r.
void orc_fanouts(void* h, int t, int64_t* out) {
  State& s = *(State*)h;
  for (int64_t r = 0; r < s.N[t]; ++r) out[r] = to64(smul(s.down[t][r], s.up[t][r]));
}

// Join result by hash-join DFS, first `limit` tuples in DFS order
// (lexicographic by row ids); returns the number written.
int64_t orc_materialize(void* h, int64_t limit, int32_t* out) {
  State& s = *(State*)h;
  Emitter em{out, limit, 0, s.n};
  std::vector<int32_t> rows(s.n);
  if (limit > 0 && s.n > 0) dfs(s, 0, rows, em);
  return em.count;
}

// The same DFS with the root's rows restricted to [lo, hi): the result
// tuples whose root row lies in that range, first `limit` of them in DFS
// order. Disjoint ranges give disjoint parts of the result (so threads can
// expand them side by side); [0, N_0) is orc_materialize.
int64_t orc_materialize_range(void* h, int64_t lo, int64_t hi, int64_t limit, int32_t* out) {
  State& s = *(State*)h;
  Emitter em{out, limit, 0, s.n};
  if (limit <= 0 || s.n == 0) return 0;
  std::vector<int32_t> rows(s.n);
  lo = std::max<int64_t>(lo, 0);
  hi = std::min<int64_t>(hi, s.N[0]);
  for (int64_t r = lo; r < hi; ++r) {
    rows[0] = (int32_t)r;
    if (!dfs(s, 1, rows, em)) break;
  }
  return em.count;
}

// Join result by an all-combinations nested loop (tiny inputs only): every
// combination of one row per table, kept when it agrees on every edge.
int64_t orc_brute_force(void* h, int64_t limit, int32_t* out) {
  State& s = *(State*)h;
  int n = s.n;
  for (int t = 0; t < n; ++t)
    if (s.N[t] == 0) return 0;
  std::vector<int32_t> rows(n, 0);
  Emitter em{out, limit, 0, n};
  while (true) {
    bool ok = true;
    for (int t = 1; t < n && ok; ++t)
      ok = s.key(t, s.sep[t], rows[t]) == s.key(s.par[t], s.pcol[t], rows[s.par[t]]);
    if (ok && !em.emit(rows)) break;
    int t = n - 1;
    while (t >= 0 && ++rows[t] == s.N[t]) rows[t--] = 0;
    if (t < 0) break;
  }
  return em.count;
}

// Sort result tuples (row-major, count x n) by all attribute values, then row ids.
void orc_sort_canonical(void* h, int32_t* tuples, int64_t count) {
  State& s = *(State*)h;
  int n = s.n;
  std::vector<std::vector<int64_t>> keys(count);
  for (int64_t i = 0; i < count; ++i) keys[i] = tuple_sort_key(s, tuples + i * n);
  std::vector<int64_t> idx(count);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  std::vector<int32_t> tmp(tuples, tuples + count * n);
  for (int64_t i = 0; i < count; ++i)
    for (int t = 0; t < n; ++t) tuples[i * n + t] = tmp[idx[i] * n + t];
}

// Checks result tuples (row-major, count x n row ids, int64) against the
// definition of the sorted result: every row id is a row of its table, every
// tuple agrees on every join edge (Sec. 1.1), and every tuple comes strictly
// after the one before it in the result order (attribute values in
// result-column order, then the row ids; Definition 1).  The tuples are split
// over `threads` threads.  Returns -1 if all pass, else the index of the first
// tuple that fails.
int64_t orc_check_tuples(void* h, const int64_t* tuples, int64_t count, int threads) {
  State& s = *(State*)h;
  const int n = s.n;
  std::vector<std::pair<int, int>> cols;  // (table, column) of every result column
  for (int t = 0; t < n; ++t)
    for (int c : s.sigma_cols(t)) cols.push_back({t, c});
  auto valid = [&](const int64_t* r) {
    for (int t = 0; t < n; ++t)
      if (r[t] < 0 || r[t] >= s.N[t]) return false;
    for (int t = 1; t < n; ++t)
      if (s.key(t, s.sep[t], r[t]) != s.key(s.par[t], s.pcol[t], r[s.par[t]])) return false;
    return true;
  };
  auto before = [&](const int64_t* a, const int64_t* b) {  // a strictly before b
    for (auto& tc : cols) {
      const int32_t x = s.key(tc.first, tc.second, a[tc.first]), y = s.key(tc.first, tc.second, b[tc.first]);
      if (x != y) return x < y;
    }
    for (int t = 0; t < n; ++t)
      if (a[t] != b[t]) return a[t] < b[t];
    return false;
  };
  if (threads < 1) threads = 1;
  std::vector<int64_t> first_bad(threads, -1);
  auto work = [&](int id) {
    const int64_t lo = count * id / threads, hi = count * (id + 1) / threads;
    for (int64_t i = lo; i < hi; ++i) {
      const int64_t* r = tuples + i * n;
      // the tuple before a range's first belongs to another range: its row
      // ids are checked here before they index the tables
      if (!valid(r) || (i > 0 && ((i == lo && !valid(r - n)) || !before(r - n, r)))) {
        first_bad[id] = i;
        return;
      }
    }
  };
  std::vector<std::thread> th;
  for (int i = 0; i < threads; ++i) th.emplace_back(work, i);
  for (auto& x : th) x.join();
  for (int64_t b : first_bad)
    if (b >= 0) return b;
  return -1;
}

// Value of result column `level` (attribute values in result-column order).
int orc_n_levels(void* h) {
  State& s = *(State*)h;
  int L = 0;
  for (int t = 0; t < s.n; ++t) L += (int)s.sigma_cols(t).size();
  return L;
}

// The GFJS of Definition 1 over sorted tuples: for every result column i, one
// (value, frequency) pair per run of equal values *within a run of equal
// values of columns 0..i-1* (per distinct prefix, as the recursive generator
// emits them).  Writes level-major into vals/freqs (capacity count per level)
// and the run count of each level into nruns.
void orc_gfjs(void* h, const int32_t* tuples, int64_t count, int32_t* vals, int64_t* freqs, int64_t* nruns) {
  State& s = *(State*)h;
  int n = s.n;
  std::vector<std::pair<int, int>> lv;  // (table, column) per level
  for (int t = 0; t < n; ++t)
    for (int c : s.sigma_cols(t)) lv.push_back({t, c});
  int L = (int)lv.size();
  for (int i = 0; i < L; ++i) {
    int64_t k = -1;
    for (int64_t r = 0; r < count; ++r) {
      bool same = r > 0;
      for (int j = 0; j <= i && same; ++j) {
        int32_t a = s.key(lv[j].first, lv[j].second, tuples[r * n + lv[j].first]);
        int32_t b = s.key(lv[j].first, lv[j].second, tuples[(r - 1) * n + lv[j].first]);
        same = a == b;
      }
      if (!same) {
        ++k;
        vals[(int64_t)i * count + k] = s.key(lv[i].first, lv[i].second, tuples[r * n + lv[i].first]);
        freqs[(int64_t)i * count + k] = 0;
      }
      freqs[(int64_t)i * count + k] += 1;
    }
    nruns[i] = k + 1;
  }
}

// The result tuple of rank R in the sorted result.  Walks the tables in order,
// choosing the value group of each from the counts of the tuples below every
// candidate; the row ids are then the mixed-radix digits of the remainder
// (table 0 most significant).  Returns 0, or 6 if R is out of range.
int orc_unrank(void* h, int64_t R, int32_t* tuple) {
  State& s = *(State*)h;
  if (R < 0 || (i128)R >= s.Q) return 6;
  int n = s.n;
  i128 rem = R;
  std::vector<int32_t> rep(n);
  std::vector<int64_t> gsize(n);
  std::vector<std::vector<int32_t>> grows(n);
  Groups scratch;
  for (int t = 0; t < n; ++t) {
    const Groups& cand = candidates(s, t, rep, scratch);
    bool found = false;
    for (auto& kv : cand) {
      rep[t] = kv.second[0];
      gsize[t] = (int64_t)kv.second.size();
      i128 c = prefix_count(s, t, gsize, rep);
      if (rem < c) {
        grows[t] = kv.second;
        found = true;
        break;
      }
      rem -= c;
    }
    if (!found) return 6;
  }
  for (int t = n - 1; t >= 0; --t) {
    tuple[t] = grows[t][(int64_t)(rem % gsize[t])];
    rem /= gsize[t];
  }
  return 0;
}

// Rank of a result tuple in the sorted result (inverse of orc_unrank).
// Returns 0, or 2 if the tuple is not in the join result.
int orc_rank(void* h, const int32_t* tuple, int64_t* R) {
  State& s = *(State*)h;
  int n = s.n;
  for (int t = 1; t < n; ++t)
    if (s.key(t, s.sep[t], tuple[t]) != s.key(s.par[t], s.pcol[t], tuple[s.par[t]])) return 2;
  i128 rank = 0;
  std::vector<int32_t> rep(n);
  std::vector<int64_t> gsize(n);
  std::vector<int64_t> pos(n);
  Groups scratch;
  for (int t = 0; t < n; ++t) {
    const Groups& cand = candidates(s, t, rep, scratch);
    std::vector<int32_t> mine = s.canon_key(t, tuple[t]);
    for (auto& kv : cand) {
      rep[t] = kv.second[0];
      gsize[t] = (int64_t)kv.second.size();
      if (kv.first == mine) {
        pos[t] = std::find(kv.second.begin(), kv.second.end(), tuple[t]) - kv.second.begin();
        break;
      }
      rank += prefix_count(s, t, gsize, rep);
    }
  }
  i128 rr = 0;
  for (int t = 0; t < n; ++t) rr = rr * gsize[t] + pos[t];
  rank += rr;
  *R = to64(rank);
  return 0;
}

// ---------------------------------------------------------------------------
// Early projections (Sec. 3.7): only some attributes are output attributes.
// The projected result is the bag of the join result's tuples restricted to
// the output attributes (every tuple keeps its multiplicity).
//
// mask[t] bit c marks key column c of table t as an output attribute.  A join
// attribute is a single attribute seen from the two tables of its edge, so a
// mark on either side counts for both.  A table is kept in the projected
// generator if it has an output attribute besides its separator (the root: any
// output attribute) or a kept child; every other table is deleted, i.e. only
// its completions count.  Supported when the root is kept and every kept
// non-root table's separator is an output attribute (otherwise two kept tables
// would be linked through a summed-out variable).
// Returns 0 and the normalized mask in `out`, or -1 if unsupported.
// ---------------------------------------------------------------------------
int orc_projection(void* h, const uint32_t* mask, uint32_t* out, int32_t* kept) {
  State& s = *(State*)h;
  int n = s.n;
  std::vector<uint32_t> m(mask, mask + n);
  for (int t = 1; t < n; ++t) {
    bool mark = ((m[t] >> s.sep[t]) & 1u) || ((m[s.par[t]] >> s.pcol[t]) & 1u);
    if (mark) {
      m[t] |= 1u << s.sep[t];
      m[s.par[t]] |= 1u << s.pcol[t];
    }
  }
  std::vector<int32_t> k(n, 0);
  for (int t = n - 1; t >= 0; --t) {
    uint32_t own = t == 0 ? m[t] : (m[t] & ~(1u << s.sep[t]));
    k[t] = own != 0;
    for (int ch : s.children[t]) k[t] |= k[ch];
  }
  if (out) std::copy(m.begin(), m.end(), out);
  if (kept) std::copy(k.begin(), k.end(), kept);
  if (n == 0 || !k[0] || m[0] == 0) return -1;
  for (int t = 1; t < n; ++t)
    if (k[t] && !((m[t] >> s.sep[t]) & 1u)) return -1;
  return 0;
}

// Projected entries of kept table t: the distinct values of its output
// columns (the separator first, then the others in declared order), each with
//   c = sum over the rows with those values of the product, over the deleted
//       children, of the completions of the child's subtree at the row's value,
//   U = product of the kept children's messages at the entry's values,
//   D = completions outside t's subtree (1 at the root),
//   F = sum of the rows' fan-outs = the number of result tuples whose t-part
//       projects to the entry.
// Only entries with F > 0.  Keys are written in declared order of the output
// columns (row-major, entries x output columns).  Returns the entry count,
// -1 if the projection is unsupported, -2 if t is deleted.
int64_t orc_projected_table(void* h, const uint32_t* mask, int t, int32_t* keys, int64_t* c, int64_t* U, int64_t* D,
                            int64_t* F) {
  State& s = *(State*)h;
  int n = s.n;
  std::vector<uint32_t> m(n);
  std::vector<int32_t> kept(n);
  if (orc_projection(h, mask, m.data(), kept.data()) != 0) return -1;
  if (!kept[t]) return -2;
  std::vector<int> ocols;  // sort order: separator, then the others in declared order
  if (t > 0) ocols.push_back(s.sep[t]);
  for (int cc = 0; cc < s.K[t]; ++cc)
    if (((m[t] >> cc) & 1u) && (t == 0 || cc != s.sep[t])) ocols.push_back(cc);
  std::vector<int> declared;
  for (int cc = 0; cc < s.K[t]; ++cc)
    if ((m[t] >> cc) & 1u) declared.push_back(cc);
  struct Acc {
    i128 c = 0, f = 0;
    int32_t rep = 0;
  };
  std::map<std::vector<int32_t>, Acc> g;
  for (int64_t r = 0; r < s.N[t]; ++r) {
    std::vector<int32_t> key;
    for (int cc : ocols) key.push_back(s.key(t, cc, r));
    i128 w = 1;
    for (int ch : s.children[t])
      if (!kept[ch]) w = smul(w, lookup(s.sumdown[ch], s.key(t, s.pcol[ch], r)));
    Acc& a = g[key];
    if (a.c == 0 && a.f == 0) a.rep = (int32_t)r;
    a.c = sadd(a.c, w);
    a.f = sadd(a.f, smul(s.down[t][r], s.up[t][r]));
  }
  int64_t e = 0;
  for (auto& kv : g) {
    if (kv.second.f == 0) continue;
    int32_t r0 = kv.second.rep;
    i128 u = 1;
    for (int ch : s.children[t])
      if (kept[ch]) u = smul(u, lookup(s.sumdown[ch], s.key(t, s.pcol[ch], r0)));
    if (keys)
      for (size_t i = 0; i < declared.size(); ++i) keys[e * (int64_t)declared.size() + i] = s.key(t, declared[i], r0);
    if (c) c[e] = to64(kv.second.c);
    if (U) U[e] = to64(u);
    if (D) D[e] = to64(s.up[t][r0]);
    if (F) F[e] = to64(kv.second.f);
    ++e;
  }
  return e;
}

// ---------------------------------------------------------------------------
// Weighted join size W = sum over result tuples of the product of their row
// weights, and dW/dw_r, in __float128.  With all weights 1, W is the join size.
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

struct WCounts {
  std::vector<std::vector<f128>> down, up;
  std::vector<std::unordered_map<int32_t, f128>> sum, upv;
  f128 W = 0;
};

f128 wlook(const std::unordered_map<int32_t, f128>& m, int32_t v) {
  auto it = m.find(v);
  return it == m.end() ? 0 : it->second;
}

// down(t,r) = w_r * prod over children of the summed weights of the matching
// subtrees; W = sum over root rows.  `w` holds per-table weight arrays.
void wcount(const State& s, const std::vector<std::vector<f128>>& w, WCounts& o, bool with_up) {
  int n = s.n;
  o.down.assign(n, {});
  o.sum.assign(n, {});
  for (int t = n - 1; t >= 0; --t) {
    o.down[t].assign(s.N[t], 0);
    for (int64_t r = 0; r < s.N[t]; ++r) {
      f128 d = w[t][r];
      for (int ch : s.children[t]) d *= wlook(o.sum[ch], s.key(t, s.pcol[ch], r));
      o.down[t][r] = d;
    }
    if (t > 0)
      for (int64_t r = 0; r < s.N[t]; ++r) o.sum[t][s.key(t, s.sep[t], r)] += o.down[t][r];
  }
  o.W = 0;
  for (int64_t r = 0; r < s.N[0]; ++r) o.W += o.down[0][r];
  if (!with_up) return;
  o.up.assign(n, {});
  o.upv.assign(n, {});
  o.up[0].assign(s.N[0], 1);
  for (int t = 1; t < n; ++t) {
    int p = s.par[t];
    for (int64_t r = 0; r < s.N[p]; ++r) {
      f128 term = o.up[p][r] * w[p][r];
      for (int sib : s.children[p])
        if (sib != t) term *= wlook(o.sum[sib], s.key(p, s.pcol[sib], r));
      o.upv[t][s.key(p, s.pcol[t], r)] += term;
    }
    o.up[t].assign(s.N[t], 0);
    for (int64_t r = 0; r < s.N[t]; ++r) o.up[t][r] = wlook(o.upv[t], s.key(t, s.sep[t], r));
  }
}

std::vector<std::vector<f128>> wload(const State& s, const double* const* w) {
  std::vector<std::vector<f128>> v(s.n);
  for (int t = 0; t < s.n; ++t) {
    v[t].resize(s.N[t]);
    for (int64_t r = 0; r < s.N[t]; ++r) v[t][r] = w ? (f128)w[t][r] : (f128)1;
  }
  return v;
}

}  // namespace

extern "C" {

// W and every dW/dw_r (rounded to double).  grad[t] may be NULL to skip a table.
double orc_weighted(void* h, const double* const* w, double* const* grad) {
  State& s = *(State*)h;
  auto wv = wload(s, w);
  WCounts o;
  wcount(s, wv, o, grad != nullptr);
  if (grad)
    for (int t = 0; t < s.n; ++t) {
      if (!grad[t]) continue;
      for (int64_t r = 0; r < s.N[t]; ++r) {
        f128 below = 1;  // product of the children's summed weights
        for (int ch : s.children[t]) below *= wlook(o.sum[ch], s.key(t, s.pcol[ch], r));
        grad[t][r] = (double)(below * o.up[t][r]);
      }
    }
  return (double)o.W;
}

// Central finite differences (W(w + h e_r) - W(w - h e_r)) / (2h) with
// h = hfrac * w_r, each W recomputed from scratch in __float128, for the rows
// `rows` of table t.  W is multilinear in each weight, so the difference
// quotient has no truncation error.  Runs on `threads` CPU threads.
void orc_weighted_fd(void* h, const double* const* w, int t, const int64_t* rows, int64_t nrows,
                     double hfrac, int threads, double* out) {
  State& s = *(State*)h;
  auto base = wload(s, w);
  if (threads < 1) threads = 1;
  auto work = [&](int tid) {
    auto wv = base;
    WCounts o;
    for (int64_t i = tid; i < nrows; i += threads) {
      int64_t r = rows[i];
      f128 w0 = base[t][r];
      f128 hh = (f128)hfrac * w0;
      wv[t][r] = w0 + hh;
      wcount(s, wv, o, false);
      f128 wp = o.W;
      wv[t][r] = w0 - hh;
      wcount(s, wv, o, false);
      f128 wm = o.W;
      wv[t][r] = w0;
      out[i] = (double)((wp - wm) / (2 * hh));
    }
  };
  std::vector<std::thread> th;
  for (int i = 0; i < threads; ++i) th.emplace_back(work, i);
  for (auto& x : th) x.join();
}

}  // extern "C"
