// Graphical Join -- CPU ORACLE for natural joins over named attributes,
// cyclic ones included.  TEST INFRASTRUCTURE ONLY: only the test-suite may
// load it; the product library never does, and it shares no code with the
// HIP path.
//
// A query is a set of tables whose key columns carry attribute ids; the
// natural join (Sec. 1.1) is every combination of one row per table such
// that all columns carrying the same attribute hold the same value.  Nothing
// here follows the paper's algorithms: the result is enumerated by
// backtracking over the tables in order, each table's candidate rows found in
// a hash index on the columns whose attributes earlier tables have bound, and
// (for tiny inputs) by an all-combinations nested loop.
#include <algorithm>
#include <array>
#include <cstdint>
#include <map>
#include <unordered_map>
#include <vector>

namespace {

struct VecHash {
  size_t operator()(const std::vector<int32_t>& v) const {
    uint64_t h = 1469598103934665603ull;
    for (int32_t x : v) {
      h ^= (uint32_t)x;
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

struct Nat {
  int n = 0;
  std::vector<int64_t> N;
  std::vector<std::vector<const int32_t*>> col;
  std::vector<std::vector<int32_t>> attr;
  // bound[t]: (column of t, earlier table, its column) for attributes bound before t
  std::vector<std::vector<std::array<int, 3>>> bound;
  std::vector<std::unordered_map<std::vector<int32_t>, std::vector<int32_t>, VecHash>> index;
};

struct Emit {
  int32_t* out;
  int64_t limit, count = 0;
  int n;
  bool push(const std::vector<int32_t>& rows) {
    if (count >= limit) return false;
    if (out)
      for (int t = 0; t < n; ++t) out[count * n + t] = rows[t];
    ++count;
    return count < limit;
  }
};

bool dfs(const Nat& s, int t, std::vector<int32_t>& rows, Emit& em) {
  if (t == s.n) return em.push(rows);
  std::vector<int32_t> key;
  for (auto& b : s.bound[t]) key.push_back(s.col[b[1]][b[2]][rows[b[1]]]);
  auto it = s.index[t].find(key);
  if (it == s.index[t].end()) return true;
  for (int32_t r : it->second) {
    // columns of t that carry the same attribute twice must agree too
    bool ok = true;
    for (size_t i = 0; i < s.attr[t].size() && ok; ++i)
      for (size_t j = i + 1; j < s.attr[t].size() && ok; ++j)
        if (s.attr[t][i] == s.attr[t][j] && s.col[t][i][r] != s.col[t][j][r]) ok = false;
    if (!ok) continue;
    rows[t] = r;
    if (!dfs(s, t + 1, rows, em)) return false;
  }
  return true;
}

}  // namespace

extern "C" {

// cols[t * 8 + c]: int32 column c of table t; attr[t * 8 + c]: its attribute id.
void* orc_nat_open(int32_t n, const int64_t* n_rows, const int32_t* n_keys, const int32_t* const* cols,
                   const int32_t* attr) {
  Nat* s = new Nat();
  s->n = n;
  s->N.assign(n_rows, n_rows + n);
  s->col.resize(n);
  s->attr.resize(n);
  s->bound.resize(n);
  s->index.resize(n);
  std::map<int32_t, std::pair<int, int>> first;  // attribute -> first (table, column)
  for (int t = 0; t < n; ++t) {
    for (int c = 0; c < n_keys[t]; ++c) {
      s->col[t].push_back(cols[t * 8 + c]);
      s->attr[t].push_back(attr[t * 8 + c]);
    }
    for (int c = 0; c < n_keys[t]; ++c) {
      auto it = first.find(attr[t * 8 + c]);
      if (it != first.end()) s->bound[t].push_back({c, it->second.first, it->second.second});
    }
    for (int c = 0; c < n_keys[t]; ++c)
      if (!first.count(attr[t * 8 + c])) first[attr[t * 8 + c]] = {t, c};
    for (int64_t r = 0; r < s->N[t]; ++r) {
      std::vector<int32_t> key;
      for (auto& b : s->bound[t]) key.push_back(s->col[t][b[0]][r]);
      s->index[t][key].push_back((int32_t)r);
    }
  }
  return s;
}

void orc_nat_close(void* h) { delete (Nat*)h; }

// First `limit` result row combinations (row ids, row-major n per tuple) in
// backtracking order; returns the number written (out may be null: counting).
int64_t orc_nat_materialize(void* h, int64_t limit, int32_t* out) {
  Nat& s = *(Nat*)h;
  Emit em{out, limit, 0, s.n};
  std::vector<int32_t> rows(s.n);
  if (limit > 0 && s.n > 0) dfs(s, 0, rows, em);
  return em.count;
}

// All-combinations nested loop (tiny inputs): every combination of one row per
// table kept when every pair of columns with the same attribute agrees.
int64_t orc_nat_brute_force(void* h, int64_t limit, int32_t* out) {
  Nat& s = *(Nat*)h;
  int n = s.n;
  for (int t = 0; t < n; ++t)
    if (s.N[t] == 0) return 0;
  std::vector<std::pair<int, int>> cols;
  for (int t = 0; t < n; ++t)
    for (size_t c = 0; c < s.attr[t].size(); ++c) cols.push_back({t, (int)c});
  std::vector<int32_t> rows(n, 0);
  Emit em{out, limit, 0, n};
  while (true) {
    bool ok = true;
    for (size_t i = 0; i < cols.size() && ok; ++i)
      for (size_t j = i + 1; j < cols.size() && ok; ++j) {
        auto [ti, ci] = cols[i];
        auto [tj, cj] = cols[j];
        if (s.attr[ti][ci] == s.attr[tj][cj] && s.col[ti][ci][rows[ti]] != s.col[tj][cj][rows[tj]]) ok = false;
      }
    if (ok && !em.push(rows)) break;
    int t = n - 1;
    while (t >= 0 && ++rows[t] == s.N[t]) rows[t--] = 0;
    if (t < 0) break;
  }
  return em.count;
}

}  // extern "C"
