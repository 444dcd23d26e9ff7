// Host-side plan of a set of tables (one query or a batch of queries) and the
// device buffers of its factors / summaries.
#pragma once
#include <string>
#include <vector>

#include "gj_internal.h"

struct gj_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  gj_alloc_fn alloc = nullptr;
  gj_free_fn free_fn = nullptr;
  void* user = nullptr;
  gj_tune tune{};
  std::string err;  // message of the last failed call made with this context
};

namespace gjh {

// Records a failure message: on the calling thread, and on the context of the
// entry point running on this thread (if it has one, see CtxScope).
void set_error(const char* fmt, ...);

// Names the context of the entry point running on this thread for as long as
// the scope lives, so that set_error records on it.
struct CtxScope {
  gj_ctx* prev;
  explicit CtxScope(const gj_ctx* c);
  ~CtxScope();
};
#define GJ_SCOPE(c) gjh::CtxScope gj_scope_((c))

// A device allocation made through the context's allocator.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

class Arena {
 public:
  explicit Arena(gj_ctx* c) : ctx(c) {}
  ~Arena() { release(); }
  // returns nullptr on failure (error already set)
  void* get(size_t bytes);
  template <typename T>
  T* get_n(int64_t n) {
    return reinterpret_cast<T*>(get((size_t)std::max<int64_t>(n, 1) * sizeof(T)));
  }
  void release();
  gj_ctx* ctx;
  std::vector<Buf> bufs;
};

struct HTable {
  int64_t n = 0;
  int k = 0;
  const int32_t* cols[MAXK] = {};
  int parent = -1;  // global index
  int sep = 0, pcol = 0;
  int query = 0, local = 0;
  std::vector<int> children;  // global indices, ascending
  int depth = 0, height = 0;
};

struct WL {
  int off = 0, n = 0;  // range in the work-item array
  int toff = 0, tn = 0;  // range in the table-id array
};

struct Plan {
  gj_ctx* ctx = nullptr;
  int nq = 0, nt = 0;
  std::vector<int> qfirst;  // nq + 1
  std::vector<HTable> ht;
  std::vector<TDesc> td;
  int64_t S = 0, key_slots = 0, link_slots = 0, agg_slots = 0, hist_slots = 0, word_units = 0, didx_slots = 0;
  int max_height = 0, max_depth = 0, max_passes = 0;
  // work lists
  std::vector<WorkItem> wl_host;
  std::vector<int32_t> tabs_host;
  WL all;                    // GJ_TILE tiles of every table
  WL allw[2];                // the same, split by sort-word width
  std::vector<WL> sort[2];   // [wide][pass]
  std::vector<WL> up;        // [height]
  std::vector<WL> down;      // [depth]: parents at depth-1 that have children
  std::vector<WL> dred;      // [depth]: (child at depth, slice) items of the bucket sums
  std::vector<char> dfall;   // [depth]: a child at this depth takes the atomic scatter
  std::vector<char> dbuck;   // [depth]: a child at this depth is summed by buckets
  int64_t dhist_slots = 0;
  WorkItem* d_wl = nullptr;
  int32_t* d_tabs = nullptr;
  TDesc* d_desc = nullptr;
  int sort_items[2] = {16, 8};
  int radix_bits = 8;
  // bucket passes + in-LDS sort for 128-bit-word tables of at least
  // local_rows rows (0: never; set only where the build may wait for the host)
  bool allow_local = false;
  int64_t local_rows = 0;
  WL local;                  // GJ_LOCAL_TILE tiles of those tables
  std::vector<WL> local_full;  // per such table: its sort tiles, for the full sort
  std::vector<int8_t> sort_kind;  // per table: 0 per-digit passes, 1 bucket sort, 2 bucket sort redone in full

  WL add_list(const std::vector<int>& tables, int tile, bool sort_tiles);
};

// Validates `nq` graphs; fills the host tables of the plan (no device work).
gj_status plan_tables(Plan& P, int nq, const int* q_off, const gj_table* tables, const gj_join_graph* graphs);
// Assigns slots, reads the key ranges on the device (one synchronization),
// picks the sort-word layout, builds the work lists and uploads everything.
gj_status plan_device(Plan& P, Arena& A, FPtrs& F);
// Factor build kernels (asynchronous, capturable).
void launch_factors(const Plan& P, const FPtrs& F, hipStream_t s);
// Summary kernels (asynchronous, capturable).
void launch_summary(const Plan& P, const FPtrs& F, const SPtrs& S, hipStream_t s);
gj_status alloc_summary(const Plan& P, Arena& A, SPtrs& S);
// Joint potential of several factors (pjoin.hip): n entries over nv
// variables, keys SoA with `stride` per variable, ascending, and frequencies.
struct PotentialOut {
  int64_t n = 0;
  int nv = 0;
  int64_t stride = 1;
  int32_t* keys = nullptr;
  int64_t* freq = nullptr;
};
// Tables with their bit set in `indicator` only filter: their frequency is
// counted in another clique's potential.
gj_status potential_join(gj_ctx* ctx, const gj_factors* f, const std::vector<int>& tabs,
                         const std::vector<std::vector<int>>& tvar, int nv, Arena& A, PotentialOut& out,
                         uint32_t indicator = 0);
// Factors of single-table queries with columns ordered by attribute id (pjoin.hip).
gj_status sorted_factors(gj_ctx* ctx, int n, const gj_table* tables, const gj_natural_query* q,
                         std::vector<int32_t>& vars, std::vector<std::vector<int>>& tvar, gj_factors** out);
// Host copy of the plan's device counters (synchronizes the stream).
gj_status read_counters(const Plan& P, const FPtrs& F, hipStream_t s, std::vector<int64_t>& out);
// Makes a summary's host-side state (entry counts, join size) current: reads
// it with one synchronization if it was computed without a read-back.
// GJ_E_OVERFLOW if the summary's query overflowed.
gj_status summary_host(const gj_summary* s);

gj_status check(hipError_t e, const char* what);

}  // namespace gjh

struct gj_factors {
  gj_ctx* ctx = nullptr;
  gjh::Plan plan;
  gjh::Arena arena;
  FPtrs F{};
  std::vector<int64_t> cnt_host;  // host copy of the counters
  int64_t* ecount = nullptr;       // per entry slot: frequency (filled on the first view)
  int refs = 1;
  explicit gj_factors(gj_ctx* c) : ctx(c), arena(c) {}
};

struct gj_summary {
  gj_ctx* ctx = nullptr;
  gj_factors* f = nullptr;
  gjh::Arena arena;
  SPtrs S{};
  int query = 0;        // which query of the plan this summary describes
  bool borrowed = false;  // part of a batch: not freed by gj_free_summary
  std::vector<int64_t> cnt_host;
  int64_t join_size = 0;
  // computed without reading anything back (gj_summarize_batch): cnt_host,
  // join_size and status are read on first use (gjh::summary_host)
  bool host_stale = false;
  int32_t status = GJ_OK;
  bool projected = false;  // entries over output attributes only: no row ids
  // result columns (table, key column) and their attribute ids when they are
  // not "the root's columns, then every other table's non-separator columns"
  std::vector<std::pair<int, int>> result_cols;
  std::vector<int32_t> result_attr;
  explicit gj_summary(gj_ctx* c) : ctx(c), arena(c) {}
};

// Value columns re-laid out in a factor's grouped row order.
struct gj_colset {
  gj_ctx* ctx = nullptr;
  gj_factors* f = nullptr;  // holds a reference
  int query = 0;
  gjh::Arena arena;
  int n_cols = 0;
  int tab[GJ_MAX_OUT_COLS] = {};
  int32_t* col[GJ_MAX_OUT_COLS] = {};
  explicit gj_colset(gj_ctx* c) : ctx(c), arena(c) {}
};
