/*
 * gj.h -- C ABI of the Graphical Join hot path on AMD MI355X (gfx950).
 *
 * The library answers acyclic natural equi-join queries (Sec. 1.1 of the
 * paper: tables T_0..T_{n-1}, already filtered, joined on equal key values)
 * the Graphical Join way (Sec. 3):
 *
 *   gj_build_factors  one group-by count per table: the table's factor
 *                     (potential, Sec. 3.2) = every distinct key tuple with
 *                     its frequency, plus the row ids grouped by tuple.
 *   gj_summarize      sum-product message passing over the join tree
 *                     (Sec. 2.2 Eq. 4 / Sec. 3.3 Algorithm 2 upward, the
 *                     generation order of Sec. 3.5 Algorithms 3-4 downward):
 *                     the join size (Eq. 3's Z) and the run-length summary of
 *                     the result, i.e. for every surviving factor entry its
 *                     count c, completions below U, completions outside D and
 *                     run length F = c*U*D.
 *   gj_desummarize    materializes any row range of the join result, sorted
 *                     by all attribute values (Definition 1) with row ids as
 *                     the tie-break, as row-id tuples (Sec. 3.6).
 *
 * Conventions
 *   - "device" pointers are HIP device memory on the context's device; "host"
 *     pointers are ordinary host memory.  Every call is ordered on the
 *     context's stream; a call that returns a host value synchronizes it.
 *   - Inputs (key columns, weights) are borrowed for the duration of the call
 *     only.  Factors, summaries and saved states are owned by the library and
 *     allocated through the context's allocator; output chunks are owned by
 *     the caller.
 *   - Every entry point returns a gj_status; out-parameters are written only
 *     on GJ_OK.  gj_last_error(ctx) gives the message of the last failed call
 *     made with that context (or with an object made by it); calls that take
 *     no context (gj_validate, gj_junction_tree_build) leave theirs per thread,
 *     returned for ctx = NULL.
 *   - Join graph: table 0 is the root; for t >= 1, parent[t] < t and table t
 *     joins its parent on  key[t][sep_col[t]] == key[parent[t]][parent_col[t]].
 *     Composite separators and cyclic queries are rejected (GJ_E_GRAPH).
 *   - Counts are exact int64.  If the join size is >= 2^63-1 the call reports
 *     GJ_E_OVERFLOW (every value of the summary is bounded by the join size,
 *     so nothing else can overflow).
 */
#ifndef GJ_H
#define GJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GJ_OK = 0,
  GJ_E_INVALID = 1,  /* bad argument (null pointer, size, key too wide to pack) */
  GJ_E_GRAPH = 2,    /* join graph is not a rooted tree with one separator per edge */
  GJ_E_OVERFLOW = 3, /* join size does not fit below 2^63-1 */
  GJ_E_OOM = 4,      /* the allocator returned NULL */
  GJ_E_DEVICE = 5,   /* a HIP runtime call failed */
  GJ_E_RANGE = 6     /* first_row beyond the join size */
} gj_status;

#define GJ_MAX_TABLES 16 /* per query */
#define GJ_MAX_KEYS 8    /* key columns per table */
#define GJ_MAX_CHILDREN 8
#define GJ_MAX_OUT_COLS 16 /* value columns per materialized row */
#define GJ_MAX_ATTRS 64    /* distinct attributes of a natural-join query */
#define GJ_MAX_CLIQUE_TABLES 8 /* tables joined into one maxclique's potential */

typedef struct gj_ctx gj_ctx;
typedef struct gj_factors gj_factors;
typedef struct gj_summary gj_summary;
typedef struct gj_wstate gj_wstate;
typedef struct gj_batch gj_batch;

/* Device-memory allocator: returns `bytes` of device memory ordered on the
 * context stream, or NULL.  Python passes PyTorch's caching allocator. */
typedef void* (*gj_alloc_fn)(size_t bytes, void* user);
typedef void (*gj_free_fn)(void* ptr, void* user);

/* Context: device, stream (hipStream_t; NULL = default stream) and allocator
 * (both NULL = hipMallocAsync/hipFreeAsync on the stream). */
gj_status gj_ctx_create(int device, void* hip_stream, gj_alloc_fn alloc, gj_free_fn free_fn, void* user,
                        gj_ctx** out);
void gj_ctx_destroy(gj_ctx* ctx);
/* Message of the last failed call made with `ctx` or with a factor set,
 * summary, column set, batch, potential or saved state made by it ("" if
 * none); ctx = NULL: the last failure on the calling thread, which is where
 * calls without a context (gj_validate, gj_junction_tree_build, and a
 * gj_ctx_create that fails) record theirs.  The string lives until the next
 * failure recorded in the same place.  A context is used by one thread at a
 * time (its calls are ordered on one stream), so its message is not shared
 * between threads. */
const char* gj_last_error(const gj_ctx* ctx);

/* One input table: n_keys int32 key columns (device pointers, SoA, n_rows each).
 * `keys` itself is a host array of n_keys device pointers.  Only the columns
 * that appear in the query are passed (Sec. 3.2: one node per join or output
 * attribute); payload columns are not. */
typedef struct {
  int64_t n_rows;
  int32_t n_keys; /* 1..GJ_MAX_KEYS */
  const int32_t* const* keys;
} gj_table;

/* Join tree (Sec. 3.2, qualitative part): host arrays of n_tables entries. */
typedef struct {
  int32_t n_tables; /* 1..GJ_MAX_TABLES */
  const int32_t* parent;     /* parent[0] = -1, parent[t] < t */
  const int32_t* sep_col;    /* column of t equal to ...           (ignored for t = 0) */
  const int32_t* parent_col; /* ... this column of parent[t]       (ignored for t = 0) */
} gj_join_graph;

/* Host-only check of a join graph against the tables' key counts: GJ_OK or
 * GJ_E_GRAPH / GJ_E_INVALID with a message.  Runs no device code. */
gj_status gj_validate(const gj_table* tables, const gj_join_graph* graph);

/* ---- stage 1: factors (Sec. 3.2 quantitative learning: one scan per table) ----
 * Builds every table's factor on the device.  Entries of the root are ordered
 * by its key columns in declared order; entries of any other table by its
 * separator column first, then its other columns in declared order; all
 * comparisons as signed int32.  Rows inside an entry ascend by row id.  A
 * table whose key columns' value ranges and row ids need more than 128 bits
 * has its widest columns ranked among their distinct values for the sort
 * (one more group-by per such column, with a host synchronization); it is
 * refused (GJ_E_INVALID) only if ranks do not make it fit either. */
gj_status gj_build_factors(gj_ctx* ctx, const gj_table* tables, const gj_join_graph* graph, gj_factors** out);

/* View of table t's factor (device pointers valid while the factors live):
 *   keys[c]  int32[n_entries]  key column c (declared order) of every entry
 *   count    int64[n_entries]  the entry's frequency (the potential's count,
 *                              Sec. 3.2) = end - start
 *   start    int32[n_entries]  first position of the entry's rows in perm
 *   end      int32[n_entries]  one past the last
 *   perm     int32[n_rows]     row ids grouped by entry, ascending inside one
 * The first view of a factor set synchronizes the stream (entry counts) and
 * fills `count` for every table with one small kernel. */
typedef struct {
  int64_t n_entries;
  int64_t n_rows;
  int32_t n_keys;
  const int32_t* keys[GJ_MAX_KEYS];
  const int64_t* count;
  const int32_t* start;
  const int32_t* end;
  const int32_t* perm;
} gj_factor_view;
gj_status gj_factor_table(const gj_factors* f, int32_t t, gj_factor_view* v);
/* How table t's rows were sorted for the group-by (host only, no device work):
 * *kind = 0: one global radix pass per digit; 1: global passes over the top
 * two digits, then each run of equal top bits sorted in LDS (gj_tune
 * sort_local_rows); 2: as 1, but a run was longer than one block holds and
 * the table was sorted again by the per-digit passes.  Same entries in every
 * case. */
gj_status gj_factor_sort(const gj_factors* f, int32_t t, int32_t* kind);
void gj_free_factors(gj_factors* f);

/* ---- stage 2: summary (Sec. 3.3 Algorithm 2 upward; Sec. 3.5 downward) ----
 * Upward, leaves to root (the perfect elimination order on a tree):
 *   U_t(e) = prod over children ch of M_ch(e[parent_col[ch]]), 1 at leaves,
 *   M_t(s) = sum over entries e of t with separator s of c_t(e) * U_t(e),
 *   join size = sum over root entries of c_0 * U_0 (Z of Eq. 3).
 * Downward, root to leaves (the conditioning of Algorithm 4):
 *   D_0 = 1,  D_t(s) = sum over parent entries e' with e'[parent_col[t]] = s of
 *   c_p(e') * D_p(e') * prod over siblings of M_sib, and F = c * U * D.
 * Only entries with F > 0 survive (Sec. 3.3: entries of frequency < 1 are
 * excluded, which is how unneeded intermediate results are avoided).
 * `join_size` (host) receives the join size. */
gj_status gj_summarize(gj_ctx* ctx, const gj_factors* f, gj_summary** out, int64_t* join_size);

/* The same upward and downward passes for n_queries factor sets (each made
 * by gj_build_factors, all distinct, all on ctx) with nothing read back to
 * the host: every query's kernels are launched in stream order and query i's
 * join size and status (GJ_OK, or GJ_E_OVERFLOW when it is >= 2^63-1) are
 * written to d_join_sizes[i] (int64) and d_status[i] (int32), device arrays
 * owned by the caller.  outs (host array of n_queries):
 *   outs[i] == NULL on entry: a summary of factors[i] is allocated through the
 *     context's allocator and returned in outs[i];
 *   outs[i] == a summary made earlier for factors[i] (by gj_summarize or by
 *     this call): it is recomputed in place, allocating nothing.
 * A call that is given every summary allocates nothing and never waits for
 * the device, so it can be recorded into a HIP graph (capture the context's
 * stream, call, end the capture); each replay recomputes every summary from
 * the factors' current contents.  The host side of a summary computed this
 * way (entry counts, join size) is read with one synchronization by its first
 * view, expansion, save or gj_summary_join_size, which return GJ_E_OVERFLOW
 * for a query that overflowed.  Arguments are checked before anything is
 * launched: null pointers, factors of another context or of a batch, the same
 * factors twice, a summary made for other factors -> GJ_E_INVALID. */
gj_status gj_summarize_batch(gj_ctx* ctx, const gj_factors* const* factors, int32_t n_queries, gj_summary** outs,
                             int64_t* d_join_sizes, int32_t* d_status);

/* Surviving entries of table t in factor order (device pointers):
 *   keys[c] int32, c/U/D/F int64; F = c*U*D is the entry's run length in the
 *   result and U*D the fan-out of each of its rows.  `pre` (int64) is the
 *   exclusive prefix sum of c*U inside the entry's separator group (over the
 *   whole table for the root): the offset of the entry's block in the order. */
typedef struct {
  int64_t n_entries;
  int32_t n_keys;
  const int32_t* keys[GJ_MAX_KEYS];
  const int64_t* c;
  const int64_t* U;
  const int64_t* D;
  const int64_t* F;
  const int64_t* pre;
} gj_summary_view;
gj_status gj_summary_table(const gj_summary* s, int32_t t, gj_summary_view* v);

/* Edge into table t >= 1: separator values s (ascending, int32) with
 * M_t(s) * D_t(s) > 0 and both messages (int64). */
typedef struct {
  int64_t n;
  const int32_t* s;
  const int64_t* M;
  const int64_t* D;
} gj_edge_view;
gj_status gj_summary_edge(const gj_summary* s, int32_t t, gj_edge_view* v);
/* Join size of a summary (-1: NULL, or its query overflowed). */
int64_t gj_summary_join_size(const gj_summary* s);
void gj_free_summary(gj_summary* s);

/* ---- stage 3: desummarization (Sec. 3.6) ----
 * Writes result rows [first_row, first_row + n_rows) of the sorted result
 * (sorted by all attribute values -- the root's columns in declared order,
 * then each further table's non-separator columns in declared order, table by
 * table -- ties broken by the row ids (r_0, .., r_{n-1})) as row-major
 * [n_rows x n_tables] row ids of `rowid_bytes` (4: int32, 8: int64) each into
 * device buffer `out`.  Rows past the join size are not written; *n_written
 * (host) receives the count.  first_row > join size -> GJ_E_RANGE.  For
 * summaries whose middle tables hold one entry per group (gj_desum_kernel)
 * the call may take stream-ordered scratch from the context's allocator for
 * root-entry records (at most a quarter of the output bytes, released before
 * it returns); if that allocation fails the records are decoded in place. */
gj_status gj_desummarize(gj_ctx* ctx, const gj_summary* s, int64_t first_row, int64_t n_rows, int32_t rowid_bytes,
                         void* out, int64_t* n_written);

/* Paper-literal GFJS (Definition 1, as Algorithms 3-4 emit it: one run per
 * distinct value prefix) of result rows [first_row, first_row + n_rows).
 * Result column i (same order as above) gets runs (values[i][k],
 * freqs[i][k]) for k < n_runs[i]; each values[i] / freqs[i] is a caller device
 * buffer of n_rows entries (int32 / int64), n_runs a host array of
 * gj_result_columns(s) entries. */
int32_t gj_result_columns(const gj_summary* s);
gj_status gj_unroll_gfjs(gj_ctx* ctx, const gj_summary* s, int64_t first_row, int64_t n_rows,
                         int32_t* const* values, int64_t* const* freqs, int64_t* n_runs);

/* ---- value columns: payload gather in the expansion ----
 * Materializes attribute or payload values instead of row ids (Sec. 3.6
 * replaces every run by copies of its value).  A column set names n_cols
 * (1..GJ_MAX_OUT_COLS) int32 device columns: column j (data[j], a host array
 * of device pointers) holds one value per row of table tab[j], in row order --
 * a key column or any payload column of that table.  gj_colset_create copies
 * each column once into the factor's grouped row order (one gather through the
 * row permutation), so the expansion reads values the way it reads row ids.
 * The columns are borrowed for the duration of the call only.  The set holds a
 * reference to the summary's factors; free it with gj_free_colset.  A
 * projected summary has no rows: GJ_E_INVALID. */
typedef struct gj_colset gj_colset;
gj_status gj_colset_create(gj_ctx* ctx, const gj_summary* s, int32_t n_cols, const int32_t* tab,
                           const int32_t* const* data, gj_colset** out);
void gj_free_colset(gj_colset* cs);
/* Rows [first_row, first_row + n_rows) of the sorted result (the order of
 * gj_desummarize) as row-major [n_rows x n_cols] int32 values: element j of a
 * row is column j of the set at that result row's row id of table tab[j].
 * `out` is a 16-byte aligned device buffer; rows past the join size are not
 * written and *n_written (host) receives the count; first_row > join size ->
 * GJ_E_RANGE; a set made for other factors -> GJ_E_INVALID.  Like
 * gj_desummarize, it takes the keyed-lookup expansion where gj_desum_kernel
 * says so, and may then take stream-ordered scratch for root-entry records
 * (released before it returns; decoded in place if the allocation fails). */
gj_status gj_desummarize_values(gj_ctx* ctx, const gj_summary* s, const gj_colset* cs, int64_t first_row,
                                int64_t n_rows, int32_t* out, int64_t* n_written);

/* ---- early projections (Sec. 3.7) ----
 * Only some attributes are output attributes.  out_cols[t] (host, one word per
 * table) has bit c set if key column c of table t is one; a join attribute
 * marked on either table of its edge counts for both.  The projected result is
 * every join result tuple restricted to the output attributes, each keeping its
 * multiplicity, sorted by all of them.  Non-output attributes are removed
 * before the generator is built: a table with no output attribute besides its
 * separator (the root: none at all) and no kept descendant is deleted -- only
 * its subtree's completions count, as a frequency carried by its parent's
 * entries -- and every kept table's entries are grouped by its output columns.
 * Returns a projected summary (views index the kept tables 0..k-1 in their
 * original order; gj_summary_n_tables gives k; keys are the output columns in
 * declared order; c is the projected frequency, an int64 that can exceed any
 * row count) and the join size in *join_size (host).
 * Supported when table 0 holds an output attribute and every kept table's
 * separator is an output attribute; otherwise two kept tables would be linked
 * through a summed-out attribute and the generator would need a fill-in edge:
 * GJ_E_GRAPH (root the query at a table that holds output attributes).  No
 * output attribute, a bit beyond a table's columns, or more than
 * GJ_MAX_OUT_COLS result columns: GJ_E_INVALID.  A projected summary has no
 * row ids: gj_desummarize, gj_unroll_gfjs and gj_colset_create reject it. */
gj_status gj_summarize_projected(gj_ctx* ctx, const gj_factors* f, const uint32_t* out_cols, gj_summary** out,
                                 int64_t* join_size);
/* Tables described by a summary (for a projected one, the kept tables). */
int32_t gj_summary_n_tables(const gj_summary* s);
/* Rows [first_row, first_row + n_rows) of the sorted result as attribute
 * values, row-major [n_rows x gj_result_columns(s)] int32: the root's columns
 * in declared order, then each further table's columns other than its
 * separator, in table order.  On a projected summary these are the output
 * attributes; on any other summary every attribute of every result row.  An
 * entry tuple of the summary is one run of identical rows, so this is
 * run-length decoding.  `out` is a 16-byte aligned device buffer; *n_written
 * (host) receives the count; first_row > join size -> GJ_E_RANGE. */
gj_status gj_desummarize_projected(gj_ctx* ctx, const gj_summary* s, int64_t first_row, int64_t n_rows, int32_t* out,
                                   int64_t* n_written);

/* ---- storing and reloading a summary (compute-and-store, load-and-desummarize) ----
 * gj_summary_save writes summary s to the file `path` (host) as its columns
 * in a fixed binary layout: per table the surviving entries' keys, c, U, D,
 * F and block offsets, the edge's (s, M, D) and the child records, and, if
 * with_rows is nonzero, each entry's (count, first position) and the grouped
 * row ids (a projected summary has none: GJ_E_INVALID).  *bytes_written
 * (host, may be NULL) receives the file size.  gj_summary_load reads such a
 * file into a new summary on ctx's device: views, gj_summary_join_size,
 * gj_result_columns and gj_desummarize_projected work on it, and when it was
 * saved with rows also gj_desummarize, gj_colset_create and gj_unroll_gfjs,
 * all with the results of the summary it was saved from.  An unreadable file,
 * a different version or a malformed header: GJ_E_INVALID.  Free it with
 * gj_free_summary. */
gj_status gj_summary_save(gj_ctx* ctx, const gj_summary* s, const char* path, int32_t with_rows,
                          int64_t* bytes_written);
gj_status gj_summary_load(gj_ctx* ctx, const char* path, gj_summary** out);

/* Checks a file written by gj_summary_save on the host alone, with no device
 * and no context: the header and table headers, then every section read in
 * full with the checks gj_summary_load applies before any copy to the device
 * (entry counts >= 1; child records, (count, first) pairs and row ids inside
 * their tables), and no data after the last section.  On success *info (host,
 * may be NULL) receives the table count, the flags, the join size, each
 * table's surviving entries and rows, and the file size.  An unreadable,
 * truncated, inconsistent or longer file: GJ_E_INVALID with the reason in
 * gj_last_error(NULL). */
typedef struct {
  int32_t n_tables, projected, with_rows;
  int64_t join_size;
  int64_t entries[GJ_MAX_TABLES];
  int64_t rows[GJ_MAX_TABLES];
  int64_t bytes;
} gj_summary_file_info;
gj_status gj_summary_file_check(const char* path, gj_summary_file_info* info);

/* ---- cyclic queries: natural joins over named attributes (Sec. 2.2.1, 3.2.1, 3.4) ----
 * A natural-join query names the attribute of every key column: column c of
 * table t carries attribute id attr[t * GJ_MAX_KEYS + c] (>= 0), and all
 * columns with the same id must hold equal values.  Its graph has one node per
 * attribute and a clique per table; cycles are allowed. */
typedef struct {
  int32_t n_tables;      /* 1..GJ_MAX_TABLES */
  const int32_t* n_keys; /* host [n_tables], 1..GJ_MAX_KEYS each */
  const int32_t* attr;   /* host [n_tables * GJ_MAX_KEYS] */
} gj_natural_query;

/* Junction tree of maxcliques (Sec. 2.2.1): min fill-in triangulation of the
 * attribute graph, its maxcliques, and a maximal spanning tree over separator
 * sizes (running intersection property).  Attributes are numbered 0..n_attrs-1
 * by ascending id (attr_id maps back); cliques are attribute bitmasks numbered
 * in tree order (parent[i] < i, parent[0] = -1; clique 0 holds table 0's
 * attributes); table t is assigned to the first clique holding all its
 * attributes.  Host only: no device work.  More than GJ_MAX_ATTRS attributes,
 * bad counts or negative ids: GJ_E_INVALID; a disconnected query: GJ_E_GRAPH. */
typedef struct {
  int32_t n_attrs;
  int32_t attr_id[GJ_MAX_ATTRS];
  int32_t elim_order[GJ_MAX_ATTRS]; /* attribute indices in elimination order */
  int32_t n_fill;                   /* fill-in edges added */
  int32_t n_cliques;
  uint64_t clique[GJ_MAX_ATTRS];
  int32_t parent[GJ_MAX_ATTRS];
  int32_t table_clique[GJ_MAX_TABLES];
} gj_junction_tree;
gj_status gj_junction_tree_build(const gj_natural_query* q, gj_junction_tree* out);

/* POTENTIAL-JOIN (Sec. 3.2.1, Algorithm 1): the joint potential of the
 * frequency tables of q's tables (1..GJ_MAX_CLIQUE_TABLES; tables[t] holds the
 * key columns whose attributes q names) over all their attributes -- every
 * combination of attribute values on which all tables agree, with the product
 * of the tables' frequencies of their parts.  Variables are the attributes in
 * ascending id order; entries ascend lexicographically.  Worst-case optimal:
 * values are bound one variable at a time, extending only prefixes that every
 * table holding the variable shares.  More than 2^31-1 entries, a table naming
 * an attribute twice: GJ_E_INVALID / GJ_E_GRAPH.  The view's device pointers
 * live until gj_free_potential. */
typedef struct gj_potential gj_potential;
typedef struct {
  int64_t n_entries;
  int32_t n_vars;
  int32_t attr[GJ_MAX_ATTRS];        /* attribute id of each variable */
  const int32_t* keys[GJ_MAX_ATTRS]; /* device int32[n_entries] per variable */
  const int64_t* freq;               /* device int64[n_entries] */
} gj_potential_view;
gj_status gj_potential_join(gj_ctx* ctx, const gj_table* tables, const gj_natural_query* q, gj_potential** out);
gj_status gj_potential_table(const gj_potential* p, gj_potential_view* v);
void gj_free_potential(gj_potential* p);

/* Summary of a natural-join query, cyclic or not (Sec. 3.4: the same inference
 * on the junction tree of maxcliques).  tables[t] holds the key columns whose
 * attributes q names.  The junction tree comes from gj_junction_tree_build; each
 * maxclique's potential is the POTENTIAL-JOIN of the tables assigned to it (a
 * clique variable no assigned table holds is restricted by the distinct
 * projection of a table holding it, which filters without counting); the tree
 * of clique potentials is summarized like an acyclic query, a separator of
 * several attributes becoming one column holding the index of the value
 * combination.  The summary's tables are the cliques (views: keys = the
 * clique's attributes in ascending id order, then separator index columns;
 * c = the potential's frequency).  It has no row ids: gj_desummarize_projected
 * writes the result as values, one column per attribute (the root clique's
 * attributes, then each further clique's attributes outside its separator;
 * gj_result_attribute names them), sorted by those columns.  *join_size
 * (host) receives the join size.  Errors: as gj_junction_tree_build and
 * gj_potential_join, a clique with more than GJ_MAX_CLIQUE_TABLES tables or
 * more than GJ_MAX_KEYS columns, more than GJ_MAX_TABLES cliques:
 * GJ_E_GRAPH; GJ_E_OVERFLOW. */
gj_status gj_summarize_cyclic(gj_ctx* ctx, const gj_table* tables, const gj_natural_query* q, gj_summary** out,
                              int64_t* join_size);
/* Attribute id of result column j of a summary made by gj_summarize_cyclic (-1 otherwise). */
int32_t gj_result_attribute(const gj_summary* s, int32_t j);

/* ---- weighted join and its adjoint ----
 * Every row r of table t carries a weight w_t[r]; W = sum over result tuples of
 * the product of their rows' weights (W = join size at unit weights).  The
 * forward pass is the upward pass with c_t(e) replaced by the summed weights
 * of e's rows, in float64.  w[t] are device arrays of n_rows(t) weights of
 * `w_dtype` (0: float32, 1: float64), accumulated in float64.  *d_W (device
 * float64) receives W; *saved keeps what the backward pass needs. */
gj_status gj_weighted_forward(gj_ctx* ctx, const gj_factors* f, const void* const* w, int32_t w_dtype, double* d_W,
                              gj_wstate** saved);
/* Adjoint of the forward pass (= the downward pass): grad_w[t][r] =
 * (*d_gradW) * dW/dw_t[r] = gradW * U(e(r)) * D(e(r)), written in w_dtype into
 * device arrays grad_w[t] (n_rows(t) each). */
gj_status gj_weighted_backward(gj_ctx* ctx, const gj_wstate* st, const double* d_gradW, void* const* grad_w);
void gj_free_wstate(gj_wstate* st);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid allocation:
 * W and every row's gradient in one call, the results of gj_weighted_forward
 * followed by gj_weighted_backward, with no allocation and no host
 * synchronization.  Arguments as there; d_gradW (device float64) scales the
 * gradients, NULL meaning 1; *d_W (device) receives W and grad_w[t] (device,
 * n_rows(t) values of w_dtype) the gradients.  The call's intermediate state
 * (36 bytes per row and a little more) lives in one fixed device array of
 * GJ_NOALLOC_SCRATCH_BYTES that every device running the library holds until
 * the process ends; a query that needs more -> GJ_E_INVALID, naming the size.
 * Every call on a device shares that array: calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller. */
#define GJ_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
gj_status gj_weighted_grad_noalloc(gj_ctx* ctx, const gj_factors* f, const void* const* w, int32_t w_dtype,
                                   const double* d_gradW, double* d_W, void* const* grad_w);

/* ---- batched queries ----
 * Plans n_queries independent queries (tables of query q are
 * tables[q_off[q] .. q_off[q+1]), graphs[q] its join tree): reads the key
 * ranges once (one synchronization), sizes every workspace for the worst case,
 * and records the factor build + summary of every query as one HIP graph of
 * one kernel launch per stage and tree level, each launch covering every
 * query; nothing in it allocates or waits for the host.  tune = NULL uses the
 * context's tile sizes. */
typedef struct {
  int32_t sort_items;   /* keys per thread in 64-bit radix-sort tiles (8 or 16;
                           128-bit tiles always take 8) */
  int32_t radix_bits;   /* digit width of the radix sort (4..8) */
  int32_t desum_rounds; /* staging rounds per lane of the expansion kernel (1..1024),
                           or 0: as many as make about 640 bytes of output per lane
                           and at least 16 tuples */
  int32_t desum_stage;  /* tuples per lane per LDS staging round: 2, 4 or 8 */
  int32_t batch_task_rows; /* rows (or sort keys) per task of the persistent batch
                              kernel's plan (256..2^24), or 0: 16384 */
  int32_t desum_general;   /* 0: gj_desummarize takes the keyed-lookup expansion for
                              the summaries it applies to (gj_desum_kernel); 1: always
                              the general expansion kernel (same result) */
  int32_t sort_local_rows; /* gj_build_factors only: a table of at least this many rows
                              whose sort words take 128 bits is sorted by two global
                              passes over its top digits and an LDS sort of each run
                              of equal top bits, instead of one global pass per digit
                              (0: never; default 2^20).  Same result; a run longer
                              than one block holds makes the build wait for the host
                              once and sort that table in full. */
} gj_tune;
gj_status gj_batch_create(gj_ctx* ctx, int32_t n_queries, const int32_t* q_off, const gj_table* tables,
                          const gj_join_graph* graphs, const gj_tune* tune, gj_batch** out);
/* Replays the recorded graph on `hip_stream` (NULL = context stream):
 * recomputes every factor and summary from the (same) input columns.  Reads on
 * the context's stream (views, gj_download) are ordered after the launch. */
gj_status gj_batch_launch(gj_batch* b, void* hip_stream);
/* The same replay (the launch-per-stage graph). */
gj_status gj_batch_launch_kernels(gj_batch* b, void* hip_stream);
/* The factor build + summary of every query in ONE persistent kernel launch
 * (blocks take tasks -- a few tiles of one stage of one table -- from a device
 * queue in dependency order; a task waits, bounded, only for the earlier
 * stages of its own table).  Switched off: returns GJ_E_INVALID. */
gj_status gj_batch_launch_persistent(gj_batch* b, void* hip_stream);
/* Tasks and stage instances of the persistent kernel's plan, and its grid
 * (0: not set up). */
gj_status gj_batch_info(const gj_batch* b, int32_t* n_tasks, int32_t* n_stages, int32_t* grid);
/* The launch-per-stage work without a graph, the kernels launched one by one. */
gj_status gj_batch_launch_eager(gj_batch* b, void* hip_stream);
/* Device arrays of n_queries entries: join sizes (int64) and statuses (int32,
 * GJ_OK or GJ_E_OVERFLOW), written by every launch. */
const int64_t* gj_batch_join_sizes(const gj_batch* b);
const int32_t* gj_batch_status(const gj_batch* b);
/* Summary of query q as a borrowed gj_summary (valid until the batch is freed
 * or relaunched; do not free it). */
gj_status gj_batch_summary(gj_batch* b, int32_t q, const gj_summary** out);
void gj_free_batch(gj_batch* b);

/* Launch shape of the general expansion kernel that gj_desummarize (n_cols =
 * 0, rowid_bytes 4 or 8) or gj_desummarize_values (n_cols value columns,
 * rowid_bytes 4) uses for n_rows rows of an n_tables-table summary under
 * `tune` (NULL: defaults) -- for summaries that gj_desum_kernel reports 0 for,
 * or under desum_general = 1.  Host
 * only, no device work: lets tests and tuners check every setting's launch
 * against the kernel's limits.  GJ_E_INVALID for arguments or shapes the
 * kernel does not support (the expansion entry points then fail the same way). */
typedef struct {
  int32_t stage;           /* tuples per lane per LDS staging round */
  int32_t tuples_per_lane; /* tuples a lane writes (a multiple of stage) */
  int32_t kernel_tables;   /* table count of the kernel instance (exact up to 8, else 16) */
  int32_t change_bits;     /* bits of the per-round change mask = stage * kernel_tables (<= 64) */
  int32_t seg_bytes;       /* bytes a lane stages per round (whole 16-byte units) */
  int64_t blocks;          /* 256-thread blocks (a multiple of 8) */
  int64_t lds_bytes;       /* dynamic LDS allocated per block */
  int64_t lds_used;        /* LDS the actual columns use (<= lds_bytes) */
} gj_desum_launch;
gj_status gj_desum_launch_config(int32_t n_tables, int32_t rowid_bytes, int32_t n_cols, int64_t n_rows,
                                 const gj_tune* tune, gj_desum_launch* out);

/* Which kernel gj_desummarize and gj_desummarize_values take for summary s on
 * this context: 1 for the keyed-lookup expansion, 0 for the general one (the
 * result is the same).  The keyed-lookup expansion (Sec. 3.6's order, decoded
 * per rank) applies to row-id summaries of two or more tables in which every
 * table other than the root and the innermost table holds exactly one
 * surviving entry per surviving group (MC == GC in gj_summary_table), as a
 * dimension joined on its key does; the context's tune can switch it off
 * (desum_general).  Reads the summary's counts, which a batch summary fetches
 * on first use. */
gj_status gj_desum_kernel(gj_ctx* ctx, const gj_summary* s, int32_t* kind);

/* Plumbing for bindings and tests: copies `bytes` of device memory to host
 * memory on the context stream and waits for it. */
gj_status gj_download(gj_ctx* ctx, void* host_dst, const void* dev_src, size_t bytes);

/* Sets the default tile sizes used by later calls on this context. */
gj_status gj_ctx_set_tune(gj_ctx* ctx, const gj_tune* tune);

#ifdef __cplusplus
}
#endif
#endif /* GJ_H */
