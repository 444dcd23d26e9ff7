// Storing and reloading a summary (the paper's compute-and-store and
// load-and-desummarize modes, Sec. 3.6: the GFJS is written per column and
// read back for desummarization; Tables 2-4).  The file is the summary's own
// columns, one array after another in a fixed order (little-endian, no
// padding), so saving and loading are plain copies between device and file:
//
//   header   magic "GJSUMM01", int32 version, n_tables, projected, with_rows,
//            int64 join size
//   table t  int32 k, sep, pcol, parent, is_root; int64 entries, groups, rows
//   then per table, in table order:
//     keys     k x entries int32 (column-major)
//     c, U, D, F, pre          entries int64 each
//     s, M, D (edge, t >= 1)   groups int32, int64, int64
//     child records (t >= 1)   entries(parent) x 32 bytes
//     with_rows: (count, first) entries x int2, then the grouped row ids rows x int32
//
// A reloaded summary answers the views, gj_desummarize_projected and (when
// saved with its rows) gj_desummarize, gj_desummarize_values and
// gj_unroll_gfjs exactly as the summary it was saved from.
#include <cstdio>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace gjh;

namespace {

const char MAGIC[8] = {'G', 'J', 'S', 'U', 'M', 'M', '0', '1'};
const int32_t VERSION = 1;

struct TabHdr {
  int32_t k, sep, pcol, parent, is_root;
  int64_t entries, groups, rows;
};

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

gj_status dev_to_file(gj_ctx* ctx, FILE* f, const void* src, size_t bytes, std::vector<char>& buf, int64_t& total) {
  if (!bytes) return GJ_OK;
  buf.resize(bytes);
  gj_status st = check(hipMemcpyAsync(buf.data(), src, bytes, hipMemcpyDeviceToHost, ctx->stream), "save");
  if (!st) st = check(hipStreamSynchronize(ctx->stream), "save");
  if (st) return st;
  if (fwrite(buf.data(), 1, bytes, f) != bytes) {
    set_error("gj_summary_save: write failed");
    return GJ_E_INVALID;
  }
  total += (int64_t)bytes;
  return GJ_OK;
}

// Reads `bytes` from the file into device memory.  `ok` (if given) checks the
// host copy first: indices that the kernels follow must stay inside their
// arrays whatever the file holds.
template <typename T>
gj_status file_to_dev(gj_ctx* ctx, FILE* f, T* dst, size_t bytes, std::vector<char>& buf,
                      bool (*ok)(const T*, size_t, const int64_t*) = nullptr, const int64_t* lim = nullptr) {
  if (!bytes) return GJ_OK;
  buf.resize(bytes);
  if (fread(buf.data(), 1, bytes, f) != bytes) {
    set_error("gj_summary_load: truncated file");
    return GJ_E_INVALID;
  }
  if (ok && !ok(reinterpret_cast<const T*>(buf.data()), bytes / sizeof(T), lim)) {
    set_error("gj_summary_load: inconsistent summary file (an index out of range)");
    return GJ_E_INVALID;
  }
  gj_status st = check(hipMemcpyAsync(dst, buf.data(), bytes, hipMemcpyHostToDevice, ctx->stream), "load");
  if (!st) st = check(hipStreamSynchronize(ctx->stream), "load");
  return st;
}

// lim[0]: entries of the child table
bool crec_ok(const ChildRec* r, size_t n, const int64_t* lim) {
  for (size_t i = 0; i < n; ++i)
    if (r[i].first < 0 || r[i].first > r[i].end || r[i].end > lim[0] || r[i].M < 0) return false;
  return true;
}
// lim[0]: rows of the table
bool ccs_ok(const int2* r, size_t n, const int64_t* lim) {
  for (size_t i = 0; i < n; ++i)
    if (r[i].x < 1 || r[i].y < 0 || (int64_t)r[i].x + r[i].y > lim[0]) return false;
  return true;
}
bool rows_ok(const int32_t* r, size_t n, const int64_t* lim) {
  for (size_t i = 0; i < n; ++i)
    if (r[i] < 0 || r[i] >= lim[0]) return false;
  return true;
}
bool count_ok(const int64_t* r, size_t n, const int64_t*) {
  for (size_t i = 0; i < n; ++i)
    if (r[i] < 1) return false;
  return true;
}

}  // namespace

extern "C" {

gj_status gj_summary_save(gj_ctx* ctx, const gj_summary* s, const char* path, int32_t with_rows,
                          int64_t* bytes_written) {
  GJ_SCOPE(ctx);
  if (!ctx || !s || !path) {
    set_error("gj_summary_save: null argument");
    return GJ_E_INVALID;
  }
  if (with_rows && s->projected) {
    set_error("gj_summary_save: a projected summary has no rows to save");
    return GJ_E_INVALID;
  }
  if (with_rows && !s->f->F.perm) {
    set_error("gj_summary_save: this summary was loaded without its rows");
    return GJ_E_INVALID;
  }
  if (gj_status st = summary_host(s)) return st;
  const Plan& P = s->f->plan;
  const int base = P.qfirst[s->query];
  const int n = P.qfirst[s->query + 1] - base;
  File fh;
  fh.f = fopen(path, "wb");
  if (!fh.f) {
    set_error("gj_summary_save: cannot open %s", path);
    return GJ_E_INVALID;
  }
  int64_t total = 0;
  std::vector<char> buf;
  auto put = [&](const void* p, size_t b) -> bool {
    total += (int64_t)b;
    return fwrite(p, 1, b, fh.f) == b;
  };
  const int32_t hdr[4] = {VERSION, n, s->projected ? 1 : 0, with_rows ? 1 : 0};
  bool ok = put(MAGIC, 8) && put(hdr, sizeof hdr) && put(&s->join_size, 8);
  std::vector<TabHdr> th(n);
  for (int t = 0; t < n && ok; ++t) {
    const TDesc& d = P.td[base + t];
    const int g = base + t;
    th[t] = TabHdr{d.k, d.sep, d.pcol, d.parent >= 0 ? d.parent - base : -1, d.is_root,
                   s->cnt_host[g * CNT_STRIDE + CNT_MC], s->cnt_host[g * CNT_STRIDE + CNT_GC], d.n};
    ok = put(&th[t], sizeof(TabHdr));
  }
  if (!ok) {
    set_error("gj_summary_save: write failed");
    return GJ_E_INVALID;
  }
  gj_status st = GJ_OK;
  for (int t = 0; t < n && !st; ++t) {
    const TDesc& d = P.td[base + t];
    const int64_t E = th[t].entries, G = th[t].groups;
    for (int c = 0; c < d.k && !st; ++c)
      st = dev_to_file(ctx, fh.f, s->S.ckey + d.key_off + (int64_t)c * d.n, E * 4, buf, total);
    const int64_t* cols[5] = {s->S.cc, s->S.cU, s->S.cD, s->S.cF, s->S.cpre};
    for (int i = 0; i < 5 && !st; ++i) st = dev_to_file(ctx, fh.f, cols[i] + d.off, E * 8, buf, total);
    if (t > 0 && !st) {
      st = dev_to_file(ctx, fh.f, s->S.cgval + d.off, G * 4, buf, total);
      if (!st) st = dev_to_file(ctx, fh.f, s->S.cgM + d.off, G * 8, buf, total);
      if (!st) st = dev_to_file(ctx, fh.f, s->S.cgD + d.off, G * 8, buf, total);
      if (!st) st = dev_to_file(ctx, fh.f, s->S.crec + d.link_off, th[th[t].parent].entries * sizeof(ChildRec), buf,
                                total);
    }
    if (with_rows && !st) {
      st = dev_to_file(ctx, fh.f, s->S.ccs + d.off, E * sizeof(int2), buf, total);
      if (!st) st = dev_to_file(ctx, fh.f, s->f->F.perm + d.off, d.n * 4, buf, total);
    }
  }
  if (st) return st;
  if (bytes_written) *bytes_written = total;
  return GJ_OK;
}

gj_status gj_summary_load(gj_ctx* ctx, const char* path, gj_summary** out) {
  GJ_SCOPE(ctx);
  if (!ctx || !path || !out) {
    set_error("gj_summary_load: null argument");
    return GJ_E_INVALID;
  }
  File fh;
  fh.f = fopen(path, "rb");
  if (!fh.f) {
    set_error("gj_summary_load: cannot open %s", path);
    return GJ_E_INVALID;
  }
  char magic[8];
  int32_t hdr[4];
  int64_t join_size = 0;
  if (fread(magic, 1, 8, fh.f) != 8 || memcmp(magic, MAGIC, 8) != 0 || fread(hdr, sizeof hdr, 1, fh.f) != 1 ||
      hdr[0] != VERSION || fread(&join_size, 8, 1, fh.f) != 1) {
    set_error("gj_summary_load: %s is not a summary file of this version", path);
    return GJ_E_INVALID;
  }
  const int n = hdr[1];
  const bool projected = hdr[2] != 0, with_rows = hdr[3] != 0;
  if (n < 1 || n > GJ_MAX_TABLES || join_size < 0) {
    set_error("gj_summary_load: bad header in %s", path);
    return GJ_E_INVALID;
  }
  std::vector<TabHdr> th(n);
  if (fread(th.data(), sizeof(TabHdr), n, fh.f) != (size_t)n) {
    set_error("gj_summary_load: truncated file");
    return GJ_E_INVALID;
  }
  for (int t = 0; t < n; ++t) {
    const TabHdr& h = th[t];
    const bool bad = h.k < 1 || h.k > GJ_MAX_KEYS || (t == 0) != (h.parent < 0) || (t > 0 && h.parent >= t) ||
                     h.entries < 0 || h.groups < 0 || h.rows < 0 || h.rows > INT32_MAX || h.entries > INT32_MAX ||
                     h.groups > INT32_MAX || (with_rows && h.entries > h.rows) ||
                     (t > 0 && (h.sep < 0 || h.sep >= h.k || h.pcol < 0 || h.pcol >= th[h.parent].k));
    if (bad) {
      set_error("gj_summary_load: bad table header %d in %s", t, path);
      return GJ_E_INVALID;
    }
  }
  // a compact layout: table t owns cap_t slots (entries, groups and rows fit)
  gj_factors* f = new gj_factors(ctx);
  f->plan.ctx = ctx;
  Plan& P = f->plan;
  P.nq = 1;
  P.nt = n;
  P.qfirst = {0, n};
  P.td.assign(n, TDesc{});
  int64_t off = 0, koff = 0, loff = 0;
  for (int t = 0; t < n; ++t) {
    const TabHdr& h = th[t];
    TDesc& d = P.td[t];
    // slots of the table: its rows (their ids), else its entries and groups
    d.n = with_rows ? h.rows : std::max(h.entries, h.groups);
    d.off = off;
    d.key_off = koff;
    d.k = h.k;
    d.sep = h.sep;
    d.pcol = h.pcol;
    d.parent = h.parent;
    d.is_root = h.is_root;
    d.query = 0;
    if (t > 0) {
      d.link_off = loff;
      loff += std::max<int64_t>(th[h.parent].entries, 1);
      TDesc& dp = P.td[h.parent];
      if (dp.nchild < GJ_MAX_CHILDREN) {
        dp.child[dp.nchild] = t;
        dp.child_col[dp.nchild] = h.pcol;
        ++dp.nchild;
      }
    }
    off += std::max<int64_t>(d.n, 1);
    koff += (int64_t)h.k * std::max<int64_t>(d.n, 1);
  }
  P.S = off;
  P.key_slots = koff;
  P.link_slots = loff;
  gj_summary* s = new gj_summary(ctx);
  s->f = f;
  s->projected = projected;
  s->join_size = join_size;
  s->cnt_host.assign((size_t)n * CNT_STRIDE, 0);
  for (int t = 0; t < n; ++t) {
    s->cnt_host[t * CNT_STRIDE + CNT_MC] = th[t].entries;
    s->cnt_host[t * CNT_STRIDE + CNT_GC] = th[t].groups;
  }
  f->cnt_host = s->cnt_host;
  Arena& A = s->arena;
  SPtrs& S = s->S;
  S.ckey = A.get_n<int32_t>(P.key_slots);
  S.cc = A.get_n<int64_t>(P.S);
  S.cU = A.get_n<int64_t>(P.S);
  S.cD = A.get_n<int64_t>(P.S);
  S.cF = A.get_n<int64_t>(P.S);
  S.cpre = A.get_n<int64_t>(P.S);
  S.cgval = A.get_n<int32_t>(P.S);
  S.cgM = A.get_n<int64_t>(P.S);
  S.cgD = A.get_n<int64_t>(P.S);
  S.crec = A.get_n<ChildRec>(P.link_slots);
  S.ccs = A.get_n<int2>(P.S);
  if (with_rows) f->F.perm = f->arena.get_n<int32_t>(P.S);
  void* need[] = {S.ckey, S.cc, S.cU, S.cD, S.cF, S.cpre, S.cgval, S.cgM, S.cgD, S.crec, S.ccs};
  bool oom = with_rows && !f->F.perm;
  for (void* p : need) oom |= !p;
  if (oom) {
    gj_free_summary(s);
    return GJ_E_OOM;
  }
  std::vector<char> buf;
  gj_status st = GJ_OK;
  for (int t = 0; t < n && !st; ++t) {
    const TDesc& d = P.td[t];
    const int64_t E = th[t].entries, G = th[t].groups;
    for (int c = 0; c < d.k && !st; ++c) st = file_to_dev(ctx, fh.f, S.ckey + d.key_off + (int64_t)c * d.n, E * 4, buf);
    st = file_to_dev(ctx, fh.f, S.cc + d.off, E * 8, buf, count_ok);
    int64_t* cols[4] = {S.cU, S.cD, S.cF, S.cpre};
    for (int i = 0; i < 4 && !st; ++i) st = file_to_dev(ctx, fh.f, cols[i] + d.off, E * 8, buf);
    if (t > 0 && !st) {
      st = file_to_dev(ctx, fh.f, S.cgval + d.off, G * 4, buf);
      if (!st) st = file_to_dev(ctx, fh.f, S.cgM + d.off, G * 8, buf);
      if (!st) st = file_to_dev(ctx, fh.f, S.cgD + d.off, G * 8, buf);
      if (!st)
        st = file_to_dev(ctx, fh.f, S.crec + d.link_off, th[d.parent].entries * sizeof(ChildRec), buf, crec_ok,
                         &th[t].entries);
    }
    if (with_rows && !st) {
      st = file_to_dev(ctx, fh.f, S.ccs + d.off, E * sizeof(int2), buf, ccs_ok, &th[t].rows);
      if (!st) st = file_to_dev(ctx, fh.f, f->F.perm + d.off, th[t].rows * 4, buf, rows_ok, &th[t].rows);
    }
  }
  if (st) {
    gj_free_summary(s);
    return st;
  }
  *out = s;
  return GJ_OK;
}

}  // extern "C"
