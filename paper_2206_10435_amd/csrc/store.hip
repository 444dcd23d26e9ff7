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
//     child records (t >= 1)   entries(parent) x 16 bytes (first, end, c0, st0 int32)
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
const int32_t VERSION = 2;  // 2: 16-byte child records

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
  if (!dst) return GJ_OK;  // checking only
  gj_status st = check(hipMemcpyAsync(dst, buf.data(), bytes, hipMemcpyHostToDevice, ctx->stream), "load");
  if (!st) st = check(hipStreamSynchronize(ctx->stream), "load");
  return st;
}

// lim[0]: entries of the child table
bool crec_ok(const ChildRec* r, size_t n, const int64_t* lim) {
  for (size_t i = 0; i < n; ++i)
    if (r[i].first < 0 || r[i].first > r[i].end || r[i].end > lim[0]) return false;
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

struct FileHdr {
  int32_t n = 0;
  bool projected = false, with_rows = false;
  int64_t join_size = 0;
  std::vector<TabHdr> th;
};

// Header and table headers, checked on the host: counts in range, a tree in
// table order, key columns that exist.
gj_status read_headers(FILE* f, const char* path, FileHdr& h) {
  char magic[8];
  int32_t hdr[4];
  if (fread(magic, 1, 8, f) != 8 || memcmp(magic, MAGIC, 8) != 0 || fread(hdr, sizeof hdr, 1, f) != 1 ||
      hdr[0] != VERSION || fread(&h.join_size, 8, 1, f) != 1) {
    set_error("gj_summary_load: %s is not a summary file of this version", path);
    return GJ_E_INVALID;
  }
  h.n = hdr[1];
  h.projected = hdr[2] != 0;
  h.with_rows = hdr[3] != 0;
  if (h.n < 1 || h.n > GJ_MAX_TABLES || h.join_size < 0) {
    set_error("gj_summary_load: bad header in %s", path);
    return GJ_E_INVALID;
  }
  h.th.resize(h.n);
  if (fread(h.th.data(), sizeof(TabHdr), h.n, f) != (size_t)h.n) {
    set_error("gj_summary_load: truncated file");
    return GJ_E_INVALID;
  }
  for (int t = 0; t < h.n; ++t) {
    const TabHdr& x = h.th[t];
    const bool bad = x.k < 1 || x.k > GJ_MAX_KEYS || (t == 0) != (x.parent < 0) || (t > 0 && x.parent >= t) ||
                     x.entries < 0 || x.groups < 0 || x.rows < 0 || x.rows > INT32_MAX || x.entries > INT32_MAX ||
                     x.groups > INT32_MAX || (h.with_rows && x.entries > x.rows) ||
                     (t > 0 && (x.sep < 0 || x.sep >= x.k || x.pcol < 0 || x.pcol >= h.th[x.parent].k));
    if (bad) {
      set_error("gj_summary_load: bad table header %d in %s", t, path);
      return GJ_E_INVALID;
    }
  }
  return GJ_OK;
}

enum Section { SEC_KEY, SEC_C, SEC_U, SEC_D, SEC_F, SEC_PRE, SEC_GVAL, SEC_GM, SEC_GD, SEC_CREC, SEC_CCS, SEC_ROWS };

// Reads every section in file order, checks the ones whose indices the
// kernels follow, and copies each to dst(section, table, key column) unless
// that is null.  The file must end after the last section.
template <typename DstFn>
gj_status read_sections(gj_ctx* ctx, FILE* f, const FileHdr& h, DstFn dst) {
  std::vector<char> buf;
  gj_status st = GJ_OK;
  for (int t = 0; t < h.n && !st; ++t) {
    const TabHdr& x = h.th[t];
    const int64_t E = x.entries, G = x.groups;
    for (int c = 0; c < x.k && !st; ++c)
      st = file_to_dev(ctx, f, static_cast<int32_t*>(dst(SEC_KEY, t, c)), E * 4, buf);
    if (!st) st = file_to_dev(ctx, f, static_cast<int64_t*>(dst(SEC_C, t, 0)), E * 8, buf, count_ok);
    const Section cols[4] = {SEC_U, SEC_D, SEC_F, SEC_PRE};
    for (int i = 0; i < 4 && !st; ++i) st = file_to_dev(ctx, f, static_cast<int64_t*>(dst(cols[i], t, 0)), E * 8, buf);
    if (t > 0 && !st) {
      st = file_to_dev(ctx, f, static_cast<int32_t*>(dst(SEC_GVAL, t, 0)), G * 4, buf);
      if (!st) st = file_to_dev(ctx, f, static_cast<int64_t*>(dst(SEC_GM, t, 0)), G * 8, buf);
      if (!st) st = file_to_dev(ctx, f, static_cast<int64_t*>(dst(SEC_GD, t, 0)), G * 8, buf);
      if (!st)
        st = file_to_dev(ctx, f, static_cast<ChildRec*>(dst(SEC_CREC, t, 0)),
                         h.th[x.parent].entries * sizeof(ChildRec), buf, crec_ok, &x.entries);
    }
    if (h.with_rows && !st) {
      st = file_to_dev(ctx, f, static_cast<int2*>(dst(SEC_CCS, t, 0)), E * sizeof(int2), buf, ccs_ok, &x.rows);
      if (!st) st = file_to_dev(ctx, f, static_cast<int32_t*>(dst(SEC_ROWS, t, 0)), x.rows * 4, buf, rows_ok, &x.rows);
    }
  }
  if (!st && fgetc(f) != EOF) {
    set_error("gj_summary_load: data after the last section");
    st = GJ_E_INVALID;
  }
  return st;
}

}  // namespace

extern "C" {

gj_status gj_summary_file_check(const char* path, gj_summary_file_info* info) {
  if (!path) {
    set_error("gj_summary_file_check: null path");
    return GJ_E_INVALID;
  }
  File fh;
  fh.f = fopen(path, "rb");
  if (!fh.f) {
    set_error("gj_summary_file_check: cannot open %s", path);
    return GJ_E_INVALID;
  }
  FileHdr h;
  gj_status st = read_headers(fh.f, path, h);
  if (!st) st = read_sections(nullptr, fh.f, h, [](Section, int, int) -> void* { return nullptr; });
  if (st) return st;
  if (info) {
    *info = gj_summary_file_info{};
    info->n_tables = h.n;
    info->projected = h.projected ? 1 : 0;
    info->with_rows = h.with_rows ? 1 : 0;
    info->join_size = h.join_size;
    for (int t = 0; t < h.n; ++t) {
      info->entries[t] = h.th[t].entries;
      info->rows[t] = h.th[t].rows;
    }
    info->bytes = (int64_t)ftell(fh.f);
  }
  return GJ_OK;
}

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
  FileHdr H;
  if (gj_status st = read_headers(fh.f, path, H)) return st;
  const int n = H.n;
  const bool projected = H.projected, with_rows = H.with_rows;
  const int64_t join_size = H.join_size;
  const std::vector<TabHdr>& th = H.th;
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
  int32_t* perm = f->F.perm;
  auto dst = [&](Section sec, int t, int c) -> void* {
    const TDesc& d = P.td[t];
    switch (sec) {
      case SEC_KEY: return S.ckey + d.key_off + (int64_t)c * d.n;
      case SEC_C: return S.cc + d.off;
      case SEC_U: return S.cU + d.off;
      case SEC_D: return S.cD + d.off;
      case SEC_F: return S.cF + d.off;
      case SEC_PRE: return S.cpre + d.off;
      case SEC_GVAL: return S.cgval + d.off;
      case SEC_GM: return S.cgM + d.off;
      case SEC_GD: return S.cgD + d.off;
      case SEC_CREC: return S.crec + d.link_off;
      case SEC_CCS: return S.ccs + d.off;
      case SEC_ROWS: return perm + d.off;
    }
    return nullptr;
  };
  gj_status st = read_sections(ctx, fh.f, H, dst);
  if (st) {
    gj_free_summary(s);
    return st;
  }
  *out = s;
  return GJ_OK;
}

}  // extern "C"
