// Stage 3 -- desummarization (Sec. 3.6) of a summary whose tables strictly
// between the root and the innermost table are keyed lookups: every surviving
// group of those tables holds one surviving entry (a dimension joined on its
// key, as in a star schema's fact-to-dimension links).
//
// The result order is the general one (desum_kernel.h): root entry, then each
// later table's entry inside its group, then the row ids as a mixed-radix
// number, table 0 most significant.  With one entry per group in the middle
// tables, a rank R decodes as
//   e_0   = the root entry whose block [pre_0(e_0), pre_0(e_0) + c_0 U_0) holds R,
//   e_t   = the only entry of the group that e_parent(t) links to (0 < t < n-1),
//   e_n-1 = the entry of the innermost group with P pre(e) <= R - pre_0(e_0),
//           P = c_0 c_1 ... c_n-2 (the product of the counts above it),
// and the offset inside that entry's block, R - pre_0(e_0) - P pre(e_n-1),
// splits into the row indexes (r_0, .., r_n-1) over the counts.
//
// Everything above the innermost table depends on the root entry only, so
// the expansion works in two levels.  A root entry's record -- its count and
// start, the middle tables' row ids (through their child records) and the
// innermost group's entry range and first entry -- is decoded once; a
// wavefront holds the records of 64 consecutive root entries, one per lane,
// in its LDS, and expands ranks 64 at a time, one per lane: a lane counts the
// held entries that start at or before its rank (a ballot for those before
// the window, byte marks in the LDS for those inside it), reads that entry's
// record from the LDS and gathers only the root's and the innermost table's
// row ids.  The tuples leave through the wave's LDS
// as contiguous 16-byte stores.  64 consecutive ranks span at most 64 root
// entries (every surviving entry's block is at least one rank), so a window
// that starts past the held entries reloads them from its first lane's entry.
//
// Decoding a record takes three dependent reads (the child records, a
// grandchild's record, the row ids), and reads issued while the expansion's
// stores stream out wait long.  So when the records of the chunk's root
// entries take at most a quarter of its output bytes, a pass of their own
// writes them first (k_unit_records, int32 arrays), and the expansion loads a
// wave's 64 records with one sequential read; otherwise (root entries of one
// or two tuples each) the expansion decodes them in place.
#include "desum_kernel.h"

namespace {

constexpr int UNIT_WAVE_TUPLES = 4096;  // tuples per wavefront (one cooperative locate each)

// Fields of a root entry's record, int32 each.  When the innermost table too
// holds one entry per group (TS), its group is that entry alone and the range
// fields are left out.
enum : int {
  F_C0 = 0,  // row count, negated when a middle count is above 1
  F_ST0,     // first position in the root's perm; its row id when the count is 1
  F_GC,      // innermost group: count of its first entry
  F_GST,     // perm start of its first entry
  F_GF,      // first surviving entry (not with TS)
  F_GE       // one past its last (not with TS)
};
// First field after the fixed ones: the middle tables' row ids (tables 1 ..
// n-2), or with value columns one slot per output column (its value when its
// table is a middle table, or the root's for a root entry of one row).
constexpr int f_mid(bool ts) { return ts ? 4 : 6; }
constexpr int n_fields(int n, bool ts, int n_cols) { return f_mid(ts) + (n_cols > 0 ? n_cols : n - 2); }

// LDS of one wavefront of the expansion: 64 records of nf fields, their block
// offsets, the window's entry-start marks and one window of tuples.
constexpr int unit_wave_lds(int nf, int tuple_bytes) { return 64 * nf * 4 + 64 * 8 + 64 + 64 * tuple_bytes; }

// The record of root entry x (fields as above; f[f_mid(TS) + t - 1] for middle
// table t, or with value columns (NC > 0) f[f_mid(TS) + j] for column j).
template <int N, bool TS, int NC, bool NT = false>
__device__ __forceinline__ void decode_entry(const gjk::DesumArgs& a, int n, int32_t x,
                                             int32_t (&f)[n_fields(N, TS, NC)]) {
  constexpr int FM = f_mid(TS);
  const int tl = n - 1;
  typedef int v4i __attribute__((ext_vector_type(4)));
  int2 cs;
  if constexpr (NT) {
    const uint64_t w = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(a.tab[0].ccs + x));
    cs.x = (int32_t)(uint32_t)w;
    cs.y = (int32_t)(uint32_t)(w >> 32);
  } else {
    cs = a.tab[0].ccs[x];
  }
  int32_t ent[N], pos[N];
  bool big = false;
  int32_t gf = 0, ge = 0, gc = 1, gst = 0;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    ent[t] = 0;
    pos[t] = 0;
  }
  ent[0] = x;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    if (t < n) {
      const int pt = a.tab[t].parent;
      int32_t ep = ent[0];
#pragma unroll
      for (int i = 1; i < N; ++i)
        if (i == pt) ep = ent[i];
      int4 rc;
      if (NT && pt == 0) {
        const v4i w = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(a.tab[t].crec + ep));
        rc.x = w.x;
        rc.y = w.y;
        rc.z = w.z;
        rc.w = w.w;
      } else {
        rc = *reinterpret_cast<const int4*>(a.tab[t].crec + ep);
      }
      ent[t] = rc.x;
      if (t < tl) {
        pos[t] = rc.w;
        big = big || rc.z != 1;
      } else {
        gf = rc.x;
        ge = rc.y;
        gc = rc.z;
        gst = rc.w;
      }
    }
  }
  f[F_C0] = big ? -cs.x : cs.x;
  // one row and no middle count above 1: the root's row index is always 0
  const bool one = cs.x == 1 && !big;
  f[F_GC] = gc;
  f[F_GST] = gst;
  if constexpr (!TS) {
    f[F_GF] = gf;
    f[F_GE] = ge;
  }
  if constexpr (NC == 0) {
    f[F_ST0] = one ? a.tab[0].perm[cs.y] : cs.y;
#pragma unroll
    for (int t = 1; t < N - 1; ++t) f[FM + t - 1] = t < tl ? a.tab[t].perm[pos[t]] : 0;
  } else {
    f[F_ST0] = cs.y;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      int32_t val = 0;
      if (j < a.n_cols) {
        const int tj = a.col_tab[j];
        int32_t pj = cs.y;  // the root's first row
#pragma unroll
        for (int t = 1; t < N; ++t)
          if (t == tj) pj = pos[t];
        if ((tj >= 1 && tj < tl) || (tj == 0 && one)) val = a.col_src[j][pj];
      }
      f[FM + j] = val;
    }
  }
}

// range[0], range[1]: the root entries of the chunk's first and last ranks
// (one wave).
__global__ void __launch_bounds__(64) k_unit_range(gjk::DesumArgs a, int64_t* __restrict__ range) {
  const int ln = lane_id();
  const int32_t nroot = (int32_t)a.n_root;
  const int32_t e_first = find_block(a.tab[0].cpre, 0, nroot, 1, (uint64_t)a.first, ln);
  const int32_t e_last = find_block(a.tab[0].cpre, e_first, nroot, 1, (uint64_t)(a.first + a.n_rows - 1), ln);
  if (ln == 0) {
    range[0] = e_first;
    range[1] = e_last;
  }
}

// Records of root entries range[0] .. range[1], field f of entry range[0] + i
// at rec[f * cap + i].
template <int N, bool TS, int NC>
__global__ void __launch_bounds__(GJ_BLOCK) k_unit_records(gjk::DesumArgs a, const int64_t* __restrict__ range,
                                                           int32_t* __restrict__ rec, int64_t cap) {
  constexpr int NF = n_fields(N, TS, NC);
  const int n = (N <= 8 && NC == 0) ? N : a.n_tables;
  const int nf = n_fields(n, TS, NC == 0 ? 0 : a.n_cols);
  const int64_t i = (int64_t)blockIdx.x * GJ_BLOCK + threadIdx.x;
  const int64_t e0 = range[0];
  if (i > range[1] - e0 || i >= cap) return;
  int32_t f[NF];
  decode_entry<N, TS, NC, true>(a, n, (int32_t)(e0 + i), f);
#pragma unroll
  for (int k = 0; k < NF; ++k)
    if (k < nf) __builtin_nontemporal_store(f[k], rec + k * cap + i);
}

// NC == 0: the output columns are the row ids of the n tables (N <= 8 is the
// exact table count).  NC > 0: the output columns are a.n_cols <= NC int32
// value columns, column j read from a.col_src[j] at the group position of
// table a.col_tab[j]; N is then an upper bound of the table count.
template <int N, typename WT, bool REC, bool TS, int NC>
__global__ void __launch_bounds__(GJ_BLOCK) k_desum_unit(gjk::DesumArgs a, const int64_t* __restrict__ range,
                                                         const int32_t* __restrict__ rec, int64_t cap) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int NF = n_fields(N, TS, NC);  // fields of a record
  constexpr int FM = f_mid(TS);
  constexpr int NCOL = NC == 0 ? N : NC;  // register capacity for output columns
  const int n = (N <= 8 && NC == 0) ? N : a.n_tables;
  const int nc = NC == 0 ? n : a.n_cols;
  const int nf = n_fields(n, TS, NC == 0 ? 0 : nc);
  const int tl = n - 1;  // innermost table, a leaf
  const int ln = lane_id();
  // XCD-aware order: consecutive wave ranges on the same XCD
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t w0 = ((int64_t)lb * GJ_WAVES + wave_id()) * UNIT_WAVE_TUPLES;
  if (w0 >= a.n_rows) return;  // wave-uniform
  const int64_t w1 = min(a.n_rows, w0 + (int64_t)UNIT_WAVE_TUPLES);
  const int tb = nc * (int)sizeof(WT);  // tuple bytes
  unsigned char* wl = lds_raw + (int64_t)wave_id() * unit_wave_lds(NF, NCOL * (int)sizeof(WT));
  int32_t* tab = reinterpret_cast<int32_t*>(wl);                      // records, [field * 64 + lane]
  uint64_t* toff = reinterpret_cast<uint64_t*>(wl + 64 * NF * 4);     // their block offsets
  unsigned char* mark = wl + 64 * NF * 4 + 64 * 8;                    // entry starts in a window
  unsigned char* stage = wl + 64 * NF * 4 + 64 * 8 + 64;              // one window of tuples
  unsigned char* dst_base = reinterpret_cast<unsigned char*>(a.out);

  const int64_t* __restrict__ pre0 = a.tab[0].cpre;
  const int32_t nroot = (int32_t)a.n_root;
  int64_t r0 = 0;  // first root entry with a record
  int32_t lo = 0, hi = nroot;
  if constexpr (REC) {
    r0 = range[0];
    lo = (int32_t)r0;
    hi = (int32_t)range[1] + 1;
  }

  // ---- the records of root entries C .. C+63 and their block offsets ----
  int32_t C = 0;
  uint64_t v = 0, vn = 0;
  auto load_table = [&](int32_t c) {
    C = __builtin_amdgcn_readfirstlane(c);
    // lanes past the chunk's last root entry repeat it (their offsets are
    // ~0, so no rank selects them)
    const int32_t x = min(C + ln, hi - 1);
    v = C + ln < hi ? (uint64_t)pre0[C + ln] : ~0ull;
    vn = C + 64 < hi ? (uint64_t)pre0[C + 64] : ~0ull;
    int32_t f[NF];
    if constexpr (REC) {
      const int32_t* rp = rec + (x - r0);
#pragma unroll
      for (int k = 0; k < NF; ++k) f[k] = k < nf ? rp[k * cap] : 0;
    } else {
      decode_entry<N, TS, NC>(a, n, x, f);
    }
    // every read of the previous records precedes this point in the wave's
    // program order
#pragma unroll
    for (int k = 0; k < NF; ++k)
      if (k < nf) tab[k * 64 + ln] = f[k];
    toff[ln] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // With records: the next 64 (entries C+64 ..) are held in registers,
  // loaded when the wave moves to the current ones, so that moving on writes
  // registers into the LDS instead of waiting for a read queued behind the
  // window's stores.  A window reaching into them reads their fields from
  // the owning lanes.
  int32_t fb[NF];
  uint64_t vb = ~0ull, vnn = ~0ull;  // their block offsets; the start of entry C+128
#pragma unroll
  for (int k = 0; k < NF; ++k) fb[k] = 0;
  auto prefetch_next = [&]() {
    const int32_t xb = C + 64 + ln;
    const int32_t xc = min(xb, hi - 1);
    vb = xb < hi ? (uint64_t)pre0[xb] : ~0ull;
    vnn = C + 128 < hi ? (uint64_t)pre0[C + 128] : ~0ull;
    const int32_t* rp = rec + (xc - r0);
#pragma unroll
    for (int k = 0; k < NF; ++k) fb[k] = k < nf ? rp[k * cap] : 0;
  };
  auto move_on = [&]() {
    C = __builtin_amdgcn_readfirstlane(C + 64);
    v = vb;
    vn = vnn;
#pragma unroll
    for (int k = 0; k < NF; ++k)
      if (k < nf) tab[k * 64 + ln] = fb[k];
    toff[ln] = vb;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    prefetch_next();
  };
  // root entry of the wave's first rank (every lane the same rank: the
  // cooperative search of the general kernel)
  load_table(find_block(pre0, lo, hi, 1, (uint64_t)(a.first + w0), ln));
  if constexpr (REC) prefetch_next();

  for (int64_t t0 = w0; t0 < w1; t0 += 64) {
    // ---- the lane's root entry and its record ----
    // Ranks Rw + li, li = 0..last, of the window; the held entries start at
    // v_k (lane k), so a lane's entry is the number of held entries starting
    // at or before Rw + li, minus one: those starting at or before Rw (a
    // ballot) plus those starting at window positions 1..li (marks in LDS).
    const uint64_t Rw = (uint64_t)(a.first + t0);
    const int last = (int)min((int64_t)63, w1 - 1 - t0);
    const int li = min(ln, last);  // lanes past the range repeat the last rank
    // the held entries must reach the window's last rank (the entry after
    // them starts at vn); else reload from the entry of Rw: the last held
    // entry starting at or before Rw, or the one after the held entries
    // (the previous window ended inside them)
    if constexpr (REC) {
      // Rw's entry lies in the held or the next 64 (the previous window
      // ended in the held ones and a window spans at most 64 entries), so
      // the window ends inside the two sets
      if (vn <= Rw) move_on();
    } else {
      for (int it = 0; it < 2 && vn <= Rw + (uint64_t)last; ++it) {
        const int n0 = __popcll(__ballot(v <= Rw));
        load_table(vn <= Rw ? C + 64 : C + n0 - 1);
      }
    }
    const int n0 = __popcll(__ballot(v <= Rw)) + (REC ? __popcll(__ballot(vb <= Rw)) : 0);
    // window positions of the entry starts (0: at or before Rw, 64: after)
    const int d = v <= Rw ? 0 : (v - Rw < 64 ? (int)(v - Rw) : 64);
    const int db = vb <= Rw ? 0 : (vb - Rw < 64 ? (int)(vb - Rw) : 64);
    mark[ln] = 0;
    if (d >= 1 && d <= 63) mark[d] = 1;
    if (REC && db >= 1 && db <= 63) mark[db] = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int cnt = 0;  // starts at positions 1..li (bytes of 0 or 1, position 0 never marked)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t w = *reinterpret_cast<const uint64_t*>(mark + 8 * k);
      const int hi_byte = li - 8 * k;  // last byte of this word at or before li
      const uint64_t m = hi_byte < 0 ? 0ull : hi_byte >= 7 ? ~0ull : (~0ull >> (8 * (7 - hi_byte)));
      cnt += __popcll(w & m);
    }
    const int jj = n0 - 1 + cnt;  // 0..63 held, 64..127 next (records only)
    const int j6 = jj & 63;
    const int32_t e0 = C + jj;
    int32_t g[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) g[k] = k < nf ? tab[k * 64 + j6] : 0;
    uint64_t vj = toff[j6];
    if (REC && __any(jj >= 64)) {
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        const int32_t x = __shfl(fb[k], j6);
        if (jj >= 64) g[k] = x;
      }
      const uint64_t x = __shfl(vb, j6);
      if (jj >= 64) vj = x;
    }
    const uint64_t R1 = Rw + (uint64_t)li - vj;
    const int32_t c0 = g[F_C0];
    const int32_t st0 = g[F_ST0];
    const int32_t gf = TS ? 0 : g[F_GF];
    const int32_t ge = TS ? 1 : g[F_GE];
    int32_t c = g[F_GC];
    int32_t st = g[F_GST];

    // ---- innermost entry inside its group, the row indexes ----
    const gjk::DTab& T = a.tab[tl];
    const bool big = c0 < 0;
    // P: the product of the counts above the innermost table; with a middle
    // count above 1 (rare) the middle tables' child records are read again
    uint64_t P = (uint32_t)(big ? -c0 : c0);
    int32_t cm[N], pm[N], rm[N];  // middle counts, perm starts and row indexes (big only)
#pragma unroll
    for (int t = 0; t < N; ++t) {
      cm[t] = 1;
      pm[t] = 0;
      rm[t] = 0;
    }
    if (__any(big)) {
      if (big) {
        int32_t ent[N];
#pragma unroll
        for (int t = 0; t < N; ++t) ent[t] = 0;
        ent[0] = e0;
#pragma unroll
        for (int t = 1; t < N; ++t) {
          if (t < tl) {
            const int pt = a.tab[t].parent;
            int32_t ep = ent[0];
#pragma unroll
            for (int i = 1; i < N; ++i)
              if (i == pt) ep = ent[i];
            const int4 rc = *reinterpret_cast<const int4*>(a.tab[t].crec + ep);
            ent[t] = rc.x;
            cm[t] = rc.z;
            pm[t] = rc.w;
            P *= (uint64_t)rc.z;
          }
        }
      }
    }
    uint64_t R2 = R1;
    if (!TS && __any(ge - gf > 1)) {
      const int32_t x = find_block(T.cpre, gf, ge, P, R1, ln);
      if (x != gf) {
        R2 -= P * (uint64_t)T.cpre[x];
        const int2 cs = T.ccs[x];
        c = cs.x;
        st = cs.y;
      }
    }
    // R2 < P * c: the row indexes, innermost fastest
    uint64_t q = 0;
    uint32_t rt = (uint32_t)R2;
    if (P != 1) {
      if ((R2 >> 32) == 0) {
        q = (uint32_t)R2 / (uint32_t)c;
        rt = (uint32_t)R2 - (uint32_t)q * (uint32_t)c;
      } else {
        q = R2 / (uint64_t)c;
        rt = (uint32_t)(R2 - q * (uint64_t)c);
      }
    }
    if (__any(big)) {
      if (big) {
        // middle tables from the innermost side: r_t = q mod c_t
#pragma unroll
        for (int t = N - 1; t >= 1; --t) {
          if (t < tl) {
            const uint64_t qt = q / (uint64_t)cm[t];
            rm[t] = (int32_t)(q - qt * (uint64_t)cm[t]);
            q = qt;
          }
        }
      }
    }
    // the gathers: the root's and the innermost table's rows (the root's held
    // in the record for a one-row entry), a middle table's only when its row
    // index is not 0
    int32_t rid[NCOL];
    if constexpr (NC == 0) {
#pragma unroll
      for (int t = 0; t < N; ++t) {
        rid[t] = 0;
        if (t >= 1 && t < tl) rid[t] = rm[t] != 0 ? a.tab[t].perm[pm[t] + rm[t]] : g[FM + t - 1];
      }
      rid[0] = c0 == 1 ? st0 : a.tab[0].perm[st0 + (int32_t)q];
      rid[tl] = T.perm[st + (int32_t)rt];
    } else {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        rid[j] = 0;
        if (j < nc) {
          const int tj = a.col_tab[j];
          const int32_t* src = a.col_src[j];
          if (tj == tl) {
            rid[j] = src[st + (int32_t)rt];
          } else if (tj == 0) {
            rid[j] = c0 == 1 ? g[FM + j] : src[st0 + (int32_t)q];
          } else {
            int32_t r = 0, p = 0;
#pragma unroll
            for (int t = 1; t < N; ++t)
              if (t == tj) {
                r = rm[t];
                p = pm[t];
              }
            rid[j] = r != 0 ? src[p + r] : g[FM + j];
          }
        }
      }
    }

    // ---- the window through the wave's LDS ----
    const int nv = (int)min((int64_t)64, w1 - t0);
    WT* my = reinterpret_cast<WT*>(stage + ln * tb);
#pragma unroll
    for (int t = 0; t < NCOL; ++t)
      if (t < nc) my[t] = NC == 0 ? (WT)(uint32_t)rid[t] : (WT)rid[t];  // row ids are non-negative
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // window start: 64 tuples from a multiple of 64, so 16-byte aligned
    unsigned char* dst = dst_base + t0 * tb;
    const int bytes = nv * tb;
    for (int u = ln; u * 16 < bytes; u += 64) {
      const unsigned char* sp = stage + u * 16;
      if (u * 16 + 16 <= bytes) {
        const uint4 val = *reinterpret_cast<const uint4*>(sp);
        uint32_t* d = reinterpret_cast<uint32_t*>(dst + u * 16);
        __builtin_nontemporal_store(val.x, d);
        __builtin_nontemporal_store(val.y, d + 1);
        __builtin_nontemporal_store(val.z, d + 2);
        __builtin_nontemporal_store(val.w, d + 3);
      } else {
        for (int x = u * 16; x < bytes; x += 4)
          *reinterpret_cast<uint32_t*>(dst + x) = *reinterpret_cast<const uint32_t*>(stage + x);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int N, typename WT, bool TS, int NC>
void launch_unit(hipStream_t s, const gjk::DesumArgs& a, int blocks, int64_t* range, int32_t* rec, int64_t cap) {
  const size_t lds = (size_t)GJ_WAVES * unit_wave_lds(n_fields(N, TS, NC), (NC == 0 ? N : NC) * (int)sizeof(WT));
  if (rec) {
    hipLaunchKernelGGL(k_unit_range, dim3(1), dim3(64), 0, s, a, range);
    const int64_t rb = (cap + GJ_BLOCK - 1) / GJ_BLOCK;
    hipLaunchKernelGGL((k_unit_records<N, TS, NC>), dim3((unsigned)rb), dim3(GJ_BLOCK), 0, s, a, range, rec, cap);
    hipLaunchKernelGGL((k_desum_unit<N, WT, true, TS, NC>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a, range, rec,
                       cap);
  } else {
    hipLaunchKernelGGL((k_desum_unit<N, WT, false, TS, NC>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a, range, rec,
                       cap);
  }
}

// row ids: exact table count up to 8, else the instance for any count
template <int N>
void launch_rows(hipStream_t s, const gjk::DesumArgs& a, int rowid_bytes, int blocks, int64_t* range, int32_t* rec,
                 int64_t cap, bool tl_single) {
  if (rowid_bytes == 4) {
    if (tl_single)
      launch_unit<N, int32_t, true, 0>(s, a, blocks, range, rec, cap);
    else
      launch_unit<N, int32_t, false, 0>(s, a, blocks, range, rec, cap);
  } else {
    if (tl_single)
      launch_unit<N, int64_t, true, 0>(s, a, blocks, range, rec, cap);
    else
      launch_unit<N, int64_t, false, 0>(s, a, blocks, range, rec, cap);
  }
}

// value columns: at most 4, 8 or 16 tables and 4, 8 or 16 columns
template <int N, int NC>
void launch_values_nc(hipStream_t s, const gjk::DesumArgs& a, int blocks, int64_t* range, int32_t* rec, int64_t cap,
                      bool tl_single) {
  if (tl_single)
    launch_unit<N, int32_t, true, NC>(s, a, blocks, range, rec, cap);
  else
    launch_unit<N, int32_t, false, NC>(s, a, blocks, range, rec, cap);
}

template <int N>
void launch_values_n(hipStream_t s, const gjk::DesumArgs& a, int blocks, int64_t* range, int32_t* rec, int64_t cap,
                     bool tl_single) {
  if (a.n_cols <= 4)
    launch_values_nc<N, 4>(s, a, blocks, range, rec, cap, tl_single);
  else if (a.n_cols <= 8)
    launch_values_nc<N, 8>(s, a, blocks, range, rec, cap, tl_single);
  else
    launch_values_nc<N, GJ_MAX_OUT_COLS>(s, a, blocks, range, rec, cap, tl_single);
}

}  // namespace

namespace gjk {

int64_t desum_unit_blocks(int64_t n_rows) {
  const int64_t waves = (n_rows + UNIT_WAVE_TUPLES - 1) / UNIT_WAVE_TUPLES;
  const int64_t blocks = (waves + GJ_WAVES - 1) / GJ_WAVES;
  return (blocks + 7) / 8 * 8;  // whole XCD rounds for the block remap
}

int64_t desum_unit_record_bytes(int64_t cap, int n_tables, bool tl_single, int n_cols) {
  return cap * (int64_t)n_fields(n_tables, tl_single, n_cols) * 4;
}

int64_t desum_unit_record_entries(int64_t n_root, int64_t n_rows, int n_tables, bool tl_single, int n_cols,
                                  int tuple_bytes) {
  // the chunk's ranks span at most min(n_root, n_rows) root entries; records
  // only when they take at most a quarter of the chunk's output bytes
  const int64_t cap = std::min(n_root, n_rows);
  const int64_t rec_bytes = desum_unit_record_bytes(cap, n_tables, tl_single, n_cols);
  return rec_bytes * 4 <= n_rows * (int64_t)tuple_bytes ? cap : 0;
}

int desummarize_unit(hipStream_t s, const DesumArgs& a0, int rowid_bytes, int n_tables, bool tl_single, int64_t* range,
                     int32_t* rec, int64_t cap) {
  if (a0.n_rows <= 0) return 0;
  const bool values = a0.n_cols > 0;
  if (n_tables < 2 || n_tables > GJ_MAX_TABLES || (rowid_bytes != 4 && rowid_bytes != 8) ||
      (values && (rowid_bytes != 4 || a0.n_cols > GJ_MAX_OUT_COLS)) ||
      (rec && (!range || cap < std::min(a0.n_root, a0.n_rows))))
    return -1;
  const int64_t blocks = desum_unit_blocks(a0.n_rows);
  if (blocks > 0x7fffffff || (rec && (cap + GJ_BLOCK - 1) / GJ_BLOCK > 0x7fffffff)) return -1;
  DesumArgs a = a0;
  a.n_tables = n_tables;
  const int nb = (int)blocks;
  if (values) {
    if (n_tables <= 4)
      launch_values_n<4>(s, a, nb, range, rec, cap, tl_single);
    else if (n_tables <= 8)
      launch_values_n<8>(s, a, nb, range, rec, cap, tl_single);
    else
      launch_values_n<GJ_MAX_TABLES>(s, a, nb, range, rec, cap, tl_single);
    return 0;
  }
  switch (n_tables) {
    case 2: launch_rows<2>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    case 3: launch_rows<3>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    case 4: launch_rows<4>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    case 5: launch_rows<5>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    case 6: launch_rows<6>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    case 7: launch_rows<7>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    case 8: launch_rows<8>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
    default: launch_rows<GJ_MAX_TABLES>(s, a, rowid_bytes, nb, range, rec, cap, tl_single); break;
  }
  return 0;
}

}  // namespace gjk
