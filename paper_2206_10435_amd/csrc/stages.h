// Device bodies of the factor-build and summary stages.
//
// Each body processes one work unit -- a tile of a table, one digit of a
// table, or a whole table -- and takes its LDS from the caller, so the same
// code runs as one kernel launch per stage (factor.hip, summary.hip: every
// block one unit of a work list) and inside the persistent batch kernel
// (batch.hip: any block runs any unit of any stage).  Bodies return only on
// block-uniform conditions, so every __syncthreads is reached by the whole
// block.  What they compute is described where they are launched.
#pragma once
#include "gj_internal.h"

namespace {

// ---------------------------------------------------------------------------
// sort words
// ---------------------------------------------------------------------------
template <int WIDE>
struct WordT;
template <>
struct WordT<0> {
  typedef uint64_t type;
};
template <>
struct WordT<1> {
  typedef W128 type;
};

__device__ __forceinline__ uint32_t digit_of(uint64_t w, int shift, uint32_t mask) {
  return (uint32_t)(w >> shift) & mask;
}
__device__ __forceinline__ uint32_t digit_of(const W128& w, int shift, uint32_t mask) {
  return (uint32_t)shr128_lo(w.lo, w.hi, shift) & mask;
}
// any bit at position >= s set?
__device__ __forceinline__ bool high_bits(uint64_t x, int s) { return s < 64 && (x >> s) != 0; }
__device__ __forceinline__ bool high_bits(const W128& x, int s) {
  if (s < 64) return (x.lo >> s) != 0 || x.hi != 0;
  return s < 128 && (x.hi >> (s - 64)) != 0;
}
__device__ __forceinline__ uint64_t wxor(uint64_t a, uint64_t b) { return a ^ b; }
__device__ __forceinline__ W128 wxor(const W128& a, const W128& b) { return W128{a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ uint64_t wlow(uint64_t a) { return a; }
__device__ __forceinline__ uint64_t wlow(const W128& a) { return a.lo; }
__device__ __forceinline__ uint32_t field_of(uint64_t w, int pos, int bits) {
  return bits == 0 ? 0u : (uint32_t)(w >> pos) & (uint32_t)((1ULL << bits) - 1);
}
__device__ __forceinline__ uint32_t field_of(const W128& w, int pos, int bits) {
  return bits == 0 ? 0u : (uint32_t)shr128_lo(w.lo, w.hi, pos) & (uint32_t)((1ULL << bits) - 1);
}

template <int WIDE>
__device__ __forceinline__ typename WordT<WIDE>::type* word_ptr(uint64_t* base, const TDesc& d) {
  return reinterpret_cast<typename WordT<WIDE>::type*>(base + d.word_off);
}

// Lanes of the wavefront holding the same `bits`-bit digit (and valid).
__device__ __forceinline__ uint64_t match_digit(uint32_t dig, bool valid, int bits) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    bool bit = (dig >> b) & 1u;
    uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// LDS bytes of each body (the persistent kernel takes the largest).
constexpr int LDS_UPSWEEP = GJ_WAVES * 256 * 4;
// downsweep: wh [GJ_WAVES][256], gb [256], ls [256], sh [GJ_WAVES], then the staged tile
constexpr int DS_GB = GJ_WAVES * 256 * 4;
constexpr int DS_LS = DS_GB + 256 * 4;
constexpr int DS_SH = DS_LS + 256 * 4;
constexpr int DS_STAGE = DS_SH + 16;
template <int WIDE, int ITEMS>
constexpr int lds_downsweep() {
  return DS_STAGE + GJ_BLOCK * ITEMS * (int)sizeof(typename WordT<WIDE>::type);
}
constexpr int LDS_SCAN64 = GJ_WAVES * 8;
constexpr int LDS_SCAN32 = GJ_WAVES * 4;
constexpr int LDS_SEG = 64 + GJ_BLOCK * 8;  // shv, shf, incl
#define DOWN_HASH 2048
constexpr int LDS_DOWN = DOWN_HASH * 4 + DOWN_HASH * 8;

// ---------------------------------------------------------------------------
// factor build
// ---------------------------------------------------------------------------

// One sort word per row of tile w: key fields above the row id.  It also
// counts the first radix pass's digits of every sort tile it covers (the
// counts that pass's upsweep would read the words again for).
constexpr int LDS_PACK = 2 * 256 * 4;  // a pack tile covers at most two sort tiles
template <int WIDE>
__device__ __forceinline__ void pack_body(const WorkItem w, const TDesc* __restrict__ D, uint64_t* __restrict__ words0,
                                          uint32_t* __restrict__ hist, void* lds) {
  uint32_t* h = reinterpret_cast<uint32_t*>(lds);
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  auto* out = word_ptr<WIDE>(words0, d);
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  const bool count = d.npasses > 0;
  const int nd = 1 << d.dbits;
  const uint32_t mask = (uint32_t)nd - 1;
  if (count) {
    for (int i = threadIdx.x; i < 2 * 256; i += GJ_BLOCK) h[i] = 0;
    __syncthreads();
  }
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    if (i >= d.n) break;
    uint64_t lo = (uint64_t)i, hi = 0;
#pragma unroll
    for (int c = 0; c < MAXK; ++c) {
      if (c < d.k && d.fbits[c] > 0) {
        uint64_t f = (uint64_t)((uint32_t)d.col[c][i] - d.kmin[c]);
        int p = d.rb + d.fshift[c];
        if (WIDE) {
          if (p < 64) {
            lo |= f << p;
            if (p > 32) hi |= f >> (64 - p);
          } else {
            hi |= f << (p - 64);
          }
        } else {
          lo |= f << p;
        }
      }
    }
    if constexpr (WIDE) {
      const W128 word{lo, hi};
      out[i] = word;
      if (count) atomicAdd(&h[((i - base) / d.sort_tile) * 256 + digit_of(word, d.sh0, mask)], 1u);
    } else {
      out[i] = lo;
      if (count) atomicAdd(&h[((i - base) / d.sort_tile) * 256 + digit_of(lo, d.sh0, mask)], 1u);
    }
  }
  if (count) {
    __syncthreads();
    const int nst = GJ_TILE / d.sort_tile;
    const int64_t st0 = base / d.sort_tile;
    for (int k = threadIdx.x; k < nst * nd; k += GJ_BLOCK) {
      const int64_t st = st0 + k / nd;
      if (st < d.ntiles_sort) hist[d.hist_off + (int64_t)(k % nd) * d.ntiles_sort + st] = h[(k / nd) * 256 + k % nd];
    }
  }
}

// Radix sort, one LSD pass = upsweep + digit scan + downsweep.
// Tile = GJ_BLOCK * ITEMS keys; wave v of the block owns keys
// [v*64*ITEMS, (v+1)*64*ITEMS) of the tile, visited in rounds of 64 so that
// (round, lane) order is the input order (needed for stability).
template <int WIDE, int ITEMS>
__device__ __forceinline__ void upsweep_body(const WorkItem w, const TDesc* __restrict__ D, uint64_t* words0,
                                             uint64_t* words1, uint32_t* __restrict__ hist, int pass, void* lds) {
  uint32_t(*wh)[256] = reinterpret_cast<uint32_t(*)[256]>(lds);
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const int db = d.dbits;
  const int nd = 1 << db;
  const uint32_t mask = (uint32_t)nd - 1;
  const int shift = d.sh0 + pass * db;
  const auto* in = word_ptr<WIDE>((pass & 1) ? words1 : words0, d);
  for (int i = threadIdx.x; i < GJ_WAVES * 256; i += GJ_BLOCK) (&wh[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)w.tile * (GJ_BLOCK * ITEMS);
  const int64_t cnt = min((int64_t)GJ_BLOCK * ITEMS, d.n - base);
  const int wv = wave_id();
  // counts only: any order, so block-strided loads and LDS adds into the
  // wave's own histogram
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t li = (int64_t)r * GJ_BLOCK + threadIdx.x;
    if (li < cnt) atomicAdd(&wh[wv][digit_of(in[base + li], shift, mask)], 1u);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < nd; g += GJ_BLOCK) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < GJ_WAVES; ++v) s += wh[v][g];
    hist[d.hist_off + (int64_t)g * d.ntiles_sort + w.tile] = s;
  }
}

// Digit g of table t: exclusive scan of that digit's counts over the table's
// tiles, in place; the digit total goes to dtot.
__device__ __forceinline__ void digit_scan_body(int t, int g, const TDesc* __restrict__ D, uint32_t* __restrict__ hist,
                                                uint32_t* __restrict__ dtot, void* lds) {
  uint32_t* sh = reinterpret_cast<uint32_t*>(lds);
  const TDesc& d = D[t];
  if (g >= (1 << d.dbits)) return;
  uint32_t* row = hist + d.hist_off + (int64_t)g * d.ntiles_sort;
  uint32_t carry = 0;
  for (int64_t i0 = 0; i0 < d.ntiles_sort; i0 += GJ_BLOCK) {
    int64_t i = i0 + threadIdx.x;
    uint32_t v = i < d.ntiles_sort ? row[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_excl_sum(v, sh, tot);
    if (i < d.ntiles_sort) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[t * 256 + g] = carry;
}

template <int WIDE, int ITEMS>
__device__ __forceinline__ void downsweep_body(const WorkItem w, const TDesc* __restrict__ D, uint64_t* words0,
                                               uint64_t* words1, const uint32_t* __restrict__ hist,
                                               const uint32_t* __restrict__ dtot, int pass, void* lds) {
  typedef typename WordT<WIDE>::type Word;
  unsigned char* L = reinterpret_cast<unsigned char*>(lds);
  uint32_t(*wh)[256] = reinterpret_cast<uint32_t(*)[256]>(L);
  uint32_t* gb = reinterpret_cast<uint32_t*>(L + DS_GB);
  uint32_t* ls = reinterpret_cast<uint32_t*>(L + DS_LS);
  uint32_t* sh = reinterpret_cast<uint32_t*>(L + DS_SH);
  Word* stage = reinterpret_cast<Word*>(L + DS_STAGE);
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const int db = d.dbits;
  const int nd = 1 << db;
  const uint32_t mask = (uint32_t)nd - 1;
  const int shift = d.sh0 + pass * db;
  const Word* in = word_ptr<WIDE>((pass & 1) ? words1 : words0, d);
  Word* out = word_ptr<WIDE>((pass & 1) ? words0 : words1, d);
  const int tid = threadIdx.x;
  for (int i = tid; i < GJ_WAVES * 256; i += GJ_BLOCK) (&wh[0][0])[i] = 0;
  // global start of every digit of this tile inside the table's output
  {
    uint32_t tot = tid < nd ? dtot[w.t * 256 + tid] : 0u;
    uint32_t T;
    uint32_t dbase = block_excl_sum(tot, sh, T);
    if (tid < nd) gb[tid] = dbase + hist[d.hist_off + (int64_t)tid * d.ntiles_sort + w.tile];
  }
  __syncthreads();
  const int64_t base = (int64_t)w.tile * (GJ_BLOCK * ITEMS);
  const int64_t cnt = min((int64_t)GJ_BLOCK * ITEMS, d.n - base);
  const int wv = wave_id(), ln = lane_id();
  Word key[ITEMS];
  uint32_t dig[ITEMS];
  uint32_t rank[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    int64_t li = (int64_t)wv * 64 * ITEMS + r * 64 + ln;
    bool valid = li < cnt;
    if (valid) key[r] = in[base + li];
    dig[r] = valid ? digit_of(key[r], shift, mask) : 0u;
    uint64_t peers = match_digit(dig[r], valid, db);
    uint64_t below = peers & lanemask_lt();
    uint32_t prev = wh[wv][dig[r]];
    rank[r] = prev + (uint32_t)__popcll(below);
    if (valid && below == 0) wh[wv][dig[r]] = prev + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t cntd = 0;
  if (tid < nd) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < GJ_WAVES; ++v) {
      uint32_t c = wh[v][tid];
      wh[v][tid] = s;
      s += c;
    }
    cntd = s;
  }
  {
    uint32_t T;
    uint32_t lstart = block_excl_sum(cntd, sh, T);
    if (tid < nd) ls[tid] = lstart;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    int64_t li = (int64_t)wv * 64 * ITEMS + r * 64 + ln;
    if (li < cnt) stage[ls[dig[r]] + wh[wv][dig[r]] + rank[r]] = key[r];
  }
  __syncthreads();
  for (int j = tid; j < cnt; j += GJ_BLOCK) {
    Word k = stage[j];
    uint32_t g = digit_of(k, shift, mask);
    out[gb[g] + (j - ls[g])] = k;
  }
}

// Runs: entry heads (key change) and separator-group heads (separator field
// change; the root is one group).  Counts per tile, then the write pass.
template <int WIDE>
__device__ __forceinline__ void run_flags(const typename WordT<WIDE>::type* wv, const TDesc& d, int64_t i, bool& head,
                                          bool& shead) {
  if (i == 0) {
    head = true;
    shead = true;
    return;
  }
  auto x = wxor(wv[i], wv[i - 1]);
  head = high_bits(x, d.rb);
  shead = !d.is_root && high_bits(x, d.rb + d.sepshift);
}

template <int WIDE>
__device__ __forceinline__ void runs_count_body(const WorkItem w, const TDesc* __restrict__ D, uint64_t* words0,
                                                uint64_t* words1, uint64_t* __restrict__ agg, void* lds) {
  uint64_t* sh = reinterpret_cast<uint64_t*>(lds);
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const auto* wv = word_ptr<WIDE>(d.final_buf ? words1 : words0, d);
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  uint64_t acc = 0;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    if (i < d.n) {
      bool h, s;
      run_flags<WIDE>(wv, d, i, h, s);
      acc += (uint64_t)h | ((uint64_t)s << 32);
    }
  }
  uint64_t tot;
  block_excl_sum(acc, sh, tot);
  if (threadIdx.x == 0) agg[d.agg_off + w.tile] = tot;
}

#ifndef RW_RP
#define RW_RP 1  // rounds of the run writer whose loads go before their stores (2 and 4 slower)
#endif
template <int WIDE>
__device__ __forceinline__ void runs_write_body(const WorkItem w, const TDesc* __restrict__ D, uint64_t* words0,
                                                uint64_t* words1, const uint64_t* __restrict__ agg, const FPtrs& P,
                                                void* lds) {
  uint64_t* sh = reinterpret_cast<uint64_t*>(lds);
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const auto* wv = word_ptr<WIDE>(d.final_buf ? words1 : words0, d);
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  const int64_t off = d.off;
  const uint64_t rbmask = d.rb == 0 ? 0ULL : ((1ULL << d.rb) - 1);
  uint64_t carry = agg[d.agg_off + w.tile];
  // RW_RP rounds at a time: their words and run flags first, then each
  // round's scan and stores (a wave's loads return only after its earlier
  // stores)
  for (int r0 = 0; r0 < GJ_ROUNDS; r0 += RW_RP) {
    typename WordT<WIDE>::type wd[RW_RP];
    bool hv[RW_RP], sv[RW_RP], nhv[RW_RP], nsv[RW_RP];
#pragma unroll
    for (int u = 0; u < RW_RP; ++u) {
      const int64_t i = base + (r0 + u) * GJ_BLOCK + threadIdx.x;
      hv[u] = sv[u] = nhv[u] = nsv[u] = false;
      if (i < d.n) {
        run_flags<WIDE>(wv, d, i, hv[u], sv[u]);
        if (i + 1 == d.n) {
          nhv[u] = true;
          nsv[u] = true;
        } else {
          run_flags<WIDE>(wv, d, i + 1, nhv[u], nsv[u]);
          if (d.is_root) nsv[u] = false;
        }
        wd[u] = wv[i];
      }
    }
#pragma unroll
    for (int u = 0; u < RW_RP; ++u) {
      const int64_t i = base + (r0 + u) * GJ_BLOCK + threadIdx.x;
      const bool h = hv[u], s = sv[u];
      uint64_t v = (uint64_t)h | ((uint64_t)s << 32);
      uint64_t tot;
      uint64_t ex = block_excl_sum(v, sh, tot) + carry;
      carry += tot;
      if (i >= d.n) continue;
      const int64_t e = (int64_t)(uint32_t)ex + (h ? 0 : -1);
      const int64_t g = (int64_t)(ex >> 32) + (s ? 0 : -1);
      const auto word = wd[u];
      P.perm[off + i] = (int32_t)(wlow(word) & rbmask);
      if (h) {
        P.estart[off + e] = (int32_t)i;
        P.egrp[off + e] = (int32_t)g;
        for (int c = 0; c < d.k; ++c) {
          uint32_t f = field_of(word, d.rb + d.fshift[c], d.fbits[c]);
          P.ekey[d.key_off + (int64_t)c * d.n + e] = d.vmap[c] ? d.vmap[c][f] : (int32_t)(f + d.kmin[c]);
        }
      }
      if (s) {
        P.glo[off + g] = (int32_t)e;
        int sc = d.is_root ? 0 : d.sep;
        uint32_t f = field_of(word, d.rb + d.fshift[sc], d.fbits[sc]);
        P.gval[off + g] = d.vmap[sc] ? d.vmap[sc][f] : (int32_t)(f + d.kmin[sc]);
      }
      if (nhv[u]) P.eend[off + e] = (int32_t)(i + 1);
      if (nsv[u]) P.ghi[off + g] = (int32_t)(e + 1);
    }
  }
}

// Dense separator index of tables whose separator values span a small range:
// didx[didx_off + gval(g) - dmin] = g for every separator group g.
__device__ __forceinline__ void group_index_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F) {
  const TDesc& d = D[w.t];
  if (d.didx_off < 0) return;
  const int64_t G = F.cnt[w.t * CNT_STRIDE + CNT_G];
  if (G == d.drange) return;  // every value is a group: the lookup needs no table
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t g = base + r * GJ_BLOCK + threadIdx.x;
    if (g >= G) break;
    F.didx[d.didx_off + ((int64_t)F.gval[d.off + g] - d.dmin)] = (int32_t)g;
  }
}

// Table t: exclusive scan (in place) of the table's tile aggregates, each a
// pair of 32-bit counts packed in a uint64 (no carry can cross the halves:
// counts are < 2^31); the totals go to cnt[t][ca], cnt[t][cb].
__device__ __forceinline__ void tile_scan_pair_body(int t, const TDesc* __restrict__ D, uint64_t* __restrict__ agg,
                                                    int64_t* __restrict__ cnt, int ca, int cb, void* lds) {
  uint64_t* sh = reinterpret_cast<uint64_t*>(lds);
  const TDesc& d = D[t];
  uint64_t carry = 0;
  for (int64_t i0 = 0; i0 < d.ntiles; i0 += GJ_BLOCK) {
    int64_t i = i0 + threadIdx.x;
    uint64_t v = i < d.ntiles ? agg[d.agg_off + i] : 0ULL;
    uint64_t tot;
    uint64_t ex = block_excl_sum(v, sh, tot);
    if (i < d.ntiles) agg[d.agg_off + i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    cnt[t * CNT_STRIDE + ca] = (int64_t)(uint32_t)carry;
    cnt[t * CNT_STRIDE + cb] = (int64_t)(carry >> 32);
  }
}

// ---------------------------------------------------------------------------
// summary
// ---------------------------------------------------------------------------

// Frequency of an entry: its row count, or the given count of a projected
// factor (where an entry stands for many rows of a deleted subtree).
__device__ __forceinline__ uint64_t entry_count(const FPtrs& F, int64_t se) {
  return F.ecnt ? (uint64_t)F.ecnt[se] : (uint64_t)(F.eend[se] - F.estart[se]);
}

// index of v in the ascending array a[0..n), or -1
__device__ __forceinline__ int32_t find_sorted(const int32_t* __restrict__ a, int64_t n, int32_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && a[lo] == v) ? (int32_t)lo : -1;
}

// A leaf with one row per group (a key column such as a primary key, with the
// rows' own counts): every group sends 1 (c = 1, U = 1).
__device__ __forceinline__ bool unit_leaf(const TDesc* __restrict__ D, const FPtrs& F, int ch) {
  return D[ch].nchild == 0 && F.ecnt == nullptr && F.cnt[ch * CNT_STRIDE + CNT_G] == D[ch].n;
}

// U per entry of tile w (looking each child value up in the child's group
// index or its sorted separator values, which also records the entry ->
// child-group link), and the tile aggregate of a segmented scan of c*U.
__device__ __forceinline__ void up_agg_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                            const SPtrs& S, void* lds) {
  uint64_t* shv = reinterpret_cast<uint64_t*>(lds);
  uint32_t* shf = reinterpret_cast<uint32_t*>(shv + GJ_WAVES);
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  uint64_t av = 0;
  uint32_t af = 0;
  if (base < M) {
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
      uint64_t cu = 0;
      uint32_t head = 0;
      if (e < M) {
        const int64_t se = d.off + e;
        uint64_t U = 1;
        uint64_t mi[MAXC];
#pragma unroll
        for (int i = 0; i < MAXC; ++i) {
          mi[i] = 1;
          if (i < d.nchild) {
            const int ch = d.child[i];
            const TDesc& dc = D[ch];
            const int32_t v = F.ekey[d.key_off + (int64_t)d.child_col[i] * d.n + e];
            int32_t j;
            if (dc.didx_off >= 0) {
              const int64_t x = (int64_t)v - dc.dmin;
              // when every value of the range is a group (a key column such
              // as a primary key), the group index is the offset itself
              const bool all = F.cnt[ch * CNT_STRIDE + CNT_G] == dc.drange;
              j = (x < 0 || x >= dc.drange) ? -1 : all ? (int32_t)x : F.didx[dc.didx_off + x];
            } else {
              j = find_sorted(F.gval + dc.off, F.cnt[ch * CNT_STRIDE + CNT_G], v);
            }
            S.link[dc.link_off + e] = j;
            const uint64_t m = j < 0 ? 0ULL : unit_leaf(D, F, ch) ? 1ULL : (uint64_t)S.Mg[dc.off + j];
            mi[i] = m;
            U = smul(U, m);
          }
        }
        // each child's product of the other children's messages, for the
        // children summed by buckets in the downward pass (it multiplies the
        // product in instead of gathering the messages again); for a unit
        // leaf it is U itself, which that pass reads instead
        {
          uint64_t pre = 1;
#pragma unroll
          for (int i = 0; i < MAXC; ++i) {
            if (i < d.nchild) {
              uint64_t x = pre;
#pragma unroll
              for (int i2 = i + 1; i2 < MAXC; ++i2)
                if (i2 < d.nchild) x = smul(x, mi[i2]);
              if (D[d.child[i]].dbucketed && !unit_leaf(D, F, d.child[i]))
                S.xprod[D[d.child[i]].link_off + e] = (int64_t)x;
              pre = smul(pre, mi[i]);
            }
          }
        }
        const uint64_t c = entry_count(F, se);
        cu = smul(c, U);
        S.U[se] = (int64_t)U;
        if (!d.is_root) head = (e == 0 || F.egrp[se] != F.egrp[se - 1]) ? 1u : 0u;
      }
      if (d.is_root) {
        // the root is one group: its tile aggregate is a plain (saturating)
        // sum, kept per thread and reduced once below
        av = sadd(av, cu);
        continue;
      }
      uint64_t tv;
      uint32_t tf;
      block_seg_incl(cu, head, shv, shf, tv, tf);
      av = tf ? tv : sadd(av, tv);
      af |= tf;
    }
  }
  if (d.is_root) {  // uniform
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) av = sadd(av, (uint64_t)__shfl_xor((long long)av, o, 64));
    if (lane_id() == 0) shv[wave_id()] = av;
    __syncthreads();
    av = 0;
#pragma unroll
    for (int v = 0; v < GJ_WAVES; ++v) av = sadd(av, shv[v]);
    af = (w.tile == 0 && M > 0) ? 1u : 0u;  // the head of the root's one group is entry 0
  }
  if (threadIdx.x == 0) {
    F.agg[d.agg_off + w.tile] = av;
    F.agg2[d.agg_off + w.tile] = af;
  }
}

// Table t: carry-in value of every tile of the segmented scan (exclusive),
// written over the tile aggregate.
__device__ __forceinline__ void seg_tiles_body(int t, const TDesc* __restrict__ D, const FPtrs& F, void* lds) {
  uint64_t* shv = reinterpret_cast<uint64_t*>(lds);
  uint32_t* shf = reinterpret_cast<uint32_t*>(shv + GJ_WAVES);
  uint64_t* incl = reinterpret_cast<uint64_t*>(reinterpret_cast<unsigned char*>(lds) + 64);
  const TDesc& d = D[t];
  uint64_t cv = 0;
  for (int64_t i0 = 0; i0 < d.ntiles; i0 += GJ_BLOCK) {
    const int64_t i = i0 + threadIdx.x;
    uint64_t v = 0;
    uint32_t f = 0;
    if (i < d.ntiles) {
      v = F.agg[d.agg_off + i];
      f = (uint32_t)F.agg2[d.agg_off + i];
    }
    uint64_t tv;
    uint32_t tf;
    block_seg_incl(v, f, shv, shf, tv, tf);
    const uint64_t mine = f ? v : sadd(cv, v);  // inclusive, with the carry
    incl[threadIdx.x] = mine;
    __syncthreads();
    const uint64_t ex = threadIdx.x == 0 ? cv : incl[threadIdx.x - 1];
    if (i < d.ntiles) F.agg[d.agg_off + i] = ex;
    cv = incl[GJ_BLOCK - 1];
    __syncthreads();
  }
}

// Exclusive prefix of c*U inside each separator group (the block offsets of
// desummarization), the group totals M, and the root's join size.
#ifndef US_RP
#define US_RP 1  // rounds of the upward scan whose loads go before their stores (4 slower)
#endif
__device__ __forceinline__ void up_scan_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                             const SPtrs& S, void* lds) {
  uint64_t* shv = reinterpret_cast<uint64_t*>(lds);
  uint32_t* shf = reinterpret_cast<uint32_t*>(shv + GJ_WAVES);
  uint64_t* incl = reinterpret_cast<uint64_t*>(reinterpret_cast<unsigned char*>(lds) + 64);
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  uint64_t cv = F.agg[d.agg_off + w.tile];
  // US_RP rounds at a time: their loads first, then each round's scan and
  // stores (a wave's loads return only after its earlier stores)
  for (int r0 = 0; r0 < GJ_ROUNDS; r0 += US_RP) {
    uint64_t cuv[US_RP];
    uint32_t hd[US_RP], lst[US_RP];
    int32_t grp[US_RP];
#pragma unroll
    for (int u = 0; u < US_RP; ++u) {
      const int64_t e = base + (r0 + u) * GJ_BLOCK + threadIdx.x;
      const int64_t se = d.off + e;
      cuv[u] = 0;
      hd[u] = 0;
      lst[u] = 0;
      grp[u] = 0;
      if (e < M) {
        cuv[u] = smul(entry_count(F, se), (uint64_t)S.U[se]);
        grp[u] = F.egrp[se];
        hd[u] = (e == 0 || grp[u] != F.egrp[se - 1]) ? 1u : 0u;
        lst[u] = ((e + 1 == M) || F.egrp[se + 1] != grp[u]) ? 1u : 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < US_RP; ++u) {
      const int64_t e = base + (r0 + u) * GJ_BLOCK + threadIdx.x;
      const int64_t se = d.off + e;
      uint64_t v = cuv[u];
      uint32_t f = hd[u];
      uint64_t tv;
      uint32_t tf;
      block_seg_incl(v, f, shv, shf, tv, tf);
      const uint64_t mine = f ? v : sadd(cv, v);
      incl[threadIdx.x] = mine;
      __syncthreads();
      if (e < M) {
        const uint64_t ex = hd[u] ? 0ULL : (threadIdx.x == 0 ? cv : incl[threadIdx.x - 1]);
        S.pre[se] = (int64_t)ex;
        if (lst[u]) {
          S.Mg[d.off + grp[u]] = (int64_t)mine;
          if (d.is_root) {
            S.qsize[d.query] = (int64_t)mine;
            S.qstatus[d.query] = mine >= SATV ? GJ_E_OVERFLOW : GJ_OK;
          }
        }
      }
      cv = incl[GJ_BLOCK - 1];
      __syncthreads();
    }
  }
}

// Downward messages into the children of tile w's table.  The terms of one
// tile are first summed per child group in an LDS hash table (linear
// probing; a key that finds no slot goes straight to global memory), so a
// heavily shared separator value costs one global atomic per tile instead of
// one per parent entry.
// SKIP_BUCKETED: children marked dbucketed are left to the bucketed pass
// below (the launch-per-stage path); without it every child is scattered
// here.
template <bool SKIP_BUCKETED = false>
__device__ __forceinline__ void down_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                          const SPtrs& S, void* lds) {
  int32_t* hkey = reinterpret_cast<int32_t*>(lds);
  unsigned long long* hval = reinterpret_cast<unsigned long long*>(reinterpret_cast<unsigned char*>(lds) + DOWN_HASH * 4);
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  for (int ci = 0; ci < d.nchild; ++ci) {
    const TDesc& dt = D[d.child[ci]];
    if (SKIP_BUCKETED && dt.dbucketed) continue;
    for (int i = threadIdx.x; i < DOWN_HASH; i += GJ_BLOCK) {
      hkey[i] = -1;
      hval[i] = 0;
    }
    __syncthreads();
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
      if (e >= M) break;
      const int64_t se = d.off + e;
      const uint64_t U = (uint64_t)S.U[se];
      if (U == 0) continue;
      const uint64_t Dp = d.is_root ? 1ULL : (uint64_t)S.Dg[d.off + F.egrp[se]];
      if (Dp == 0) continue;
      const uint64_t c = entry_count(F, se);
      const int32_t j = S.link[dt.link_off + e];
      // c * Dp * product of the other children's messages: U / M_ci when U
      // is exact (U > 0, so every message is > 0), else the product itself
      uint64_t term = smul(c, Dp);
      if (U < SATV) {
        term = smul(term, U / (uint64_t)S.Mg[dt.off + j]);
      } else {
        for (int i = 0; i < d.nchild; ++i) {
          if (i == ci) continue;
          const TDesc& dc = D[d.child[i]];
          term = smul(term, (uint64_t)S.Mg[dc.off + S.link[dc.link_off + e]]);
        }
      }
      uint32_t h = ((uint32_t)j * 2654435761u) >> 21;  // 11 bits
      bool placed = false;
#pragma unroll 1
      for (int p = 0; p < 8 && !placed; ++p) {
        const uint32_t slot = (h + p) & (DOWN_HASH - 1);
        const int32_t prev = atomicCAS(&hkey[slot], -1, j);
        if (prev == -1 || prev == j) {
          atomicAdd(&hval[slot], (unsigned long long)term);
          placed = true;
        }
      }
      if (!placed) atomicAdd((unsigned long long*)(S.Dg + dt.off + j), (unsigned long long)term);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < DOWN_HASH; i += GJ_BLOCK) {
      const int32_t j = hkey[i];
      if (j >= 0) atomicAdd((unsigned long long*)(S.Dg + dt.off + j), hval[i]);
    }
    __syncthreads();
  }
}

// ---- downward pass by buckets of the child's groups ----
// Child table ch of parent t (ch marked dbucketed): every
// parent entry e with a group j in ch is one item (j, c_e * D_t(e's group) *
// product of e's other children's messages), 0 when U_e or that D is 0.  A
// parent tile orders its items by bucket (j >> sh, 2^sh groups a bucket) in
// LDS and writes them to the tile's own slots in that order, with the start
// of every bucket; a reduce block then takes one bucket over a range of
// tiles, sums the bucket's runs per group in LDS and writes the sums to D of
// the bucket's groups (or adds them, when other tile ranges share the
// bucket).  Sums of integers: the order of the items does not change them.

// buckets of 2^sh groups, at most DOWN_BUCKETS of them (sh <= 12 below DOWN_MAX_GROUPS)
__device__ __forceinline__ int down_shift(int64_t G) {
  int sh = 0;
  while (((G - 1) >> sh) >= DOWN_BUCKETS) ++sh;
  return sh;
}
constexpr int DOWN_ACC = (DOWN_MAX_GROUPS / DOWN_BUCKETS);  // groups of one bucket at most
constexpr int DT_STAGE = 2 * DOWN_BUCKETS * 4 + LDS_SCAN32 + 16;
constexpr int LDS_DTILE = DT_STAGE + GJ_TILE * 12;
constexpr int DOWN_RTILES = 8 * GJ_BLOCK;  // tiles of one reduce range at most
#ifndef DOWN_RUNS
#define DOWN_RUNS 4  // runs per 16-lane group in flight in the bucket sums
#endif
constexpr int LDS_DRED = DOWN_ACC * 8 + (2 * DOWN_RTILES + 1) * 4 + LDS_SCAN32 + 12;

// Parent tile: each bucketed child's items in bucket order at the tile's
// slots [tile * GJ_TILE, ...) of the child's item arrays; bucket b's run
// starts at dhist[dhist_off + b * ntiles + tile] inside the tile (row
// DOWN_BUCKETS: the tile's item count).
__device__ __forceinline__ void down_tile_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                               const SPtrs& S, void* lds) {
  static_assert(GJ_BLOCK == DOWN_BUCKETS, "one thread per bucket");
  unsigned char* L = reinterpret_cast<unsigned char*>(lds);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(L);
  uint32_t* start = cnt + DOWN_BUCKETS;
  uint32_t* sh = start + DOWN_BUCKETS;
  int32_t* skey = reinterpret_cast<int32_t*>(L + DT_STAGE);
  uint64_t* sval = reinterpret_cast<uint64_t*>(skey + GJ_TILE);
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  const int tid = threadIdx.x;
  bool any = false;
  for (int ci = 0; ci < d.nchild; ++ci) any |= D[d.child[ci]].dbucketed != 0;
  if (!any) return;  // uniform: this parent's children take the atomic scatter
  // the entry part of every item, once per entry: c * D of its group (0 if U = 0)
  uint64_t cd[GJ_ROUNDS];
#pragma unroll
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + tid;
    cd[r] = 0;
    if (e < M) {
      const int64_t se = d.off + e;
      const uint64_t U = (uint64_t)S.U[se];
      const uint64_t Dp = d.is_root ? 1ULL : (uint64_t)S.Dg[d.off + F.egrp[se]];
      if (U != 0 && Dp != 0) cd[r] = smul(entry_count(F, se), Dp);
    }
  }
  for (int ci = 0; ci < d.nchild; ++ci) {
    const int ch = d.child[ci];
    const TDesc& dc = D[ch];
    if (!dc.dbucketed) continue;
    const int32_t* link = S.link + dc.link_off;
    const int shb = down_shift(F.cnt[ch * CNT_STRIDE + CNT_G]);
    cnt[tid] = 0;
    // every load of this child first (a wave's loads return only after its
    // earlier stores): links and products into registers, the stores last
    const bool unit = unit_leaf(D, F, ch);  // the product of the other messages is U
    int32_t jv[GJ_ROUNDS];
    uint64_t xv[GJ_ROUNDS];
#pragma unroll
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      const int64_t e = base + r * GJ_BLOCK + tid;
      jv[r] = -1;
      xv[r] = 0;
      if (e < M) {
        jv[r] = link[e];
        xv[r] = unit ? (uint64_t)S.U[d.off + e] : (uint64_t)S.xprod[dc.link_off + e];
      }
    }
    __syncthreads();
    int32_t rk[GJ_ROUNDS];  // rank inside the bucket (-1: no item)
#pragma unroll
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      rk[r] = -1;
      if (jv[r] >= 0) rk[r] = (int32_t)atomicAdd(&cnt[jv[r] >> shb], 1u);
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t st = block_excl_sum(cnt[tid], sh, tot);
    start[tid] = st;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      if (rk[r] < 0) continue;
      const uint32_t p = start[jv[r] >> shb] + (uint32_t)rk[r];
      skey[p] = jv[r];
      sval[p] = cd[r] ? smul(cd[r], xv[r]) : 0ULL;
    }
    __syncthreads();
    int32_t* okey = S.dkey + dc.link_off + base;
    int64_t* oval = S.dval + dc.link_off + base;
    for (uint32_t i = tid; i < tot; i += GJ_BLOCK) {
      okey[i] = skey[i];
      oval[i] = (int64_t)sval[i];
    }
    S.dhist[dc.dhist_off + (int64_t)tid * d.ntiles + w.tile] = st;
    if (tid == 0) S.dhist[dc.dhist_off + (int64_t)DOWN_BUCKETS * d.ntiles + w.tile] = tot;
    __syncthreads();
  }
}

// Reduce item (child ch, x): bucket x / ns, tile range x % ns of ns ranges of
// dslice(ch) parent tiles each.  The range's runs of the bucket are laid end
// to end (prefix of their lengths in LDS) and the block's threads take
// consecutive items of that sequence, so a wave reads whole lines.
__device__ __forceinline__ void down_reduce_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                                 const SPtrs& S, void* lds) {
  const int ch = w.t;
  if (!D[ch].dbucketed) return;
  unsigned char* L = reinterpret_cast<unsigned char*>(lds);
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(L);
  uint32_t* rbeg = reinterpret_cast<uint32_t*>(L + DOWN_ACC * 8);  // run start in the flat sequence
  uint32_t* rsrc = rbeg + DOWN_RTILES + 1;                          // run start in the tile's slots
  uint32_t* shs = rsrc + DOWN_RTILES;
  const TDesc& dc = D[ch];
  const TDesc& dp = D[dc.parent];
  const int64_t G = F.cnt[ch * CNT_STRIDE + CNT_G];
  const int sh = down_shift(G);
  const int nb = G > 0 ? (int)((G - 1) >> sh) + 1 : 0;
  const int TS = dc.dslice;  // tiles per range (<= DOWN_RTILES)
  const int ns = (dp.ntiles + TS - 1) / TS;
  const int b = w.tile / ns;
  const int x = w.tile - b * ns;
  if (b >= nb) return;
  const int64_t Mp = F.cnt[dc.parent * CNT_STRIDE + CNT_M];
  const int t0 = x * TS;
  const int nt = (int)max<int64_t>(0, min<int64_t>((int64_t)TS, (Mp + GJ_TILE - 1) / GJ_TILE - t0));
  if (nt == 0) return;  // uniform: D of the bucket's groups is already 0
  const int64_t g0 = (int64_t)b << sh;
  const int ng = (int)min((int64_t)1 << sh, G - g0);
  for (int i = threadIdx.x; i < ng; i += GJ_BLOCK) acc[i] = 0;
  const uint32_t* hb = S.dhist + dc.dhist_off + (int64_t)b * dp.ntiles + t0;
  uint32_t carry = 0;
  for (int i0 = 0; i0 < nt; i0 += GJ_BLOCK) {
    const int i = i0 + threadIdx.x;
    uint32_t s0 = 0, len = 0;
    if (i < nt) {
      s0 = hb[i];
      len = hb[dp.ntiles + i] - s0;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_sum(len, shs, tot);
    if (i < nt) {
      rbeg[i] = carry + ex;
      rsrc[i] = s0;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) rbeg[nt] = carry;
  __syncthreads();
  const int64_t o = dc.link_off + (int64_t)t0 * GJ_TILE;
  // each run (a tile's items of this bucket, contiguous) by a group of 16
  // lanes, DOWN_RUNS runs per group at a time, every lane's loads before its adds
  constexpr int RG = 16, NRG = GJ_BLOCK / RG;
  const int q = threadIdx.x / RG, ql = threadIdx.x % RG;
  for (int i0 = q; i0 < nt; i0 += DOWN_RUNS * NRG) {
    uint32_t len[DOWN_RUNS];
    int64_t at0[DOWN_RUNS];
    uint32_t lm = 0;
#pragma unroll
    for (int r = 0; r < DOWN_RUNS; ++r) {
      const int i = i0 + r * NRG;
      len[r] = 0;
      at0[r] = 0;
      if (i < nt) {
        len[r] = rbeg[i + 1] - rbeg[i];
        at0[r] = o + (int64_t)i * GJ_TILE + rsrc[i];
      }
      lm = max(lm, len[r]);
    }
    for (uint32_t k = ql; k < lm; k += 2 * RG) {
      int32_t key[2 * DOWN_RUNS];
      uint64_t val[2 * DOWN_RUNS];
#pragma unroll
      for (int u = 0; u < 2 * DOWN_RUNS; ++u) {
        const uint32_t kk = k + (u & 1) * RG;
        key[u] = -1;
        if (kk < len[u >> 1]) {
          key[u] = S.dkey[at0[u >> 1] + kk];
          val[u] = (uint64_t)S.dval[at0[u >> 1] + kk];
        }
      }
#pragma unroll
      for (int u = 0; u < 2 * DOWN_RUNS; ++u)
        if (key[u] >= 0) atomicAdd(&acc[key[u] - g0], (unsigned long long)val[u]);
    }
  }
  __syncthreads();
  unsigned long long* Dg = reinterpret_cast<unsigned long long*>(S.Dg + dc.off + g0);
  if (ns == 1) {
    for (int i = threadIdx.x; i < ng; i += GJ_BLOCK) Dg[i] = acc[i];
  } else {
    for (int i = threadIdx.x; i < ng; i += GJ_BLOCK)
      if (acc[i]) atomicAdd(&Dg[i], acc[i]);
  }
}

// Survivors: entries with c > 0, U > 0 and D > 0, groups with M > 0 and D > 0
// (a row count is never 0; a projected frequency can be).
__device__ __forceinline__ bool entry_survives(const TDesc& d, const FPtrs& F, const SPtrs& S, int64_t se) {
  if (S.U[se] == 0 || (F.ecnt && F.ecnt[se] == 0)) return false;
  return d.is_root || S.Dg[d.off + F.egrp[se]] > 0;
}
__device__ __forceinline__ bool group_survives(const TDesc& d, const SPtrs& S, int64_t sg) {
  return S.Mg[sg] > 0 && (d.is_root || S.Dg[sg] > 0);
}

__device__ __forceinline__ void compact_count_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                                   const SPtrs& S, void* lds) {
  uint64_t* sh = reinterpret_cast<uint64_t*>(lds);
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t G = F.cnt[w.t * CNT_STRIDE + CNT_G];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  uint64_t acc = 0;
  if (base < M) {
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
      if (e < M && entry_survives(d, F, S, d.off + e)) acc += 1;
      if (e < G && group_survives(d, S, d.off + e)) acc += 1ULL << 32;
    }
  }
  uint64_t tot;
  block_excl_sum(acc, sh, tot);
  if (threadIdx.x == 0) F.agg[d.agg_off + w.tile] = tot;
}

#ifndef CW_RP
#define CW_RP 1  // rounds of the compaction whose loads go before their stores (2 measured
                 // the same, 4 lost occupancy)
#endif
static_assert(GJ_ROUNDS % CW_RP == 0, "whole groups of rounds");
__device__ __forceinline__ void compact_write_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                                   const SPtrs& S, void* lds) {
  uint64_t* sh = reinterpret_cast<uint64_t*>(lds);
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t G = F.cnt[w.t * CNT_STRIDE + CNT_G];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  uint64_t carry = F.agg[d.agg_off + w.tile];
  // CW_RP rounds at a time: every load of those rounds, then their prefix
  // scans, then their stores (a wave's loads return only after its earlier
  // stores)
  for (int r0 = 0; r0 < GJ_ROUNDS; r0 += CW_RP) {
    bool es[CW_RP], gs[CW_RP];
    uint64_t c[CW_RP], U[CW_RP], Dv[CW_RP], pre[CW_RP], gM[CW_RP], gD[CW_RP];
    int32_t est[CW_RP], gv[CW_RP];
    int32_t key[CW_RP][MAXK];
#pragma unroll
    for (int u = 0; u < CW_RP; ++u) {
      const int64_t e = base + (r0 + u) * GJ_BLOCK + threadIdx.x;
      const int64_t se = d.off + e;
      es[u] = e < M && entry_survives(d, F, S, se);
      gs[u] = e < G && group_survives(d, S, se);
      if (es[u]) {
        c[u] = entry_count(F, se);
        U[u] = (uint64_t)S.U[se];
        Dv[u] = d.is_root ? 1ULL : (uint64_t)S.Dg[d.off + F.egrp[se]];
        pre[u] = (uint64_t)S.pre[se];
        est[u] = F.estart[se];
#pragma unroll
        for (int k = 0; k < MAXK; ++k)
          if (k < d.k) key[u][k] = F.ekey[d.key_off + (int64_t)k * d.n + e];
      }
      if (gs[u]) {
        gv[u] = F.gval[se];
        gM[u] = (uint64_t)S.Mg[se];
        gD[u] = d.is_root ? 1ULL : (uint64_t)S.Dg[se];
      }
    }
    int64_t ci[CW_RP], gi[CW_RP];
#pragma unroll
    for (int u = 0; u < CW_RP; ++u) {
      uint64_t tot;
      const uint64_t ex = block_excl_sum((uint64_t)es[u] | ((uint64_t)gs[u] << 32), sh, tot) + carry;
      carry += tot;
      ci[u] = (int64_t)(uint32_t)ex;
      gi[u] = (int64_t)(ex >> 32);
    }
#pragma unroll
    for (int u = 0; u < CW_RP; ++u) {
      const int64_t e = base + (r0 + u) * GJ_BLOCK + threadIdx.x;
      const int64_t se = d.off + e;
      if (e < M) {
        S.e2c[se] = (int32_t)ci[u];
        if (es[u]) {
          const int64_t sc = d.off + ci[u];
#pragma unroll
          for (int k = 0; k < MAXK; ++k)
            if (k < d.k) S.ckey[d.key_off + (int64_t)k * d.n + ci[u]] = key[u][k];
          S.cc[sc] = (int64_t)c[u];
          S.cU[sc] = (int64_t)U[u];
          S.cD[sc] = (int64_t)Dv[u];
          S.cF[sc] = (int64_t)smul(smul(c[u], U[u]), Dv[u]);
          S.cpre[sc] = (int64_t)pre[u];
          S.cstart[sc] = est[u];
          S.ccs[sc] = make_int2((int)c[u], est[u]);
        }
      }
      if (e < G) {
        S.g2c[se] = gs[u] ? (int32_t)gi[u] : -1;
        if (gs[u]) {
          const int64_t sg = d.off + gi[u];
          S.cgval[sg] = gv[u];
          S.cgM[sg] = (int64_t)gM[u];
          S.cgD[sg] = (int64_t)gD[u];
        }
      }
    }
  }
}

// Second compaction pass (needs every e2c / g2c).  What a child's group
// contributes to its parents' records depends on the group only, so every
// group's record is built once (group_recs) and copied to the records of the
// surviving parent entries that link to it (compact_links).
__device__ __forceinline__ void group_recs_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                                const SPtrs& S) {
  const TDesc& d = D[w.t];
  if (d.is_root) return;
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t G = F.cnt[w.t * CNT_STRIDE + CNT_G];
  const int64_t Mc = F.cnt[w.t * CNT_STRIDE + CNT_MC];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t g = base + r * GJ_BLOCK + threadIdx.x;
    if (g >= G) break;
    const int64_t sg = d.off + g;
    const int32_t gc = S.g2c[sg];
    if (gc < 0) continue;  // no surviving parent entry links here
    const int32_t glo = F.glo[sg], ghi = F.ghi[sg];
    ChildRec rc;
    rc.first = glo < M ? S.e2c[d.off + glo] : (int32_t)Mc;
    rc.end = ghi < M ? S.e2c[d.off + ghi] : (int32_t)Mc;
    const int2 cs0 = rc.first < rc.end ? S.ccs[d.off + rc.first] : make_int2(0, 0);
    rc.c0 = cs0.x;
    rc.st0 = cs0.y;
    S.grec[sg] = rc;
  }
}

__device__ __forceinline__ void compact_links_body(const WorkItem w, const TDesc* __restrict__ D, const FPtrs& F,
                                                   const SPtrs& S) {
  const TDesc& d = D[w.t];
  if (d.nchild == 0) return;
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  int32_t ci[GJ_ROUNDS];  // compacted index of each surviving entry, else -1
#pragma unroll
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    ci[r] = -1;
    if (e < M && entry_survives(d, F, S, d.off + e)) ci[r] = S.e2c[d.off + e];
  }
  // one child at a time, every round's gathers before its stores (a wave's
  // loads return only after its earlier stores)
  for (int i = 0; i < d.nchild; ++i) {
    const TDesc& dc = D[d.child[i]];
    const int4* grec = reinterpret_cast<const int4*>(S.grec + dc.off);
    int4* crec = reinterpret_cast<int4*>(S.crec + dc.link_off);
    const int32_t* link = S.link + dc.link_off + base + threadIdx.x;
    // a leaf with one row per group all of whose entries survive: group g is
    // entry g, of one row, at perm position g -- its record needs no gather
    const int ch = d.child[i];
    const bool unit = unit_leaf(D, F, ch) && F.cnt[ch * CNT_STRIDE + CNT_MC] == dc.n;
    int4 rec[GJ_ROUNDS];
#pragma unroll
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      // a surviving entry's child group survives (its message and its
      // downward message are both > 0)
      rec[r] = make_int4(0, 0, 0, 0);
      if (ci[r] >= 0) {
        const int32_t g = link[r * GJ_BLOCK];
        rec[r] = unit ? make_int4(g, g + 1, 1, g) : grec[g];
      }
    }
#pragma unroll
    for (int r = 0; r < GJ_ROUNDS; ++r)
      if (ci[r] >= 0) crec[ci[r]] = rec[r];
  }
}

}  // namespace
