// Internal definitions shared by the HIP translation units of libgj.
//
// Memory layout.  A *plan* is a set of tables (one query, or many queries of a
// batch).  Every per-row and per-entry array is one flat device array of S
// "slots": table t owns slots [off_t, off_t + n_t).  A table has at most n_t
// factor entries and at most n_t separator groups, so entry e of table t lives
// at slot off_t + e and group g at slot off_t + g -- nothing is sized by data,
// which is what lets a whole batch be recorded as a graph with no host
// synchronization.  Kernels walk (table, tile) work lists and skip tiles past
// the table's actual entry count, read from device memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gj.h"

#define GJ_BLOCK 256
#define GJ_WAVES (GJ_BLOCK / 64)
#define MAXK GJ_MAX_KEYS
#define MAXC GJ_MAX_CHILDREN

// device counters per table (int64): cnt[t * CNT_STRIDE + CNT_x]
#define CNT_STRIDE 8
#define CNT_M 0   // factor entries
#define CNT_G 1   // separator groups (the root has one group: the whole table)
#define CNT_MC 2  // surviving entries
#define CNT_GC 3  // surviving groups

#define SATV 0x7fffffffffffffffULL

struct WorkItem {
  int32_t t;
  int32_t tile;
};

struct TDesc {
  const int32_t* col[MAXK];  // input key columns (valid while factors are built)
  int64_t n;                 // rows
  int64_t off;               // slot offset
  int64_t key_off;           // entry keys: ekey[key_off + c * n + e]
  int64_t link_off;          // (t >= 1) link[link_off + parent entry] -> group of t
  int64_t agg_off;           // tile aggregates of this table
  int64_t hist_off;          // radix histogram region (2^dbits * ntiles_sort)
  int64_t word_off;          // sort words start at words[b] + word_off (uint64 units)
  int32_t k, sep, parent, pcol;
  int32_t nchild, query, depth, height;
  int32_t child[MAXC];
  int32_t child_col[MAXC];  // column of this table that child i joins on
  uint32_t kmin[MAXK];      // per declared column: minimum value (as uint32 of int32)
  // per declared column: null, or the column's distinct values in ascending
  // order when col[c] holds each row's rank among them (a column compressed
  // so that the table's key fits the sort word; field f decodes to vmap[c][f])
  const int32_t* vmap[MAXK];
  int32_t fshift[MAXK];     // per declared column: field position above the row-id bits
  int32_t fbits[MAXK];      // per declared column: field width
  int32_t rb;               // row-id bits (low bits of every sort word)
  int32_t keybits;          // total key bits
  int32_t wide;             // 1: 128-bit words, 0: 64-bit words
  int32_t npasses, dbits;   // radix passes over the key bits and digit width
  int32_t sh0;              // bit position of digit 0 of the passes (rb, or the top digits' base)
  int32_t local;            // 1: the passes take the top two digits, buckets are sorted in LDS
  int32_t npasses_full;     // passes of the plain radix sort (host only)
  int32_t sort_tile;        // keys per sort tile
  int32_t final_buf;        // word buffer (0/1) holding the sorted words
  int32_t sepshift;         // (t >= 1) separator field position within the key bits
  int32_t ntiles_sort;      // ceil(n / sort_tile)
  int32_t ntiles;           // ceil(n / GJ_TILE)
  int32_t is_root;
  // (t >= 1) separator value -> group: didx[didx_off + v - dmin] for v in
  // [dmin, dmin + drange) when the values are dense enough (didx_off >= 0)
  int64_t didx_off;
  int64_t drange;
  int32_t dmin;
  // (t >= 1) downward pass by buckets of this table's groups: start of
  // bucket b's items inside parent tile x at dhist[dhist_off + b *
  // ntiles(parent) + x] (row DOWN_BUCKETS: the tile's item count); a reduce
  // block takes one bucket over dslice parent tiles
  int64_t dhist_off;
  int32_t dslice;
  int32_t dbucketed;  // (t >= 1) this table's downward message is summed by buckets
};

// Downward pass by buckets (buckets of at most 2^12 groups, at most 256
// buckets): for a child of at most this many rows whose parent has at least
// DOWN_PARENT_RATIO times as many (a large table's foreign key into a
// smaller one: few repeats of a child group inside a parent tile for the
// LDS table of the atomic scatter to merge).
#define DOWN_MAX_GROUPS (1 << 20)
#define DOWN_BUCKETS 256
#define DOWN_PARENT_RATIO 4

// Positions per block of the in-LDS bucket sort of large 128-bit-word tables.
#define GJ_LOCAL_TILE 704

// Rows / entries per tile of the flat kernels (rounds of GJ_BLOCK elements).
#define GJ_ROUNDS 16
#define GJ_TILE (GJ_BLOCK * GJ_ROUNDS)

// Pointers of a plan's factor arrays.
struct FPtrs {
  uint64_t* words[2];  // sort words, 16 bytes per slot
  int32_t* perm;
  int32_t* ekey;
  int32_t* estart;
  int32_t* eend;
  int32_t* egrp;
  int32_t* gval;
  int32_t* glo;
  int32_t* ghi;
  int64_t* cnt;
  uint32_t* hist;
  uint32_t* dtot;
  int32_t* mm;
  uint64_t* agg;  // tile aggregates (scratch)
  uint64_t* agg2;
  int64_t* ecnt;  // projected factors: entry frequencies (null: the row counts)
  int32_t* didx;  // dense separator value -> group indexes (see TDesc)
  int32_t* lflag;  // per table: a bucket did not fit the in-LDS sort
};

// Pointers of a plan's summary arrays.
// What the expansion needs of a child table when its parent entry changes,
// in one 16-byte record per (child table, surviving parent entry): the child's
// group as a range [first, end) of its surviving entries, and the row count
// and first perm position of entry `first`.  (The group's upward message M,
// needed only to locate a rank, is cpre + c*U of the group's last entry.)
struct __align__(16) ChildRec {
  int32_t first, end, c0, st0;
};

struct SPtrs {
  int64_t* U;
  int64_t* pre;
  int64_t* Mg;
  int64_t* Dg;
  int32_t* link;
  int32_t* e2c;
  int32_t* g2c;
  int32_t* ckey;
  int64_t* cc;
  int64_t* cU;
  int64_t* cD;
  int64_t* cF;
  int64_t* cpre;
  int32_t* cstart;
  int32_t* cgval;
  int64_t* cgM;
  int64_t* cgD;
  int2* ccs;  // surviving entry -> (row count, first position in perm)
  ChildRec* crec;  // surviving parent entry -> the child's group (see ChildRec)
  ChildRec* grec;  // (t >= 1) group of t -> its record (the same for every parent entry)
  int64_t* xprod;  // (t >= 1) parent entry -> product of its other children's messages (link layout)
  int32_t* dkey;   // (t >= 1) downward items: child group, placed bucket by bucket (link layout)
  int64_t* dval;   //          and the item's term
  uint32_t* dhist; // per-(bucket, parent tile) start of the bucket's items in the tile (see TDesc)
  int64_t* qsize;
  int32_t* qstatus;
};

// ---------------------------------------------------------------------------
// Saturating non-negative int64 arithmetic (values kept in [0, 2^63-1]).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sadd(uint64_t a, uint64_t b) {
  uint64_t s = a + b;  // a, b <= 2^63-1: no wrap
  return s > SATV ? SATV : s;
}
__device__ __forceinline__ uint64_t smul(uint64_t a, uint64_t b) {
  uint64_t hi = __umul64hi(a, b);
  uint64_t lo = a * b;
  return (hi != 0 || lo > SATV) ? SATV : lo;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ULL : (~0ULL >> (64 - l));
}

// ---------------------------------------------------------------------------
// Wave / block scans (64-lane wavefronts, GJ_BLOCK threads).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(v, o, 64);
    if (l >= o) v += y;
  }
  return v;
}

// Block-wide exclusive sum of one value per thread; returns the exclusive
// prefix and writes the block total.  `sh` needs GJ_WAVES elements.
template <typename T>
__device__ __forceinline__ T block_excl_sum(T v, T* sh, T& total) {
  T inc = wave_incl_sum(v);
  if (lane_id() == 63) sh[wave_id()] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < GJ_WAVES; ++w) {
    T x = sh[w];
    if (w < wave_id()) before += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + inc - v;
}

// Segmented saturating scan.  A pair (v, f): f = 1 when a segment starts at or
// before this position within the span the pair summarizes.  Combining a left
// pair a with a right pair b gives (b.f ? b.v : a.v + b.v, a.f | b.f).
__device__ __forceinline__ void seg_combine(uint64_t& v, uint32_t& f, uint64_t lv, uint32_t lf) {
  // (lv, lf) is the left operand, (v, f) the right one (updated in place)
  if (!f) v = sadd(lv, v);
  f |= lf;
}

__device__ __forceinline__ void wave_seg_incl(uint64_t& v, uint32_t& f) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t y = __shfl_up(v, o, 64);
    uint32_t fy = __shfl_up(f, o, 64);
    if (l >= o) seg_combine(v, f, y, fy);
  }
}

// Block-wide inclusive segmented scan; returns the block aggregate in (tv, tf).
// `shv`/`shf` need GJ_WAVES elements.
__device__ __forceinline__ void block_seg_incl(uint64_t& v, uint32_t& f, uint64_t* shv, uint32_t* shf,
                                               uint64_t& tv, uint32_t& tf) {
  wave_seg_incl(v, f);
  if (lane_id() == 63) {
    shv[wave_id()] = v;
    shf[wave_id()] = f;
  }
  __syncthreads();
  uint64_t cv = 0;
  uint32_t cf = 0;  // combination of the waves before this one
  uint64_t av = 0;
  uint32_t af = 0;  // all waves
#pragma unroll
  for (int w = 0; w < GJ_WAVES; ++w) {
    uint64_t x = shv[w];
    uint32_t fx = shf[w];
    if (w < wave_id()) {
      cv = fx ? x : sadd(cv, x);
      cf |= fx;
    }
    av = fx ? x : sadd(av, x);
    af |= fx;
  }
  __syncthreads();
  seg_combine(v, f, cv, cf);
  tv = av;
  tf = af;
}

// 128-bit sort word.
struct W128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ uint64_t shr128_lo(uint64_t lo, uint64_t hi, int s) {
  // low 64 bits of (hi:lo) >> s, 0 <= s < 128
  if (s == 0) return lo;
  if (s < 64) return (lo >> s) | (hi << (64 - s));
  return hi >> (s - 64);
}
