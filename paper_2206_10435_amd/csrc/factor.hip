// Stage 1 -- factors (Sec. 3.2, quantitative learning): one group-by count per
// table.  A table's factor is every distinct key tuple with its frequency; the
// GPU form is a sort of the rows by key tuple followed by run detection:
//
//   minmax   per-column range of every table (host picks field widths)
//   pack     one sort word per row: key fields (separator field most
//            significant for non-root tables) above the row id
//   radix    LSD radix sort over the key bits only; each pass is an upsweep
//            (per-tile digit counts), a digit scan and a downsweep that ranks
//            keys inside the tile with wavefront ballots, stages the tile in
//            LDS in digit order and writes contiguous digit runs.  LSD is
//            stable and the words start in row order, so rows inside an entry
//            come out ascending by row id.
//   runs     entry / separator-group boundaries, their exclusive scan, and the
//            entry arrays (keys, row range, group) plus the grouped row ids.
#include "gj_internal.h"
#include "kernels.h"

namespace {

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

// ---------------------------------------------------------------------------
// Per-tile column ranges (no atomics: every tile writes its own slot), then
// one block per table reduces its tiles.
__global__ void __launch_bounds__(GJ_BLOCK) k_minmax(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                     int32_t* __restrict__ mmt) {
  __shared__ int32_t sh[2][GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int c = 0; c < d.k; ++c) {
    const int32_t* col = d.col[c];
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      int64_t i = base + r * GJ_BLOCK + threadIdx.x;
      if (i < d.n) {
        int32_t v = col[i];
        lo = min(lo, v);
        hi = max(hi, v);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane_id() == 0) {
      sh[0][wave_id()] = lo;
      sh[1][wave_id()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = 1; v < GJ_WAVES; ++v) {
        lo = min(lo, sh[0][v]);
        hi = max(hi, sh[1][v]);
      }
      mmt[((d.agg_off + w.tile) * MAXK + c) * 2 + 0] = lo;
      mmt[((d.agg_off + w.tile) * MAXK + c) * 2 + 1] = hi;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(GJ_BLOCK) k_minmax_reduce(const int32_t* __restrict__ tabs,
                                                            const TDesc* __restrict__ D,
                                                            const int32_t* __restrict__ mmt, int32_t* __restrict__ mm) {
  __shared__ int32_t sh[2][GJ_WAVES];
  const int t = tabs[blockIdx.x];
  const TDesc& d = D[t];
  for (int c = 0; c < d.k; ++c) {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int64_t i = threadIdx.x; i < d.ntiles; i += GJ_BLOCK) {
      lo = min(lo, mmt[((d.agg_off + i) * MAXK + c) * 2 + 0]);
      hi = max(hi, mmt[((d.agg_off + i) * MAXK + c) * 2 + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane_id() == 0) {
      sh[0][wave_id()] = lo;
      sh[1][wave_id()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = 1; v < GJ_WAVES; ++v) {
        lo = min(lo, sh[0][v]);
        hi = max(hi, sh[1][v]);
      }
      mm[(t * MAXK + c) * 2 + 0] = lo;
      mm[(t * MAXK + c) * 2 + 1] = hi;
    }
    __syncthreads();
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v0, int32_t v1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (i & 1) ? v1 : v0;
}

// ---------------------------------------------------------------------------
template <int WIDE>
__global__ void __launch_bounds__(GJ_BLOCK) k_pack(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                   uint64_t* __restrict__ words0) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  auto* out = word_ptr<WIDE>(words0, d);
  const int64_t base = (int64_t)w.tile * GJ_TILE;
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
      out[i] = W128{lo, hi};
    } else {
      out[i] = lo;
    }
  }
}

// ---------------------------------------------------------------------------
// Radix sort, one LSD pass = upsweep + digit scan + downsweep.
// Tile = GJ_BLOCK * ITEMS keys; wave v of the block owns keys
// [v*64*ITEMS, (v+1)*64*ITEMS) of the tile, visited in rounds of 64 so that
// (round, lane) order is the input order (needed for stability).
// ---------------------------------------------------------------------------
template <int WIDE, int ITEMS>
__global__ void __launch_bounds__(GJ_BLOCK) k_upsweep(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                      uint64_t* words0, uint64_t* words1, uint32_t* __restrict__ hist,
                                                      int pass) {
  __shared__ uint32_t wh[GJ_WAVES][256];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const int db = d.dbits;
  const int nd = 1 << db;
  const uint32_t mask = (uint32_t)nd - 1;
  const int shift = d.rb + pass * db;
  const auto* in = word_ptr<WIDE>((pass & 1) ? words1 : words0, d);
  for (int i = threadIdx.x; i < GJ_WAVES * 256; i += GJ_BLOCK) (&wh[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)w.tile * (GJ_BLOCK * ITEMS);
  const int64_t cnt = min((int64_t)GJ_BLOCK * ITEMS, d.n - base);
  const int wv = wave_id(), ln = lane_id();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    int64_t li = (int64_t)wv * 64 * ITEMS + r * 64 + ln;
    bool valid = li < cnt;
    uint32_t dig = valid ? digit_of(in[base + li], shift, mask) : 0u;
    uint64_t peers = match_digit(dig, valid, db);
    bool leader = valid && (peers & lanemask_lt()) == 0;
    if (leader) wh[wv][dig] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < nd; g += GJ_BLOCK) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < GJ_WAVES; ++v) s += wh[v][g];
    hist[d.hist_off + (int64_t)g * d.ntiles_sort + w.tile] = s;
  }
}

// One block per (table, digit): exclusive scan of that digit's counts over the
// table's tiles, in place; the digit total goes to dtot.
__global__ void __launch_bounds__(GJ_BLOCK) k_digit_scan(const int32_t* __restrict__ tabs,
                                                         const TDesc* __restrict__ D, uint32_t* __restrict__ hist,
                                                         uint32_t* __restrict__ dtot) {
  __shared__ uint32_t sh[GJ_WAVES];
  const int t = tabs[blockIdx.x >> 8];
  const int g = blockIdx.x & 255;
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
__global__ void __launch_bounds__(GJ_BLOCK) k_downsweep(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                        uint64_t* words0, uint64_t* words1,
                                                        const uint32_t* __restrict__ hist,
                                                        const uint32_t* __restrict__ dtot, int pass) {
  typedef typename WordT<WIDE>::type Word;
  __shared__ uint32_t wh[GJ_WAVES][256];
  __shared__ uint32_t gb[256];
  __shared__ uint32_t ls[256];
  __shared__ uint32_t sh[GJ_WAVES];
  __shared__ Word stage[GJ_BLOCK * ITEMS];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const int db = d.dbits;
  const int nd = 1 << db;
  const uint32_t mask = (uint32_t)nd - 1;
  const int shift = d.rb + pass * db;
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

// ---------------------------------------------------------------------------
// Runs: entry heads (key change) and separator-group heads (separator field
// change; the root is one group).  Counts per tile, then the write pass.
// ---------------------------------------------------------------------------
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
__global__ void __launch_bounds__(GJ_BLOCK) k_runs_count(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                         uint64_t* words0, uint64_t* words1,
                                                         uint64_t* __restrict__ agg) {
  __shared__ uint64_t sh[GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
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

template <int WIDE>
__global__ void __launch_bounds__(GJ_BLOCK) k_runs_write(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                         uint64_t* words0, uint64_t* words1,
                                                         const uint64_t* __restrict__ agg, FPtrs P) {
  __shared__ uint64_t sh[GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  if (d.wide != WIDE) return;
  const auto* wv = word_ptr<WIDE>(d.final_buf ? words1 : words0, d);
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  const int64_t off = d.off;
  const uint64_t rbmask = d.rb == 0 ? 0ULL : ((1ULL << d.rb) - 1);
  uint64_t carry = agg[d.agg_off + w.tile];
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    bool valid = i < d.n;
    bool h = false, s = false, nh = false, ns = false;
    if (valid) {
      run_flags<WIDE>(wv, d, i, h, s);
      if (i + 1 == d.n) {
        nh = true;
        ns = true;
      } else {
        run_flags<WIDE>(wv, d, i + 1, nh, ns);
        if (d.is_root) ns = false;
      }
    }
    uint64_t v = (uint64_t)h | ((uint64_t)s << 32);
    uint64_t tot;
    uint64_t ex = block_excl_sum(v, sh, tot) + carry;
    carry += tot;
    if (!valid) continue;
    const int64_t e = (int64_t)(uint32_t)ex + (h ? 0 : -1);
    const int64_t g = (int64_t)(ex >> 32) + (s ? 0 : -1);
    auto word = wv[i];
    P.perm[off + i] = (int32_t)(wlow(word) & rbmask);
    if (h) {
      P.estart[off + e] = (int32_t)i;
      P.egrp[off + e] = (int32_t)g;
      for (int c = 0; c < d.k; ++c) {
        uint32_t f = field_of(word, d.rb + d.fshift[c], d.fbits[c]);
        P.ekey[d.key_off + (int64_t)c * d.n + e] = (int32_t)(f + d.kmin[c]);
      }
    }
    if (s) {
      P.glo[off + g] = (int32_t)e;
      int sc = d.is_root ? 0 : d.sep;
      uint32_t f = field_of(word, d.rb + d.fshift[sc], d.fbits[sc]);
      P.gval[off + g] = (int32_t)(f + d.kmin[sc]);
    }
    if (nh) P.eend[off + e] = (int32_t)(i + 1);
    if (ns) P.ghi[off + g] = (int32_t)(e + 1);
  }
}

}  // namespace

// Dense separator index of tables whose separator values span a small range:
// didx[didx_off + gval(g) - dmin] = g for every separator group g.
__global__ void __launch_bounds__(GJ_BLOCK) k_group_index(const WorkItem* __restrict__ wl,
                                                          const TDesc* __restrict__ D, FPtrs F) {
  const WorkItem w = wl[blockIdx.x];
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

// Entry frequencies as int64 (the factor view's count column).
__global__ void __launch_bounds__(GJ_BLOCK) k_entry_counts(const WorkItem* __restrict__ wl,
                                                           const TDesc* __restrict__ D, FPtrs F,
                                                           int64_t* __restrict__ out) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    if (e >= M) break;
    const int64_t se = d.off + e;
    out[se] = F.ecnt ? F.ecnt[se] : (int64_t)(F.eend[se] - F.estart[se]);
  }
}

// One block per table: exclusive scan (in place) of the table's tile
// aggregates, each a pair of 32-bit counts packed in a uint64 (no carry can
// cross the halves: counts are < 2^31); the totals go to cnt[t][ca], cnt[t][cb].
__global__ void __launch_bounds__(GJ_BLOCK) k_tile_scan_pair(const int32_t* __restrict__ tabs,
                                                             const TDesc* __restrict__ D, uint64_t* __restrict__ agg,
                                                             int64_t* __restrict__ cnt, int ca, int cb) {
  __shared__ uint64_t sh[GJ_WAVES];
  const int t = tabs[blockIdx.x];
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
// Host launchers
// ---------------------------------------------------------------------------
namespace gjk {

void fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v0, int32_t v1) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(GJ_BLOCK), 0, s, p, n, v0, v1);
}

void minmax(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
            int32_t* mmt, int32_t* mm) {
  if (nwl > 0) hipLaunchKernelGGL(k_minmax, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, mmt);
  if (ntab > 0) hipLaunchKernelGGL(k_minmax_reduce, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, mmt, mm);
}

void pack(hipStream_t s, int wide, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& P) {
  if (nwl <= 0) return;
  if (wide)
    hipLaunchKernelGGL(k_pack<1>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0]);
  else
    hipLaunchKernelGGL(k_pack<0>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0]);
}

void radix_pass(hipStream_t s, int wide, int items, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab,
                const TDesc* D, const FPtrs& P, int pass) {
  if (nwl <= 0) return;
#define GJ_RADIX_CASE(W, I)                                                                                        \
  if (wide == W && items == I) {                                                                                   \
    hipLaunchKernelGGL((k_upsweep<W, I>), dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.hist, \
                       pass);                                                                                      \
    hipLaunchKernelGGL(k_digit_scan, dim3(ntab * 256), dim3(GJ_BLOCK), 0, s, tabs, D, P.hist, P.dtot);            \
    hipLaunchKernelGGL((k_downsweep<W, I>), dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1],       \
                       P.hist, P.dtot, pass);                                                                      \
    return;                                                                                                        \
  }
  GJ_RADIX_CASE(0, 8)
  GJ_RADIX_CASE(0, 16)
  GJ_RADIX_CASE(1, 8)
#undef GJ_RADIX_CASE
}

void runs(hipStream_t s, int wide, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
          const FPtrs& P) {
  if (nwl <= 0) return;
  if (wide)
    hipLaunchKernelGGL(k_runs_count<1>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg);
  else
    hipLaunchKernelGGL(k_runs_count<0>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg);
}

void runs_scan(hipStream_t s, const int32_t* tabs, int ntab, const TDesc* D, const FPtrs& P) {
  if (ntab > 0)
    hipLaunchKernelGGL(k_tile_scan_pair, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, P.agg, P.cnt, CNT_M, CNT_G);
}

void runs_write(hipStream_t s, int wide, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& P) {
  if (nwl <= 0) return;
  if (wide)
    hipLaunchKernelGGL(k_runs_write<1>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg, P);
  else
    hipLaunchKernelGGL(k_runs_write<0>, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, P.words[0], P.words[1], P.agg, P);
}

void group_index(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F) {
  if (nwl > 0) hipLaunchKernelGGL(k_group_index, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F);
}

void entry_counts(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, int64_t* out) {
  if (nwl > 0) hipLaunchKernelGGL(k_entry_counts, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, out);
}

void tile_scan_pair(hipStream_t s, const int32_t* tabs, int ntab, const TDesc* D, uint64_t* agg, int64_t* cnt, int ca,
                    int cb) {
  if (ntab > 0) hipLaunchKernelGGL(k_tile_scan_pair, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, agg, cnt, ca, cb);
}

}  // namespace gjk
