// Stage 1 -- the group-by of the factor build (Sec. 3.2), for large tables
// whose sort words are 128 bits wide.
//
// The radix sort of such a table takes only its two most significant digits
// as global passes (the ordinary upsweep / scan / downsweep, shifted to the
// top of the key): every run of words with equal top bits -- a bucket -- is
// then contiguous and, the passes being stable, in row order.  What is left
// is sorting each bucket by the bits below, which needs no more global
// traffic: a block takes whole buckets into its LDS and sorts them there.
//
// Block b owns the table's positions [b T, (b+1) T), T = GJ_LOCAL_TILE.  Its
// range runs from the first bucket head at or after b T to the first head at
// or after (b+1) T (or the table's end), so the ranges of consecutive blocks
// meet and cover the table in whole buckets; a block whose tile holds no
// head owns nothing.  The block loads its tile and then looks ahead, a chunk
// at a time, for the end of its last bucket; a range longer than the LDS
// holds (LS_CAP words) raises the table's flag and is left alone, and the
// host then sorts that table in full (the bucket order is a valid input for
// it).  Otherwise the block finds the key bits that vary inside its range
// (bits above them are equal there) and orders the range by them in LDS:
// one stable pass over the top 8 varying bits (ranking by wave ballots in
// input order, as the global passes do) splits it into sub-buckets of about
// 1/256 of its words, and each word's place inside its sub-bucket is the
// number of smaller words there.  A whole word compares as (key, row id),
// since the row-id bits sit below the key, so equal keys come out in row
// order, as the run writer needs.  A sub-bucket of more than LS_SMALL words
// (keys that share most of their varying bits) takes stable LSD passes over
// every varying digit instead.  The range goes to the other word buffer.
#include "stages.h"

namespace {

// 512 threads and one 1920-word buffer (40 KB of LDS with the histograms):
// four blocks share a CU.  (A first form -- 1024 threads, two 4096-word
// buffers, one block a CU, eight LSD passes -- took 3.6 ms for 5e7 words,
// against 0.87 ms for this one.)  With tiles of 704 positions a bucket of up
// to 1216 words fits wherever it starts.
constexpr int LS_BLOCK = 512;
constexpr int LS_CAP = 1920;  // longest range a block sorts
constexpr int LS_WAVES = LS_BLOCK / 64;
constexpr int LS_ITEMS = (LS_CAP + LS_BLOCK - 1) / LS_BLOCK;  // most words per lane and LDS pass
constexpr int LS_CHUNK = 512;                                 // words per look-ahead step
constexpr int LS_SMALL = 96;  // longest sub-bucket ranked by counting
static_assert(GJ_LOCAL_TILE < LS_CAP, "look-ahead room");
static_assert(LS_CHUNK <= LS_BLOCK, "one look-ahead word per thread");
static_assert(LS_CAP * 2 <= LS_WAVES * 256 * 4, "the indexes fit the histograms' room");

struct LsShared {
  W128 buf[LS_CAP];  // the range (a pass permutes it in place through registers)
  union {
    uint32_t wh[LS_WAVES][256];  // in a pass: per wave, digit counts, then their prefix over waves
    uint16_t idx[LS_CAP];        // after the counting: the word that goes to each place
  };
  uint32_t dstart[257];        // digit starts in the pass's output, then m
  uint32_t wmax[4];
  uint64_t orr[LS_WAVES][2];
  uint32_t wsum[4];  // the 256 digits' scan: waves 0..3
  int32_t pos[2];  // first head in the tile, first head past it
};

// Lowest position (block-wide) whose lane raised `head`; pos starts at INT_MAX.
__device__ __forceinline__ void note_head(bool head, int j, int32_t* pos) {
  const uint64_t b = __ballot(head);
  if (b != 0 && lane_id() == __ffsll((long long)b) - 1) atomicMin(pos, j);
}

// One stable LDS pass: the m words at S.buf[src ..] ordered by their 8-bit
// digit at `shift` into S.buf[0 ..], ranked by wave ballots in input order
// (wave v takes words [v 64 R, (v+1) 64 R), R rounds of 64).  Every word is
// in a register before the first store.  Leaves digit g's words at
// [S.dstart[g], S.dstart[g + 1]); returns the largest digit count.
__device__ __forceinline__ int lds_pass(LsShared& S, int src, int m, int R, int shift) {
  const int tid = threadIdx.x, wv = wave_id(), ln = lane_id();
  for (int i = tid; i < LS_WAVES * 256; i += LS_BLOCK) (&S.wh[0][0])[i] = 0;
  __syncthreads();
  W128 key[LS_ITEMS];
  uint32_t dig[LS_ITEMS], rank[LS_ITEMS];
#pragma unroll
  for (int r = 0; r < LS_ITEMS; ++r) {
    if (r >= R) break;
    const int j = wv * 64 * R + r * 64 + ln;
    const bool valid = j < m;
    if (valid) key[r] = S.buf[src + j];
    dig[r] = valid ? (uint32_t)shr128_lo(key[r].lo, key[r].hi, shift) & 255u : 0u;
    const uint64_t peers = match_digit(dig[r], valid, 8);
    const uint64_t below = peers & lanemask_lt();
    const uint32_t prev = S.wh[wv][dig[r]];
    rank[r] = prev + (uint32_t)__popcll(below);
    if (valid && below == 0) S.wh[wv][dig[r]] = prev + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t total = 0, inc = 0;
  if (tid < 256) {
#pragma unroll
    for (int v = 0; v < LS_WAVES; ++v) {
      const uint32_t c = S.wh[v][tid];
      S.wh[v][tid] = total;
      total += c;
    }
    inc = wave_incl_sum(total);
    uint32_t mx = total;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (ln == 63) {
      S.wsum[wv] = inc;
      S.wmax[wv] = mx;
    }
  }
  __syncthreads();
  if (tid < 256) {
    uint32_t before = 0;
    for (int v = 0; v < wv; ++v) before += S.wsum[v];
    S.dstart[tid] = before + inc - total;
    if (tid == 0) S.dstart[256] = (uint32_t)m;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < LS_ITEMS; ++r) {
    if (r >= R) break;
    const int j = wv * 64 * R + r * 64 + ln;
    if (j < m) S.buf[S.dstart[dig[r]] + S.wh[wv][dig[r]] + rank[r]] = key[r];
  }
  __syncthreads();
  return (int)max(max(S.wmax[0], S.wmax[1]), max(S.wmax[2], S.wmax[3]));
}

__global__ void __launch_bounds__(LS_BLOCK) k_local_sort(const WorkItem* __restrict__ wl,
                                                         const TDesc* __restrict__ D, uint64_t* words0,
                                                         uint64_t* words1, int32_t* __restrict__ flag) {
  __shared__ LsShared S;
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int tid = threadIdx.x, wv = wave_id(), ln = lane_id();
  const int64_t t0 = (int64_t)w.tile * GJ_LOCAL_TILE;
  const int64_t avail = d.n - t0;  // words from t0 to the table's end (> 0)
  const int tn = (int)min((int64_t)GJ_LOCAL_TILE, avail);
  const W128* in = word_ptr<1>(words0, d);
  W128* out = word_ptr<1>(words1, d);
  const int sh0 = d.sh0;

  for (int j = tid; j < tn; j += LS_BLOCK) S.buf[j] = in[t0 + j];
  if (tid < 2) S.pos[tid] = INT_MAX;
  __syncthreads();
  // first bucket head in the tile
#pragma unroll
  for (int k = 0; k < (GJ_LOCAL_TILE + LS_BLOCK - 1) / LS_BLOCK; ++k) {
    const int j = k * LS_BLOCK + tid;
    bool head = false;
    if (j < tn) {
      if (j == 0)
        head = t0 == 0 || high_bits(wxor(in[t0 - 1], S.buf[0]), sh0);
      else
        head = high_bits(wxor(S.buf[j - 1], S.buf[j]), sh0);
    }
    note_head(head, j, &S.pos[0]);
  }
  __syncthreads();
  const int s_off = S.pos[0];
  if (s_off == INT_MAX) return;  // the tile lies inside a bucket that starts earlier
  // end of the last bucket that starts in the tile
  int e_off = tn;
  if (avail > GJ_LOCAL_TILE) {
    e_off = -1;
    for (int c0 = GJ_LOCAL_TILE; c0 < LS_CAP; c0 += LS_CHUNK) {
      if ((int64_t)c0 >= avail) {
        e_off = (int)avail;
        break;
      }
      const int cend = (int)min((int64_t)min(c0 + LS_CHUNK, LS_CAP), avail);
      const int j = c0 + tid;
      if (j < cend) S.buf[j] = in[t0 + j];
      __syncthreads();
      if (tid < LS_CHUNK) note_head(j < cend && high_bits(wxor(S.buf[j - 1], S.buf[j]), sh0), j, &S.pos[1]);
      __syncthreads();
      const int h = S.pos[1];
      if (h != INT_MAX) {
        e_off = h;
        break;
      }
      if (cend == avail) {
        e_off = (int)avail;
        break;
      }
    }
    if (e_off < 0) {  // the range does not fit: the host sorts this table in full
      if (tid == 0) flag[w.t] = 1;
      return;
    }
  }
  const int m = e_off - s_off;

  // key bits that vary inside the range (row-id bits excluded)
  uint64_t olo = 0, ohi = 0;
  {
    const W128 f = S.buf[s_off];
    for (int j = s_off + tid; j < e_off; j += LS_BLOCK) {
      const W128 x = S.buf[j];
      olo |= x.lo ^ f.lo;
      ohi |= x.hi ^ f.hi;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      olo |= __shfl_xor(olo, o, 64);
      ohi |= __shfl_xor(ohi, o, 64);
    }
    if (ln == 0) {
      S.orr[wv][0] = olo;
      S.orr[wv][1] = ohi;
    }
    __syncthreads();
    olo = ohi = 0;
#pragma unroll
    for (int v = 0; v < LS_WAVES; ++v) {
      olo |= S.orr[v][0];
      ohi |= S.orr[v][1];
    }
    const int rb = d.rb;
    if (rb >= 64) {
      olo = 0;
      ohi &= rb == 64 ? ~0ULL : ~((1ULL << (rb - 64)) - 1);
    } else if (rb > 0) {
      olo &= ~((1ULL << rb) - 1);
    }
  }
  const int hb = ohi ? 127 - __clzll((long long)ohi) : (olo ? 63 - __clzll((long long)olo) : -1);
  const int npass = hb < d.rb ? 0 : (hb - d.rb) / 8 + 1;

  const int R = (m + LS_BLOCK - 1) / LS_BLOCK;  // words per lane and pass, over every wave
  W128* o = out + t0 + s_off;
  if (npass == 0) {
    for (int j = tid; j < m; j += LS_BLOCK) o[j] = S.buf[s_off + j];
    return;
  }
  // the top varying digit first: sub-buckets of about m / 256 words
  const int top = max(d.rb, hb - 7);
  const int big = lds_pass(S, s_off, m, R, top);
  if (top > d.rb && big <= LS_SMALL) {
    // each word's place inside its sub-bucket: the number of smaller words
    // there (whole words compare as (key, row id), the order wanted)
    for (int j = tid; j < m; j += LS_BLOCK) {
      const W128 x = S.buf[j];
      const uint32_t g = (uint32_t)shr128_lo(x.lo, x.hi, top) & 255u;
      const int a = S.dstart[g], e = S.dstart[g + 1];
      int rank = a;
      for (int k = a; k < e; ++k) {
        const W128 y = S.buf[k];
        rank += (y.hi < x.hi || (y.hi == x.hi && y.lo < x.lo)) ? 1 : 0;
      }
      S.idx[rank] = (uint16_t)j;
    }
    __syncthreads();
    for (int j = tid; j < m; j += LS_BLOCK) o[j] = S.buf[S.idx[j]];
    return;
  }
  if (top > d.rb) {
    // a long sub-bucket: LSD passes over every varying digit (stable, so
    // equal keys keep their row order)
    for (int p = 0; p < npass; ++p) {
      const int shift = d.rb + 8 * p;
      if (((uint32_t)shr128_lo(olo, ohi, shift) & 255u) == 0) continue;  // digit constant in the range
      lds_pass(S, 0, m, R, shift);
    }
  }
  for (int j = tid; j < m; j += LS_BLOCK) o[j] = S.buf[j];
}

}  // namespace

namespace gjk {

void local_sort(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F) {
  if (nwl > 0)
    hipLaunchKernelGGL(k_local_sort, dim3(nwl), dim3(LS_BLOCK), 0, s, wl, D, F.words[0], F.words[1], F.lflag);
}

}  // namespace gjk
