// Stage 2 -- summary.  Integer sum-product message passing over the join tree.
//
// Upward (Sec. 3.3, Algorithm 2; variable elimination Eq. 4 from the leaves):
// for every entry e of table t, U_t(e) = product over t's children ch of the
// child's message at e's value of the joining column (1 at a leaf); the
// message of t is M_t(s) = sum of c_t(e) * U_t(e) over t's entries with
// separator value s, and the root's sum is the join size (Eq. 3's Z).
//   k_up_agg    U per entry (looking each child value up in the child's
//               sorted separator values, which also records the entry ->
//               child-group link), tile aggregates of a segmented scan of c*U
//   k_seg_tiles carry-in of every tile
//   k_up_scan   exclusive prefix of c*U inside each separator group (the block
//               offsets used by desummarization) and the group totals M
// Downward (Sec. 3.5, Algorithms 3-4 condition each level on the levels
// above): D_t(s) = sum over parent entries e' with value s in the joining
// column of c_p(e') * D_p(e') * product of the other children's messages;
// scattered with 64-bit atomics (exact: every partial sum is bounded by the
// join size once the upward pass has not overflowed).
// Compaction keeps entries with F = c*U*D > 0 and groups with M*D > 0 (Sec.
// 3.3: entries of frequency below 1 are excluded) and re-links them.
#include "gj_internal.h"
#include "kernels.h"

namespace {

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

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void __launch_bounds__(GJ_BLOCK) k_up_agg(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                     FPtrs F, SPtrs S) {
  __shared__ uint64_t shv[GJ_WAVES];
  __shared__ uint32_t shf[GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
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
#pragma unroll
        for (int i = 0; i < MAXC; ++i) {
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
            const uint64_t m = j >= 0 ? (uint64_t)S.Mg[dc.off + j] : 0ULL;
            U = smul(U, m);
          }
        }
        const uint64_t c = entry_count(F, se);
        cu = smul(c, U);
        S.U[se] = (int64_t)U;
        head = (e == 0 || F.egrp[se] != F.egrp[se - 1]) ? 1u : 0u;
      }
      uint64_t tv;
      uint32_t tf;
      block_seg_incl(cu, head, shv, shf, tv, tf);
      av = tf ? tv : sadd(av, tv);
      af |= tf;
    }
  }
  if (threadIdx.x == 0) {
    F.agg[d.agg_off + w.tile] = av;
    F.agg2[d.agg_off + w.tile] = af;
  }
}

// One block per table: carry-in value of every tile of the segmented scan
// (exclusive), written over the tile aggregate.
__global__ void __launch_bounds__(GJ_BLOCK) k_seg_tiles(const int32_t* __restrict__ tabs, const TDesc* __restrict__ D,
                                                        FPtrs F) {
  __shared__ uint64_t shv[GJ_WAVES];
  __shared__ uint32_t shf[GJ_WAVES];
  __shared__ uint64_t incl[GJ_BLOCK];
  const int t = tabs[blockIdx.x];
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

__global__ void __launch_bounds__(GJ_BLOCK) k_up_scan(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                      FPtrs F, SPtrs S) {
  __shared__ uint64_t shv[GJ_WAVES];
  __shared__ uint32_t shf[GJ_WAVES];
  __shared__ uint64_t incl[GJ_BLOCK];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  uint64_t cv = F.agg[d.agg_off + w.tile];
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    const int64_t se = d.off + e;
    uint64_t cu = 0;
    uint32_t head = 0;
    const bool valid = e < M;
    if (valid) {
      const uint64_t c = entry_count(F, se);
      cu = smul(c, (uint64_t)S.U[se]);
      head = (e == 0 || F.egrp[se] != F.egrp[se - 1]) ? 1u : 0u;
    }
    uint64_t v = cu;
    uint32_t f = head;
    uint64_t tv;
    uint32_t tf;
    block_seg_incl(v, f, shv, shf, tv, tf);
    const uint64_t mine = f ? v : sadd(cv, v);
    incl[threadIdx.x] = mine;
    __syncthreads();
    if (valid) {
      const uint64_t ex = head ? 0ULL : (threadIdx.x == 0 ? cv : incl[threadIdx.x - 1]);
      S.pre[se] = (int64_t)ex;
      const bool last = (e + 1 == M) || F.egrp[se + 1] != F.egrp[se];
      if (last) {
        S.Mg[d.off + F.egrp[se]] = (int64_t)mine;
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

// Downward messages into the children of the tables in the work list.  The
// terms of one tile are first summed per child group in an LDS hash table
// (linear probing; a key that finds no slot goes straight to global memory),
// so a heavily shared separator value costs one global atomic per tile
// instead of one per parent entry.
#define DOWN_HASH 2048
__global__ void __launch_bounds__(GJ_BLOCK) k_down(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                   FPtrs F, SPtrs S) {
  __shared__ int32_t hkey[DOWN_HASH];
  __shared__ unsigned long long hval[DOWN_HASH];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  for (int ci = 0; ci < d.nchild; ++ci) {
    const TDesc& dt = D[d.child[ci]];
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

// Survivors per tile: entries with c > 0, U > 0 and D > 0, groups with M > 0
// and D > 0 (a row count is never 0; a projected frequency can be).
__device__ __forceinline__ bool entry_survives(const TDesc& d, const FPtrs& F, const SPtrs& S, int64_t se) {
  if (S.U[se] == 0 || (F.ecnt && F.ecnt[se] == 0)) return false;
  return d.is_root || S.Dg[d.off + F.egrp[se]] > 0;
}
__device__ __forceinline__ bool group_survives(const TDesc& d, const SPtrs& S, int64_t sg) {
  return S.Mg[sg] > 0 && (d.is_root || S.Dg[sg] > 0);
}

__global__ void __launch_bounds__(GJ_BLOCK) k_compact_count(const WorkItem* __restrict__ wl,
                                                            const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  __shared__ uint64_t sh[GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
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

__global__ void __launch_bounds__(GJ_BLOCK) k_compact_write(const WorkItem* __restrict__ wl,
                                                            const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  __shared__ uint64_t sh[GJ_WAVES];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t G = F.cnt[w.t * CNT_STRIDE + CNT_G];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  uint64_t carry = F.agg[d.agg_off + w.tile];
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    const int64_t se = d.off + e;
    const bool ve = e < M, vg = e < G;
    const bool es = ve && entry_survives(d, F, S, se);
    const bool gs = vg && group_survives(d, S, se);
    uint64_t tot;
    const uint64_t ex = block_excl_sum((uint64_t)es | ((uint64_t)gs << 32), sh, tot) + carry;
    carry += tot;
    const int64_t ci = (int64_t)(uint32_t)ex;
    const int64_t gi = (int64_t)(ex >> 32);
    if (ve) {
      S.e2c[se] = (int32_t)ci;
      if (es) {
        const int64_t sc = d.off + ci;
        const uint64_t c = entry_count(F, se);
        const uint64_t U = (uint64_t)S.U[se];
        const uint64_t Dv = d.is_root ? 1ULL : (uint64_t)S.Dg[d.off + F.egrp[se]];
        for (int k = 0; k < d.k; ++k)
          S.ckey[d.key_off + (int64_t)k * d.n + ci] = F.ekey[d.key_off + (int64_t)k * d.n + e];
        S.cc[sc] = (int64_t)c;
        S.cU[sc] = (int64_t)U;
        S.cD[sc] = (int64_t)Dv;
        S.cF[sc] = (int64_t)smul(smul(c, U), Dv);
        S.cpre[sc] = S.pre[se];
        S.cstart[sc] = F.estart[se];
        S.ccs[sc] = make_int2((int)c, F.estart[se]);
      }
    }
    if (vg) {
      S.g2c[se] = gs ? (int32_t)gi : -1;
      if (gs) {
        const int64_t sg = d.off + gi;
        S.cgval[sg] = F.gval[se];
        S.cgM[sg] = S.Mg[se];
        S.cgD[sg] = d.is_root ? 1 : S.Dg[se];
      }
    }
  }
}

// Second compaction pass (needs every e2c / g2c).  What a child's group
// contributes to its parents' records depends on the group only, so every
// group's record is built once (k_group_recs) and copied to the records of
// the surviving parent entries that link to it (k_compact_links).
__global__ void __launch_bounds__(GJ_BLOCK) k_group_recs(const WorkItem* __restrict__ wl,
                                                         const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  const WorkItem w = wl[blockIdx.x];
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
    rc.M = S.cgM[d.off + gc];
    rc.unused = 0;
    S.grec[sg] = rc;
  }
}

__global__ void __launch_bounds__(GJ_BLOCK) k_compact_links(const WorkItem* __restrict__ wl,
                                                            const TDesc* __restrict__ D, FPtrs F, SPtrs S) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  if (d.nchild == 0) return;
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    if (e >= M) break;
    const int64_t se = d.off + e;
    if (!entry_survives(d, F, S, se)) continue;
    const int32_t ci = S.e2c[se];
    for (int i = 0; i < d.nchild; ++i) {
      const TDesc& dc = D[d.child[i]];
      // a surviving entry's child group survives (its message and its
      // downward message are both > 0)
      S.crec[dc.link_off + ci] = S.grec[dc.off + S.link[dc.link_off + e]];
    }
  }
}

__global__ void k_export_status(const int64_t* __restrict__ qsize, const int32_t* __restrict__ qstatus,
                                int64_t* __restrict__ out_size, int32_t* __restrict__ out_status) {
  if (threadIdx.x == 0) {
    *out_size = *qsize;
    *out_status = *qstatus;
  }
}

}  // namespace

namespace gjk {

void export_status(hipStream_t s, const int64_t* qsize, const int32_t* qstatus, int64_t* out_size,
                   int32_t* out_status) {
  hipLaunchKernelGGL(k_export_status, dim3(1), dim3(64), 0, s, qsize, qstatus, out_size, out_status);
}

void fill_i64(hipStream_t s, int64_t* p, int64_t n, int64_t v) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 4096);
  hipLaunchKernelGGL(k_fill_i64, dim3(blocks), dim3(GJ_BLOCK), 0, s, p, n, v);
}

void up_pass(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
             const FPtrs& F, const SPtrs& S) {
  if (nwl <= 0) return;
  hipLaunchKernelGGL(k_up_agg, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  hipLaunchKernelGGL(k_seg_tiles, dim3(ntab), dim3(GJ_BLOCK), 0, s, tabs, D, F);
  hipLaunchKernelGGL(k_up_scan, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
}

void down_pass(hipStream_t s, const WorkItem* wl, int nwl, const TDesc* D, const FPtrs& F, const SPtrs& S) {
  if (nwl > 0) hipLaunchKernelGGL(k_down, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
}

void compact(hipStream_t s, const WorkItem* wl, int nwl, const int32_t* tabs, int ntab, const TDesc* D,
             const FPtrs& F, const SPtrs& S) {
  if (nwl <= 0) return;
  hipLaunchKernelGGL(k_compact_count, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  tile_scan_pair(s, tabs, ntab, D, F.agg, F.cnt, CNT_MC, CNT_GC);
  hipLaunchKernelGGL(k_compact_write, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  hipLaunchKernelGGL(k_group_recs, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
  hipLaunchKernelGGL(k_compact_links, dim3(nwl), dim3(GJ_BLOCK), 0, s, wl, D, F, S);
}

}  // namespace gjk
