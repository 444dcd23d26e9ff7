// Stage 3 -- desummarization (Sec. 3.6): write result rows [first, first+n)
// of the sorted result as row-id tuples.  Write-bandwidth bound.
//
// Order.  The result is sorted by all attribute values (Definition 1) and then
// by the row ids.  With the root's entries ordered by its columns and every
// other table's entries ordered by (separator, other columns), that order is:
// the root entry, then table 1's entry inside its separator group, ...,
// table n-1's entry, then the row ids (r_0, .., r_{n-1}) as a mixed-radix
// number over the entries' row lists (table 0 most significant).
//
// Block sizes.  With entries e_0..e_{t-1} fixed, the tuples below are
// P * prod_{j >= t, parent(j) < t} M_j, P = c_0(e_0)...c_{t-1}(e_{t-1}); the
// block of entry e_t inside its group is K * c_t(e_t) U_t(e_t) with
// K = P * prod_{j > t, parent(j) < t} M_j, at offset K * pre_t(e_t), where
// pre_t is the exclusive prefix of c*U in the group.  So a rank is located by
// one binary search per table (multiplications only; every product is
// bounded by the join size) and a mixed-radix split of the rest.
//
// Each lane locates the first of its L consecutive tuples and then walks them
// with an odometer (rows fastest, then entries; no division).  A round of KS
// tuples is produced in two loops: a control loop that only advances the
// odometer and records the perm position of every row id (entry metadata is
// read as fused (count, start) and (first, end) records; the innermost table,
// always a leaf, has consecutive row ranges for the entries of a group, so
// its next start is the current start plus count and its counts are read
// four at a time), then a data loop that issues all KS x n row-id gathers at
// once, so a round waits for memory once.  Tuples are staged in LDS per
// wavefront and flushed as 16-byte units that cover whole lines.  Block
// indices are remapped so that each XCD (own L2) expands one contiguous part
// of the range and re-reads the same entries.
#pragma once
#include <type_traits>

#include "desum.h"
#include "gj_internal.h"
#include "kernels.h"

namespace {

constexpr int CW = 4;  // innermost counts read per refill

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Largest x in [lo, hi) with K * pre[x] <= R, where pre is strictly
// increasing on [lo, hi) (surviving entries have c*U >= 1) and pre[lo] = 0.
// K * pre[x] never exceeds the join size for x in [lo, hi), so no product
// overflows.  Must be called by all 64 lanes of the wave.
//
// When every lane searches the same range (the usual case: a wave's targets
// are a few thousand consecutive ranks), the wave searches it together: each
// lane reads one of 64 evenly spaced probes, every lane finds its own slot
// among them by a binary search over the probes held by the other lanes
// (lane permutes, no memory), and the range shrinks to the union of the
// lanes' slots.  That takes about log64 of the range in dependent loads
// instead of log2.  Lanes whose targets spread over the range finish alone.
__device__ __forceinline__ int32_t find_block(const int64_t* __restrict__ pre, int32_t lo, int32_t hi, uint64_t K,
                                              uint64_t R, int ln) {
  int32_t x0 = lo, x1 = hi;
  const int32_t lo_u = __builtin_amdgcn_readfirstlane(lo);
  const int32_t hi_u = __builtin_amdgcn_readfirstlane(hi);
  if (__all(lo == lo_u && hi == hi_u)) {
    int32_t L0 = lo_u, H0 = hi_u;
    while (true) {
      const int32_t W = H0 - L0;
      if (W <= 1) {
        x0 = L0;
        x1 = L0 + 1;
        break;
      }
      const bool exact = W <= 64;
      const int32_t p = exact ? L0 + ln : L0 + (int32_t)(((int64_t)W * ln) >> 6);
      const uint64_t v = p < H0 ? (uint64_t)pre[p] : ~0ull;
      // slot j: the largest probe index with K * v_j <= R (probe 0 = pre[L0]
      // qualifies for every lane, as the range holds every lane's answer)
      int j = 0;
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) {
        const uint64_t vs = __shfl(v, j + s);
        if (vs != ~0ull && K * vs <= R) j += s;
      }
      if (exact) {
        x0 = L0 + j;
        x1 = x0 + 1;
        break;
      }
      x0 = L0 + (int32_t)(((int64_t)W * j) >> 6);
      x1 = j < 63 ? L0 + (int32_t)(((int64_t)W * (j + 1)) >> 6) : H0;
      const int32_t nL0 = wave_min_i32(x0), nH0 = wave_max_i32(x1);
      if (nH0 - nL0 > W / 2) break;  // the lanes' targets spread out
      L0 = nL0;
      H0 = nH0;
    }
  }
  while (x1 - x0 > 1) {
    const int32_t mid = (int32_t)(((int64_t)x0 + x1) >> 1);
    if (K * (uint64_t)pre[mid] <= R)
      x0 = mid;
    else
      x1 = mid;
  }
  return x0;
}

// NC == 0: the output columns are the row ids of the n tables (N <= 8 is the
// exact table count).  NC > 0: the output columns are a.n_cols <= NC value
// columns, column j read from a.col_src[j] at the group position of table
// a.col_tab[j]; N is then an upper bound of the table count.
template <int N, int NC, typename WT, int KS>
__global__ void __launch_bounds__(GJ_BLOCK) k_desum(gjk::DesumArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int n = (N <= 8 && NC == 0) ? N : a.n_tables;
  constexpr int NCOL = NC == 0 ? N : NC;  // register capacity for output columns
  const int nc = NC == 0 ? n : a.n_cols;
  const int tl = n - 1;  // innermost table: a leaf
  const int L = a.tuples_per_lane;
  // XCD-aware block order: consecutive logical blocks on the same XCD
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t glane = (int64_t)lb * GJ_BLOCK + threadIdx.x;
  const int64_t my0 = glane * L;  // first tuple of this lane within the chunk
  const int64_t mycnt = max((int64_t)0, min((int64_t)L, a.n_rows - my0));
  const int ln = lane_id();

  int32_t e[N], gh[N], r[N], c[N], st[N], cur[NCOL];
  int32_t cw[CW];  // counts of innermost entries cwb .. cwb+CW-1
  int32_t cwb = 0;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    e[t] = 0;
    gh[t] = 0;
    r[t] = 0;
    c[t] = 1;
    st[t] = 0;
  }
#pragma unroll
  for (int j = 0; j < NCOL; ++j) cur[j] = 0;
#pragma unroll
  for (int i = 0; i < CW; ++i) cw[i] = 1;

// counts of the innermost entries from e[tl] on (clamped inside the group)
#define GJ_CW_FILL()                                                                   \
  do {                                                                                 \
    cwb = e[tl];                                                                       \
    const int2* cs = a.tab[tl].ccs;                                                    \
    _Pragma("unroll") for (int i = 0; i < CW; ++i) cw[i] = cs[min(cwb + i, gh[tl] - 1)].x; \
  } while (0)

  // wave-uniform: the searches below are cooperative, so every lane of a wave
  // with any work locates (lanes past the range take the range's last rank
  // and write nothing)
  if ((glane - ln) * L < a.n_rows) {
    // ---- locate rank first + my0 ----
    uint64_t R = (uint64_t)(a.first + min(my0, a.n_rows - 1));
    uint64_t P = 1;
    int32_t lo[N], fc[N], fs[N];
    uint64_t mg[N];
    uint32_t have_mg = 0;  // bit j: mg[j] read
#pragma unroll
    for (int t = 0; t < N; ++t) {
      lo[t] = 0;
      mg[t] = 1;
      fc[t] = 1;
      fs[t] = 0;
    }
    gh[0] = (int32_t)a.n_root;
#pragma unroll
    for (int t = 0; t < N; ++t) {
      if (t < n) {
        const gjk::DTab& T = a.tab[t];
        // The pending messages scale only a search over more than one entry:
        // a group of one entry (a dimension joined on its key) needs neither
        // them nor its block offset (0, the group's first) nor its count and
        // start (in the child record), so its locate reads no random line.
        uint64_t Kt = P;
        if (gh[t] - lo[t] > 1) {
#pragma unroll
          for (int j = t + 1; j < N; ++j) {
            if (j < n && a.tab[j].parent < t) {
              if (!((have_mg >> j) & 1)) {
                // the group's message: the block offset of its last entry plus that block
                const gjk::DTab& C = a.tab[j];
                const int32_t x = gh[j] - 1;
                mg[j] = (uint64_t)C.cpre[x] + (uint64_t)C.ccs[x].x * (uint64_t)C.cU[x];
                have_mg |= 1u << j;
              }
              Kt *= mg[j];
            }
          }
        }
        const int32_t x0 = find_block(T.cpre, lo[t], gh[t], Kt, R, ln);
        e[t] = x0;
        if (t == 0 || x0 != lo[t]) {
          R -= Kt * (uint64_t)T.cpre[x0];
          const int2 cs = T.ccs[x0];
          c[t] = cs.x;
          st[t] = cs.y;
        } else {
          c[t] = fc[t];
          st[t] = fs[t];
        }
        P *= (uint64_t)c[t];
        // children: their group (entry range, first entry's count and start)
        // under this entry
#pragma unroll
        for (int j = t + 1; j < N; ++j) {
          if (j < n && a.tab[j].parent == t) {
            const int4 rc = *reinterpret_cast<const int4*>(a.tab[j].crec + e[t]);
            lo[j] = rc.x;
            gh[j] = rc.y;
            fc[j] = rc.z;
            fs[j] = rc.w;
          }
        }
      }
    }
#pragma unroll
    for (int t = N - 1; t >= 0; --t) {
      if (t < n) {
        r[t] = (int32_t)(R % (uint64_t)c[t]);
        R /= (uint64_t)c[t];
      }
    }
    cwb = e[tl] - CW;  // the counts window is read on the first advance inside the group
  }

  const int wv = wave_id();
  // A lane's staged round is one segment of KS*nc values, upl whole 16-byte
  // units (the launcher picks KS so), placed in a slot of uplp units, the next
  // power of two.  Unit u of lane l's segment is stored at unit u ^ swz(l):
  // without it the lanes of a write instruction, one slot apart, fall into
  // the same banks.  Row-id launches whose segment is not a power of two of
  // units (6 tables of int64 ids: 12 units) use slots of exactly upl units
  // instead, unswizzled: the padding would cost a quarter of the LDS and with
  // it occupancy, which bounds expansions of short runs (the general flush
  // below handles that layout).
  const int seg_bytes = KS * nc * (int)sizeof(WT);
  const int upl = seg_bytes >> 4;
  int uplp = 1;
  while (uplp < upl) uplp <<= 1;
  const bool tight = NC == 0 && uplp != upl;
  const int slot = (tight ? upl : uplp) << 4;
  unsigned char* wlds = lds_raw + (int64_t)wv * 64 * slot;
  auto swz = [&](int l) -> int {
    return tight ? 0 : ((((l * uplp) >> 3) ^ ((l * uplp) >> 4)) & (uplp - 1));
  };
  const int my_swz = swz(ln);
  unsigned char* my_seg = wlds + (int64_t)ln * slot;
  unsigned char* dst_base = reinterpret_cast<unsigned char*>(a.out);
  const int64_t wave_lane0 = glane - ln;
  const int64_t tup_bytes = (int64_t)nc * (int64_t)sizeof(WT);
  const int rounds = (L + KS - 1) / KS;
  int64_t done = 0;
  // row ids tuple 0 of the next round needs (the first round reads them all)
  uint32_t next0 = (uint32_t)((1ull << N) - 1);
  for (int rd = 0; rd < rounds; ++rd) {
    const int kcnt = (int)max((int64_t)0, min((int64_t)KS, mycnt - done));
    // ---- control: perm positions of the row ids that change ----
    // chg bit (k*N + t): tuple k of the round needs a new row id for table t
    int32_t pos[KS][N];
    static_assert(KS * N <= 64, "change mask is 64 bits");
    using MT = typename std::conditional<KS * N <= 32, uint32_t, uint64_t>::type;
    MT chg = (MT)next0;
    uint32_t nx = 0;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int t = 0; t < N; ++t) pos[k][t] = st[t] + r[t];
      if (k < kcnt && done + k + 1 < mycnt) {
        bool carry = true;
#pragma unroll
        for (int t = N - 1; t >= 0; --t) {
          if (t < n && carry) {
            if (++r[t] < c[t])
              carry = false;
            else
              r[t] = 0;
            if (k + 1 < KS)
              chg |= (MT)1 << ((k + 1) * N + t);
            else
              nx |= 1u << t;
          }
        }
        if (carry) {
          // every row list wrapped: next entry tuple
          if (k + 1 < KS)
            chg |= (MT)(((MT)1 << N) - 1) << ((k + 1) * N);
          else
            nx = (uint32_t)((1ull << N) - 1);
          if (e[tl] + 1 < gh[tl]) {
            // next entry of the innermost group: rows follow the current ones
            st[tl] += c[tl];
            ++e[tl];
            if (e[tl] - cwb >= CW) GJ_CW_FILL();
            const int d = e[tl] - cwb;
            int32_t v = cw[0];
#pragma unroll
            for (int i = 1; i < CW; ++i)
              if (d == i) v = cw[i];
            c[tl] = v;
          } else {
            // the deepest table with a next entry in its group advances ...
            int tc = -1;
#pragma unroll
            for (int t = N - 1; t >= 0; --t) {
              if (t < n && tc < 0) {
                ++e[t];
                if (e[t] < gh[t]) tc = t;
              }
            }
#pragma unroll
            for (int t = 0; t < N; ++t) {
              if (t < n && t == tc) {
                const int2 cs = a.tab[t].ccs[e[t]];
                c[t] = cs.x;
                st[t] = cs.y;
              }
            }
            // ... and every later table restarts at the first entry of the
            // group under its parent's (possibly new) entry: one record each
#pragma unroll
            for (int t = 1; t < N; ++t) {
              if (t < n && t > tc) {
                const int pt = a.tab[t].parent;
                int32_t ep = 0;
#pragma unroll
                for (int i = 0; i < N; ++i)
                  if (i == pt) ep = e[i];
                const int4 rc = *reinterpret_cast<const int4*>(a.tab[t].crec + ep);
                e[t] = rc.x;
                gh[t] = rc.y;
                c[t] = rc.z;
                st[t] = rc.w;
              }
            }
            cwb = e[tl] - CW;
          }
        }
      }
    }
    // tuple 0 of the next round reads what the last advance of this round
    // changed (re-reading every row id at each round start costs a random
    // line per table and lane when runs are short)
    next0 = nx;
    // ---- data: gathers of the columns whose table moved (exec-masked), all
    //      issued before the first use, then the round into the wave's staging ----
    int32_t v[KS][NCOL];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int j = 0; j < NCOL; ++j) {
        if (j < nc) {
          const int tj = NC == 0 ? j : a.col_tab[j];
          int32_t pj = pos[k][0];
          if (NC == 0) {
            pj = pos[k][j];
          } else {
#pragma unroll
            for (int t = 1; t < N; ++t)
              if (tj == t) pj = pos[k][t];
          }
          const int32_t* src = NC == 0 ? a.tab[j].perm : a.col_src[j];
          if (k < kcnt && ((chg >> (k * N + tj)) & 1)) v[k][j] = src[pj];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int j = 0; j < NCOL; ++j) {
        if (j < nc) {
          const int tj = NC == 0 ? j : a.col_tab[j];
          if (k < kcnt && ((chg >> (k * N + tj)) & 1)) cur[j] = v[k][j];
          const int off = (k * nc + j) * (int)sizeof(WT);
          // row ids are non-negative: zero-extended to the output width
          *reinterpret_cast<WT*>(my_seg + ((((off >> 4) ^ my_swz)) << 4) + (off & 15)) = (WT)(uint32_t)cur[j];
        }
      }
    }
    // ---- flush: lane ln writes 16-byte units of every lane's segment ----
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      const unsigned char* src = reinterpret_cast<const unsigned char*>(wlds);
      // every lane of the wave staged a whole round (all but the range's end)
      const bool wave_full = (wave_lane0 + 63) * L + done + KS <= a.n_rows;
      if (wave_full && !tight) {
        // slot unit q = ln + 64 i is unit (ln mod uplp) of lane ln / uplp + i * 64 / uplp
        // (swz(sl) with sl * uplp = sl0 * uplp + 64 i, split into its parts);
        // units past the segment (u >= upl) are padding and not written
        const int lsh = __builtin_ctz(uplp);
        const int u = ln & (uplp - 1);
        const int sl0 = ln >> lsh;
        const int step = 64 >> lsh;
        const int sa = (sl0 * uplp) >> 3, sb = (sl0 * uplp) >> 4;
        const unsigned char* rbase = src + sl0 * slot;
        unsigned char* dst = dst_base + ((wave_lane0 + sl0) * L + done) * tup_bytes + u * 16;
        const int64_t dstep = (int64_t)step * L * tup_bytes;
        const bool mine = u < upl;
#pragma unroll
        for (int i = 0; i < uplp; ++i) {
          const int sw = ((sa + 8 * i) ^ (sb + 4 * i)) & (uplp - 1);
          if (mine) {
            const uint4 val = *reinterpret_cast<const uint4*>(rbase + i * step * slot + ((u ^ sw) << 4));
            __builtin_nontemporal_store(val.x, reinterpret_cast<uint32_t*>(dst));
            __builtin_nontemporal_store(val.y, reinterpret_cast<uint32_t*>(dst) + 1);
            __builtin_nontemporal_store(val.z, reinterpret_cast<uint32_t*>(dst) + 2);
            __builtin_nontemporal_store(val.w, reinterpret_cast<uint32_t*>(dst) + 3);
          }
          dst += dstep;
        }
      } else if (wave_full) {
        // unpadded slots: unit q = ln + 64 i is unit q % upl of lane q / upl
        for (int q = ln; q < 64 * upl; q += 64) {
          const int sl = q / upl;
          const int u = q - sl * upl;
          const uint4 val = *reinterpret_cast<const uint4*>(src + sl * slot + (u << 4));
          unsigned char* dst = dst_base + ((wave_lane0 + sl) * L + done) * tup_bytes + (u << 4);
          __builtin_nontemporal_store(val.x, reinterpret_cast<uint32_t*>(dst));
          __builtin_nontemporal_store(val.y, reinterpret_cast<uint32_t*>(dst) + 1);
          __builtin_nontemporal_store(val.z, reinterpret_cast<uint32_t*>(dst) + 2);
          __builtin_nontemporal_store(val.w, reinterpret_cast<uint32_t*>(dst) + 3);
        }
      } else {
        for (int q = ln; q < 64 * upl; q += 64) {
          const int sl = q / upl;
          const int u = q - sl * upl;
          // tuples lane sl wrote this round (fewer than KS only at the end)
          const int64_t tup0 = (wave_lane0 + sl) * L + done;
          const int64_t scnt = max((int64_t)0, min((int64_t)KS, min((int64_t)L - done, a.n_rows - tup0)));
          const int64_t bytes = scnt * tup_bytes;
          const int64_t b0 = (int64_t)u * 16;
          if (b0 >= bytes) continue;
          unsigned char* dst = dst_base + tup0 * tup_bytes + b0;
          const unsigned char* sp = src + (int64_t)sl * slot + ((u ^ swz(sl)) << 4);
          if (b0 + 16 <= bytes) {
            const uint4 val = *reinterpret_cast<const uint4*>(sp);
            __builtin_nontemporal_store(val.x, reinterpret_cast<uint32_t*>(dst));
            __builtin_nontemporal_store(val.y, reinterpret_cast<uint32_t*>(dst) + 1);
            __builtin_nontemporal_store(val.z, reinterpret_cast<uint32_t*>(dst) + 2);
            __builtin_nontemporal_store(val.w, reinterpret_cast<uint32_t*>(dst) + 3);
          } else {
            for (int64_t x = 0; x < bytes - b0; x += 4)
              *reinterpret_cast<uint32_t*>(dst + x) = *reinterpret_cast<const uint32_t*>(sp + x);
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    done += KS;
  }
#undef GJ_CW_FILL
}

}  // namespace
