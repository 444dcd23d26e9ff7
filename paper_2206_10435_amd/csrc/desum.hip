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
#include "desum.h"
#include "gj_internal.h"
#include "kernels.h"

namespace {

constexpr int CW = 4;  // innermost counts read per refill

template <int N, typename WT, int KS>
__global__ void __launch_bounds__(GJ_BLOCK) k_desum(gjk::DesumArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // exact table count for N <= 8 (compile-time), runtime for the generic case
  const int n = N <= 8 ? N : a.n_tables;
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

  int32_t e[N], gh[N], r[N], c[N], st[N], cur[N];
  int32_t cw[CW];  // counts of innermost entries cwb .. cwb+CW-1
  int32_t cwb = 0;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    e[t] = 0;
    gh[t] = 0;
    r[t] = 0;
    c[t] = 1;
    st[t] = 0;
    cur[t] = 0;
  }
#pragma unroll
  for (int i = 0; i < CW; ++i) cw[i] = 1;

// counts of the innermost entries from e[tl] on (clamped inside the group)
#define GJ_CW_FILL()                                                                   \
  do {                                                                                 \
    cwb = e[tl];                                                                       \
    const int2* cs = a.tab[tl].ccs;                                                    \
    _Pragma("unroll") for (int i = 0; i < CW; ++i) cw[i] = cs[min(cwb + i, gh[tl] - 1)].x; \
  } while (0)

  if (mycnt > 0) {
    // ---- locate rank first + my0 ----
    uint64_t R = (uint64_t)(a.first + my0);
    uint64_t P = 1;
    int32_t g[N];
    uint64_t mg[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      g[t] = 0;
      mg[t] = 1;
    }
#pragma unroll
    for (int t = 0; t < N; ++t) {
      if (t < n) {
        const gjk::DTab& T = a.tab[t];
        int64_t lo;
        if (t == 0) {
          lo = 0;
          gh[t] = (int32_t)a.n_root;
        } else {
          lo = T.cglo[g[t]];
          gh[t] = T.cghi[g[t]];
        }
        uint64_t Kt = P;
#pragma unroll
        for (int j = t + 1; j < N; ++j)
          if (j < n && a.tab[j].parent < t) Kt *= mg[j];
        // largest x in [lo, hi) with Kt * pre[x] <= R (pre[lo] == 0)
        int64_t x0 = lo, x1 = gh[t];
        while (x1 - x0 > 1) {
          const int64_t mid = (x0 + x1) >> 1;
          if (Kt * (uint64_t)T.cpre[mid] <= R)
            x0 = mid;
          else
            x1 = mid;
        }
        e[t] = (int32_t)x0;
        R -= Kt * (uint64_t)T.cpre[x0];
        const int2 cs = T.ccs[x0];
        c[t] = cs.x;
        st[t] = cs.y;
        P *= (uint64_t)c[t];
#pragma unroll
        for (int j = t + 1; j < N; ++j) {
          if (j < n && a.tab[j].parent == t) {
            g[j] = a.tab[j].clink[e[t]];
            mg[j] = (uint64_t)a.tab[j].cgM[g[j]];
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
    GJ_CW_FILL();
  }

  const int wv = wave_id();
  WT* wlds = reinterpret_cast<WT*>(lds_raw) + (int64_t)wv * 64 * KS * n;
  int32_t* lds_cnt = reinterpret_cast<int32_t*>(lds_raw + (size_t)GJ_BLOCK * KS * n * sizeof(WT)) + wv * 64;
  unsigned char* dst_base = reinterpret_cast<unsigned char*>(a.out);
  const int rounds = (L + KS - 1) / KS;
  int64_t done = 0;
  for (int rd = 0; rd < rounds; ++rd) {
    const int kcnt = (int)max((int64_t)0, min((int64_t)KS, mycnt - done));
    // ---- control: perm positions of the row ids that change ----
    // chg bit (k*N + t): tuple k of the round needs a new row id for table t
    int32_t pos[KS][N];
    static_assert(KS * N <= 64, "change mask is 64 bits");
    uint64_t chg = 0;
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
            if (k + 1 < KS) chg |= 1ull << ((k + 1) * N + t);
          }
        }
        if (carry) {
          // every row list wrapped: next entry tuple
          if (k + 1 < KS) chg |= (N == 64 ? ~0ull : ((1ull << N) - 1)) << ((k + 1) * N);
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
            int tc = -1;
#pragma unroll
            for (int t = N - 1; t >= 0; --t) {
              if (t < n && tc < 0) {
                ++e[t];
                if (e[t] < gh[t]) tc = t;
              }
            }
#pragma unroll
            for (int t = 1; t < N; ++t) {
              if (t < n && t > tc) {
                const int pt = a.tab[t].parent;
                int32_t ep = 0;
#pragma unroll
                for (int i = 0; i < N; ++i)
                  if (i == pt) ep = e[i];
                const int2 lr = a.tab[t].clr[ep];
                e[t] = lr.x;
                gh[t] = lr.y;
              }
            }
#pragma unroll
            for (int t = 0; t < N; ++t) {
              if (t < n && t >= tc) {
                const int2 cs = a.tab[t].ccs[e[t]];
                c[t] = cs.x;
                st[t] = cs.y;
              }
            }
            GJ_CW_FILL();
          }
        }
      }
    }
    // the first tuple of a round after the lane's first round reuses the row
    // ids of the previous round's last tuple unless they changed across the
    // round boundary, which the previous round's control loop cannot know:
    // gather them all for k = 0.
    chg |= (1ull << N) - 1;
    // ---- data: gathers of changed row ids only (exec-masked), all issued
    //      before the first use, then the round into the wave's staging ----
    int32_t v[KS][N];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int t = 0; t < N; ++t) {
        v[k][t] = 0;
        if (t < n && k < kcnt && ((chg >> (k * N + t)) & 1ull)) v[k][t] = a.tab[t].perm[pos[k][t]];
      }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int t = 0; t < N; ++t) {
        if (t < n) {
          if ((chg >> (k * N + t)) & 1ull) cur[t] = v[k][t];
          wlds[((int64_t)ln * KS + k) * n + t] = (WT)cur[t];
        }
      }
    }
    // ---- flush: lane ln writes 16-byte units of every lane's segment ----
    lds_cnt[ln] = kcnt;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      const int seg_bytes = KS * n * (int)sizeof(WT);
      const int upl = seg_bytes >> 4;
      const unsigned char* src = reinterpret_cast<const unsigned char*>(wlds);
      const int64_t wave_lane0 = glane - ln;
      for (int q = ln; q < 64 * upl; q += 64) {
        const int sl = q / upl;
        const int u = q - sl * upl;
        const int64_t bytes = (int64_t)lds_cnt[sl] * n * (int64_t)sizeof(WT);
        const int64_t b0 = (int64_t)u * 16;
        if (b0 >= bytes) continue;
        const int64_t tup0 = (wave_lane0 + sl) * L + done;
        unsigned char* dst = dst_base + tup0 * n * (int64_t)sizeof(WT) + b0;
        const unsigned char* sp = src + (int64_t)sl * seg_bytes + b0;
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
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    done += KS;
  }
#undef GJ_CW_FILL
}

template <int N, typename WT>
void launch_nw(hipStream_t s, const gjk::DesumArgs& a, int ks, int blocks) {
  if (ks == 8 && N * 8 > 64) ks = 4;  // the change mask holds KS * N bits
  const size_t lds = (size_t)GJ_BLOCK * ks * N * sizeof(WT) + GJ_BLOCK * sizeof(int32_t);
  if (ks == 2) {
    hipLaunchKernelGGL((k_desum<N, WT, 2>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  } else if (ks == 8) {
    if constexpr (N * 8 <= 64) hipLaunchKernelGGL((k_desum<N, WT, 8>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  } else {
    hipLaunchKernelGGL((k_desum<N, WT, 4>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  }
}

template <int N>
void launch_n(hipStream_t s, const gjk::DesumArgs& a, int rowid_bytes, int ks, int blocks) {
  if (rowid_bytes == 4)
    launch_nw<N, int32_t>(s, a, ks, blocks);
  else
    launch_nw<N, int64_t>(s, a, ks, blocks);
}

}  // namespace

namespace gjk {

int desummarize(hipStream_t s, const DesumArgs& a0, int rowid_bytes, int n_tables, int rounds_per_lane, int stage) {
  DesumArgs a = a0;
  const int ks = (stage == 2 || stage == 4 || stage == 8) ? stage : 4;
  const int rs = ks;
  if (a0.n_rows <= 0) return 0;
  if (n_tables > GJ_MAX_TABLES) return -1;
  a.n_tables = n_tables;
  a.k_round = ks;
  a.tuples_per_lane = rs * std::max(1, rounds_per_lane);
  // a smaller per-lane range when the chunk would not fill the chip
  while (a.tuples_per_lane > rs && a.n_rows / a.tuples_per_lane < 256LL * 1024) a.tuples_per_lane /= 2;
  a.tuples_per_lane = std::max(rs, a.tuples_per_lane / rs * rs);
  const int64_t lanes = (a.n_rows + a.tuples_per_lane - 1) / a.tuples_per_lane;
  int64_t blocks = (lanes + GJ_BLOCK - 1) / GJ_BLOCK;
  blocks = (blocks + 7) / 8 * 8;  // whole XCD rounds for the block remap
  if (blocks > 0x7fffffff) return -1;
  switch (n_tables) {
    case 1: launch_n<1>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 2: launch_n<2>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 3: launch_n<3>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 4: launch_n<4>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 5: launch_n<5>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 6: launch_n<6>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 7: launch_n<7>(s, a, rowid_bytes, ks, (int)blocks); break;
    case 8: launch_n<8>(s, a, rowid_bytes, ks, (int)blocks); break;
    default: launch_n<GJ_MAX_TABLES>(s, a, rowid_bytes, ks, (int)blocks); break;
  }
  return 0;
}

}  // namespace gjk
