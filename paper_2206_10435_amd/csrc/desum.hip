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
// Each lane locates the first of its `L` consecutive tuples and then walks
// them with an odometer (rows fastest, then entries, no division).  Tuples go
// through LDS so that each wavefront store instruction writes whole 128-byte
// lines.  Block indices are remapped so that each XCD (own L2) expands one
// contiguous part of the range and re-reads the same entries.
#include "gj_internal.h"
#include "kernels.h"
#include "desum.h"

namespace {

template <int N, typename WT>
__global__ void __launch_bounds__(GJ_BLOCK) k_desum(gjk::DesumArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int n = a.n_tables;
  const int K = a.k_round;  // tuples per lane per round
  const int L = a.tuples_per_lane;
  // XCD-aware block order: consecutive logical blocks on the same XCD
  const int nb = gridDim.x;
  const int per_xcd = nb / 8;
  const int b = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (b % 8) * per_xcd + b / 8 : b;
  const int64_t glane = (int64_t)lb * GJ_BLOCK + threadIdx.x;
  const int64_t my0 = glane * L;  // first tuple of this lane within the chunk
  const int64_t mycnt = max((int64_t)0, min((int64_t)L, a.n_rows - my0));
  const int wv = wave_id(), ln = lane_id();
  WT* wlds = reinterpret_cast<WT*>(lds_raw) + (int64_t)wv * 64 * K * n;
  int32_t* lds_cnt = reinterpret_cast<int32_t*>(lds_raw + (size_t)GJ_BLOCK * K * n * sizeof(WT)) + wv * 64;

  int32_t e[N], g[N], r[N], c[N], st[N];
  uint64_t mg[N];
  WT rid[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    e[t] = 0;
    g[t] = 0;
    r[t] = 0;
    c[t] = 1;
    st[t] = 0;
    mg[t] = 1;
    rid[t] = 0;
  }
  if (mycnt > 0) {
    // ---- locate rank first + my0 ----
    uint64_t R = (uint64_t)(a.first + my0);
    uint64_t P = 1;
#pragma unroll
    for (int t = 0; t < N; ++t) {
      if (t < n) {
        const gjk::DTab& T = a.tab[t];
        int64_t lo, hi;
        if (t == 0) {
          lo = 0;
          hi = a.n_root;
        } else {
          lo = T.cglo[g[t]];
          hi = T.cghi[g[t]];
        }
        uint64_t Kt = P;
#pragma unroll
        for (int j = t + 1; j < N; ++j)
          if (j < n && a.tab[j].parent < t) Kt *= mg[j];
        // largest x in [lo, hi) with Kt * pre[x] <= R (pre[lo] == 0)
        int64_t x0 = lo, x1 = hi;  // invariant: answer in [x0, x1)
        while (x1 - x0 > 1) {
          int64_t mid = (x0 + x1) >> 1;
          if (Kt * (uint64_t)T.cpre[mid] <= R)
            x0 = mid;
          else
            x1 = mid;
        }
        e[t] = (int32_t)x0;
        R -= Kt * (uint64_t)T.cpre[x0];
        c[t] = (int32_t)T.cc[x0];
        st[t] = T.cstart[x0];
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
        rid[t] = (WT)a.tab[t].perm[st[t] + r[t]];
      }
    }
  }

  // ---- expand: rounds of K tuples through LDS ----
  const int rounds = (L + K - 1) / K;
  WT* out = reinterpret_cast<WT*>(a.out);
  int64_t done = 0;
  for (int rd = 0; rd < rounds; ++rd) {
    const int64_t kcnt = max((int64_t)0, min((int64_t)K, mycnt - done));
    for (int k = 0; k < kcnt; ++k) {
#pragma unroll
      for (int t = 0; t < N; ++t)
        if (t < n) wlds[((int64_t)ln * K + k) * n + t] = rid[t];
      if (done + k + 1 < mycnt) {
        // odometer: rows first
        bool carry = true;
#pragma unroll
        for (int t = N - 1; t >= 0; --t) {
          if (t < n && carry) {
            if (++r[t] < c[t])
              carry = false;
            else
              r[t] = 0;
            rid[t] = (WT)a.tab[t].perm[st[t] + r[t]];
          }
        }
        if (carry) {
          // every row list wrapped: next entry tuple
          int tc = -1;
#pragma unroll
          for (int t = N - 1; t >= 0; --t) {
            if (t < n && tc < 0) {
              ++e[t];
              const int64_t hi = (t == 0) ? a.n_root : (int64_t)a.tab[t].cghi[g[t]];
              if (e[t] < hi) tc = t;
            }
          }
#pragma unroll
          for (int t = 0; t < N; ++t) {
            if (t > 0 && t < n && t > tc) {
              const int pt = a.tab[t].parent;
              int32_t ep = 0;
#pragma unroll
              for (int i = 0; i < N; ++i)
                if (i == pt) ep = e[i];
              g[t] = a.tab[t].clink[ep];
              e[t] = a.tab[t].cglo[g[t]];
            }
          }
#pragma unroll
          for (int t = 0; t < N; ++t) {
            if (t < n && t >= tc) {
              const gjk::DTab& T = a.tab[t];
              c[t] = (int32_t)T.cc[e[t]];
              st[t] = T.cstart[e[t]];
              r[t] = 0;
              rid[t] = (WT)T.perm[st[t]];
            }
          }
        }
      }
    }
    lds_cnt[ln] = (int32_t)kcnt;
    __syncthreads();
    // flush: lane ln writes 16-byte units of every lane's segment
    const int seg_bytes = K * n * (int)sizeof(WT);
    const int upl = seg_bytes >> 4;  // 16-byte units per lane segment
    const unsigned char* src = reinterpret_cast<const unsigned char*>(wlds);
    unsigned char* dst_base = reinterpret_cast<unsigned char*>(out);
    const int64_t wave_lane0 = glane - ln;
    for (int q = ln; q < 64 * upl; q += 64) {
      const int sl = q / upl;
      const int u = q - sl * upl;
      const int64_t bytes = (int64_t)lds_cnt[sl] * n * (int64_t)sizeof(WT);
      const int64_t b0 = (int64_t)u * 16;
      if (b0 >= bytes) continue;
      const int64_t tup0 = (wave_lane0 + sl) * L + done;  // same `done` for every lane of the wave
      unsigned char* dst = dst_base + tup0 * n * (int64_t)sizeof(WT) + b0;
      const unsigned char* s = src + (int64_t)sl * seg_bytes + b0;
      if (b0 + 16 <= bytes) {
        *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(s);
      } else {
        for (int64_t x = 0; x < bytes - b0; x += 4)
          *reinterpret_cast<uint32_t*>(dst + x) = *reinterpret_cast<const uint32_t*>(s + x);
      }
    }
    __syncthreads();
    done += K;
  }
}

template <int N>
void launch_n(hipStream_t s, const gjk::DesumArgs& a, int rowid_bytes, int blocks, size_t lds) {
  if (rowid_bytes == 4)
    hipLaunchKernelGGL((k_desum<N, int32_t>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  else
    hipLaunchKernelGGL((k_desum<N, int64_t>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
}

}  // namespace

namespace gjk {

// Tuples per lane per LDS round: the most that fit 240 bytes (so a block's
// staging stays below 64 KB) with the round a whole number of 128-byte lines,
// else of 16-byte units.
int desum_round(int n_tables, int rowid_bytes) {
  const int tb = n_tables * rowid_bytes;
  for (int k = 240 / tb; k >= 1; --k)
    if ((k * tb) % 128 == 0) return k;
  for (int k = 240 / tb; k >= 1; --k)
    if ((k * tb) % 16 == 0) return k;
  return 4;  // tb is a multiple of 4, so 4 tuples are a multiple of 16 bytes
}

int desummarize(hipStream_t s, const DesumArgs& a0, int rowid_bytes, int n_tables, int rounds_per_lane) {
  DesumArgs a = a0;
  a.n_tables = n_tables;
  a.k_round = desum_round(n_tables, rowid_bytes);
  a.tuples_per_lane = a.k_round * rounds_per_lane;
  if (a.n_rows <= 0) return 0;
  int64_t lanes = (a.n_rows + a.tuples_per_lane - 1) / a.tuples_per_lane;
  int64_t blocks = (lanes + GJ_BLOCK - 1) / GJ_BLOCK;
  blocks = (blocks + 7) / 8 * 8;  // whole XCD rounds for the block remap
  if (blocks > 0x7fffffff) return -1;
  size_t lds = (size_t)GJ_BLOCK * a.k_round * n_tables * rowid_bytes + GJ_BLOCK * sizeof(int32_t);
  switch (n_tables) {
    case 1: launch_n<1>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 2: launch_n<2>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 3: launch_n<3>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 4: launch_n<4>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 5: launch_n<5>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 6: launch_n<6>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 7: launch_n<7>(s, a, rowid_bytes, (int)blocks, lds); break;
    case 8: launch_n<8>(s, a, rowid_bytes, (int)blocks, lds); break;
    default: launch_n<GJ_MAX_TABLES>(s, a, rowid_bytes, (int)blocks, lds); break;
  }
  return 0;
}

}  // namespace gjk
