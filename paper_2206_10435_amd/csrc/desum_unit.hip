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
// splits into the row indexes (r_0, .., r_n-1) over the counts.  Nothing of
// it depends on a neighbouring tuple, so a wavefront takes 64 consecutive
// ranks at once, one per lane: the lanes' loads of the same entry fall on the
// same lines, and the 64 tuples leave through the wave's LDS as contiguous
// 16-byte stores.  The general kernel instead walks each lane's own range,
// and when the root entry changes every few tuples (short innermost groups),
// its lanes restart at different times and the wave waits for each restart.
//
// Root entries of a window: the wave holds the block offsets of 64
// consecutive root entries, one per lane, and each lane finds its entry by a
// binary search over the other lanes' values (lane permutes).  64
// consecutive ranks span at most 64 entries, as every surviving entry's block
// is at least one rank, so a window falls outside the held entries only when
// it starts past them; the wave then reloads from its first lane's entry.
#include "desum_kernel.h"

namespace {

constexpr int UNIT_WINDOWS = 2;       // windows of 64 ranks decoded together (their loads overlap)
constexpr int UNIT_WAVE_TUPLES = 4096;  // tuples per wavefront (one cooperative locate each)

// j: the largest lane index with v_j <= R (v_0 <= R), and v_j itself.
// Values of lanes past the root are ~0 and never selected.
__device__ __forceinline__ int lane_search(uint64_t v, uint64_t R, uint64_t& vj) {
  int j = 0;
  vj = __shfl(v, 0);
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    const uint64_t vs = __shfl(v, j + s);
    if (vs <= R) {
      j += s;
      vj = vs;
    }
  }
  return j;
}

template <int N, typename WT>
__global__ void __launch_bounds__(GJ_BLOCK) k_desum_unit(gjk::DesumArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int J = UNIT_WINDOWS;
  const int n = N <= 8 ? N : a.n_tables;
  const int tl = n - 1;  // innermost table, a leaf
  const int ln = lane_id();
  // XCD-aware order: consecutive wave ranges on the same XCD
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t w0 = ((int64_t)lb * GJ_WAVES + wave_id()) * UNIT_WAVE_TUPLES;
  if (w0 >= a.n_rows) return;  // wave-uniform
  const int64_t w1 = min(a.n_rows, w0 + (int64_t)UNIT_WAVE_TUPLES);
  const int tb = n * (int)sizeof(WT);  // tuple bytes
  unsigned char* stage = lds_raw + (int64_t)wave_id() * 64 * N * (int)sizeof(WT);
  unsigned char* dst_base = reinterpret_cast<unsigned char*>(a.out);

  const int64_t* __restrict__ pre0 = a.tab[0].cpre;
  const int2* __restrict__ ccs0 = a.tab[0].ccs;
  const int32_t nroot = (int32_t)a.n_root;
  // root entry of the wave's first rank (every lane the same rank: the
  // cooperative search of the general kernel)
  int32_t C = find_block(pre0, 0, nroot, 1, (uint64_t)(a.first + w0), ln);
  C = __builtin_amdgcn_readfirstlane(C);
  uint64_t v = C + ln < nroot ? (uint64_t)pre0[C + ln] : ~0ull;
  uint64_t vn = C + 64 < nroot ? (uint64_t)pre0[C + 64] : ~0ull;

  for (int64_t s0 = w0; s0 < w1; s0 += 64 * J) {
    // ---- root entry and the offset inside its block, per window ----
    int32_t e0[J];
    uint64_t R1[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t off = min(s0 + 64 * j + ln, w1 - 1);  // lanes past the range repeat the last rank
      const uint64_t R = (uint64_t)(a.first + off);
      uint64_t vj;
      int jj = lane_search(v, R, vj);
      // a lane on the held range's last entry may be past it (the entry
      // after it starts at vn); the window then starts at or after the
      // first lane's entry, and one reload from there holds the whole window
      for (int it = 0; it < 4 && !__all(jj < 63 || R < vn); ++it) {
        const int j0 = __shfl(jj, 0);
        const uint64_t R0 = __shfl(R, 0);
        C += (j0 < 63 || R0 < vn) ? j0 : 64;
        C = __builtin_amdgcn_readfirstlane(C);
        v = C + ln < nroot ? (uint64_t)pre0[C + ln] : ~0ull;
        vn = C + 64 < nroot ? (uint64_t)pre0[C + 64] : ~0ull;
        jj = lane_search(v, R, vj);
      }
      e0[j] = C + jj;
      R1[j] = R - vj;
    }
    // ---- records: the root entry's (count, start), the middle tables'
    //      only entries through the child records, the innermost group ----
    int32_t pos[J][N];  // perm position of each table's row id
    int32_t c0[J], gf[J], ge[J], gc[J];
    bool big[J];        // a middle table's count is above 1 (rare: full split)
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int2 cs = ccs0[e0[j]];
      c0[j] = cs.x;
      int32_t ent[N];  // entry of each table (the middle tables' only one)
#pragma unroll
      for (int t = 0; t < N; ++t) {
        ent[t] = 0;
        pos[j][t] = 0;
      }
      pos[j][0] = cs.y;
      ent[0] = e0[j];
      big[j] = false;
      gf[j] = ge[j] = 0;
      gc[j] = 1;
#pragma unroll
      for (int t = 1; t < N; ++t) {
        if (t < n) {
          const int pt = a.tab[t].parent;
          int32_t ep = ent[0];
#pragma unroll
          for (int i = 1; i < N; ++i)
            if (i == pt) ep = ent[i];
          const int4 rc = *reinterpret_cast<const int4*>(a.tab[t].crec + ep);
          ent[t] = rc.x;
          pos[j][t] = rc.w;
          if (t < tl) {
            big[j] = big[j] || rc.z != 1;
          } else {
            gf[j] = rc.x;
            ge[j] = rc.y;
            gc[j] = rc.z;
          }
        }
      }
    }
    // ---- innermost entry inside its group, then the row indexes ----
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const gjk::DTab& T = a.tab[tl];
      // P: the product of the counts above the innermost table
      uint64_t P = (uint64_t)c0[j];
      if (__any(big[j])) {
        if (big[j]) {
          int32_t ent[N];
#pragma unroll
          for (int t = 0; t < N; ++t) ent[t] = 0;
          ent[0] = e0[j];
#pragma unroll
          for (int t = 1; t < N; ++t) {
            if (t < n && t < tl) {
              const int pt = a.tab[t].parent;
              int32_t ep = ent[0];
#pragma unroll
              for (int i = 1; i < N; ++i)
                if (i == pt) ep = ent[i];
              const int4 rc = *reinterpret_cast<const int4*>(a.tab[t].crec + ep);
              ent[t] = rc.x;
              P *= (uint64_t)rc.z;
            }
          }
        }
      }
      uint64_t R2 = R1[j];
      int32_t c = gc[j];
      if (__any(ge[j] - gf[j] > 1)) {
        const int32_t x = find_block(T.cpre, gf[j], ge[j], P, R1[j], ln);
        if (x != gf[j]) {
          R2 -= P * (uint64_t)T.cpre[x];
          const int2 cs = T.ccs[x];
          c = cs.x;
          pos[j][tl] = cs.y;
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
      pos[j][tl] += (int32_t)rt;
      if (__any(big[j])) {
        if (big[j]) {
          // middle tables from the innermost side: r_t = q mod c_t
          int32_t cm[N], ent[N];
#pragma unroll
          for (int t = 0; t < N; ++t) {
            cm[t] = 1;
            ent[t] = 0;
          }
          ent[0] = e0[j];
#pragma unroll
          for (int t = 1; t < N; ++t) {
            if (t < n && t < tl) {
              const int pt = a.tab[t].parent;
              int32_t ep = ent[0];
#pragma unroll
              for (int i = 1; i < N; ++i)
                if (i == pt) ep = ent[i];
              const int4 rc = *reinterpret_cast<const int4*>(a.tab[t].crec + ep);
              ent[t] = rc.x;
              cm[t] = rc.z;
            }
          }
#pragma unroll
          for (int t = N - 1; t >= 1; --t) {
            if (t < tl) {
              const uint64_t qt = q / (uint64_t)cm[t];
              pos[j][t] += (int32_t)(q - qt * (uint64_t)cm[t]);
              q = qt;
            }
          }
        }
      }
      pos[j][0] += (int32_t)q;
    }
    // ---- row ids, then each window through the wave's LDS ----
    int32_t rid[J][N];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int t = 0; t < N; ++t) rid[j][t] = t < n ? a.tab[t].perm[pos[j][t]] : 0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t t0 = s0 + 64 * j;  // first tuple of the window
      if (t0 >= w1) break;             // wave-uniform
      const int nv = (int)min((int64_t)64, w1 - t0);
      WT* my = reinterpret_cast<WT*>(stage + ln * tb);
#pragma unroll
      for (int t = 0; t < N; ++t)
        if (t < n) my[t] = (WT)(uint32_t)rid[j][t];  // row ids are non-negative
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
}

template <int N>
void launch_unit(hipStream_t s, const gjk::DesumArgs& a, int rowid_bytes, int blocks) {
  const size_t lds = (size_t)GJ_WAVES * 64 * N * rowid_bytes;
  if (rowid_bytes == 4)
    hipLaunchKernelGGL((k_desum_unit<N, int32_t>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  else
    hipLaunchKernelGGL((k_desum_unit<N, int64_t>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
}

}  // namespace

namespace gjk {

int64_t desum_unit_blocks(int64_t n_rows) {
  const int64_t waves = (n_rows + UNIT_WAVE_TUPLES - 1) / UNIT_WAVE_TUPLES;
  const int64_t blocks = (waves + GJ_WAVES - 1) / GJ_WAVES;
  return (blocks + 7) / 8 * 8;  // whole XCD rounds for the block remap
}

int desummarize_unit(hipStream_t s, const DesumArgs& a0, int rowid_bytes, int n_tables) {
  if (a0.n_rows <= 0) return 0;
  if (n_tables < 2 || n_tables > GJ_MAX_TABLES || (rowid_bytes != 4 && rowid_bytes != 8) || a0.n_cols != 0)
    return -1;
  const int64_t blocks = desum_unit_blocks(a0.n_rows);
  if (blocks > 0x7fffffff) return -1;
  DesumArgs a = a0;
  a.n_tables = n_tables;
  switch (n_tables) {
    case 2: launch_unit<2>(s, a, rowid_bytes, (int)blocks); break;
    case 3: launch_unit<3>(s, a, rowid_bytes, (int)blocks); break;
    case 4: launch_unit<4>(s, a, rowid_bytes, (int)blocks); break;
    case 5: launch_unit<5>(s, a, rowid_bytes, (int)blocks); break;
    case 6: launch_unit<6>(s, a, rowid_bytes, (int)blocks); break;
    case 7: launch_unit<7>(s, a, rowid_bytes, (int)blocks); break;
    case 8: launch_unit<8>(s, a, rowid_bytes, (int)blocks); break;
    default: launch_unit<GJ_MAX_TABLES>(s, a, rowid_bytes, (int)blocks); break;
  }
  return 0;
}

}  // namespace gjk
