// Desummarization of a projected summary (Sec. 3.7 early projections, then
// Sec. 3.6): the result has no row ids, only the output attributes, and every
// entry tuple (e_0, .., e_{n-1}) of the projected factors is one run of
// identical value tuples whose length is the product of the entries'
// frequencies c_t(e_t) (int64: a projected entry stands for whole deleted
// subtrees).  Writing rows [first, first + n) is therefore run-length
// decoding: a lane locates its first tuple exactly as the row-id expansion
// does (one search per table over the block offsets K * pre, here with the
// wave-cooperative search), then repeats the entry tuple's values until the
// run ends and steps the entry odometer (the deepest table with a next entry
// in its group advances; every later table restarts at the first entry of the
// group under its parent's entry).  Rounds of KS tuples are staged per
// wavefront in LDS and flushed as 16-byte units; a wave inside a single run
// skips all of that and fills its range.
#include "desum_kernel.h"

namespace {

template <int N, int NC, int KS>
__global__ void __launch_bounds__(GJ_BLOCK) k_expand_runs(gjk::RunArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int n = a.n_tables;
  const int nc = a.n_cols;
  const int L = a.tuples_per_lane;
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t glane = (int64_t)lb * GJ_BLOCK + threadIdx.x;
  const int64_t my0 = glane * L;
  const int64_t mycnt = max((int64_t)0, min((int64_t)L, a.n_rows - my0));
  const int ln = lane_id();

  int32_t e[N], gh[N];
  uint64_t c[N];
  int32_t val[NC];
  uint64_t left = 0;  // tuples left in the current run, the current one included
#pragma unroll
  for (int t = 0; t < N; ++t) {
    e[t] = 0;
    gh[t] = 0;
    c[t] = 1;
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) val[j] = 0;

  if ((glane - ln) * L < a.n_rows) {  // wave-uniform (cooperative search)
    uint64_t R = (uint64_t)(a.first + min(my0, a.n_rows - 1));
    uint64_t P = 1;
    int32_t lo[N];
    uint64_t mg[N];
    uint32_t have_mg = 0;  // bit j: mg[j] read
#pragma unroll
    for (int t = 0; t < N; ++t) {
      lo[t] = 0;
      mg[t] = 1;
    }
    gh[0] = (int32_t)a.n_root;
#pragma unroll
    for (int t = 0; t < N; ++t) {
      if (t < n) {
        const gjk::RunTab& T = a.tab[t];
        // pending messages only for a search over more than one entry, and
        // no block offset for a group's first entry (0).  The frequency is
        // read from cc: the record's 32-bit count cannot hold a projected one.
        uint64_t Kt = P;
        if (gh[t] - lo[t] > 1) {
#pragma unroll
          for (int j = t + 1; j < N; ++j) {
            if (j < n && a.tab[j].parent < t) {
              if (!((have_mg >> j) & 1)) {
                // the group's message: the block offset of its last entry plus that block
                const gjk::RunTab& C = a.tab[j];
                const int32_t y = gh[j] - 1;
                mg[j] = (uint64_t)C.cpre[y] + (uint64_t)C.cc[y] * (uint64_t)C.cU[y];
                have_mg |= 1u << j;
              }
              Kt *= mg[j];
            }
          }
        }
        const int32_t x = find_block(T.cpre, lo[t], gh[t], Kt, R, ln);
        e[t] = x;
        if (x != lo[t]) R -= Kt * (uint64_t)T.cpre[x];
        c[t] = (uint64_t)T.cc[x];
        P *= c[t];
#pragma unroll
        for (int j = t + 1; j < N; ++j) {
          if (j < n && a.tab[j].parent == t) {
            const int4 rc = *reinterpret_cast<const int4*>(a.tab[j].crec + x);
            lo[j] = rc.x;
            gh[j] = rc.y;
          }
        }
      }
    }
    left = P - R;  // R: offset inside the run of the entry tuple
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j < nc) {
        const int tj = a.col_tab[j];
        int32_t ej = e[0];
#pragma unroll
        for (int t = 1; t < N; ++t)
          if (tj == t) ej = e[t];
        val[j] = a.col_key[j][ej];
      }
    }
  }

  // A wave whose whole range lies inside one run (the usual case when runs
  // are long, as for a projection's products of frequencies) writes one value
  // tuple repeated: a coalesced fill of 16-byte units, with no staging.  Lane
  // 0's run covers the wave's range when its remaining length reaches the
  // range's end; every lane then holds the same values.
  {
    const int64_t wbase = (glane - ln) * L;  // first tuple of the wave
    const int64_t wspan = 64LL * L;
    bool one_run = false;
    if (wbase < a.n_rows && wbase + wspan <= a.n_rows) {
      const uint32_t l_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)left);
      const uint32_t l_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(left >> 32));
      one_run = (((uint64_t)l_hi << 32) | l_lo) >= (uint64_t)wspan;
    }
    if (one_run) {
      // int32 index x of the wave's region holds column x mod nc; the region
      // starts at a tuple boundary and spans 64 L nc values (whole units)
      uint4* dst = reinterpret_cast<uint4*>(a.out + wbase * nc);
      const int units = L * nc / 4;  // per lane
      int ph = (4 * ln) % nc;        // column of the lane's first value
      const int step = 256 % nc;     // 64 units further on
      auto pick = [&](int col) -> int32_t {
        int32_t x = val[0];
#pragma unroll
        for (int j = 1; j < NC; ++j)
          if (j == col) x = val[j];
        return x;
      };
      for (int i = 0; i < units; ++i) {
        int c1 = ph + 1, c2 = ph + 2, c3 = ph + 3;
        c1 -= c1 >= nc ? nc : 0;
        c2 -= c2 >= nc ? nc : 0;
        c2 -= c2 >= nc ? nc : 0;
        c3 -= c3 >= nc ? nc : 0;
        c3 -= c3 >= nc ? nc : 0;
        c3 -= c3 >= nc ? nc : 0;
        uint4* d = dst + ln + 64 * i;
        __builtin_nontemporal_store((uint32_t)pick(ph), reinterpret_cast<uint32_t*>(d));
        __builtin_nontemporal_store((uint32_t)pick(c1), reinterpret_cast<uint32_t*>(d) + 1);
        __builtin_nontemporal_store((uint32_t)pick(c2), reinterpret_cast<uint32_t*>(d) + 2);
        __builtin_nontemporal_store((uint32_t)pick(c3), reinterpret_cast<uint32_t*>(d) + 3);
        ph += step;
        ph -= ph >= nc ? nc : 0;
      }
      return;
    }
  }

  const int wv = wave_id();
  const int seg = KS * nc;  // int32 values per lane and round (a multiple of 4)
  const int upl = seg >> 2;  // 16-byte units per lane segment
  // a lane's segment sits in a slot of the next power of two of units; unit u
  // is stored at unit u ^ swz(l), so lanes a slot apart use different banks
  int uplp = 1;
  while (uplp < upl) uplp <<= 1;
  const int slot = uplp << 2;  // int32 values per slot
  int32_t* wlds = reinterpret_cast<int32_t*>(lds_raw) + (int64_t)wv * 64 * slot;
  int32_t* my_seg = wlds + (int64_t)ln * slot;
  auto swz = [&](int l) -> int { return (((l * uplp) >> 3) ^ ((l * uplp) >> 4)) & (uplp - 1); };
  const int my_swz = swz(ln);
  const int64_t wave_lane0 = glane - ln;
  const int rounds = (L + KS - 1) / KS;
  int32_t* out = a.out;
  for (int rd = 0; rd < rounds; ++rd) {
    const int64_t done = (int64_t)rd * KS;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        if (j < nc) {
          const int w = k * nc + j;
          my_seg[(((w >> 2) ^ my_swz) << 2) + (w & 3)] = val[j];
        }
      }
      if (done + k + 1 < mycnt) {
        if (--left == 0) {
          // next entry tuple: the deepest table with a next entry in its group
          int tc = -1;
#pragma unroll
          for (int t = N - 1; t >= 0; --t) {
            if (t < n && tc < 0) {
              ++e[t];
              if (e[t] < gh[t]) tc = t;
            }
          }
#pragma unroll
          for (int t = 0; t < N; ++t)
            if (t < n && t == tc) c[t] = (uint64_t)a.tab[t].cc[e[t]];
          // later tables restart at the first entry of their group
#pragma unroll
          for (int t = 1; t < N; ++t) {
            if (t < n && t > tc) {
              const int pt = a.tab[t].parent;
              int32_t ep = 0;
#pragma unroll
              for (int i = 0; i < N; ++i)
                if (i == pt) ep = e[i];
              const ChildRec rc = a.tab[t].crec[ep];
              e[t] = rc.first;
              gh[t] = rc.end;
              c[t] = (uint64_t)a.tab[t].cc[rc.first];
            }
          }
          left = 1;
#pragma unroll
          for (int t = 0; t < N; ++t)
            if (t < n) left *= c[t];
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (j < nc) {
              const int tj = a.col_tab[j];
              if (tj >= tc) {
                int32_t ej = e[0];
#pragma unroll
                for (int t = 1; t < N; ++t)
                  if (tj == t) ej = e[t];
                val[j] = a.col_key[j][ej];
              }
            }
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // flush: lane ln writes 16-byte units of every lane's segment
    for (int q = ln; q < 64 * upl; q += 64) {
      const int sl = q / upl;
      const int u = q - sl * upl;
      const int64_t tup0 = (wave_lane0 + sl) * L + done;
      const int64_t scnt = max((int64_t)0, min((int64_t)KS, min((int64_t)L - done, a.n_rows - tup0)));
      const int64_t words = scnt * nc;
      const int64_t w0 = (int64_t)u * 4;
      if (w0 >= words) continue;
      int32_t* dst = out + tup0 * nc + w0;
      const int32_t* sp = wlds + (int64_t)sl * slot + ((u ^ swz(sl)) << 2);
      if (w0 + 4 <= words) {
        const uint4 v = *reinterpret_cast<const uint4*>(sp);
        __builtin_nontemporal_store(v.x, reinterpret_cast<uint32_t*>(dst));
        __builtin_nontemporal_store(v.y, reinterpret_cast<uint32_t*>(dst) + 1);
        __builtin_nontemporal_store(v.z, reinterpret_cast<uint32_t*>(dst) + 2);
        __builtin_nontemporal_store(v.w, reinterpret_cast<uint32_t*>(dst) + 3);
      } else {
        for (int64_t x = 0; x < words - w0; ++x) dst[x] = sp[x];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int N, int NC>
void launch_r(hipStream_t s, const gjk::RunArgs& a, int blocks) {
  constexpr int KS = NC <= 4 ? 8 : 4;
  const size_t lds = gjk::staging_bytes(KS, a.n_cols, (int)sizeof(int32_t));
  hipLaunchKernelGGL((k_expand_runs<N, NC, KS>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
}

template <int N>
void launch_rn(hipStream_t s, const gjk::RunArgs& a, int blocks) {
  if (a.n_cols <= 4)
    launch_r<N, 4>(s, a, blocks);
  else if (a.n_cols <= 8)
    launch_r<N, 8>(s, a, blocks);
  else
    launch_r<N, GJ_MAX_OUT_COLS>(s, a, blocks);
}

}  // namespace

namespace gjk {

int expand_runs(hipStream_t s, const RunArgs& a0, int rounds_per_lane) {
  RunArgs a = a0;
  if (a.n_rows <= 0) return 0;
  if (a.n_cols < 1 || a.n_cols > GJ_MAX_OUT_COLS || a.n_tables < 1 || a.n_tables > GJ_MAX_TABLES) return -1;
  const int ks = a.n_cols <= 4 ? 8 : 4;
  // rounds_per_lane 0: about 640 bytes of output per lane, at least 16 tuples
  a.tuples_per_lane =
      rounds_per_lane > 0 ? ks * rounds_per_lane : std::max(ks, std::max(16, 640 / (a.n_cols * 4)) / ks * ks);
  while (a.tuples_per_lane > ks && a.n_rows / a.tuples_per_lane < 256LL * 1024) a.tuples_per_lane /= 2;
  a.tuples_per_lane = std::max(ks, a.tuples_per_lane / ks * ks);
  const int64_t lanes = (a.n_rows + a.tuples_per_lane - 1) / a.tuples_per_lane;
  int64_t blocks = (lanes + GJ_BLOCK - 1) / GJ_BLOCK;
  blocks = (blocks + 7) / 8 * 8;
  if (blocks > 0x7fffffff) return -1;
  if (a.n_tables <= 4)
    launch_rn<4>(s, a, (int)blocks);
  else if (a.n_tables <= 8)
    launch_rn<8>(s, a, (int)blocks);
  else
    launch_rn<GJ_MAX_TABLES>(s, a, (int)blocks);
  return 0;
}

}  // namespace gjk
