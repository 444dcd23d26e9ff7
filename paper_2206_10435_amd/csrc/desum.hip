// Stage 3 -- desummarization (Sec. 3.6): launchers of the expansion kernel
// for row-id output (the kernel itself is in desum_kernel.h).
#include "desum_kernel.h"

namespace {
template <int N, typename WT>
void launch_nw(hipStream_t s, const gjk::DesumArgs& a, int ks, int blocks) {
  if (ks == 8 && N * 8 > 64) ks = 4;  // the change mask holds KS * N bits
  const size_t lds = gjk::staging_bytes(ks, N, (int)sizeof(WT), true);
  if (ks == 2) {
    hipLaunchKernelGGL((k_desum<N, 0, WT, 2>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  } else if (ks == 8) {
    if constexpr (N * 8 <= 64) hipLaunchKernelGGL((k_desum<N, 0, WT, 8>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  } else {
    hipLaunchKernelGGL((k_desum<N, 0, WT, 4>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  }
}

template <int N>
void launch_n(hipStream_t s, const gjk::DesumArgs& a, int rowid_bytes, int ks, int blocks) {
  if (rowid_bytes == 4)
    launch_nw<N, int32_t>(s, a, ks, blocks);
  else
    launch_nw<N, int64_t>(s, a, ks, blocks);
}

__global__ void k_gather_rows(const int32_t* __restrict__ perm, const int32_t* __restrict__ data, int64_t n,
                              int32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = data[perm[i]];
}

}  // namespace

namespace gjk {

void gather_rows(hipStream_t s, const int32_t* perm, const int32_t* data, int64_t n, int32_t* out) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 8192);
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks), dim3(GJ_BLOCK), 0, s, perm, data, n, out);
}

int desummarize(hipStream_t s, const DesumArgs& a0, int rowid_bytes, int n_tables, int rounds_per_lane, int stage) {
  DesumArgs a = a0;
  const bool values = a0.n_cols > 0;
  if (values && (a0.n_cols > GJ_MAX_OUT_COLS || rowid_bytes != 4)) return -1;
  int ks = values ? value_round(n_tables, a0.n_cols) : (stage == 2 || stage == 4 || stage == 8) ? stage : 4;
  // a lane's staged round must be whole 16-byte units (int32 ids, odd n)
  while (!values && (ks * n_tables * rowid_bytes) % 16 != 0) ks *= 2;
  const int rs = ks;
  if (a0.n_rows <= 0) return 0;
  if (n_tables > GJ_MAX_TABLES) return -1;
  a.n_tables = n_tables;
  a.k_round = ks;
  // rounds_per_lane 0: about 640 bytes of output per lane, at least 16 tuples
  // (measured best for tuples of 12 to 64 bytes, row ids or values)
  const int tup_bytes = values ? a0.n_cols * 4 : n_tables * rowid_bytes;
  a.tuples_per_lane = rounds_per_lane > 0 ? rs * rounds_per_lane
                                          : std::max(rs, std::max(16, 640 / tup_bytes) / rs * rs);
  // a smaller per-lane range when the chunk would not fill the chip
  while (a.tuples_per_lane > rs && a.n_rows / a.tuples_per_lane < 256LL * 1024) a.tuples_per_lane /= 2;
  a.tuples_per_lane = std::max(rs, a.tuples_per_lane / rs * rs);
  const int64_t lanes = (a.n_rows + a.tuples_per_lane - 1) / a.tuples_per_lane;
  int64_t blocks = (lanes + GJ_BLOCK - 1) / GJ_BLOCK;
  blocks = (blocks + 7) / 8 * 8;  // whole XCD rounds for the block remap
  if (blocks > 0x7fffffff) return -1;
  if (values) {
    launch_values(s, a, (int)blocks);
    return 0;
  }
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
