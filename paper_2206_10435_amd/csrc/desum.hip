// Stage 3 -- desummarization (Sec. 3.6): launchers of the expansion kernel
// for row-id output (the kernel itself is in desum_kernel.h).
#include "desum_kernel.h"

namespace {
template <int N, typename WT>
void launch_nw(hipStream_t s, const gjk::DesumArgs& a, int ks, int blocks) {
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

DesumPlan desum_plan(int n_tables, int rowid_bytes, int n_cols, int64_t n_rows, int rounds_per_lane, int stage) {
  DesumPlan p{};
  const bool values = n_cols > 0;
  if (n_tables < 1 || n_tables > GJ_MAX_TABLES || n_rows < 0 || (values && (n_cols > GJ_MAX_OUT_COLS || rowid_bytes != 4)) ||
      (!values && rowid_bytes != 4 && rowid_bytes != 8))
    return p;  // ok = 0
  // the kernel instance: exact table count up to 8, else compiled for 16;
  // value launches for at most 4, 8 or 16 tables
  p.kernel_tables = values ? (n_tables <= 4 ? 4 : n_tables <= 8 ? 8 : GJ_MAX_TABLES)
                           : (n_tables <= 8 ? n_tables : GJ_MAX_TABLES);
  int ks = values ? value_round(n_tables, n_cols) : (stage == 2 || stage == 4 || stage == 8) ? stage : 4;
  // a lane's staged round must be whole 16-byte units (int32 ids, odd n)
  while (!values && (ks * n_tables * rowid_bytes) % 16 != 0) ks *= 2;
  const int rs = ks;
  // the change mask holds KS * N bits
  if (!values && ks == 8 && p.kernel_tables * 8 > 64) ks = 4;
  p.stage = ks;
  const int nc = values ? n_cols : n_tables;
  const int wb = values ? 4 : rowid_bytes;
  // rounds_per_lane 0: about 768 bytes of row ids per lane (measured best for
  // 4 tables with long runs, 24-32 tuples of 32 B, and for 6 tables with runs
  // of about 9 tuples, 12-16 tuples of 48 B), about 640 bytes of values, and at
  // least 16 tuples
  const int tup_bytes = nc * wb;
  const int lane_bytes = values ? 640 : 768;
  int L = rounds_per_lane > 0 ? rs * rounds_per_lane : std::max(rs, std::max(16, lane_bytes / tup_bytes) / rs * rs);
  // a smaller per-lane range when the range would not fill the chip
  while (L > rs && n_rows / L < 256LL * 1024) L /= 2;
  L = std::max(rs, L / rs * rs);
  p.tuples_per_lane = L;
  const int64_t lanes = (n_rows + L - 1) / L;
  int64_t blocks = (lanes + GJ_BLOCK - 1) / GJ_BLOCK;
  blocks = (blocks + 7) / 8 * 8;  // whole XCD rounds for the block remap
  p.blocks = blocks;
  p.lds_bytes = values ? (int64_t)staging_bytes(ks, n_cols, 4) : (int64_t)staging_bytes(ks, p.kernel_tables, wb, true);
  p.lds_used = (int64_t)staging_bytes(ks, nc, wb, !values);
  p.seg_bytes = ks * nc * wb;
  p.ok = blocks <= 0x7fffffff && p.seg_bytes % 16 == 0 && ks * p.kernel_tables <= 64 && L % ks == 0;
  return p;
}

int desummarize(hipStream_t s, const DesumArgs& a0, int rowid_bytes, int n_tables, int rounds_per_lane, int stage) {
  if (a0.n_rows <= 0) return 0;
  const DesumPlan p = desum_plan(n_tables, rowid_bytes, a0.n_cols, a0.n_rows, rounds_per_lane, stage);
  if (!p.ok) return -1;
  DesumArgs a = a0;
  a.n_tables = n_tables;
  a.k_round = p.stage;
  a.tuples_per_lane = p.tuples_per_lane;
  const int blocks = (int)p.blocks;
  if (a0.n_cols > 0) {
    launch_values(s, a, blocks);
    return 0;
  }
  const int ks = p.stage;
  switch (n_tables) {
    case 1: launch_n<1>(s, a, rowid_bytes, ks, blocks); break;
    case 2: launch_n<2>(s, a, rowid_bytes, ks, blocks); break;
    case 3: launch_n<3>(s, a, rowid_bytes, ks, blocks); break;
    case 4: launch_n<4>(s, a, rowid_bytes, ks, blocks); break;
    case 5: launch_n<5>(s, a, rowid_bytes, ks, blocks); break;
    case 6: launch_n<6>(s, a, rowid_bytes, ks, blocks); break;
    case 7: launch_n<7>(s, a, rowid_bytes, ks, blocks); break;
    case 8: launch_n<8>(s, a, rowid_bytes, ks, blocks); break;
    default: launch_n<GJ_MAX_TABLES>(s, a, rowid_bytes, ks, blocks); break;
  }
  return 0;
}

}  // namespace gjk

extern "C" gj_status gj_desum_launch_config(int32_t n_tables, int32_t rowid_bytes, int32_t n_cols, int64_t n_rows,
                                            const gj_tune* tune, gj_desum_launch* out) {
  if (!out) return GJ_E_INVALID;
  const int rounds = tune ? tune->desum_rounds : 0;
  const int stage = tune ? tune->desum_stage : 4;
  const gjk::DesumPlan p = gjk::desum_plan(n_tables, rowid_bytes, n_cols, n_rows, rounds, stage);
  if (!p.ok) return GJ_E_INVALID;
  out->stage = p.stage;
  out->tuples_per_lane = p.tuples_per_lane;
  out->kernel_tables = p.kernel_tables;
  out->change_bits = p.stage * p.kernel_tables;
  out->blocks = p.blocks;
  out->lds_bytes = p.lds_bytes;
  out->lds_used = p.lds_used;
  out->seg_bytes = p.seg_bytes;
  return GJ_OK;
}
