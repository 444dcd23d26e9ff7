// Stage 3 with value columns (payload gather): launchers of the expansion
// kernel (desum_kernel.h) for int32 value output.  A lane stages a round of KS
// tuples of n_cols values.
#include "desum_kernel.h"

namespace {

// Tuples per lane and round: the fewest of 2, 4, 8 that make a round of
// whole 16-byte units and at least 64 bytes (measured: shorter rounds keep
// fewer values in registers and more waves per SIMD, down to about one cache
// line per lane), within the change mask's KS * N <= 64 bits.
template <int N>
int val_ks(int n_cols) {
  int ks = 2;
  while (ks < 8 && ((ks * n_cols * 4) % 16 != 0 || ks * n_cols * 4 < 64)) ks *= 2;
  return ks * N > 64 ? 64 / N : ks;
}

template <int N, int NC, int KS>
void launch_val(hipStream_t s, const gjk::DesumArgs& a, int blocks) {
  if constexpr (KS * N <= 64) {
    const size_t lds = gjk::staging_bytes(KS, a.n_cols, (int)sizeof(int32_t));
    hipLaunchKernelGGL((k_desum<N, NC, int32_t, KS>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
  }
}

template <int N, int NC>
void launch_val_ks(hipStream_t s, const gjk::DesumArgs& a, int blocks) {
  const int ks = val_ks<N>(a.n_cols);
  if (ks == 2)
    launch_val<N, NC, 2>(s, a, blocks);
  else if (ks == 4)
    launch_val<N, NC, 4>(s, a, blocks);
  else
    launch_val<N, NC, 8>(s, a, blocks);
}

template <int N>
void launch_val_n(hipStream_t s, const gjk::DesumArgs& a, int blocks) {
  if (a.n_cols <= 4)
    launch_val_ks<N, 4>(s, a, blocks);
  else if (a.n_cols <= 8)
    launch_val_ks<N, 8>(s, a, blocks);
  else
    launch_val_ks<N, GJ_MAX_OUT_COLS>(s, a, blocks);
}

}  // namespace

namespace gjk {

int value_round(int n_tables, int n_cols) {
  return n_tables <= 4 ? val_ks<4>(n_cols) : n_tables <= 8 ? val_ks<8>(n_cols) : val_ks<GJ_MAX_TABLES>(n_cols);
}

void launch_values(hipStream_t s, const DesumArgs& a, int blocks) {
  if (a.n_tables <= 4)
    launch_val_n<4>(s, a, blocks);
  else if (a.n_tables <= 8)
    launch_val_n<8>(s, a, blocks);
  else
    launch_val_n<GJ_MAX_TABLES>(s, a, blocks);
}

}  // namespace gjk
