// Stage 3 with value columns (payload gather): launchers of the expansion
// kernel (desum_kernel.h) for int32 value output.  A lane stages a round of KS
// tuples of n_cols values; KS is picked so that a round is at least 128 bytes
// where the register budget allows (the change mask holds KS * N bits).
#include "desum_kernel.h"

namespace {

template <int N, int NC>
constexpr int val_ks() {
  return (NC <= 4 && N <= 8) ? 8 : 4;
}

template <int N, int NC>
void launch_val(hipStream_t s, const gjk::DesumArgs& a, int blocks) {
  constexpr int KS = val_ks<N, NC>();
  static_assert(KS * N <= 64, "change mask");
  const size_t lds = gjk::staging_bytes(KS, a.n_cols, (int)sizeof(int32_t));
  hipLaunchKernelGGL((k_desum<N, NC, int32_t, KS>), dim3(blocks), dim3(GJ_BLOCK), lds, s, a);
}

template <int N>
void launch_val_n(hipStream_t s, const gjk::DesumArgs& a, int blocks) {
  if (a.n_cols <= 4)
    launch_val<N, 4>(s, a, blocks);
  else if (a.n_cols <= 8)
    launch_val<N, 8>(s, a, blocks);
  else
    launch_val<N, GJ_MAX_OUT_COLS>(s, a, blocks);
}

template <int N>
int val_ks_n(int n_cols) {
  return n_cols <= 4 ? val_ks<N, 4>() : n_cols <= 8 ? val_ks<N, 8>() : val_ks<N, GJ_MAX_OUT_COLS>();
}

}  // namespace

namespace gjk {

int value_round(int n_tables, int n_cols) {
  return n_tables <= 4 ? val_ks_n<4>(n_cols) : n_tables <= 8 ? val_ks_n<8>(n_cols) : val_ks_n<GJ_MAX_TABLES>(n_cols);
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
