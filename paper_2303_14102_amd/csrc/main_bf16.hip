// Instantiations of the bf16-MFMA fused kernel for X stored bf16.
#include "main_kernels.h"

namespace sil {

// Split products (2 or 3) with one row block per wave at depths up to 128 run with 32-cluster
// tiles and three workgroups per CU, the other forms with 64-cluster tiles and two.  Measured on
// the 128-dimension workload with one row block: 32-cluster tiles -9% (2 products), -2% (3),
// +5% (1); two products with two row blocks (64-cluster tiles): a further -8%.
template <int DPX, int P, int METRIC>
static void run_p(const MainArgs& m, unsigned grid, hipStream_t st) {
  constexpr int NB = bf16_nb(DPX, P, SIL_BF16);
  if constexpr (P >= 2 && DPX <= 128 && NB == 1) {
    MainArgs m2 = m;
    m2.ntiles = m.ntiles * (kColTile / 32);
    k_main_bf16<DPX, NB, P, SIL_BF16, METRIC, false, 32><<<grid, 256, 0, st>>>(m2);
  } else {
    k_main_bf16<DPX, NB, P, SIL_BF16, METRIC, false><<<grid, 256, 0, st>>>(m);
  }
}

template <int DPX, int METRIC>
static void run_dp(const MainArgs& m, int products, unsigned grid, hipStream_t st) {
  if (products == 1)
    run_p<DPX, 1, METRIC>(m, grid, st);
  else if (products == 2)
    run_p<DPX, 2, METRIC>(m, grid, st);
  else
    run_p<DPX, 3, METRIC>(m, grid, st);
}

template <int METRIC>
static void run_metric(const MainArgs& m, int DPX, int products, unsigned grid, hipStream_t st) {
  with_depth(DepthsBf16{}, DPX, [&](auto dp) { run_dp<decltype(dp)::value, METRIC>(m, products, grid, st); });
}

void launch_main_bf16(const MainArgs& m, int DPX, int metric, int products, unsigned grid,
                      hipStream_t st) {
  if (metric == SIL_SQEUCLID)
    run_metric<SIL_SQEUCLID>(m, DPX, products, grid, st);
  else if (metric == SIL_COSINE)
    run_metric<SIL_COSINE>(m, DPX, products, grid, st);
  else
    run_metric<SIL_KL>(m, DPX, products, grid, st);
}

}  // namespace sil
