// Instantiations of the bf16-MFMA fused kernel for X stored fp8 e4m3 with a per-column scale.
#include "main_kernels.h"

namespace sil {

template <int DP, int METRIC>
static void run_dp(const MainArgs& m, int products, unsigned grid, hipStream_t st) {
  if (products == 1)
    k_main_bf16<DP, bf16_nb(DP, 1), 1, SIL_FP8_E4M3, METRIC, false><<<grid, 256, 0, st>>>(m);
  else if (products == 2)
    k_main_bf16<DP, bf16_nb(DP, 2), 2, SIL_FP8_E4M3, METRIC, false><<<grid, 256, 0, st>>>(m);
  else
    k_main_bf16<DP, bf16_nb(DP, 3), 3, SIL_FP8_E4M3, METRIC, false><<<grid, 256, 0, st>>>(m);
}

template <int METRIC>
static void run_metric(const MainArgs& m, int DP, int products, unsigned grid, hipStream_t st) {
  switch (DP) {
    case 16: run_dp<16, METRIC>(m, products, grid, st); break;
    case 32: run_dp<32, METRIC>(m, products, grid, st); break;
    case 64: run_dp<64, METRIC>(m, products, grid, st); break;
    case 128: run_dp<128, METRIC>(m, products, grid, st); break;
    default: run_dp<256, METRIC>(m, products, grid, st); break;
  }
}

void launch_main_fp8(const MainArgs& m, int DP, int metric, int products, unsigned grid,
                      hipStream_t st) {
  if (metric == SIL_SQEUCLID)
    run_metric<SIL_SQEUCLID>(m, DP, products, grid, st);
  else
    run_metric<SIL_COSINE>(m, DP, products, grid, st);
}

}  // namespace sil
