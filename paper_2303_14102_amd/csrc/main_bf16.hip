// Instantiations of the bf16-MFMA fused kernel for X stored bf16.
#include "main_kernels.h"

namespace sil {

template <int DPX, int METRIC>
static void run_dp(const MainArgs& m, int products, unsigned grid, hipStream_t st) {
  if (products == 1)
    k_main_bf16<DPX, bf16_nb(DPX, 1), 1, SIL_BF16, METRIC, false><<<grid, 256, 0, st>>>(m);
  else if (products == 2)
    k_main_bf16<DPX, bf16_nb(DPX, 2), 2, SIL_BF16, METRIC, false><<<grid, 256, 0, st>>>(m);
  else
    k_main_bf16<DPX, bf16_nb(DPX, 3), 3, SIL_BF16, METRIC, false><<<grid, 256, 0, st>>>(m);
}

template <int METRIC>
static void run_metric(const MainArgs& m, int DPX, int products, unsigned grid, hipStream_t st) {
  switch (DPX) {
    case 16: run_dp<16, METRIC>(m, products, grid, st); break;
    case 32: run_dp<32, METRIC>(m, products, grid, st); break;
    case 48: run_dp<48, METRIC>(m, products, grid, st); break;
    case 80: run_dp<80, METRIC>(m, products, grid, st); break;
    case 144: run_dp<144, METRIC>(m, products, grid, st); break;
    default: run_dp<272, METRIC>(m, products, grid, st); break;
  }
}

void launch_main_bf16(const MainArgs& m, int DPX, int metric, int products, unsigned grid,
                      hipStream_t st) {
  if (metric == SIL_SQEUCLID)
    run_metric<SIL_SQEUCLID>(m, DPX, products, grid, st);
  else
    run_metric<SIL_COSINE>(m, DPX, products, grid, st);
}

}  // namespace sil
