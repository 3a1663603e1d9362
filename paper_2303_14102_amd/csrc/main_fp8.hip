// Instantiations of the bf16-MFMA fused kernel for X stored fp8 e4m3 with a per-column scale.
#include "main_kernels.h"

namespace sil {

// 64-cluster tiles (the 32-cluster form of the bf16 launcher spills here: the fp8 decode holds
// more registers).
template <int DPX, int P, int METRIC>
static void run_p(const MainArgs& m, unsigned grid, hipStream_t st) {
  k_main_bf16<DPX, bf16_nb(DPX, P, SIL_FP8_E4M3), P, SIL_FP8_E4M3, METRIC, false><<<grid, 256, 0, st>>>(m);
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

void launch_main_fp8(const MainArgs& m, int DPX, int metric, int products, unsigned grid,
                      hipStream_t st) {
  if (metric == SIL_SQEUCLID)
    run_metric<SIL_SQEUCLID>(m, DPX, products, grid, st);
  else
    run_metric<SIL_COSINE>(m, DPX, products, grid, st);
}

}  // namespace sil
