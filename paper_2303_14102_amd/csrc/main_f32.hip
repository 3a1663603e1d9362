// Instantiations of the fp32-MFMA fused kernel (X stored fp32).
#include "main_kernels.h"

namespace sil {

template <int DP, int METRIC>
static void run_f32(const MainArgs& m, bool save, unsigned grid, hipStream_t st) {
  if (save)
    k_main_f32<DP, 1, METRIC, true><<<grid, 256, 0, st>>>(m);
  else
    k_main_f32<DP, 1, METRIC, false><<<grid, 256, 0, st>>>(m);
}

template <int METRIC>
static void run_f32_dp(const MainArgs& m, int DP, bool save, unsigned grid, hipStream_t st) {
  switch (DP) {
    case 16: run_f32<16, METRIC>(m, save, grid, st); break;
    case 32: run_f32<32, METRIC>(m, save, grid, st); break;
    case 64: run_f32<64, METRIC>(m, save, grid, st); break;
    case 128: run_f32<128, METRIC>(m, save, grid, st); break;
    default: run_f32<256, METRIC>(m, save, grid, st); break;
  }
}

void launch_main_f32(const MainArgs& m, int DP, int metric, bool save, unsigned grid,
                     hipStream_t st) {
  if (metric == SIL_SQEUCLID)
    run_f32_dp<SIL_SQEUCLID>(m, DP, save, grid, st);
  else
    run_f32_dp<SIL_COSINE>(m, DP, save, grid, st);
}

}  // namespace sil
