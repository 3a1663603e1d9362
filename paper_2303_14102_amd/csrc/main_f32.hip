// Instantiations of the fp32-MFMA fused kernel (X stored fp32).
#include "main_kernels.h"

namespace sil {

template <int DPX, int METRIC>
static void run_f32(const MainArgs& m, bool save, unsigned grid, hipStream_t st) {
  if (save)
    k_main_f32<DPX, 1, METRIC, true><<<grid, 256, 0, st>>>(m);
  else
    k_main_f32<DPX, 1, METRIC, false><<<grid, 256, 0, st>>>(m);
}

template <int METRIC>
static void run_f32_dp(const MainArgs& m, int DPX, bool save, unsigned grid, hipStream_t st) {
  with_depth(DepthsF32{}, DPX, [&](auto dp) { run_f32<decltype(dp)::value, METRIC>(m, save, grid, st); });
}

template <int DPX>
static void run_f32_kl(const MainArgs& m, unsigned grid, hipStream_t st) {
  k_main_f32<DPX, 1, SIL_KL, false><<<grid, 256, 0, st>>>(m);
}

void launch_main_f32(const MainArgs& m, int DPX, int metric, bool save, unsigned grid,
                     hipStream_t st) {
  if (metric == SIL_SQEUCLID) {
    run_f32_dp<SIL_SQEUCLID>(m, DPX, save, grid, st);
  } else if (metric == SIL_COSINE) {
    run_f32_dp<SIL_COSINE>(m, DPX, save, grid, st);
  } else {  // the KL divergence has no backward, so no kernels that keep a_i, b_i
    with_depth(DepthsF32{}, DPX, [&](auto dp) { run_f32_kl<decltype(dp)::value>(m, grid, st); });
  }
}

}  // namespace sil
