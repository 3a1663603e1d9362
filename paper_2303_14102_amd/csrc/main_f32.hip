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
  switch (DPX) {
    case 16: run_f32<16, METRIC>(m, save, grid, st); break;
    case 24: run_f32<24, METRIC>(m, save, grid, st); break;
    case 40: run_f32<40, METRIC>(m, save, grid, st); break;
    case 72: run_f32<72, METRIC>(m, save, grid, st); break;
    case 128: run_f32<128, METRIC>(m, save, grid, st); break;
    default: run_f32<256, METRIC>(m, save, grid, st); break;
  }
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
    switch (DPX) {
      case 16: run_f32_kl<16>(m, grid, st); break;
      case 24: run_f32_kl<24>(m, grid, st); break;
      case 40: run_f32_kl<40>(m, grid, st); break;
      case 72: run_f32_kl<72>(m, grid, st); break;
      case 128: run_f32_kl<128>(m, grid, st); break;
      default: run_f32_kl<256>(m, grid, st); break;
    }
  }
}

}  // namespace sil
