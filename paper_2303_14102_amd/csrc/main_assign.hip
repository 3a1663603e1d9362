// Instantiations of the bf16-MFMA fused kernel for the K-means assignment (X stored bf16 or fp8,
// three products, squared Euclidean): the kernels that track the argmin, run with
// MainArgs::assign set, so that the minimum covers every cluster and the finish writes the
// nearest mean's id.  64-cluster tiles: the argmin needs the registers of the larger tile form.
#include "main_kernels.h"

namespace sil {

template <int DPX, int DT>
static void run_assign(const MainArgs& m, unsigned grid, hipStream_t st) {
  k_main_bf16<DPX, bf16_nb(DPX, 3, DT), 3, DT, SIL_SQEUCLID, true><<<grid, 256, 0, st>>>(m);
}

template <int DT>
static void run_assign_dt(const MainArgs& m, int DPX, unsigned grid, hipStream_t st) {
  switch (DPX) {
    case 16: run_assign<16, DT>(m, grid, st); break;
    case 32: run_assign<32, DT>(m, grid, st); break;
    case 48: run_assign<48, DT>(m, grid, st); break;
    case 80: run_assign<80, DT>(m, grid, st); break;
    case 128: run_assign<128, DT>(m, grid, st); break;
    default: run_assign<256, DT>(m, grid, st); break;
  }
}

void launch_main_assign(const MainArgs& m, int DPX, int dtype, unsigned grid, hipStream_t st) {
  if (dtype == SIL_BF16)
    run_assign_dt<SIL_BF16>(m, DPX, grid, st);
  else
    run_assign_dt<SIL_FP8_E4M3>(m, DPX, grid, st);
}

}  // namespace sil
