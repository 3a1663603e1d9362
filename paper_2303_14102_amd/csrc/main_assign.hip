// Instantiations of the bf16-MFMA fused kernel for the K-means assignment (X stored bf16 or fp8,
// squared Euclidean): the kernels that track the argmin, run with MainArgs::assign set, so that
// the minimum covers every cluster and the finish writes the nearest mean's id.  Three products,
// or two on the exact x with folded centring (bf16 storage); one row block per wave and
// 64-cluster tiles: the argmin needs the registers.
#include "main_kernels.h"

namespace sil {

template <int DPX, int DT, int P>
static void run_assign(const MainArgs& m, unsigned grid, hipStream_t st) {
  k_main_bf16<DPX, 1, P, DT, SIL_SQEUCLID, true><<<grid, 256, 0, st>>>(m);
}

template <int DT, int P>
static void run_assign_dt(const MainArgs& m, int DPX, unsigned grid, hipStream_t st) {
  with_depth(DepthsBf16{}, DPX, [&](auto dp) { run_assign<decltype(dp)::value, DT, P>(m, grid, st); });
}

void launch_main_assign(const MainArgs& m, int DPX, int dtype, int products, unsigned grid,
                        hipStream_t st) {
  if (dtype == SIL_BF16 && products == 2)
    run_assign_dt<SIL_BF16, 2>(m, DPX, grid, st);
  else if (dtype == SIL_BF16)
    run_assign_dt<SIL_BF16, 3>(m, DPX, grid, st);
  else
    run_assign_dt<SIL_FP8_E4M3, 3>(m, DPX, grid, st);
}

}  // namespace sil
