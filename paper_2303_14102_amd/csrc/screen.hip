// Host side and small kernels of the one-product screen (squared Euclidean distance, Eq.11):
// the fp16 screen table with its error bounds, the list of rows the screen leaves to the
// two-product kernel, and the sum of their s_i.
//
// The screen value of row x and cluster k is
//     v~_k = fl32(c_k) + x16 . T16_k          (fp16 products accumulated in fp32 onto the fp32
//                                              constant, all scaled by the table's power of two
//                                              2^-f, which scales fl32(c_k) exactly)
// against the exact v_k = x . T_k + c_k, with T_k = -2 mu'_k and c_k the binary64 table values
// of the two-product form.  x is exact in fp16 (rows where it is not go to the fallback), so
//     |v~_k - v_k| <= ||x|| L1 + EC + (DPX + 16) 2^-24 (||x|| L2 + L3)
// with L1 = max_k ||T16_k - T_k||, L2 = max_k ||T16_k||, L3 = max_k |fl32(c_k)|,
// EC = max_k |fl32(c_k) - c_k| (all unscaled): Cauchy-Schwarz for the table's rounding, and the
// bound of a sum of DPX exact products and the constant accumulated in fp32 in any order (taken
// with DPX + 16 terms and twice the unit roundoff, so that it holds whatever rounding the
// accumulation uses).
#include "sil_internal.h"

namespace sil {

namespace {

__device__ __forceinline__ double wave_sum64(double v) {
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ void raise_slot(int32_t* hdr, int slot, double v) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(hdr + kHdrScreenWord) + slot;
  atomicMax(p, static_cast<unsigned long long>(__double_as_longlong(v)));
}
__device__ __forceinline__ double read_slot(const int32_t* hdr, int slot) {
  const unsigned long long* p =
      reinterpret_cast<const unsigned long long*>(hdr + kHdrScreenWord) + slot;
  return __longlong_as_double(static_cast<long long>(*p));
}

// Four clusters per wave, sixteen per workgroup.  Table row k (scaled by 2^-f, rounded to nearest
// fp16): [T_k (D entries), 0 ... (to DPX + 8)]; the constant is the fp32 c_k of the two-product
// tables (ctab), which the screen kernel scales and starts each accumulation from.
// The maxima over the workgroup's clusters raise the header slots (one atomic each); workgroup 0
// also stores the norm of the centring vector.  Empty and padding clusters get a zero row (the
// screen kernel excludes their columns).
constexpr int kTableClustersPerWave = 4;
__global__ __launch_bounds__(256) void k_screen_table(
    const int32_t* __restrict__ count, const double* __restrict__ V,
    const double* __restrict__ gmean, const float* __restrict__ mvec,
    const float* __restrict__ tscale, const double* __restrict__ c64, int32_t K, int32_t Kpad,
    int32_t D, int32_t DPX, _Float16* __restrict__ stab, float* __restrict__ rtab,
    int32_t* __restrict__ hdr) {
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int f = screen_exponent(fmax(read_slot(hdr, SC_TMAX), read_slot(hdr, SC_CMAX)));
  const double sc = ldexp(1.0, -f), usc = ldexp(1.0, f);
  const int RSS = screen_stride(DPX);
  double l1 = 0.0, l2 = 0.0, l3 = 0.0, ec = 0.0;
  for (int i = 0; i < kTableClustersPerWave; ++i) {
    const int32_t k = (static_cast<int32_t>(blockIdx.x) * 4 + wave) * kTableClustersPerWave + i;
    if (k >= Kpad) break;
    _Float16* row = stab + static_cast<int64_t>(k) * RSS;
    const int32_t n = k < K ? count[k] : 0;
    const double dn = static_cast<double>(n);
    double err2 = 0.0, nrm2 = 0.0;
    for (int l = lane; l < RSS; l += 64) {
      double g = 0.0;
      if (n > 0 && l < D) {  // the same binary64 operations as the two-product table
        const double mu = V[static_cast<int64_t>(k) * D + l] / dn;
        g = -2.0 * (mu - gmean[l]);
        if (tscale) g *= static_cast<double>(tscale[l]);  // fp8: the codes enter the GEMM
      }
      const _Float16 t = static_cast<_Float16>(static_cast<float>(g * sc));
      row[l] = t;
      // fp8: s_l mu'_kl in fp32 for the exact score of the codes (-g / 2, exact scaling)
      if (rtab && k < K && l < DPX) rtab[static_cast<int64_t>(k) * DPX + l] = static_cast<float>(-0.5 * g);
      const double back = static_cast<double>(t) * usc;
      err2 += (back - g) * (back - g);
      nrm2 += back * back;
    }
    err2 = wave_sum64(err2);
    nrm2 = wave_sum64(nrm2);
    if (lane == 0 && n > 0) {
      // the constant as the kernel takes it: the fp32 table value (its scaling by 2^-f is exact)
      const double c32 = static_cast<double>(static_cast<float>(c64[k]));
      // binary64 rounding of these few operations is far below the margins the kernel adds
      l1 = fmax(l1, sqrt(err2));
      l2 = fmax(l2, sqrt(nrm2));
      l3 = fmax(l3, fabs(c32));
      ec = fmax(ec, fabs(c32 - c64[k]));
    }
  }
  if (lane == 0) {
    red[wave][0] = l1;
    red[wave][1] = l2;
    red[wave][2] = l3;
    red[wave][3] = ec;
  }
  if (blockIdx.x == 0 && wave == 0) {
    double m2 = 0.0;
    for (int l = lane; l < D; l += 64) m2 += static_cast<double>(mvec[l]) * static_cast<double>(mvec[l]);
    m2 = wave_sum64(m2);
    if (lane == 0) raise_slot(hdr, SC_MNORM, sqrt(m2));
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int w = 0; w < 4; ++w) v = fmax(v, red[w][threadIdx.x]);
    raise_slot(hdr, SC_L1 + static_cast<int>(threadIdx.x), v);
  }
}

// Sum of the fallback workgroups' partial sums, in list order (one workgroup, fixed tree).
__global__ __launch_bounds__(1024) void k_fb_sum(const double* __restrict__ part, int rows_per_wg,
                                                 int32_t* __restrict__ hdr) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  const int64_t total = hdr[kHdrFallbackWord];
  const int64_t nwg = (total + rows_per_wg - 1) / rows_per_wg * kMainWaves;  // per wave
  double v = 0.0;
  for (int64_t i = t; i < nwg; i += 1024) v += part[i];
  sh[t] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) *reinterpret_cast<double*>(hdr + kHdrFallbackSumWord) = sh[0];
}

}  // namespace

bool screen_applies(int metric, int dtype, int DPX, int products, int flags) {
  return metric == SIL_SQEUCLID && (dtype == SIL_BF16 || dtype == SIL_FP8_E4M3) && products == 2 &&
         DPX <= kScreenMaxDPX &&
         !(flags & (SIL_FLAG_NO_SCREEN | SIL_FLAG_SAVE_FOR_GRAD));
}

hipError_t launch_screen_table(const Problem& p, const WsLayout& L, const WsPtrs& w,
                               hipStream_t st) {
  (void)L;
  const unsigned nb = static_cast<unsigned>(ceil_div(p.Kpad, 4 * kTableClustersPerWave));
  const float* tscale = p.dtype == SIL_FP8_E4M3 ? p.col_scale : nullptr;
  k_screen_table<<<nb, 256, 0, st>>>(w.count, w.V, w.gmean, w.mvec, tscale, w.c64, p.K, p.Kpad,
                                     p.D, p.DPX, static_cast<_Float16*>(w.stab),
                                     tscale ? w.rtab : nullptr, w.hdr);
  return hipGetLastError();
}

// the sum of the fallback rows' s_i (their kernels are in main_screen.hip)
hipError_t launch_fb_sum(const WsPtrs& w, int rows_per_wg, hipStream_t st) {
  k_fb_sum<<<1, 1024, 0, st>>>(w.fbpart, rows_per_wg, w.hdr);
  return hipGetLastError();
}

}  // namespace sil
