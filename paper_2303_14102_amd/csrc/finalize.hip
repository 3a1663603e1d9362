// From the per-cluster statistics to the tables the fused GEMM+epilogue kernel reads.
//
// Squared Euclidean (Eq.11).  With mu_k = Y_k / N_k and the cluster variance
// sigma_k^2 = Psi_k / N_k - ||mu_k||^2, the mean squared distance from x to cluster k is
//     m(x, k) = ||x||^2 + Psi_k/N_k - 2 x.Y_k/N_k = ||x - mu_k||^2 + sigma_k^2,
// and both sides are unchanged when x and mu_k are shifted by the same vector.  The kernels
// shift by the global mean m (centring), so that the cross term is small:
//     m(x, k) = ||x'||^2 + c_k - 2 x'.mu'_k,   x' = x - m, mu'_k = mu_k - m,
//     c_k = ||mu'_k||^2 + sigma_k^2            (uncentred: c_k = Psi_k / N_k, m = 0).
// Cosine (Eq.18), z = x/||x||, mu_k = Omega_k / N_k:
//     m(x, k) = 1 - z.mu_k = (1 - ||mu_k||^2 + ||z - mu_k||^2) / 2.
// The b-path (minimum over the other clusters) uses the GEMM form; the a-path (own cluster)
// uses the difference form, which has no cancellation.  All table entries are formed in FP64
// and rounded once.
#include "sil_internal.h"

namespace sil {

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// Global mean (centring vector), one thread per column; zeros when not centring.
__global__ __launch_bounds__(256) void k_gmean(const double* __restrict__ V,
                                               const int32_t* __restrict__ hdr, int32_t K,
                                               int32_t D, int32_t DP, int centre,
                                               double* __restrict__ gmean,
                                               float* __restrict__ mvec) {
  const int l = threadIdx.x;
  if (l >= DP) return;
  double m = 0.0;
  if (centre && l < D) {
    const double n = static_cast<double>(hdr[1]);
    for (int32_t k = 0; k < K; ++k) m += V[static_cast<int64_t>(k) * D + l];
    m = n > 0.0 ? m / n : 0.0;
  }
  gmean[l] = m;
  mvec[l] = static_cast<float>(m);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per (padded) cluster.
template <int METRIC, bool BF16TAB>
__global__ __launch_bounds__(256) void k_finalize(
    const int32_t* __restrict__ count, const double* __restrict__ V,
    const double* __restrict__ psi, const double* __restrict__ gmean, int32_t K, int32_t Kpad,
    int32_t D, int32_t DP, void* __restrict__ btab, float* __restrict__ cvec,
    float* __restrict__ atab, float* __restrict__ avec, float* __restrict__ ascale) {
  const int lane = threadIdx.x & 63;
  const int32_t k = static_cast<int32_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (k >= Kpad) return;
  const int nrep = (DP + 63) / 64;
  float* bt32 = static_cast<float*>(btab);
  uint16_t* bthi = static_cast<uint16_t*>(btab);
  uint16_t* btlo = bthi + static_cast<int64_t>(Kpad) * DP;
  const int64_t brow = static_cast<int64_t>(k) * DP;
  const int32_t n = k < K ? count[k] : 0;
  if (n == 0) {
    for (int r = 0; r < nrep; ++r) {
      const int l = lane + 64 * r;
      if (l >= DP) break;
      if (BF16TAB) {
        bthi[brow + l] = 0;
        btlo[brow + l] = 0;
      } else {
        bt32[brow + l] = 0.0f;
      }
      if (k < K) atab[brow + l] = 0.0f;
    }
    if (lane == 0) {
      cvec[k] = __builtin_inff();
      if (k < K) {
        avec[k] = 0.0f;
        ascale[k] = 0.0f;
      }
    }
    return;
  }
  const double dn = static_cast<double>(n);
  double mu2 = 0.0, muc2 = 0.0;
  for (int r = 0; r < nrep; ++r) {
    const int l = lane + 64 * r;
    if (l >= DP) break;
    const double mu = l < D ? V[static_cast<int64_t>(k) * D + l] / dn : 0.0;
    const double muc = METRIC == SIL_SQEUCLID ? mu - gmean[l] : mu;
    mu2 += mu * mu;
    muc2 += muc * muc;
    if (BF16TAB) {
      const uint16_t hi = f32_to_bf16_rne(static_cast<float>(muc));
      const uint16_t lo = f32_to_bf16_rne(static_cast<float>(muc - static_cast<double>(bf16_to_f32(hi))));
      bthi[brow + l] = hi;
      btlo[brow + l] = lo;
    } else {
      bt32[brow + l] = static_cast<float>(muc);
    }
    atab[brow + l] = static_cast<float>(muc);
  }
  mu2 = wave_sum(mu2);
  muc2 = wave_sum(muc2);
  if (lane == 0) {
    double c, av;
    if (METRIC == SIL_SQEUCLID) {
      const double mean_sq = psi[k] / dn;
      const double sigma2 = fmax(0.0, mean_sq - mu2);
      c = muc2 + sigma2;  // equals Psi_k/N_k when gmean = 0
      av = sigma2;
    } else {
      c = 1.0;
      av = fmax(0.0, 1.0 - mu2);
    }
    cvec[k] = static_cast<float>(c);
    avec[k] = static_cast<float>(av);
    ascale[k] = n >= 2 ? static_cast<float>(dn / (dn - 1.0)) : 0.0f;
  }
}

hipError_t launch_finalize(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st) {
  const int centre = p.metric == SIL_SQEUCLID && !(p.flags & SIL_FLAG_NO_CENTRE);
  k_gmean<<<1, 256, 0, st>>>(w.V, w.hdr, p.K, p.D, p.DP, centre, w.gmean, w.mvec);
  const unsigned nb = static_cast<unsigned>(ceil_div(p.Kpad, 4));
  const bool bf = p.dtype != SIL_F32;
#define SIL_FIN(MT, BF)                                                                        \
  k_finalize<MT, BF><<<nb, 256, 0, st>>>(w.count, w.V, w.psi, w.gmean, p.K, p.Kpad, p.D, p.DP, \
                                         w.btab, w.cvec, w.atab, w.avec, w.ascale)
  if (p.metric == SIL_SQEUCLID) {
    if (bf) SIL_FIN(SIL_SQEUCLID, true);
    else SIL_FIN(SIL_SQEUCLID, false);
  } else {
    if (bf) SIL_FIN(SIL_COSINE, true);
    else SIL_FIN(SIL_COSINE, false);
  }
#undef SIL_FIN
  (void)L;
  return hipGetLastError();
}

}  // namespace sil
