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
// The b-path (minimum over the other clusters) uses the GEMM form, with c_k held in its own fp32
// table and added to the cross term in the fused kernel's epilogue; the a-path (own cluster)
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

// Global mean (centring vector): one workgroup per column reduces the cluster sums in a fixed
// order; zeros when not centring.
__device__ __forceinline__ void gmean_body(const double* __restrict__ V,
                                           const int32_t* __restrict__ hdr, int32_t K, int32_t D,
                                           int centre, double* __restrict__ gmean,
                                           float* __restrict__ mvec, int l) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  double m = 0.0;
  if (centre && l < D)
    for (int32_t k = t; k < K; k += 256) m += V[static_cast<int64_t>(k) * D + l];
  sh[t] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double n = static_cast<double>(hdr[1]);
    const double mean = (centre && l < D && n > 0.0) ? sh[0] / n : 0.0;
    gmean[l] = mean;
    mvec[l] = static_cast<float>(mean);
  }
}

__global__ __launch_bounds__(256) void k_gmean(const double* __restrict__ V,
                                               const int32_t* __restrict__ hdr, int32_t K,
                                               int32_t D, int centre, double* __restrict__ gmean,
                                               float* __restrict__ mvec) {
  gmean_body(V, hdr, K, D, centre, gmean, mvec, blockIdx.x);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per (padded) cluster.  GEMM table row k (DPX entries):
//   fp32:  [alpha mu'_k (D), 0 ...]
//   bf16:  hi = [bf16(alpha mu'_k) (D), 0 ...], lo = [bf16(alpha mu'_k - hi) (D), 0 ...]
// alpha = -2 (squared Euclidean) or -1 (cosine, KL) is a power of two, so alpha mu' splits exactly
// like mu'.  The constant c_k goes to ctab (fp32), which the fused kernels add to the cross term
// before the minimum; with fold set (the folded centring of the two-product kernels) it also
// carries 2 m.mu'_k, m being the fp32 centring vector mvec.  With tscale set (fp8 codes in the
// GEMM) entry l of the table row is multiplied by the column scale tscale[l].  Empty and padding clusters get
// c_k = kEmptyC (large and finite) and a zero mean.
constexpr double kEmptyC = 1.0e30;

template <int METRIC, bool BF16TAB>
__device__ __forceinline__ void finalize_body(
    const int32_t* __restrict__ count, const double* __restrict__ V,
    const double* __restrict__ psi, const double* __restrict__ gmean, int32_t K, int32_t Kpad,
    int32_t D, int32_t DPX, int32_t RS, void* __restrict__ btab, float* __restrict__ ctab,
    float* __restrict__ atab, float* __restrict__ avec, float* __restrict__ ascale, int with_var,
    const float* __restrict__ mvec, int fold, const float* __restrict__ tscale,
    double* __restrict__ c64, double* __restrict__ smax, int64_t bid) {
  constexpr double ALPHA = METRIC == SIL_SQEUCLID ? -2.0 : -1.0;
  const int lane = threadIdx.x & 63;
  const int32_t k = static_cast<int32_t>(bid) * 4 + (threadIdx.x >> 6);
  if (k >= Kpad) return;
  const int nrep = (RS + 63) / 64;
  float* bt32 = static_cast<float*>(btab);
  uint16_t* bthi = static_cast<uint16_t*>(btab);
  uint16_t* btlo = bthi + static_cast<int64_t>(Kpad) * RS;
  const int64_t brow = static_cast<int64_t>(k) * RS;  // table row
  const int64_t arow = static_cast<int64_t>(k) * DPX; // a-path row
  const int32_t n = k < K ? count[k] : 0;
  const double dn = static_cast<double>(n);
  double mu2 = 0.0, muc2 = 0.0, mdot = 0.0, gmax = 0.0;
  for (int r = 0; r < nrep; ++r) {
    const int l = lane + 64 * r;
    if (l >= RS) break;
    double mu = 0.0, muc = 0.0;
    if (n > 0 && l < D) {
      mu = V[static_cast<int64_t>(k) * D + l] / dn;
      muc = METRIC == SIL_SQEUCLID ? mu - gmean[l] : mu;
    }
    mu2 += mu * mu;
    muc2 += muc * muc;
    if (fold && l < D) mdot = fma(static_cast<double>(mvec[l]), muc, mdot);
    double g = ALPHA * muc;  // exact scaling
    if (tscale && l < D) g *= static_cast<double>(tscale[l]);
    gmax = fmax(gmax, fabs(g));
    if (BF16TAB) {
      const uint16_t hi = f32_to_bf16_rne(static_cast<float>(g));
      bthi[brow + l] = hi;
      btlo[brow + l] = f32_to_bf16_rne(static_cast<float>(g - static_cast<double>(bf16_to_f32(hi))));
    } else {
      bt32[brow + l] = static_cast<float>(g);
    }
    if (k < K && l < DPX) atab[arow + l] = static_cast<float>(muc);
  }
  mu2 = wave_sum(mu2);
  muc2 = wave_sum(muc2);
  if (fold) mdot = wave_sum(mdot);
  if (smax)
    for (int off = 1; off < 64; off <<= 1) gmax = fmax(gmax, __shfl_xor(gmax, off, 64));
  if (lane == 0) {
    double c = kEmptyC, av = 0.0;
    if (n > 0) {
      if (METRIC == SIL_SQEUCLID) {
        const double sigma2 = fmax(0.0, psi[k] / dn - mu2);
        // equals Psi_k/N_k when the centring vector is zero; without the variance term the GEMM
        // form gives ||x' - mu'_k||^2, the K-means assignment's distance
        c = with_var ? muc2 + sigma2 : muc2;
        if (fold) c -= ALPHA * mdot;  // + 2 m.mu'_k
        av = sigma2;
      } else if (METRIC == SIL_KL) {
        // V holds sum log y and psi sum_y sum_l y: the table row is -(mean log y), the
        // constant the mean of sum_l y, which the a-path adds too
        c = psi[k] / dn;
        av = c;
      } else {  // cosine: the finish adds the 1 of 1 - z.mu_k after the minimum
        c = 0.0;
        av = fmax(0.0, 1.0 - mu2);
      }
    }
    ctab[k] = static_cast<float>(c);
    if (c64) c64[k] = c;
    if (smax) {  // the screen table's scale: largest entry and constant (see screen.hip)
      smax[0] = n > 0 ? gmax : 0.0;
      smax[1] = n > 0 ? fabs(c) : 0.0;
    }
    if (k < K) {
      avec[k] = static_cast<float>(av);
      ascale[k] = n >= 2 ? static_cast<float>(dn / (dn - 1.0)) : 0.0f;
    }
  }
}

template <int METRIC, bool BF16TAB>
__global__ __launch_bounds__(256) void k_finalize(
    const int32_t* __restrict__ count, const double* __restrict__ V,
    const double* __restrict__ psi, const double* __restrict__ gmean, int32_t K, int32_t Kpad,
    int32_t D, int32_t DPX, int32_t RS, void* __restrict__ btab, float* __restrict__ ctab,
    float* __restrict__ atab, float* __restrict__ avec, float* __restrict__ ascale, int with_var,
    const float* __restrict__ mvec, int fold, const float* __restrict__ tscale,
    int32_t* __restrict__ shdr, double* __restrict__ c64) {
  // shdr (the one-product screen): the workgroup's largest table entry and constant raise the
  // header's slots (one atomic each per workgroup)
  __shared__ double red[4][2];
  const int wave = threadIdx.x >> 6;
  red[wave][0] = 0.0;
  red[wave][1] = 0.0;
  finalize_body<METRIC, BF16TAB>(count, V, psi, gmean, K, Kpad, D, DPX, RS, btab, ctab, atab,
                                 avec, ascale, with_var, mvec, fold, tscale, c64,
                                 shdr ? red[wave] : nullptr, blockIdx.x);
  if (!shdr) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, c = 0.0;
    for (int w = 0; w < 4; ++w) {
      t = fmax(t, red[w][0]);
      c = fmax(c, red[w][1]);
    }
    unsigned long long* slot = reinterpret_cast<unsigned long long*>(shdr + kHdrScreenWord);
    atomicMax(slot + SC_TMAX, static_cast<unsigned long long>(__double_as_longlong(t)));
    atomicMax(slot + SC_CMAX, static_cast<unsigned long long>(__double_as_longlong(c)));
  }
}

hipError_t launch_finalize(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st) {
  const int centre = p.metric == SIL_SQEUCLID && !(p.flags & SIL_FLAG_NO_CENTRE);
  k_gmean<<<static_cast<unsigned>(p.DPX), 256, 0, st>>>(w.V, w.hdr, p.K, p.D, centre, w.gmean,
                                                        w.mvec);
  const unsigned nb = static_cast<unsigned>(ceil_div(p.Kpad, 4));
  const bool bf = p.dtype != SIL_F32;
  const int fold = centre && fold_centre(p.dtype, p.products, p.metric) ? 1 : 0;
  // fp8 codes in the GEMM (the two-product kernels and not the argmin ones): scaled tables
  const float* tscale =
      p.dtype == SIL_FP8_E4M3 && !p.assign && raw_x(p.dtype, p.products, p.metric) ? p.col_scale
                                                                                 : nullptr;
#define SIL_FIN(MT, BF)                                                                        \
  k_finalize<MT, BF><<<nb, 256, 0, st>>>(w.count, w.V, w.psi, w.gmean, p.K, p.Kpad, p.D, p.DPX, \
                                         table_stride(p.DPX, p.dtype), w.btab, w.ctab, w.atab,  \
                                         w.avec, w.ascale, p.assign ? 0 : 1, w.mvec, fold, tscale, \
                                         p.screen ? w.hdr : nullptr, p.screen ? w.c64 : nullptr)
  if (p.metric == SIL_SQEUCLID) {
    if (bf) SIL_FIN(SIL_SQEUCLID, true);
    else SIL_FIN(SIL_SQEUCLID, false);
  } else if (p.metric == SIL_KL) {
    if (bf) SIL_FIN(SIL_KL, true);
    else SIL_FIN(SIL_KL, false);
  } else {
    if (bf) SIL_FIN(SIL_COSINE, true);
    else SIL_FIN(SIL_COSINE, false);
  }
#undef SIL_FIN
  if (p.screen) return launch_screen_table(p, L, w, st);
  return hipGetLastError();
}


// ------------------------------------------------------------------------------------------
// batched (fp32 tables; work item blockIdx.x of the phase, as in the batched statistics)

__device__ __forceinline__ const BatchProblem& batch_item_fin(const BatchDev& b, int phase,
                                                              int64_t* local) {
  const int32_t* pre = b.prefix + phase * (b.n + 1);
  const int32_t item = static_cast<int32_t>(blockIdx.x);
  const int j = batch_locate(pre, b.n, item);
  *local = item - pre[j];
  return b.prob[j];
}

__global__ __launch_bounds__(256) void kb_gmean(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item_fin(b, BP_GMEAN, &it);
  const int centre = q.metric == SIL_SQEUCLID && !(q.flags & SIL_FLAG_NO_CENTRE);
  gmean_body(q.V, q.hdr, q.K, q.D, centre, q.gmean, q.mvec, static_cast<int>(it));
}

__global__ __launch_bounds__(256) void kb_fin(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item_fin(b, BP_FIN, &it);
  const int32_t RS = table_stride(q.DPX, SIL_F32);
  if (q.metric == SIL_SQEUCLID)
    finalize_body<SIL_SQEUCLID, false>(q.count, q.V, q.psi, q.gmean, q.K, q.Kpad, q.D, q.DPX, RS,
                                       q.btab, q.ctab, q.atab, q.avec, q.ascale, 1, nullptr, 0,
                                       nullptr, nullptr, nullptr, it);
  else
    finalize_body<SIL_COSINE, false>(q.count, q.V, q.psi, q.gmean, q.K, q.Kpad, q.D, q.DPX, RS,
                                     q.btab, q.ctab, q.atab, q.avec, q.ascale, 1, nullptr, 0,
                                     nullptr, nullptr, nullptr, it);
}

hipError_t launch_finalize_batched(const BatchLaunch& b, hipStream_t st) {
  kb_gmean<<<static_cast<unsigned>(b.items[BP_GMEAN]), 256, 0, st>>>(b.dev);
  kb_fin<<<static_cast<unsigned>(b.items[BP_FIN]), 256, 0, st>>>(b.dev);
  return hipGetLastError();
}

}  // namespace sil
