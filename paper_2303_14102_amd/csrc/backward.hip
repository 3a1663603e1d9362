// Gradient of S with respect to X (labels fixed).  Not in the paper: derived from Eq.11 and
// Eq.18 with the per-point a_i, b_i and neighbouring cluster kept by the forward call.
//
// With alpha_i,o = gS ds_i/da_i N_o/((N_o-1) N) and alpha_i,n = gS ds_i/db_i / N (o the own, n
// the neighbouring cluster; ds/da = -1/b, ds/db = a/b^2 when a <= b, -b/a^2 and 1/a otherwise,
// zero for singletons), A_k = sum_i alpha_ik and B_k = sum_i alpha_ik v_i over the two clusters
// each point touches (v = x' centred, or z = x/||x|| for cosine):
//   squared Euclidean: dX_j = 2 alpha_j,o (x'_j - mu'_o) + 2 alpha_j,n (x'_j - mu'_n)
//                             + (2 / N_o)(A_o x'_j - B_o)
//   cosine:            g = -alpha_j,o mu_o - alpha_j,n mu_n - B_o / N_o,
//                      dX_j = (g - (g.z_j) z_j) / ||x_j||
// (x' = x - m and mu' = mu - m: the centring cancels in every difference.)
//
// Kernels: kb_accum (per workgroup, A and B accumulated in LDS in FP64, written out as one
// partial per workgroup), kb_reduce (partials summed in workgroup order: deterministic),
// kb_dx (one wave per row).  When K (D+1) FP64 values do not fit in LDS, kb_accum_global adds
// straight into global memory with FP64 atomics instead.
#include "sil_internal.h"

namespace sil {

constexpr int kBwdWaves = 8;  // waves per workgroup of the accumulation kernel

struct BwdArgs {
  const float* X;
  const int32_t* labels;
  const int32_t* count;
  const int32_t* hdr;
  const float* atab;   // [K][DPX] mu' (squared Euclidean, centred) or mu (cosine)
  const float* mvec;   // [DPX]
  const float* save_a;
  const float* save_b;
  const int32_t* save_n;
  const double* gS;
  int64_t N;
  int32_t D, DPX, K;
  double* part;        // [nwg][K*(D+1)]  (A_k in column D)
  double* AB;          // [K*(D+1)] reduced
  float* dX;
};

// alpha for the own and the neighbouring cluster of row i (zero when the point is a singleton or
// max(a, b) = 0).
__device__ __forceinline__ void alphas(const BwdArgs& a, int64_t i, int32_t o, double gS,
                                       double& al_o, double& al_n) {
  al_o = 0.0;
  al_n = 0.0;
  const int32_t no = a.count[o];
  const double av = a.save_a[i], bv = a.save_b[i];
  const double mx = av > bv ? av : bv;
  if (no < 2 || !(mx > 0.0)) return;
  double dsa, dsb;
  if (av <= bv) {
    dsa = -1.0 / bv;
    dsb = av / (bv * bv);
  } else {
    dsa = -bv / (av * av);
    dsb = 1.0 / av;
  }
  const double n = static_cast<double>(a.N);
  al_o = gS * dsa * static_cast<double>(no) / static_cast<double>(no - 1) / n;
  al_n = gS * dsb / n;
}

// Point i's vector v (centred x or unit z) for the columns this lane holds: cols lane + 64 e.
template <int METRIC>
__device__ __forceinline__ void load_v(const BwdArgs& a, int64_t i, int lane, float (&v)[4],
                                       float& inv_norm) {
  const int64_t base = i * static_cast<int64_t>(a.D);
  float n2 = 0.0f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = lane + 64 * e;
    float x = c < a.D ? a.X[base + c] : 0.0f;
    if (METRIC == SIL_SQEUCLID && c < a.D) x -= a.mvec[c];
    v[e] = x;
    n2 = fmaf(x, x, n2);
  }
  inv_norm = 1.0f;
  if constexpr (METRIC == SIL_COSINE) {
    for (int off = 1; off < 64; off <<= 1) n2 += __shfl_xor(n2, off, 64);
    inv_norm = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] *= inv_norm;
  }
}

// One wave per row (grid-stride); A and B of this workgroup in LDS.
template <int METRIC>
__global__ __launch_bounds__(64 * kBwdWaves) void kb_accum(BwdArgs a) {
  extern __shared__ double sh[];  // [K*(D+1)]
  const int W = a.D + 1;
  const int64_t KW = static_cast<int64_t>(a.K) * W;
  for (int64_t q = threadIdx.x; q < KW; q += blockDim.x) sh[q] = 0.0;
  __syncthreads();
  // wave-uniform wave index: the per-row loads (labels, saves, counts) become scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double gS = *a.gS;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * kBwdWaves;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBwdWaves + wave; i < a.N; i += nw) {
    const int32_t o = a.labels[i];
    const int32_t n = a.save_n[i];
    if (o < 0 || o >= a.K) continue;
    double al_o, al_n;
    alphas(a, i, o, gS, al_o, al_n);
    if (al_o == 0.0 && al_n == 0.0) continue;
    float v[4], inv;
    load_v<METRIC>(a, i, lane, v, inv);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = lane + 64 * e;
      if (c < a.D) {
        atomicAdd(&sh[static_cast<int64_t>(o) * W + c], al_o * v[e]);
        if (n >= 0 && n < a.K) atomicAdd(&sh[static_cast<int64_t>(n) * W + c], al_n * v[e]);
      }
    }
    if (lane == 0) {
      atomicAdd(&sh[static_cast<int64_t>(o) * W + a.D], al_o);
      if (n >= 0 && n < a.K) atomicAdd(&sh[static_cast<int64_t>(n) * W + a.D], al_n);
    }
  }
  __syncthreads();
  double* out = a.part + static_cast<int64_t>(blockIdx.x) * KW;
  for (int64_t q = threadIdx.x; q < KW; q += blockDim.x) out[q] = sh[q];
}

// Same without LDS: FP64 atomics in global memory (large K * D).
template <int METRIC>
__global__ __launch_bounds__(64 * kBwdWaves) void kb_accum_global(BwdArgs a) {
  const int W = a.D + 1;
  // wave-uniform wave index: the per-row loads (labels, saves, counts) become scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double gS = *a.gS;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * kBwdWaves;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBwdWaves + wave; i < a.N; i += nw) {
    const int32_t o = a.labels[i];
    const int32_t n = a.save_n[i];
    if (o < 0 || o >= a.K) continue;
    double al_o, al_n;
    alphas(a, i, o, gS, al_o, al_n);
    if (al_o == 0.0 && al_n == 0.0) continue;
    float v[4], inv;
    load_v<METRIC>(a, i, lane, v, inv);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = lane + 64 * e;
      if (c < a.D) {
        unsafeAtomicAdd(&a.AB[static_cast<int64_t>(o) * W + c], al_o * v[e]);
        if (n >= 0 && n < a.K) unsafeAtomicAdd(&a.AB[static_cast<int64_t>(n) * W + c], al_n * v[e]);
      }
    }
    if (lane == 0) {
      unsafeAtomicAdd(&a.AB[static_cast<int64_t>(o) * W + a.D], al_o);
      if (n >= 0 && n < a.K) unsafeAtomicAdd(&a.AB[static_cast<int64_t>(n) * W + a.D], al_n);
    }
  }
}

// Squared Euclidean partials by column slice.  Workgroup b of the grid is row group b % nrg and
// slice b / nrg: it accumulates columns 64 s .. 64 s + 63 (one per lane) of the rows of its
// group, and slice 0 also the alphas themselves (A_k, slot 64).  Its LDS holds K x 65 values
// instead of K x (D + 1), so several workgroups share a CU; every row is still read once in all.
constexpr int kBwdSlice = 64;
__global__ __launch_bounds__(64 * kBwdWaves) void kb_accum_slice(BwdArgs a, int nrg) {
  extern __shared__ double sh[];  // [K * 65]
  constexpr int SW = kBwdSlice + 1;
  const int W = a.D + 1;
  const int64_t KS = static_cast<int64_t>(a.K) * SW;
  for (int64_t q = threadIdx.x; q < KS; q += blockDim.x) sh[q] = 0.0;
  __syncthreads();
  const int rg = static_cast<int>(blockIdx.x) % nrg, sl = static_cast<int>(blockIdx.x) / nrg;
  // wave-uniform wave index: the per-row loads (labels, saves, counts) become scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = sl * kBwdSlice + lane;
  const bool col_ok = c < a.D;
  const float mv = col_ok ? a.mvec[c] : 0.0f;
  const double gS = *a.gS;
  const int64_t nw = static_cast<int64_t>(nrg) * kBwdWaves;
  for (int64_t i = static_cast<int64_t>(rg) * kBwdWaves + wave; i < a.N; i += nw) {
    const int32_t o = a.labels[i];
    const int32_t n = a.save_n[i];
    if (o < 0 || o >= a.K) continue;
    double al_o, al_n;
    alphas(a, i, o, gS, al_o, al_n);
    if (al_o == 0.0 && al_n == 0.0) continue;
    const bool has_n = n >= 0 && n < a.K;
    if (col_ok) {
      const double v = static_cast<double>(a.X[i * static_cast<int64_t>(a.D) + c] - mv);
      atomicAdd(&sh[static_cast<int64_t>(o) * SW + lane], al_o * v);
      if (has_n) atomicAdd(&sh[static_cast<int64_t>(n) * SW + lane], al_n * v);
    }
    if (sl == 0 && lane == 0) {
      atomicAdd(&sh[static_cast<int64_t>(o) * SW + kBwdSlice], al_o);
      if (has_n) atomicAdd(&sh[static_cast<int64_t>(n) * SW + kBwdSlice], al_n);
    }
  }
  __syncthreads();
  double* out = a.part + static_cast<int64_t>(rg) * a.K * W;
  for (int64_t q = threadIdx.x; q < KS; q += blockDim.x) {
    const int64_t k = q / SW;
    const int j = static_cast<int>(q % SW);
    if (j < kBwdSlice) {
      if (sl * kBwdSlice + j < a.D) out[k * W + sl * kBwdSlice + j] = sh[q];
    } else if (sl == 0) {
      out[k * W + a.D] = sh[q];
    }
  }
}

// AB[q] = sum of the workgroup partials in workgroup order.
__global__ __launch_bounds__(256) void kb_reduce(const double* __restrict__ part, int nwg,
                                                 int64_t KW, double* __restrict__ AB) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= KW) return;
  double s = 0.0;
  for (int g = 0; g < nwg; ++g) s += part[static_cast<int64_t>(g) * KW + q];
  AB[q] = s;
}

__global__ void kb_zero(double* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// dX, one wave per row (grid-stride).  Rows whose status is bad get NaN (the forward S is NaN).
template <int METRIC>
__global__ __launch_bounds__(256) void kb_dx(BwdArgs a) {
  const int lane = threadIdx.x & 63;
  const int W = a.D + 1;
  const double gS = *a.gS;
  const bool bad = a.hdr[0] != 0;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
  // wave-uniform row index: the per-row loads (labels, saves, counts) become scalar loads
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) +
                   __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
       i < a.N; i += nw) {
    const int64_t base = i * static_cast<int64_t>(a.D);
    const int32_t o = a.labels[i];
    if (bad || o < 0 || o >= a.K) {
      for (int c = lane; c < a.D; c += 64) a.dX[base + c] = __builtin_nanf("");
      continue;
    }
    const int32_t n = a.save_n[i];
    const bool has_n = n >= 0 && n < a.K;
    double al_o, al_n;
    alphas(a, i, o, gS, al_o, al_n);
    float v[4], inv;
    load_v<METRIC>(a, i, lane, v, inv);
    const float fo = static_cast<float>(al_o), fn = static_cast<float>(al_n);
    const double Ao = a.AB[static_cast<int64_t>(o) * W + a.D];
    const float rn = 1.0f / static_cast<float>(a.count[o]);
    float g[4];
    float gz = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = lane + 64 * e;
      g[e] = 0.0f;
      if (c < a.D) {
        const float mo = a.atab[static_cast<int64_t>(o) * a.DPX + c];
        const float mn = has_n ? a.atab[static_cast<int64_t>(n) * a.DPX + c] : 0.0f;
        const float Bo = static_cast<float>(a.AB[static_cast<int64_t>(o) * W + c]);
        if constexpr (METRIC == SIL_SQEUCLID) {
          g[e] = 2.0f * fo * (v[e] - mo) + (has_n ? 2.0f * fn * (v[e] - mn) : 0.0f) +
                 2.0f * rn * (static_cast<float>(Ao) * v[e] - Bo);
        } else {
          g[e] = -fo * mo - (has_n ? fn * mn : 0.0f) - Bo * rn;
          gz = fmaf(g[e], v[e], gz);
        }
      }
    }
    if constexpr (METRIC == SIL_COSINE) {
      for (int off = 1; off < 64; off <<= 1) gz += __shfl_xor(gz, off, 64);
#pragma unroll
      for (int e = 0; e < 4; ++e) g[e] = (g[e] - gz * v[e]) * inv;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = lane + 64 * e;
      if (c < a.D) a.dX[base + c] = g[e];
    }
  }
}

int bwd_accum_workgroups(int64_t N) {
  const int64_t w = ceil_div(N, 64 * kBwdWaves);
  return static_cast<int>(w < 512 ? w : 512);
}

// The per-workgroup partials of A_k, B_k in LDS: up to the 160 KB of one CU (gfx950), so that
// K (D + 1) = 64 x 257 FP64 values (the 256-dimension, 64-cluster case) stay off global atomics.
bool bwd_fits_lds(int32_t K, int32_t D) {
  return static_cast<int64_t>(K) * (D + 1) * 8 <= 160 * 1024;
}

// The column-slice form (squared Euclidean): K x 65 partials per workgroup.
bool bwd_fits_slices(int32_t K) {
  return static_cast<int64_t>(K) * (kBwdSlice + 1) * 8 <= 160 * 1024;
}

hipError_t launch_backward(const Problem& p, const WsLayout& L, const WsPtrs& w, const double* gS,
                           float* dX, hipStream_t st) {
  BwdArgs a;
  a.X = static_cast<const float*>(p.X);
  a.labels = p.labels;
  a.count = w.count;
  a.hdr = w.hdr;
  a.atab = w.atab;
  a.mvec = w.mvec;
  a.save_a = w.save_a;
  a.save_b = w.save_b;
  a.save_n = w.save_n;
  a.gS = gS;
  a.N = p.N;
  a.D = p.D;
  a.DPX = p.DPX;
  a.K = p.K;
  a.part = w.gpart;
  a.AB = w.gAB;
  a.dX = dX;
  const int64_t KW = static_cast<int64_t>(p.K) * (p.D + 1);
  const int nwg = bwd_accum_workgroups(p.N);
  const bool lds = bwd_fits_lds(p.K, p.D);
  if (p.metric == SIL_SQEUCLID && bwd_fits_slices(p.K)) {
    const size_t shm = static_cast<size_t>(p.K) * (kBwdSlice + 1) * 8;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_accum_slice),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(shm));
    if (e != hipSuccess) return e;
    const int nsl = static_cast<int>(ceil_div(p.D, kBwdSlice));
    kb_accum_slice<<<static_cast<unsigned>(nwg * nsl), 64 * kBwdWaves, shm, st>>>(a, nwg);
    kb_reduce<<<static_cast<unsigned>(ceil_div(KW, 256)), 256, 0, st>>>(w.gpart, nwg, KW, w.gAB);
  } else if (lds) {
    const size_t shm = static_cast<size_t>(KW) * 8;
    if (p.metric == SIL_SQEUCLID) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_accum<SIL_SQEUCLID>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               static_cast<int>(shm));
      if (e != hipSuccess) return e;
      kb_accum<SIL_SQEUCLID><<<nwg, 64 * kBwdWaves, shm, st>>>(a);
    } else {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_accum<SIL_COSINE>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               static_cast<int>(shm));
      if (e != hipSuccess) return e;
      kb_accum<SIL_COSINE><<<nwg, 64 * kBwdWaves, shm, st>>>(a);
    }
    kb_reduce<<<static_cast<unsigned>(ceil_div(KW, 256)), 256, 0, st>>>(w.gpart, nwg, KW, w.gAB);
  } else {
    kb_zero<<<static_cast<unsigned>(ceil_div(KW, 256)), 256, 0, st>>>(w.gAB, KW);
    if (p.metric == SIL_SQEUCLID)
      kb_accum_global<SIL_SQEUCLID><<<nwg, 64 * kBwdWaves, 0, st>>>(a);
    else
      kb_accum_global<SIL_COSINE><<<nwg, 64 * kBwdWaves, 0, st>>>(a);
  }
  const unsigned gdx = static_cast<unsigned>(ceil_div(p.N, 4) < 8192 ? ceil_div(p.N, 4) : 8192);
  if (p.metric == SIL_SQEUCLID)
    kb_dx<SIL_SQEUCLID><<<gdx, 256, 0, st>>>(a);
  else
    kb_dx<SIL_COSINE><<<gdx, 256, 0, st>>>(a);
  (void)L;
  return hipGetLastError();
}

}  // namespace sil
