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
// Kernels: kb_alpha (one thread per row: the row's two alphas, formed once, into a 16-byte record
// the other kernels read with one scalar load), kb_accum (per workgroup, A and B accumulated in
// LDS in FP64, written out as one partial per workgroup), kb_reduce (partials summed in workgroup
// order), kb_dx (one wave per row).  When K (D+1) FP64 values do not fit in LDS,
// kb_accum_global adds straight into global memory with FP64 atomics instead.
#include "sil_internal.h"

namespace sil {

constexpr int kBwdWaves = 16;  // waves per workgroup of the accumulation kernels

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
  float* gtab;         // [K][DPX] per-cluster fp32 terms of dX (zero past D)
  float* htab;         // [K]
  struct Alpha* alpha; // [N]
};

// Row i's clusters and alphas: o = -1 for a row outside [0, K) (it contributes nothing and gets
// NaN), n = -1 without a neighbouring cluster; the alphas are formed in binary64 and rounded
// once to fp32 (their products with fp32 values are then exact in binary64).
struct Alpha {
  int32_t o, n;
  float ao, an;
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

__global__ __launch_bounds__(256) void kb_alpha(BwdArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int32_t o = a.labels[i];
  Alpha r{-1, -1, 0.0f, 0.0f};
  if (o >= 0 && o < a.K) {
    double ao, an;
    alphas(a, i, o, *a.gS, ao, an);
    const int32_t n = a.save_n[i];
    r.o = o;
    r.n = n >= 0 && n < a.K ? n : -1;
    r.ao = static_cast<float>(ao);
    r.an = static_cast<float>(an);
  }
  a.alpha[i] = r;
}

// This lane's columns c = lane + 64 e, clamped into [0, D) so that every load is unconditional
// (the loads of a step then issue back to back instead of each behind a branch of its own and a
// wait); ok marks the real ones, mv holds the centring vector there (squared Euclidean).
struct LaneCols {
  int cc[4];
  bool ok[4];
  float mv[4];
};

template <int METRIC>
__device__ __forceinline__ LaneCols lane_cols(const BwdArgs& a, int lane) {
  LaneCols l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = lane + 64 * e;
    l.ok[e] = c < a.D;
    l.cc[e] = l.ok[e] ? c : a.D - 1;
    l.mv[e] = METRIC == SIL_SQEUCLID ? a.mvec[l.cc[e]] : 0.0f;
  }
  return l;
}

// Row i's vector v (centred x or unit z) at this lane's columns (zero past D); i < N.
template <int METRIC>
__device__ __forceinline__ void load_v(const BwdArgs& a, const LaneCols& l, int64_t i,
                                       float (&v)[4], float& inv_norm) {
  const float* xr = a.X + i * static_cast<int64_t>(a.D);
  float n2 = 0.0f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float x = xr[l.cc[e]] - l.mv[e];
    v[e] = l.ok[e] ? x : 0.0f;
    n2 = fmaf(v[e], v[e], n2);
  }
  inv_norm = 1.0f;
  if constexpr (METRIC == SIL_COSINE) {
    for (int off = 1; off < 64; off <<= 1) n2 += __shfl_xor(n2, off, 64);
    inv_norm = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] *= inv_norm;
  }
}

// Each wave takes a few consecutive rows per step and issues all their loads (alpha records, X,
// table rows) before the first atomic or store that depends on them: one row at a time leaves
// too few bytes in flight to cover the memory latency.  kAccRows for the accumulation kernels
// (one column per lane: 256 bytes of X per row and wave), kDxRows for dX (whose table rows also
// take registers).
constexpr int kAccRows = 8;
constexpr int kDxRows = 4;

template <bool GLOBAL>
__device__ __forceinline__ void bwd_add(double* p, double v) {
  if constexpr (GLOBAL)
    unsafeAtomicAdd(p, v);
  else
    atomicAdd(p, v);
}

// Row i0 + u, clamped to the last row (its loads stay in bounds; the results are not used).
__device__ __forceinline__ int64_t bwd_row(const BwdArgs& a, int64_t i0, int u) {
  return i0 + u < a.N ? i0 + u : a.N - 1;
}

// The Alpha records of rows i0 .. i0 + R - 1 (o = -1 past the end).
template <int R>
__device__ __forceinline__ void load_alphas(const BwdArgs& a, int64_t i0, Alpha (&r)[R]) {
#pragma unroll
  for (int u = 0; u < R; ++u) r[u] = a.alpha[bwd_row(a, i0, u)];
#pragma unroll
  for (int u = 0; u < R; ++u)
    if (i0 + u >= a.N) r[u].o = -1;
}

// A and B over all D columns of the rows of this wave, into tgt ([K][D+1], LDS or global).
template <int METRIC, bool GLOBAL>
__device__ __forceinline__ void accum_rows(const BwdArgs& a, double* tgt, int64_t g, int64_t ng,
                                           int lane) {
  const int W = a.D + 1;
  const LaneCols l = lane_cols<METRIC>(a, lane);
  for (; g * kAccRows < a.N; g += ng) {
    const int64_t i0 = g * kAccRows;
    Alpha r[kAccRows];
    load_alphas(a, i0, r);
    float v[kAccRows][4], inv;
#pragma unroll
    for (int u = 0; u < kAccRows; ++u) load_v<METRIC>(a, l, bwd_row(a, i0, u), v[u], inv);
#pragma unroll
    for (int u = 0; u < kAccRows; ++u) {
      const int32_t o = r[u].o, n = r[u].n;
      if (o < 0 || (r[u].ao == 0.0f && r[u].an == 0.0f)) continue;
      const double al_o = r[u].ao, al_n = r[u].an;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (l.ok[e]) {
          bwd_add<GLOBAL>(&tgt[static_cast<int64_t>(o) * W + l.cc[e]], al_o * v[u][e]);
          if (n >= 0) bwd_add<GLOBAL>(&tgt[static_cast<int64_t>(n) * W + l.cc[e]], al_n * v[u][e]);
        }
      }
      if (lane == 0) {
        bwd_add<GLOBAL>(&tgt[static_cast<int64_t>(o) * W + a.D], al_o);
        if (n >= 0) bwd_add<GLOBAL>(&tgt[static_cast<int64_t>(n) * W + a.D], al_n);
      }
    }
  }
}

// A and B of this workgroup's rows in LDS, written out as its partial.
template <int METRIC>
__global__ __launch_bounds__(64 * kBwdWaves) void kb_accum(BwdArgs a) {
  extern __shared__ double sh[];  // [K*(D+1)]
  const int64_t KW = static_cast<int64_t>(a.K) * (a.D + 1);
  for (int64_t q = threadIdx.x; q < KW; q += blockDim.x) sh[q] = 0.0;
  __syncthreads();
  // wave-uniform wave index: the per-row loads become scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  accum_rows<METRIC, false>(a, sh, static_cast<int64_t>(blockIdx.x) * kBwdWaves + wave,
                            static_cast<int64_t>(gridDim.x) * kBwdWaves, lane);
  __syncthreads();
  double* out = a.part + static_cast<int64_t>(blockIdx.x) * KW;
  for (int64_t q = threadIdx.x; q < KW; q += blockDim.x) out[q] = sh[q];
}

// Same without LDS: FP64 atomics in global memory (large K * D).
template <int METRIC>
__global__ __launch_bounds__(64 * kBwdWaves) void kb_accum_global(BwdArgs a) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  accum_rows<METRIC, true>(a, a.AB, static_cast<int64_t>(blockIdx.x) * kBwdWaves + wave,
                           static_cast<int64_t>(gridDim.x) * kBwdWaves, lane);
}

// Squared Euclidean partials by column slice.  Workgroup b of the grid is row group b % nrg and
// slice b / nrg: it accumulates columns 64 s .. 64 s + 63 (one per lane) of the rows of its
// group, and slice 0 also the alphas themselves (A_k, slot 64).  Its LDS holds K x 65 values
// instead of K x (D + 1): the form for K (D + 1) FP64 values beyond the LDS of one CU.
constexpr int kBwdSlice = 64;
__global__ __launch_bounds__(64 * kBwdWaves) void kb_accum_slice(BwdArgs a, int nrg) {
  extern __shared__ double sh[];  // [K * 65]
  constexpr int SW = kBwdSlice + 1;
  const int W = a.D + 1;
  const int64_t KS = static_cast<int64_t>(a.K) * SW;
  for (int64_t q = threadIdx.x; q < KS; q += blockDim.x) sh[q] = 0.0;
  __syncthreads();
  const int rg = static_cast<int>(blockIdx.x) % nrg, sl = static_cast<int>(blockIdx.x) / nrg;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = sl * kBwdSlice + lane;
  const bool col_ok = c < a.D;
  const int cc = col_ok ? c : a.D - 1;  // clamped: the loads below are unconditional
  const float mv = a.mvec[cc];
  const int64_t ng = static_cast<int64_t>(nrg) * kBwdWaves;
  for (int64_t g = static_cast<int64_t>(rg) * kBwdWaves + wave; g * kAccRows < a.N; g += ng) {
    const int64_t i0 = g * kAccRows;
    Alpha r[kAccRows];
    load_alphas(a, i0, r);
    float x[kAccRows];
#pragma unroll
    for (int u = 0; u < kAccRows; ++u) x[u] = a.X[bwd_row(a, i0, u) * static_cast<int64_t>(a.D) + cc];
#pragma unroll
    for (int u = 0; u < kAccRows; ++u) {
      const int32_t o = r[u].o, n = r[u].n;
      if (o < 0 || (r[u].ao == 0.0f && r[u].an == 0.0f)) continue;
      const double al_o = r[u].ao, al_n = r[u].an;
      if (col_ok) {
        const double v = static_cast<double>(x[u] - mv);
        atomicAdd(&sh[static_cast<int64_t>(o) * SW + lane], al_o * v);
        if (n >= 0) atomicAdd(&sh[static_cast<int64_t>(n) * SW + lane], al_n * v);
      }
      if (sl == 0 && lane == 0) {
        atomicAdd(&sh[static_cast<int64_t>(o) * SW + kBwdSlice], al_o);
        if (n >= 0) atomicAdd(&sh[static_cast<int64_t>(n) * SW + kBwdSlice], al_n);
      }
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

// AB[q] = sum of the workgroup partials: workgroup b covers 64 entries q (one per lane); its
// wave w sums the partials of the w-th of kRedWaves contiguous chunks of workgroups in order,
// and the chunk sums are added in chunk order (a fixed order for given N, K, D).
constexpr int kRedWaves = 8;
__global__ __launch_bounds__(64 * kRedWaves) void kb_reduce(const double* __restrict__ part, int nwg,
                                                           int64_t KW, double* __restrict__ AB) {
  __shared__ double red[kRedWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  const int per = (nwg + kRedWaves - 1) / kRedWaves;
  const int g0 = wave * per, g1 = g0 + per < nwg ? g0 + per : nwg;
  double s = 0.0;
  if (q < KW) {
#pragma unroll 8
    for (int g = g0; g < g1; ++g) s += part[static_cast<int64_t>(g) * KW + q];
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && q < KW) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRedWaves; ++w) t += red[w][lane];
    AB[q] = t;
  }
}

__global__ void kb_zero(double* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Per-cluster fp32 terms of dX, from A_k, B_k (FP64) and N_k: gtab[k][c] = f B_k[c] / N_k for
// c < D (f = 2 squared Euclidean, 1 cosine; zero for D <= c < DPX) and htab[k] = 2 A_k / N_k
// (squared Euclidean).  Empty clusters get zeros (no row refers to them).
__global__ __launch_bounds__(256) void kb_gtab(BwdArgs a, int metric) {
  const int W = a.D + 1;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= static_cast<int64_t>(a.K) * a.DPX) return;
  const int64_t k = q / a.DPX;
  const int c = static_cast<int>(q % a.DPX);
  const int32_t nk = a.count[k];
  const double rn = nk > 0 ? 1.0 / static_cast<double>(nk) : 0.0;
  const double f = metric == SIL_SQEUCLID ? 2.0 : 1.0;
  a.gtab[q] = c < a.D ? static_cast<float>(f * a.AB[k * W + c] * rn) : 0.0f;
  if (c == 0) a.htab[k] = static_cast<float>(2.0 * a.AB[k * W + a.D] * rn);
}

// dX, one wave per kDxRows rows per step (grid-stride).  Rows whose status is bad get NaN (the
// forward S is NaN).
template <int METRIC>
__global__ __launch_bounds__(256) void kb_dx(BwdArgs a) {
  const int lane = threadIdx.x & 63;
  const bool bad = a.hdr[0] != 0;
  const LaneCols l = lane_cols<METRIC>(a, lane);
  const int64_t ng = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
  // wave-uniform row group: the alpha records and table rows of a row are wave-uniform
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) +
                   __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
       g * kDxRows < a.N; g += ng) {
    const int64_t i0 = g * kDxRows;
    // X first: its loads do not wait for the alpha records
    float v[kDxRows][4], inv[kDxRows], mo[kDxRows][4], mn[kDxRows][4], go[kDxRows][4],
        ho[kDxRows];
#pragma unroll
    for (int u = 0; u < kDxRows; ++u) load_v<METRIC>(a, l, bwd_row(a, i0, u), v[u], inv[u]);
    Alpha r[kDxRows];
    load_alphas(a, i0, r);
    // the table rows of the own and neighbouring clusters (cluster 0's for a row without one)
#pragma unroll
    for (int u = 0; u < kDxRows; ++u) {
      const int64_t o = r[u].o < 0 ? 0 : r[u].o, n = r[u].n < 0 ? o : r[u].n;
      ho[u] = a.htab[o];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        mo[u][e] = a.atab[o * a.DPX + l.cc[e]];
        mn[u][e] = a.atab[n * a.DPX + l.cc[e]];
        go[u][e] = a.gtab[o * a.DPX + l.cc[e]];
      }
    }
#pragma unroll
    for (int u = 0; u < kDxRows; ++u) {
      const int64_t i = i0 + u;
      if (i >= a.N) break;
      float* dxr = a.dX + i * static_cast<int64_t>(a.D);
      if (bad || r[u].o < 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (l.ok[e]) dxr[l.cc[e]] = __builtin_nanf("");
        continue;
      }
      const float fo = r[u].ao, fn = r[u].n < 0 ? 0.0f : r[u].an;
      float gr[4];
      float gz = 0.0f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if constexpr (METRIC == SIL_SQEUCLID) {
          gr[e] = 2.0f * fo * (v[u][e] - mo[u][e]) + 2.0f * fn * (v[u][e] - mn[u][e]) +
                  (ho[u] * v[u][e] - go[u][e]);
        } else {
          gr[e] = -fo * mo[u][e] - fn * mn[u][e] - go[u][e];
          gz = fmaf(gr[e], v[u][e], gz);
        }
      }
      if constexpr (METRIC == SIL_COSINE) {
        for (int off = 1; off < 64; off <<= 1) gz += __shfl_xor(gz, off, 64);
#pragma unroll
        for (int e = 0; e < 4; ++e) gr[e] = (gr[e] - gz * v[u][e]) * inv[u];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (l.ok[e]) dxr[l.cc[e]] = gr[e];
    }
  }
}

// dX with four consecutive columns per lane (D % 4 == 0, X and dX 16-byte aligned): one 16-byte
// load or store per lane and row for X, the tables and dX.  Lanes past D / 4 idle, so it is used
// for D > 128 only.
template <int METRIC>
__global__ __launch_bounds__(256) void kb_dx4(BwdArgs a) {
  const int lane = threadIdx.x & 63;
  const bool ok = 4 * lane < a.D;
  const int c = ok ? 4 * lane : a.D - 4;  // clamped: the loads below are unconditional
  const float4 mv = METRIC == SIL_SQEUCLID ? *reinterpret_cast<const float4*>(a.mvec + c)
                                           : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const bool bad = a.hdr[0] != 0;
  const int64_t ng = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) +
                   __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
       g * kDxRows < a.N; g += ng) {
    const int64_t i0 = g * kDxRows;
    float4 v[kDxRows], mo[kDxRows], mn[kDxRows], go[kDxRows];
    float inv[kDxRows], ho[kDxRows];
#pragma unroll
    for (int u = 0; u < kDxRows; ++u) {
      const float4 x =
          *reinterpret_cast<const float4*>(a.X + bwd_row(a, i0, u) * static_cast<int64_t>(a.D) + c);
      v[u] = ok ? make_float4(x.x - mv.x, x.y - mv.y, x.z - mv.z, x.w - mv.w)
                : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    Alpha r[kDxRows];
    load_alphas(a, i0, r);
#pragma unroll
    for (int u = 0; u < kDxRows; ++u) {
      const int64_t o = r[u].o < 0 ? 0 : r[u].o, n = r[u].n < 0 ? o : r[u].n;
      ho[u] = a.htab[o];
      mo[u] = *reinterpret_cast<const float4*>(a.atab + o * a.DPX + c);
      mn[u] = *reinterpret_cast<const float4*>(a.atab + n * a.DPX + c);
      go[u] = *reinterpret_cast<const float4*>(a.gtab + o * a.DPX + c);
    }
    if constexpr (METRIC == SIL_COSINE) {
#pragma unroll
      for (int u = 0; u < kDxRows; ++u) {
        float n2 = v[u].x * v[u].x + v[u].y * v[u].y + v[u].z * v[u].z + v[u].w * v[u].w;
        for (int off = 1; off < 64; off <<= 1) n2 += __shfl_xor(n2, off, 64);
        inv[u] = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
        v[u].x *= inv[u];
        v[u].y *= inv[u];
        v[u].z *= inv[u];
        v[u].w *= inv[u];
      }
    }
#pragma unroll
    for (int u = 0; u < kDxRows; ++u) {
      const int64_t i = i0 + u;
      if (i >= a.N) break;
      float4* dxr = reinterpret_cast<float4*>(a.dX + i * static_cast<int64_t>(a.D) + c);
      if (bad || r[u].o < 0) {
        const float q = __builtin_nanf("");
        if (ok) *dxr = make_float4(q, q, q, q);
        continue;
      }
      const float fo = r[u].ao, fn = r[u].n < 0 ? 0.0f : r[u].an;
      const float vv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
      const float mo4[4] = {mo[u].x, mo[u].y, mo[u].z, mo[u].w};
      const float mn4[4] = {mn[u].x, mn[u].y, mn[u].z, mn[u].w};
      const float go4[4] = {go[u].x, go[u].y, go[u].z, go[u].w};
      float gr[4];
      float gz = 0.0f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if constexpr (METRIC == SIL_SQEUCLID) {
          gr[e] = 2.0f * fo * (vv[e] - mo4[e]) + 2.0f * fn * (vv[e] - mn4[e]) +
                  (ho[u] * vv[e] - go4[e]);
        } else {
          gr[e] = -fo * mo4[e] - fn * mn4[e] - go4[e];
          gz = fmaf(gr[e], vv[e], gz);
        }
      }
      if constexpr (METRIC == SIL_COSINE) {
        for (int off = 1; off < 64; off <<= 1) gz += __shfl_xor(gz, off, 64);
#pragma unroll
        for (int e = 0; e < 4; ++e) gr[e] = (gr[e] - gz * vv[e]) * inv[u];
      }
      if (ok) *dxr = make_float4(gr[0], gr[1], gr[2], gr[3]);
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
  a.alpha = static_cast<Alpha*>(w.galpha);
  kb_alpha<<<static_cast<unsigned>(ceil_div(p.N, 256)), 256, 0, st>>>(a);
  const int64_t KW = static_cast<int64_t>(p.K) * (p.D + 1);
  const int nwg = bwd_accum_workgroups(p.N);
  const bool lds = bwd_fits_lds(p.K, p.D);
  // whole rows per wave where the K (D + 1) partials fit in LDS; else 64-column slices (squared
  // Euclidean) or global atomics
  if (p.metric == SIL_SQEUCLID && !lds && bwd_fits_slices(p.K)) {
    const size_t shm = static_cast<size_t>(p.K) * (kBwdSlice + 1) * 8;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_accum_slice),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(shm));
    if (e != hipSuccess) return e;
    const int nsl = static_cast<int>(ceil_div(p.D, kBwdSlice));
    kb_accum_slice<<<static_cast<unsigned>(nwg * nsl), 64 * kBwdWaves, shm, st>>>(a, nwg);
    kb_reduce<<<static_cast<unsigned>(ceil_div(KW, 64)), 64 * kRedWaves, 0, st>>>(w.gpart, nwg, KW, w.gAB);
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
    kb_reduce<<<static_cast<unsigned>(ceil_div(KW, 64)), 64 * kRedWaves, 0, st>>>(w.gpart, nwg, KW, w.gAB);
  } else {
    kb_zero<<<static_cast<unsigned>(ceil_div(KW, 256)), 256, 0, st>>>(w.gAB, KW);
    if (p.metric == SIL_SQEUCLID)
      kb_accum_global<SIL_SQEUCLID><<<nwg, 64 * kBwdWaves, 0, st>>>(a);
    else
      kb_accum_global<SIL_COSINE><<<nwg, 64 * kBwdWaves, 0, st>>>(a);
  }
  a.gtab = w.gtab;
  a.htab = w.gtab + static_cast<int64_t>(p.K) * p.DPX;
  kb_gtab<<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(p.K) * p.DPX, 256)), 256, 0, st>>>(
      a, p.metric);
  const int64_t nrows = ceil_div(p.N, 4 * kDxRows);
  const unsigned gdx = static_cast<unsigned>(nrows < 8192 ? nrows : 8192);
  const bool vec4 = p.D % 4 == 0 && p.D > 128 && reinterpret_cast<uintptr_t>(p.X) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(dX) % 16 == 0;
  if (p.metric == SIL_SQEUCLID) {
    if (vec4)
      kb_dx4<SIL_SQEUCLID><<<gdx, 256, 0, st>>>(a);
    else
      kb_dx<SIL_SQEUCLID><<<gdx, 256, 0, st>>>(a);
  } else {
    if (vec4)
      kb_dx4<SIL_COSINE><<<gdx, 256, 0, st>>>(a);
    else
      kb_dx<SIL_COSINE><<<gdx, 256, 0, st>>>(a);
  }
  (void)L;
  return hipGetLastError();
}

}  // namespace sil
