// Pass 1 of the method: per-cluster statistics in one pass over the points.
//
//   N_k                       cluster sizes
//   Y_k   = sum_{j in k} x_j                  (Eq.8)       squared Euclidean
//   Psi_k = sum_{j in k} ||x_j||^2            (Eq.5, Eq.6)
//   Omega_k = sum_{j in k} x_j / ||x_j||      (Eq.15, Eq.16) cosine
//   sum_{j in k} log x_j, sum_{j in k} sum_l x_jl              generalized KL (the Bregman
//                                              statistics of the divergence; positive entries;
//                                              each log in fp32 (the entries are fp32 or bf16
//                                              values), the sums in FP64)
//
// The paper accumulates Y and Psi together in one pass with per-worker partial sums that one
// node then adds up (footnotes to Eq.6 and Eq.9).  On the GPU the "workers" are waves, and the
// per-cluster sums are made contention-free by a counting sort of the row ids by label:
//   k_hist_lds  label histogram (LDS-privatised, validates labels; k_hist above 16384 clusters)
//   k_scan      exclusive prefix of N_k -> start of every cluster in sorted order
//   k_scatter_staged  row ids scattered to their cluster's range, each chunk counting-sorted in
//               LDS first (k_scatter, one reservation per row, above 4096 clusters)
//   k_segreduce each wave owns kSegLen consecutive sorted positions and accumulates the rows it
//               gathers in FP64 registers; a run of one cluster that lies wholly inside the
//               segment is stored directly, a run cut by a segment border goes to one of two
//               partial slots of the segment
//   k_combine   adds the partial slots of clusters that span several segments, in segment order
// No floating-point atomics are used, so the sums do not depend on the schedule except through
// the order of rows within a cluster, which the scatter leaves unspecified.
#include <algorithm>

#include "sil_internal.h"

namespace sil {

// ------------------------------------------------------------------------------------------
// element decoding (storage -> float)

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// OCP FP8 E4M3 ("fn": bias 7, no infinities, S.1111.111 is NaN, exponent 0 is subnormal), by
// the hardware conversion: gfx950's v_cvt_[pk_]f32_fp8 read the OCP encoding, and decode all 256
// codes to the values the format defines (checked bit for bit on the device, NaN codes and the
// zero's sign included).
typedef float f32x2_s __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float e4m3_to_f32(uint8_t q) {
  return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(q), 0);
}
// the four codes of a 32-bit word, lowest byte first
__device__ __forceinline__ void e4m3x4_to_f32(uint32_t w, float* out) {
  const f32x2_s lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), false);
  const f32x2_s hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), true);
  out[0] = lo[0];
  out[1] = lo[1];
  out[2] = hi[0];
  out[3] = hi[1];
}

// Stored element as double; the fp8 code times its column scale is exact in binary64.
template <int DT>
__device__ __forceinline__ double load_elem(const void* X, const float* col_scale, int64_t row,
                                            int32_t D, int32_t col) {
  const int64_t idx = row * static_cast<int64_t>(D) + col;
  if constexpr (DT == SIL_F32) {
    return static_cast<double>(static_cast<const float*>(X)[idx]);
  } else if constexpr (DT == SIL_BF16) {
    return static_cast<double>(bf16_bits_to_f32(static_cast<const uint16_t*>(X)[idx]));
  } else {
    return static_cast<double>(e4m3_to_f32(static_cast<const uint8_t*>(X)[idx])) *
           static_cast<double>(col_scale[col]);
  }
}

// ------------------------------------------------------------------------------------------

__device__ __forceinline__ void fill_zero_body(uint32_t* __restrict__ p, int64_t n_words,
                                               int64_t bid, int64_t nblk) {
  const int64_t stride = nblk * blockDim.x;
  for (int64_t i = bid * blockDim.x + threadIdx.x; i < n_words; i += stride) p[i] = 0u;
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, int64_t n_words) {
  fill_zero_body(p, n_words, blockIdx.x, gridDim.x);
}

// Label histogram; labels outside [0, K) are skipped and reported.
__device__ __forceinline__ void hist_body(const int32_t* __restrict__ labels, int64_t N, int32_t K,
                                          int32_t* __restrict__ count, int32_t* __restrict__ hdr,
                                          int64_t bid, int32_t* sh) {
  const bool in_lds = K <= kLdsHistMaxK;
  const int64_t c0 = bid * kChunk;
  const int64_t c1 = min(N, c0 + static_cast<int64_t>(kChunk));
  if (in_lds) {
    for (int k = threadIdx.x; k < K; k += blockDim.x) sh[k] = 0;
    __syncthreads();
  }
  bool bad = false;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    const int32_t k = labels[i];
    if (k < 0 || k >= K) {
      bad = true;
      continue;
    }
    if (in_lds)
      atomicAdd(&sh[k], 1);
    else
      atomicAdd(&count[k], 1);
  }
  if (bad) set_status(hdr, SIL_E_LABEL);
  if (in_lds) {
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x)
      if (sh[k]) atomicAdd(&count[k], sh[k]);
  }
}

__global__ __launch_bounds__(256) void k_hist(const int32_t* __restrict__ labels, int64_t N,
                                              int32_t K, int32_t* __restrict__ count,
                                              int32_t* __restrict__ hdr) {
  extern __shared__ int32_t sh_dyn[];
  hist_body(labels, N, K, count, hdr, blockIdx.x, sh_dyn);
}

// The sort passes for K <= kLdsHistMaxK run kSortThreads per workgroup and read the labels four
// at a time: one 16-byte load when the labels start at a 16-byte aligned address (uniform over
// the grid), four 4-byte loads otherwise and at the end of the array.  Positions past N read as
// -1 and are never counted.
constexpr int kSortThreads = 1024;

__device__ __forceinline__ int4 load_label4(const int32_t* __restrict__ labels, int64_t N,
                                            int64_t i, bool vec) {
  if (vec && i + 3 < N) return *reinterpret_cast<const int4*>(labels + i);
  int4 v;
  v.x = i < N ? labels[i] : -1;
  v.y = i + 1 < N ? labels[i + 1] : -1;
  v.z = i + 2 < N ? labels[i + 2] : -1;
  v.w = i + 3 < N ? labels[i + 3] : -1;
  return v;
}

// Label histogram, K <= kLdsHistMaxK: CHUNK labels per workgroup, every load issued before the
// first LDS atomic, then one global atomic per cluster present in the chunk.  Large chunks keep
// the number of global atomics on each count (one per workgroup) low.
// chunk `bid` of CHUNK labels, by a workgroup of kSortThreads; sh_dyn: K ints of LDS
template <int CHUNK>
__device__ __forceinline__ void hist_lds_body(const int32_t* __restrict__ labels, int64_t N,
                                              int32_t K, int32_t* __restrict__ count,
                                              int32_t* __restrict__ hdr, int64_t bid,
                                              int32_t* sh_dyn) {
  constexpr int PER = CHUNK / (kSortThreads * 4);
  const int t = threadIdx.x;
  const int64_t c0 = bid * CHUNK;
  const bool vec = (reinterpret_cast<uintptr_t>(labels) & 15) == 0;
  for (int k = t; k < K; k += kSortThreads) sh_dyn[k] = 0;
  int4 v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u)
    v[u] = load_label4(labels, N, c0 + static_cast<int64_t>(u * kSortThreads + t) * 4, vec);
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = c0 + static_cast<int64_t>(u * kSortThreads + t) * 4;
    const int32_t a[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (i + e >= N) continue;
      if (a[e] < 0 || a[e] >= K)
        bad = true;
      else
        atomicAdd(&sh_dyn[a[e]], 1);
    }
  }
  if (bad) set_status(hdr, SIL_E_LABEL);
  __syncthreads();
  for (int k = t; k < K; k += kSortThreads)
    if (const int32_t n = sh_dyn[k]) atomicAdd(&count[k], n);
}

template <int CHUNK>
__global__ __launch_bounds__(kSortThreads) void k_hist_lds(const int32_t* __restrict__ labels,
                                                           int64_t N, int32_t K,
                                                           int32_t* __restrict__ count,
                                                           int32_t* __restrict__ hdr) {
  extern __shared__ int32_t sh_dyn[];
  hist_lds_body<CHUNK>(labels, N, K, count, hdr, blockIdx.x, sh_dyn);
}

// Exclusive prefix of the cluster sizes, scatter cursors, number of valid points and of
// non-empty clusters (fewer than min_nonempty is an error).  One workgroup of 1024 threads.
__device__ __forceinline__ void scan_body(const int32_t* __restrict__ count, int32_t K,
                                          int32_t* __restrict__ offset, int32_t* __restrict__ cursor,
                                          int32_t* __restrict__ hdr, int min_nonempty) {
  __shared__ int32_t part[1024];
  __shared__ int32_t nz[1024];
  const int t = threadIdx.x;
  const int per = static_cast<int>((K + 1023) / 1024);
  const int k0 = min(K, t * per), k1 = min(K, k0 + per);
  int32_t sum = 0, nonempty = 0;
  for (int k = k0; k < k1; ++k) {
    sum += count[k];
    nonempty += count[k] > 0;
  }
  part[t] = sum;
  nz[t] = nonempty;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 partial sums
  for (int d = 1; d < 1024; d <<= 1) {
    const int32_t v = t >= d ? part[t - d] : 0;
    const int32_t w = t >= d ? nz[t - d] : 0;
    __syncthreads();
    part[t] += v;
    nz[t] += w;
    __syncthreads();
  }
  int32_t run = part[t] - sum;  // exclusive
  for (int k = k0; k < k1; ++k) {
    offset[k] = run;
    cursor[k] = run;
    run += count[k];
  }
  if (t == 1023) {
    offset[K] = part[1023];
    hdr[1] = part[1023];
    hdr[2] = nz[1023];
    if (nz[1023] < min_nonempty) set_status(hdr, SIL_E_FEW_CLUSTERS);
  }
}

__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ count, int32_t K,
                                               int32_t* __restrict__ offset,
                                               int32_t* __restrict__ cursor,
                                               int32_t* __restrict__ hdr, int min_nonempty) {
  scan_body(count, K, offset, cursor, hdr, min_nonempty);
}

// Scatter row ids into their cluster's range of the sorted order.
__device__ __forceinline__ void scatter_body(const int32_t* __restrict__ labels, int64_t N,
                                             int32_t K, int32_t* __restrict__ cursor,
                                             int32_t* __restrict__ perm,
                                             int32_t* __restrict__ lsorted, int64_t bid,
                                             int32_t* sh) {
  const bool in_lds = K <= kLdsHistMaxK;
  const int64_t c0 = bid * kChunk;
  const int64_t c1 = min(N, c0 + static_cast<int64_t>(kChunk));
  if (in_lds) {
    for (int k = threadIdx.x; k < K; k += blockDim.x) sh[k] = 0;
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
      const int32_t k = labels[i];
      if (k >= 0 && k < K) atomicAdd(&sh[k], 1);
    }
    __syncthreads();
    // reserve one block of positions per cluster present in this chunk
    for (int k = threadIdx.x; k < K; k += blockDim.x)
      if (sh[k]) sh[k] = atomicAdd(&cursor[k], sh[k]);
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
      const int32_t k = labels[i];
      if (k >= 0 && k < K) {
        const int32_t pos = atomicAdd(&sh[k], 1);
        perm[pos] = static_cast<int32_t>(i);
        lsorted[pos] = k;
      }
    }
  } else {
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
      const int32_t k = labels[i];
      if (k >= 0 && k < K) {
        const int32_t pos = atomicAdd(&cursor[k], 1);
        perm[pos] = static_cast<int32_t>(i);
        lsorted[pos] = k;
      }
    }
  }
}

// Exclusive prefix of one int per thread over a workgroup of THREADS; wsum holds THREADS/64 ints
// of LDS; *total receives the workgroup's sum.
template <int THREADS>
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* wsum, int32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < THREADS / 64; ++w) {
    const int32_t s = wsum[w];
    before += w < wv ? s : 0;
    tot += s;
  }
  *total = tot;
  return before + inc - v;
}

// The same scatter with the chunk sorted in LDS first (K <= kStageMaxK): the chunk's rows are
// counted per cluster, the counts scanned into local offsets, each present cluster's block of
// positions reserved once, the rows placed in LDS by cluster, and the chunk written out in that
// order.  A cluster's rows then go to consecutive positions from consecutive lanes, so the
// stores coalesce into whole-line writes instead of one 4-byte request per row; the larger the
// chunk, the longer those runs and the fewer the reservations.  A staged row is one word, its
// cluster in the high half and its offset in the chunk in the low half; LDS: 4 CHUNK + 8 K bytes.
constexpr int kStageMaxK = 4096;
constexpr int kStageBig = 32768, kStageSmall = 16384;  // labels per workgroup
constexpr int stage_lds(int chunk, int K) { return (chunk + 2 * K) * 4; }
static_assert(stage_lds(kStageBig, kStageMaxK) <= 160 * 1024, "staged scatter exceeds the LDS");

// chunk `bid` of CHUNK labels, by a workgroup of kSortThreads; st_dyn: stage_lds(CHUNK, K) bytes
template <int CHUNK>
__device__ __forceinline__ void scatter_staged_body(
    const int32_t* __restrict__ labels, int64_t N, int32_t K, int32_t* __restrict__ cursor,
    int32_t* __restrict__ perm, int32_t* __restrict__ lsorted, int64_t bid, uint32_t* st_dyn) {
  static_assert(CHUNK <= 65536, "row offset in the low half of a staged word");
  constexpr int PER = CHUNK / (kSortThreads * 4);
  uint32_t* staged = st_dyn;                                    // [CHUNK]
  int32_t* cnt = reinterpret_cast<int32_t*>(st_dyn + CHUNK);    // [K] counts, then cursors
  int32_t* delta = cnt + K;                                     // [K] global - local position
  int32_t* wsum = reinterpret_cast<int32_t*>(st_dyn);           // scan scratch, before placement
  const int t = threadIdx.x;
  const int64_t c0 = bid * CHUNK;
  const bool vec = (reinterpret_cast<uintptr_t>(labels) & 15) == 0;
  for (int k = t; k < K; k += kSortThreads) cnt[k] = 0;
  int4 v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u)
    v[u] = load_label4(labels, N, c0 + static_cast<int64_t>(u * kSortThreads + t) * 4, vec);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    int32_t* a = reinterpret_cast<int32_t*>(&v[u]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (a[e] < 0 || a[e] >= K) a[e] = -1;  // past N, or invalid (the histogram reports it)
      if (a[e] >= 0) atomicAdd(&cnt[a[e]], 1);
    }
  }
  __syncthreads();
  const int seg = (K + kSortThreads - 1) / kSortThreads;
  const int k0 = min(K, t * seg), k1 = min(K, k0 + seg);
  int32_t sum = 0;
  for (int k = k0; k < k1; ++k) sum += cnt[k];
  int32_t nvalid;
  int32_t run = block_excl_scan<kSortThreads>(sum, wsum, &nvalid);
  for (int k = k0; k < k1; ++k) {
    const int32_t n = cnt[k];
    if (n) delta[k] = atomicAdd(&cursor[k], n) - run;
    cnt[k] = run;  // placement cursor
    run += n;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int32_t* a = reinterpret_cast<const int32_t*>(&v[u]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (a[e] >= 0) {
        const int32_t slot = atomicAdd(&cnt[a[e]], 1);
        staged[slot] = (static_cast<uint32_t>(a[e]) << 16) |
                       static_cast<uint32_t>((u * kSortThreads + t) * 4 + e);
      }
    }
  }
  __syncthreads();
  for (int j = t; j < nvalid; j += kSortThreads) {
    const uint32_t w = staged[j];
    const int32_t k = static_cast<int32_t>(w >> 16);
    const int32_t pos = delta[k] + j;
    perm[pos] = static_cast<int32_t>(c0 + (w & 0xffffu));
    lsorted[pos] = k;
  }
}

template <int CHUNK>
__global__ __launch_bounds__(kSortThreads) void k_scatter_staged(
    const int32_t* __restrict__ labels, int64_t N, int32_t K, int32_t* __restrict__ cursor,
    int32_t* __restrict__ perm, int32_t* __restrict__ lsorted) {
  extern __shared__ uint32_t st_dyn[];
  scatter_staged_body<CHUNK>(labels, N, K, cursor, perm, lsorted, blockIdx.x, st_dyn);
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ labels, int64_t N,
                                                 int32_t K, int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ perm,
                                                 int32_t* __restrict__ lsorted) {
  extern __shared__ int32_t sh_dyn[];
  scatter_body(labels, N, K, cursor, perm, lsorted, blockIdx.x, sh_dyn);
}

// zero is done; histogram, scan and scatter
static hipError_t launch_hist_scatter(const Problem& p, const WsPtrs& w, hipStream_t st) {
  const unsigned nchunk = static_cast<unsigned>(ceil_div(p.N, kChunk));
  if (p.K <= kLdsHistMaxK) {
    const size_t lds = static_cast<size_t>(p.K) * 4;
    if (p.N >= (int64_t{1} << 24))  // enough 64K-label chunks to fill the chip
      k_hist_lds<65536><<<static_cast<unsigned>(ceil_div(p.N, 65536)), kSortThreads, lds, st>>>(
          p.labels, p.N, p.K, w.count, w.hdr);
    else
      k_hist_lds<16384><<<static_cast<unsigned>(ceil_div(p.N, 16384)), kSortThreads, lds, st>>>(
          p.labels, p.N, p.K, w.count, w.hdr);
  } else {
    k_hist<<<nchunk, 256, 0, st>>>(p.labels, p.N, p.K, w.count, w.hdr);
  }
  k_scan<<<1, 1024, 0, st>>>(w.count, p.K, w.offset, w.cursor, w.hdr, p.min_nonempty);
  if (p.K <= kStageMaxK) {
    static bool lds_set = false;  // above 64 KB of dynamic LDS the kernels must say so once
    if (!lds_set) {
      for (const void* f : {reinterpret_cast<const void*>(&k_scatter_staged<kStageBig>),
                            reinterpret_cast<const void*>(&k_scatter_staged<kStageSmall>)}) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 stage_lds(kStageBig, kStageMaxK));
        if (e != hipSuccess) return e;
      }
      lds_set = true;
    }
    // the larger chunk where the reservations dominate (many clusters) and it still makes at
    // least one workgroup per compute unit
    if (p.K >= 512 && p.N >= int64_t{256} * kStageBig)
      k_scatter_staged<kStageBig><<<static_cast<unsigned>(ceil_div(p.N, kStageBig)), kSortThreads,
                                    stage_lds(kStageBig, p.K), st>>>(p.labels, p.N, p.K, w.cursor,
                                                                     w.perm, w.lsorted);
    else
      k_scatter_staged<kStageSmall><<<static_cast<unsigned>(ceil_div(p.N, kStageSmall)),
                                      kSortThreads, stage_lds(kStageSmall, p.K), st>>>(
          p.labels, p.N, p.K, w.cursor, w.perm, w.lsorted);
  } else {
    const size_t lds = p.K <= kLdsHistMaxK ? static_cast<size_t>(p.K) * 4 : 0;
    k_scatter<<<nchunk, 256, lds, st>>>(p.labels, p.N, p.K, w.cursor, w.perm, w.lsorted);
  }
  return hipSuccess;
}

// Cluster whose sorted range contains position q (0 <= q < offset[K]): the largest k with
// offset[k] <= q, which skips empty clusters.
__device__ __forceinline__ int32_t find_cluster(const int32_t* __restrict__ offset, int32_t K,
                                                int64_t q) {
  int32_t lo = 0, hi = K;  // offset[lo] <= q < offset[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (offset[mid] <= q)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ double shfl_xor_f64(double v, int m) {
  return __shfl_xor(v, m, 64);
}

// One wave per segment of kSegLen sorted positions.  A group of G lanes handles one row at a
// time (lane covers E consecutive columns), RPW = 64/G rows per step.
template <int DT, int METRIC>
__device__ __forceinline__ void segreduce_body(
    const void* __restrict__ X, const float* __restrict__ col_scale,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ offset, int32_t K, int32_t D,
    int G, int E, int64_t nseg, double* __restrict__ V, double* __restrict__ psi,
    double* __restrict__ segpart, int32_t* __restrict__ hdr, int64_t bid) {
  const int lane = threadIdx.x & 63;
  const int64_t seg = bid * 4 + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int64_t nvalid = hdr[1];
  const int64_t p0 = seg * kSegLen;
  const int64_t p1 = min(nvalid, p0 + static_cast<int64_t>(kSegLen));
  if (p0 >= p1) return;
  const int RPW = 64 / G;
  const int g = lane / G, lig = lane % G;

  int32_t kc = find_cluster(offset, K, p0);
  int64_t rs = offset[kc], re = offset[kc + 1];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double accq = 0.0;
  bool bad_value = false, zero_norm = false, domain = false;

  auto flush = [&]() {
    for (int off = G; off < 64; off <<= 1)
      for (int e = 0; e < 4; ++e) acc[e] += shfl_xor_f64(acc[e], off);
    for (int off = 1; off < 64; off <<= 1) accq += shfl_xor_f64(accq, off);
    double* dst;
    double* dpsi;
    if (rs >= p0 && re <= p1) {  // the whole cluster lies in this segment
      dst = V + static_cast<int64_t>(kc) * D;
      dpsi = psi + kc;
    } else {
      const int slot = rs <= p0 ? 0 : 1;  // run through p0 -> slot 0, run past p1 -> slot 1
      dst = segpart + (seg * 2 + slot) * static_cast<int64_t>(D + 1);
      dpsi = dst + D;
    }
    if (g == 0)
      for (int e = 0; e < E; ++e) {
        const int col = lig * E + e;
        if (col < D) dst[col] = acc[e];
      }
    if (lane == 0) *dpsi = accq;
    for (int e = 0; e < 4; ++e) acc[e] = 0.0;
    accq = 0.0;
  };

  for (int64_t p = p0; p < p1; p += RPW) {
    const int64_t pos = p + g;
    const bool valid = pos < p1;
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    double sq = 0.0;
    if (valid) {
      const int64_t row = perm[pos];
      for (int e = 0; e < E; ++e) {
        const int col = lig * E + e;
        if (col < D) {
          const double v = load_elem<DT>(X, col_scale, row, D, col);
          bad_value |= !isfinite(v);
          if constexpr (METRIC == SIL_KL) {  // sum log y and sum_l y (positive entries only)
            domain |= !(v > 0.0);
            x[e] = v > 0.0 ? static_cast<double>(logf(static_cast<float>(v))) : 0.0;
            sq += v;
          } else {
            x[e] = v;
            sq = fma(x[e], x[e], sq);
          }
        }
      }
    }
    // row norm over the G lanes of the group
    double rowsq = sq;
    for (int off = 1; off < G; off <<= 1) rowsq += shfl_xor_f64(rowsq, off);
    if constexpr (METRIC == SIL_COSINE) {
      if (valid && rowsq == 0.0) zero_norm = true;
      const double inv = rsqrt(rowsq);  // 1 / |x| to an ulp or two
      for (int e = 0; e < 4; ++e) x[e] *= inv;
    }
    bool done = !valid;
    while (true) {
      if (!done && pos < re) {
        for (int e = 0; e < 4; ++e) acc[e] += x[e];
        if constexpr (METRIC != SIL_COSINE) accq += sq;
        done = true;
      }
      if (__all(done)) break;
      flush();
      kc = find_cluster(offset, K, re);
      rs = offset[kc];
      re = offset[kc + 1];
    }
  }
  flush();
  if (bad_value) set_status(hdr, SIL_E_NONFINITE);
  if (zero_norm) set_status(hdr, SIL_E_ZERO_NORM);
  if (domain) set_status(hdr, SIL_E_DOMAIN);
}

template <int DT, int METRIC>
__global__ __launch_bounds__(256) void k_segreduce(
    const void* __restrict__ X, const float* __restrict__ col_scale,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ offset, int32_t K, int32_t D,
    int G, int E, int64_t nseg, double* __restrict__ V, double* __restrict__ psi,
    double* __restrict__ segpart, int32_t* __restrict__ hdr) {
  segreduce_body<DT, METRIC>(X, col_scale, perm, offset, K, D, G, E, nseg, V, psi, segpart, hdr,
                             blockIdx.x);
}

// Same reduction with 16-byte row chunks and U rows in flight per lane: a lane holds E = 16 /
// sizeof(element) consecutive columns (fp32 4, bf16 8, fp8 16), a group of G = D / E lanes one
// row (G a power of two <= 64), RPW = 64 / G rows per wave step, U steps per batch.  A batch
// whose positions all lie in the current run takes the fast path; otherwise each step is
// handled as in k_segreduce.
typedef uint32_t u32x4_s __attribute__((ext_vector_type(4)));

template <int DT>
__device__ __forceinline__ void decode16(u32x4_s raw, const float* __restrict__ col_scale,
                                         int c0, double* x) {
  if constexpr (DT == SIL_F32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = static_cast<double>(__uint_as_float(raw[e]));
  } else if constexpr (DT == SIL_BF16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x[2 * e] = static_cast<double>(__uint_as_float(raw[e] << 16));
      x[2 * e + 1] = static_cast<double>(__uint_as_float(raw[e] & 0xffff0000u));
    }
  } else {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      float f[4];
      e4m3x4_to_f32(raw[w], f);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        x[4 * w + i] = static_cast<double>(f[i]) * static_cast<double>(col_scale[c0 + 4 * w + i]);
    }
  }
}

template <int DT, int METRIC>
__device__ __forceinline__ void segreduce_vec_body(
    const void* __restrict__ X, const float* __restrict__ col_scale,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ offset, int32_t K, int32_t D,
    int G, int64_t nseg, double* __restrict__ V, double* __restrict__ psi,
    double* __restrict__ segpart, int32_t* __restrict__ hdr, int64_t bid) {
  constexpr int E = DT == SIL_F32 ? 4 : DT == SIL_BF16 ? 8 : 16;
  constexpr int ESZ = 16 / E;
  constexpr int U = DT == SIL_FP8_E4M3 ? 4 : 8;  // rows in flight per lane
  const int lane = threadIdx.x & 63;
  const int64_t seg = bid * 4 + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int64_t nvalid = hdr[1];
  const int64_t p0 = seg * kSegLen;
  const int64_t p1 = min(nvalid, p0 + static_cast<int64_t>(kSegLen));
  if (p0 >= p1) return;
  const int RPW = 64 / G;
  const int g = lane / G, lig = lane % G;
  const int c0 = lig * E;
  const char* Xb = static_cast<const char*>(X);

  int32_t kc = find_cluster(offset, K, p0);
  int64_t rs = offset[kc], re = offset[kc + 1];
  double acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0;
  double accq = 0.0;
  bool bad_value = false, zero_norm = false, domain = false;

  auto flush = [&]() __attribute__((always_inline)) {
    for (int off = G; off < 64; off <<= 1)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] += shfl_xor_f64(acc[e], off);
    for (int off = 1; off < 64; off <<= 1) accq += shfl_xor_f64(accq, off);
    double* dst;
    double* dpsi;
    if (rs >= p0 && re <= p1) {
      dst = V + static_cast<int64_t>(kc) * D;
      dpsi = psi + kc;
    } else {
      const int slot = rs <= p0 ? 0 : 1;
      dst = segpart + (seg * 2 + slot) * static_cast<int64_t>(D + 1);
      dpsi = dst + D;
    }
    if (g == 0)
#pragma unroll
      for (int e = 0; e < E; ++e) dst[c0 + e] = acc[e];
    if (lane == 0) *dpsi = accq;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    accq = 0.0;
  };

  // row -> E values (scaled to unit norm for cosine) and the row's sum of squares
  auto prepare = [&](u32x4_s raw, bool valid, double* x, double& sq) __attribute__((always_inline)) {
    decode16<DT>(raw, col_scale, c0, x);
    sq = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      bad_value |= valid && !isfinite(x[e]);
      if constexpr (METRIC == SIL_KL) {  // sum log y and sum_l y (positive entries only)
        domain |= valid && !(x[e] > 0.0);
        sq += x[e];
        x[e] = x[e] > 0.0 ? static_cast<double>(logf(static_cast<float>(x[e]))) : 0.0;
      } else {
        sq = fma(x[e], x[e], sq);
      }
    }
    if constexpr (METRIC == SIL_COSINE) {
      double rowsq = sq;
      for (int off = 1; off < G; off <<= 1) rowsq += shfl_xor_f64(rowsq, off);
      if (valid && rowsq == 0.0) zero_norm = true;
      const double inv = valid ? rsqrt(rowsq) : 0.0;  // 1 / |x| to an ulp or two
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] *= inv;
    }
  };

  const int64_t batch = static_cast<int64_t>(U) * RPW;
  for (int64_t p = p0; p < p1; p += batch) {
    u32x4_s raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t pos = p + u * RPW + g;
      valid[u] = pos < p1;
      const int64_t row = valid[u] ? perm[pos] : 0;
      raw[u] = valid[u] ? *reinterpret_cast<const u32x4_s*>(Xb + (row * D + c0) * ESZ)
                        : u32x4_s{0u, 0u, 0u, 0u};
    }
    if (p + batch <= re && p + batch <= p1) {  // the whole batch belongs to the current run
#pragma unroll
      for (int u = 0; u < U; ++u) {
        double x[E], sq;
        prepare(raw[u], true, x, sq);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] += x[e];
        if constexpr (METRIC != SIL_COSINE) accq += sq;
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t pos = p + u * RPW + g;
      double x[E], sq;
      prepare(raw[u], valid[u], x, sq);
      bool done = !valid[u];
      while (true) {
        if (!done && pos < re) {
#pragma unroll
          for (int e = 0; e < E; ++e) acc[e] += x[e];
          if constexpr (METRIC != SIL_COSINE) accq += sq;
          done = true;
        }
        if (__all(done)) break;
        flush();
        kc = find_cluster(offset, K, re);
        rs = offset[kc];
        re = offset[kc + 1];
      }
    }
  }
  flush();
  if (bad_value) set_status(hdr, SIL_E_NONFINITE);
  if (zero_norm) set_status(hdr, SIL_E_ZERO_NORM);
  if (domain) set_status(hdr, SIL_E_DOMAIN);
}

template <int DT, int METRIC>
__global__ __launch_bounds__(256) void k_segreduce_vec(
    const void* __restrict__ X, const float* __restrict__ col_scale,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ offset, int32_t K, int32_t D,
    int G, int64_t nseg, double* __restrict__ V, double* __restrict__ psi,
    double* __restrict__ segpart, int32_t* __restrict__ hdr) {
  segreduce_vec_body<DT, METRIC>(X, col_scale, perm, offset, K, D, G, nseg, V, psi, segpart, hdr,
                                 blockIdx.x);
}

// Squared Euclidean statistics of fp32 or bf16 rows of RB = 64 * CH bytes (CH = 4, 8 or 16):
// the whole wave reads one row per step, lane l holding the CH bytes at offset l * CH, so a lane
// always owns the same E = CH / sizeof(element) columns and every lane sees the same row.  The
// sorted positions are wave-uniform: row ids come from scalar loads of perm, run boundaries are
// scalar branches, and Psi is reduced across the wave only when a run is stored.  Batches of U
// rows are double-buffered: the rows of batch t + 1 and the ids of batch t + 2 are in flight
// while batch t is accumulated.  Runs are stored as in k_segreduce.  METRIC is the squared
// Euclidean distance (sums of x and ||x||^2), KL (sums of log x and of the entries) or cosine
// (sums of x / ||x||).  For cosine the norms of a batch's U rows are reduced across the wave
// together: each halving step exchanges half of a lane's remaining row sums with the partner
// lane, so U rows cost about U FP64 exchanges instead of 6 U; lane l ends with the norm of row
// (l >> (6 - log2 U)), and each row's 1 / ||x|| is read from its lane with readlane.
template <int DT, int CH, int METRIC = SIL_SQEUCLID>
__device__ __forceinline__ void segreduce_row_body(
    const void* __restrict__ X, const float* __restrict__ col_scale,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ offset, int32_t K, int32_t D,
    int64_t nseg, double* __restrict__ V, double* __restrict__ psi,
    double* __restrict__ segpart, int32_t* __restrict__ hdr, int64_t bid) {
  static_assert(DT == SIL_F32 || DT == SIL_BF16 || (DT == SIL_FP8_E4M3 && CH <= 4), "row form");
  static_assert(METRIC == SIL_SQEUCLID || METRIC == SIL_KL || METRIC == SIL_COSINE, "metric");
  constexpr int ESZ = DT == SIL_F32 ? 4 : DT == SIL_BF16 ? 2 : 1;
  constexpr int E = CH / ESZ;
  constexpr int NW = CH >= 4 ? CH / 4 : 1;  // 32-bit words per lane (fp8 rows of 128 B: half of one)
  // rows per batch; cosine and 4-byte fp8 chunks halve it (the row sums and norms, or the
  // decoded values, would need twice the registers)
  constexpr int U = (NW == 1 ? 16 : NW == 2 ? 8 : 4) / (METRIC == SIL_COSINE ? 2 : 1) /
                    (DT == SIL_FP8_E4M3 && CH == 4 ? 2 : 1);
  constexpr int64_t RB = 64 * CH;
  typedef uint32_t chunk_t __attribute__((ext_vector_type(NW == 1 ? 2 : NW)));
  const int lane = threadIdx.x & 63;
  const int64_t seg = bid * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int64_t nvalid = hdr[1];
  const int64_t p0 = seg * kSegLen;
  const int64_t p1 = min(nvalid, p0 + static_cast<int64_t>(kSegLen));
  if (p0 >= p1) return;
  const char* Xl = static_cast<const char*>(X) + lane * CH;
  // fp8: the lane's columns lane * E .. + E keep their scales for every row
  float sc[DT == SIL_FP8_E4M3 ? E : 1];
  if constexpr (DT == SIL_FP8_E4M3) {
#pragma unroll
    for (int e = 0; e < E; ++e) sc[e] = col_scale[lane * E + e];
  }

  int32_t kc = find_cluster(offset, K, p0);
  int64_t rs = offset[kc], re = offset[kc + 1];
  double acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0;
  double accq = 0.0;
  bool bad_value = false, domain = false, zero_norm = false;

  auto flush = [&]() __attribute__((always_inline)) {
    for (int off = 1; off < 64; off <<= 1) accq += shfl_xor_f64(accq, off);
    double* dst;
    double* dpsi;
    if (rs >= p0 && re <= p1) {
      dst = V + static_cast<int64_t>(kc) * D;
      dpsi = psi + kc;
    } else {
      const int slot = rs <= p0 ? 0 : 1;
      dst = segpart + (seg * 2 + slot) * static_cast<int64_t>(D + 1);
      dpsi = dst + D;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) dst[lane * E + e] = acc[e];
    if (lane == 0) *dpsi = accq;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    accq = 0.0;
  };

  auto decode = [&](chunk_t raw, double* x) __attribute__((always_inline)) {
    if constexpr (DT == SIL_FP8_E4M3) {
      float f[4];
      e4m3x4_to_f32(raw[0], f);
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = static_cast<double>(f[e]) * static_cast<double>(sc[e]);
      return;
    }
#pragma unroll
    for (int w = 0; w < (NW == 1 ? 1 : NW); ++w) {
      if constexpr (DT == SIL_F32) {
        x[w] = static_cast<double>(__uint_as_float(raw[w]));
      } else if constexpr (DT == SIL_BF16) {
        x[2 * w] = static_cast<double>(__uint_as_float(raw[w] << 16));
        x[2 * w + 1] = static_cast<double>(__uint_as_float(raw[w] & 0xffff0000u));
      }
    }
  };
  // inv: 1 / ||x|| of the row (cosine only)
  auto add_row = [&](chunk_t raw, double inv) __attribute__((always_inline)) {
    double x[E];
    decode(raw, x);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      bad_value |= !isfinite(x[e]);
      if constexpr (METRIC == SIL_KL) {  // log in fp32 (x is an fp32 value), sums in FP64
        domain |= !(x[e] > 0.0);
        accq += x[e];
        acc[e] += x[e] > 0.0 ? static_cast<double>(logf(static_cast<float>(x[e]))) : 0.0;
      } else if constexpr (METRIC == SIL_COSINE) {
        acc[e] = fma(x[e], inv, acc[e]);
      } else {
        acc[e] += x[e];
        accq = fma(x[e], x[e], accq);
      }
    }
    if constexpr (METRIC == SIL_COSINE) zero_norm |= isinf(inv);
  };
  // 1 / ||x|| of the batch's U rows (cosine): the halving reduction described above
  constexpr int LU = U == 16 ? 4 : U == 8 ? 3 : U == 4 ? 2 : 1;
  static_assert((1 << LU) == U, "batch of 2, 4, 8 or 16 rows");
  auto row_inv = [&](const chunk_t* raw, double* inv) __attribute__((always_inline)) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double x[E];
      decode(raw[u], x);
      double sq = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) sq = fma(x[e], x[e], sq);
      v[u] = sq;
    }
#pragma unroll
    for (int st = 0; st < LU; ++st) {
      const int m = 32 >> st;
      const int half = U >> (st + 1);
      const bool up = (lane & m) != 0;
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const double send = up ? v[j] : v[j + half];
        const double keep = up ? v[j + half] : v[j];
        v[j] = keep + shfl_xor_f64(send, m);
      }
    }
#pragma unroll
    for (int m = 32 >> LU; m >= 1; m >>= 1) v[0] += shfl_xor_f64(v[0], m);
    const double mine = rsqrt(v[0]);  // row (lane >> (6 - LU)); +inf for a zero row
    const uint64_t b = __double_as_longlong(mine);
    const int lo = static_cast<int>(static_cast<uint32_t>(b)), hi = static_cast<int>(b >> 32);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t l = static_cast<uint32_t>(__builtin_amdgcn_readlane(lo, u << (6 - LU)));
      const uint32_t h = static_cast<uint32_t>(__builtin_amdgcn_readlane(hi, u << (6 - LU)));
      inv[u] = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(h) << 32) | l));
    }
  };

  // ids of the U positions from p; past p1 the last valid id is repeated and its row is loaded
  // but never accumulated
  auto fetch_ids = [&](int64_t p, int32_t* ids) __attribute__((always_inline)) {
    if (p + U <= p1) {
#pragma unroll
      for (int u = 0; u < U; ++u) ids[u] = perm[p + u];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) ids[u] = perm[min(p + u, p1 - 1)];
    }
  };
  auto fetch_rows = [&](const int32_t* ids, chunk_t* raw) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const char* src = Xl + static_cast<int64_t>(ids[u]) * RB;
      if constexpr (CH == 2)
        raw[u] = chunk_t{static_cast<uint32_t>(*reinterpret_cast<const uint16_t*>(src)), 0u};
      else if constexpr (NW == 1)
        raw[u] = chunk_t{*reinterpret_cast<const uint32_t*>(src), 0u};
      else
        raw[u] = *reinterpret_cast<const chunk_t*>(src);
    }
  };

  // The loads of the next batch are issued unconditionally (the last batch prefetches rows it
  // never uses) so that every iteration has the same loads in flight and the waits for batch t
  // leave batch t + 1 outstanding.
  int32_t ids[U];
  chunk_t raw[U];
  fetch_ids(p0, ids);
  fetch_rows(ids, raw);
  fetch_ids(p0 + U, ids);
  for (int64_t p = p0; p < p1; p += U) {
    chunk_t nxt[U];
    fetch_rows(ids, nxt);
    fetch_ids(p + 2 * U, ids);
    double inv[U];
    if constexpr (METRIC == SIL_COSINE) {
      row_inv(raw, inv);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) inv[u] = 1.0;
    }
    if (p + U <= re && p + U <= p1) {  // the whole batch belongs to the current run
#pragma unroll
      for (int u = 0; u < U; ++u) add_row(raw[u], inv[u]);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t pos = p + u;
        if (pos < p1) {
          while (pos >= re) {  // uniform: the run ends before this row
            flush();
            kc = find_cluster(offset, K, re);
            rs = offset[kc];
            re = offset[kc + 1];
          }
          add_row(raw[u], inv[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) raw[u] = nxt[u];
  }
  flush();
  if (bad_value) set_status(hdr, SIL_E_NONFINITE);
  if (zero_norm) set_status(hdr, SIL_E_ZERO_NORM);
  if (domain) set_status(hdr, SIL_E_DOMAIN);
}

template <int DT, int CH, int METRIC>
__global__ __launch_bounds__(256) void k_segreduce_row(
    const void* __restrict__ X, const float* __restrict__ col_scale, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ offset, int32_t K, int32_t D, int64_t nseg,
    double* __restrict__ V, double* __restrict__ psi, double* __restrict__ segpart,
    int32_t* __restrict__ hdr) {
  segreduce_row_body<DT, CH, METRIC>(X, col_scale, perm, offset, K, D, nseg, V, psi, segpart,
                                     hdr, blockIdx.x);
}

// Sums of clusters whose sorted range spans several segments.  One thread per (cluster,
// column), column D being Psi.
__device__ __forceinline__ void combine_body(const int32_t* __restrict__ offset, int32_t K,
                                             int32_t D, const double* __restrict__ segpart,
                                             double* __restrict__ V, double* __restrict__ psi,
                                             int64_t bid) {
  const int64_t t = bid * blockDim.x + threadIdx.x;
  const int64_t W = D + 1;
  if (t >= static_cast<int64_t>(K) * W) return;
  const int32_t k = static_cast<int32_t>(t / W);
  const int32_t col = static_cast<int32_t>(t % W);
  const int64_t a = offset[k], b = offset[k + 1];
  if (a == b) return;
  const int64_t s0 = a / kSegLen, s1 = (b - 1) / kSegLen;
  if (s0 == s1) return;
  // the largest cluster spans many segments: eight loads in flight at a time, each group added
  // in segment order (the same additions as one at a time)
  const int first = a != s0 * kSegLen ? 1 : 0;  // the first segment's slot
  double sum = 0.0;
  int64_t s = s0;
  for (; s + 7 <= s1; s += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = segpart[((s + u) * 2 + (s + u == s0 ? first : 0)) * W + col];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += v[u];
  }
  for (; s <= s1; ++s) sum += segpart[(s * 2 + (s == s0 ? first : 0)) * W + col];
  if (col < D)
    V[static_cast<int64_t>(k) * D + col] = sum;
  else
    psi[k] = sum;
}

__global__ __launch_bounds__(256) void k_combine(const int32_t* __restrict__ offset, int32_t K,
                                                 int32_t D, const double* __restrict__ segpart,
                                                 double* __restrict__ V,
                                                 double* __restrict__ psi) {
  combine_body(offset, K, D, segpart, V, psi, blockIdx.x);
}

// ------------------------------------------------------------------------------------------

template <int DT, int METRIC>
static void launch_seg_row(const Problem& p, const WsLayout& L, const WsPtrs& w, int ch,
                           unsigned nblk, hipStream_t st) {
#define SIL_ROW(CH)                                                                            \
  k_segreduce_row<DT, CH, METRIC><<<nblk, 256, 0, st>>>(p.X, p.col_scale, w.perm, w.offset, p.K, \
                                                        p.D, L.nseg, w.V, w.psi, w.segpart, w.hdr)
  if constexpr (DT == SIL_FP8_E4M3) {  // rows of 128 or 256 bytes
    if (ch == 2) SIL_ROW(2);
    else SIL_ROW(4);
  } else {
    if (ch == 4) SIL_ROW(4);
    else if (ch == 8) SIL_ROW(8);
    else SIL_ROW(16);
  }
#undef SIL_ROW
}

hipError_t launch_sort(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st) {
  const int64_t words = static_cast<int64_t>((L.perm - L.hdr) / 4);
  const int64_t zblocks = ceil_div(words, 256) < 2048 ? ceil_div(words, 256) : 2048;
  k_fill_zero<<<static_cast<unsigned>(zblocks), 256, 0, st>>>(
      reinterpret_cast<uint32_t*>(w.hdr), words);
  if (const hipError_t e = launch_hist_scatter(p, w, st); e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_stats(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st) {
  // zero [hdr, perm) (header .. segpart are contiguous in the layout), then the counting sort;
  // k_scan checks the non-empty clusters (the Silhouette needs a neighbouring cluster, a K-means
  // step one non-empty cluster)
  if (const hipError_t e = launch_sort(p, L, w, st); e != hipSuccess) return e;
  const unsigned nblk = static_cast<unsigned>(ceil_div(L.nseg, 4));
  // 16-byte chunks when a row splits into a power-of-two number of them
  int32_t Gv, G, E;
  stats_lanes(p.D, p.dtype, &Gv, &G, &E);
  const bool vec = Gv != 0;
  // whole-wave rows (fp32 or bf16 rows of 256, 512 or 1024 bytes; fp8 rows of 128 or 256)
  const int rowch = row_chunk(p.D, p.dtype);
#define SIL_SEG(DT, MT)                                                                         \
  do {                                                                                          \
    if (rowch)                                                                                  \
      launch_seg_row<DT, MT>(p, L, w, rowch, nblk, st);                                         \
    else if (vec)                                                                               \
      k_segreduce_vec<DT, MT><<<nblk, 256, 0, st>>>(p.X, p.col_scale, w.perm, w.offset, p.K,    \
                                                    p.D, Gv, L.nseg, w.V, w.psi, w.segpart,     \
                                                    w.hdr);                                     \
    else                                                                                        \
      k_segreduce<DT, MT><<<nblk, 256, 0, st>>>(p.X, p.col_scale, w.perm, w.offset, p.K, p.D, G, \
                                                E, L.nseg, w.V, w.psi, w.segpart, w.hdr);       \
  } while (0)
  if (p.metric == SIL_SQEUCLID) {
    if (p.dtype == SIL_F32) SIL_SEG(SIL_F32, SIL_SQEUCLID);
    else if (p.dtype == SIL_BF16) SIL_SEG(SIL_BF16, SIL_SQEUCLID);
    else SIL_SEG(SIL_FP8_E4M3, SIL_SQEUCLID);
  } else if (p.metric == SIL_KL) {  // fp32 or bf16 storage
    if (p.dtype == SIL_F32) SIL_SEG(SIL_F32, SIL_KL);
    else SIL_SEG(SIL_BF16, SIL_KL);
  } else {
    if (p.dtype == SIL_F32) SIL_SEG(SIL_F32, SIL_COSINE);
    else if (p.dtype == SIL_BF16) SIL_SEG(SIL_BF16, SIL_COSINE);
    else SIL_SEG(SIL_FP8_E4M3, SIL_COSINE);
  }
#undef SIL_SEG
  const int64_t nt = static_cast<int64_t>(p.K) * (p.D + 1);
  k_combine<<<static_cast<unsigned>(ceil_div(nt, 256)), 256, 0, st>>>(w.offset, p.K, p.D,
                                                                       w.segpart, w.V, w.psi);
  return hipGetLastError();
}


// ------------------------------------------------------------------------------------------
// batched statistics: every launch covers the work items of all problems of a batch; work item
// blockIdx.x belongs to the problem whose range in the phase's prefix contains it

__device__ __forceinline__ const BatchProblem& batch_item(const BatchDev& b, int phase,
                                                          int64_t* local) {
  const int32_t* pre = b.prefix + phase * (b.n + 1);
  const int32_t item = static_cast<int32_t>(blockIdx.x);
  const int j = batch_locate(pre, b.n, item);
  *local = item - pre[j];
  return b.prob[j];
}

__global__ __launch_bounds__(256) void kb_zero(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item(b, BP_ZERO, &it);
  const int64_t w0 = it * kZeroWordsPerItem;
  const int64_t n = q.zero_words - w0 < kZeroWordsPerItem ? q.zero_words - w0 : kZeroWordsPerItem;
  fill_zero_body(reinterpret_cast<uint32_t*>(q.hdr) + w0, n, 0, 1);
}

// kChunk labels per item (K <= kLdsHistMaxK for every batched problem)
__global__ __launch_bounds__(kSortThreads) void kb_hist(BatchDev b) {
  extern __shared__ int32_t sh_dyn[];
  int64_t it;
  const BatchProblem& q = batch_item(b, BP_HIST, &it);
  hist_lds_body<kChunk>(q.labels, q.N, q.K, q.count, q.hdr, it, sh_dyn);
}

__global__ __launch_bounds__(1024) void kb_scan(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item(b, BP_SCAN, &it);
  scan_body(q.count, q.K, q.offset, q.cursor, q.hdr, 2);
}

// kChunk labels per item, as the histogram: staged in LDS for K <= kStageMaxK
static_assert(kChunk == kStageSmall, "batched scatter items are staged chunks");
__global__ __launch_bounds__(kSortThreads) void kb_scatter(BatchDev b) {
  extern __shared__ int32_t sh_dyn[];
  int64_t it;
  const BatchProblem& q = batch_item(b, BP_HIST, &it);
  if (q.K <= kStageMaxK)
    scatter_staged_body<kStageSmall>(q.labels, q.N, q.K, q.cursor, q.perm, q.lsorted, it,
                                     reinterpret_cast<uint32_t*>(sh_dyn));
  else
    scatter_body(q.labels, q.N, q.K, q.cursor, q.perm, q.lsorted, it, sh_dyn);
}

// fp32 storage only (the batched path's storage type)
__global__ __launch_bounds__(256) void kb_seg(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item(b, BP_SEG, &it);
  if (q.metric == SIL_SQEUCLID) {
    if (q.rowch == 4)
      segreduce_row_body<SIL_F32, 4>(q.X, nullptr, q.perm, q.offset, q.K, q.D, q.nseg, q.V,
                                     q.psi, q.segpart, q.hdr, it);
    else if (q.rowch == 8)
      segreduce_row_body<SIL_F32, 8>(q.X, nullptr, q.perm, q.offset, q.K, q.D, q.nseg, q.V,
                                     q.psi, q.segpart, q.hdr, it);
    else if (q.Gv)
      segreduce_vec_body<SIL_F32, SIL_SQEUCLID>(q.X, q.col_scale, q.perm, q.offset, q.K, q.D, q.Gv,
                                                q.nseg, q.V, q.psi, q.segpart, q.hdr, it);
    else
      segreduce_body<SIL_F32, SIL_SQEUCLID>(q.X, q.col_scale, q.perm, q.offset, q.K, q.D, q.G, q.E,
                                            q.nseg, q.V, q.psi, q.segpart, q.hdr, it);
  } else {
    if (q.Gv)
      segreduce_vec_body<SIL_F32, SIL_COSINE>(q.X, q.col_scale, q.perm, q.offset, q.K, q.D, q.Gv,
                                              q.nseg, q.V, q.psi, q.segpart, q.hdr, it);
    else
      segreduce_body<SIL_F32, SIL_COSINE>(q.X, q.col_scale, q.perm, q.offset, q.K, q.D, q.G, q.E,
                                          q.nseg, q.V, q.psi, q.segpart, q.hdr, it);
  }
}

__global__ __launch_bounds__(256) void kb_combine(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item(b, BP_COMBINE, &it);
  combine_body(q.offset, q.K, q.D, q.segpart, q.V, q.psi, it);
}

// Bytes per lane of the whole-wave row reduction (fp32 or bf16 rows of 256, 512 or 1024 bytes;
// fp8 rows of 128 or 256 bytes), else 0.
int row_chunk(int32_t D, int32_t dtype) {
  if (dtype == SIL_FP8_E4M3) return (D == 128 || D == 256) ? D / 64 : 0;
  if (dtype != SIL_F32 && dtype != SIL_BF16) return 0;
  const int64_t rb = static_cast<int64_t>(D) * (dtype == SIL_F32 ? 4 : 2);
  return (rb == 256 || rb == 512 || rb == 1024) ? static_cast<int>(rb / 64) : 0;
}

// Lanes per row of the generic reduction for D columns (shared with the batch planner).
void stats_lanes(int32_t D, int32_t dtype, int32_t* Gv, int32_t* G, int32_t* E) {
  const int esz = dtype == SIL_F32 ? 4 : dtype == SIL_BF16 ? 2 : 1;
  const int per16 = 16 / esz;
  const int g = D % per16 == 0 ? D / per16 : 0;
  *Gv = (g >= 1 && g <= 64 && (g & (g - 1)) == 0) ? g : 0;
  int gg = 1;
  while (gg < D && gg < 64) gg <<= 1;
  *G = gg;
  *E = static_cast<int32_t>(ceil_div(D, gg));
}

hipError_t launch_stats_batched(const BatchLaunch& b, hipStream_t st) {
  const size_t lds = static_cast<size_t>(b.maxK) * 4;
  kb_zero<<<static_cast<unsigned>(b.items[BP_ZERO]), 256, 0, st>>>(b.dev);
  kb_hist<<<static_cast<unsigned>(b.items[BP_HIST]), kSortThreads, lds, st>>>(b.dev);
  kb_scan<<<static_cast<unsigned>(b.items[BP_SCAN]), 1024, 0, st>>>(b.dev);
  {
    // staged items: stage_lds(kChunk, K) for K <= kStageMaxK; the others K ints
    const int kst = b.maxK < kStageMaxK ? b.maxK : kStageMaxK;
    const size_t sl = std::max<size_t>(static_cast<size_t>(stage_lds(kStageSmall, kst)), lds);
    static bool lds_set = false;  // above 64 KB of dynamic LDS the kernel must say so once
    if (!lds_set) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_scatter),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               stage_lds(kStageSmall, kStageMaxK));
      if (e != hipSuccess) return e;
      lds_set = true;
    }
    kb_scatter<<<static_cast<unsigned>(b.items[BP_HIST]), kSortThreads, sl, st>>>(b.dev);
  }
  kb_seg<<<static_cast<unsigned>(b.items[BP_SEG]), 256, 0, st>>>(b.dev);
  kb_combine<<<static_cast<unsigned>(b.items[BP_COMBINE]), 256, 0, st>>>(b.dev);
  return hipGetLastError();
}

}  // namespace sil
