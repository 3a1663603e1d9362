// Dispatch of the fused GEMM+epilogue kernel, and the fixed-order reduction of S (Section II:
// S = sum_i s_i / N).
#include "main_kernels.h"

namespace sil {

// S = sum of the workgroup sums / N, in two fixed-order stages (deterministic); NaN when the
// workspace holds an error.  Stage 1: block b sums partials [b*chunk, (b+1)*chunk).
__device__ __forceinline__ double block_sum_1024(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  return sh[0];
}

__device__ __forceinline__ void reduce1_body(const double* __restrict__ bpart, int64_t nb,
                                             int64_t chunk, double* __restrict__ out, int64_t bid) {
  __shared__ double sh[1024];
  const int64_t b0 = bid * chunk;
  const int64_t b1 = min(nb, b0 + chunk);
  double v = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 1024) v += bpart[i];
  const double tot = block_sum_1024(v, sh);
  if (threadIdx.x == 0) out[bid] = tot;
}

__global__ __launch_bounds__(1024) void k_reduce1(const double* __restrict__ bpart, int64_t nb,
                                                  int64_t chunk, double* __restrict__ out) {
  reduce1_body(bpart, nb, chunk, out, blockIdx.x);
}

// mean: S = sum / N (the Silhouette); otherwise the sum itself (the K-means inertia)
// extra (may be NULL): one more partial sum, added last (the screen's fallback rows)
__device__ __forceinline__ void reduce2_body(const double* __restrict__ part, int n, int64_t N,
                                             const int32_t* __restrict__ hdr,
                                             double* __restrict__ S, int mean,
                                             const double* __restrict__ extra = nullptr) {
  __shared__ double sh[1024];
  const double v = static_cast<int>(threadIdx.x) < n ? part[threadIdx.x] : 0.0;
  double tot = block_sum_1024(v, sh);
  if (threadIdx.x == 0) {
    if (extra) tot += *extra;
    *S = hdr[0] != 0 ? __builtin_nan("") : (mean ? tot / static_cast<double>(N) : tot);
  }
}

__global__ __launch_bounds__(1024) void k_reduce2(const double* __restrict__ part, int n,
                                                  int64_t N, const int32_t* __restrict__ hdr,
                                                  double* __restrict__ S, int mean,
                                                  const double* __restrict__ extra) {
  reduce2_body(part, n, N, hdr, S, mean, extra);
}

__device__ __forceinline__ void poison_body(const int32_t* __restrict__ hdr, float* __restrict__ s,
                                            int64_t N, int64_t bid, int64_t nblk) {
  if (hdr[0] == 0) return;
  const int64_t stride = nblk * blockDim.x;
  for (int64_t i = bid * blockDim.x + threadIdx.x; i < N; i += stride) s[i] = __builtin_nanf("");
}

__global__ void k_poison(const int32_t* __restrict__ hdr, float* __restrict__ s, int64_t N) {
  poison_body(hdr, s, N, blockIdx.x, gridDim.x);
}

// K-means step: every label becomes -1 when the workspace holds an error
__global__ void k_poison_labels(const int32_t* __restrict__ hdr, int32_t* __restrict__ lab,
                                int64_t N) {
  if (hdr[0] == 0) return;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride)
    lab[i] = -1;
}

int main_rows_per_block(int dtype, int DPX, int products) {
  if (dtype == SIL_F32) return kMainWaves * 32;
  if (products < 1 || products > 3) products = 3;
  return kMainWaves * 32 * bf16_nb(DPX, products, dtype);
}

hipError_t launch_main(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st) {
  if (p.screen) return launch_screen_main(p, L, w, st);
  MainArgs m;
  m.X = p.X;
  m.col_scale = p.col_scale;
  m.perm = w.perm;
  m.lsorted = w.lsorted;
  m.hdr = w.hdr;
  m.N = p.N;
  m.D = p.D;
  m.K = p.K;
  m.btab = w.btab;
  m.piece = static_cast<int64_t>(p.Kpad) * table_stride(p.DPX, p.dtype);
  m.ctab = w.ctab;
  m.atab = w.atab;
  m.avec = w.avec;
  m.ascale = w.ascale;
  m.mvec = w.mvec;
  m.ntiles = p.Kpad / kColTile;
  m.root = (p.metric == SIL_SQEUCLID && (p.flags & SIL_FLAG_EUCLID_APPROX)) ? 1 : 0;
  m.s = p.s;
  m.bpart = w.bpart;
  m.save_a = w.save_a;
  m.save_b = w.save_b;
  m.save_n = w.save_n;
  m.labels_out = p.labels_out;
  m.assign = p.assign;
  const unsigned grid = static_cast<unsigned>(p.nblocks);
  if (p.assign) {
    if (p.dtype == SIL_F32)
      launch_main_f32(m, p.DPX, SIL_SQEUCLID, true, grid, st);
    else
      launch_main_assign(m, p.DPX, p.dtype, p.products, grid, st);
  } else if (p.dtype == SIL_F32) {
    launch_main_f32(m, p.DPX, p.metric, (p.flags & SIL_FLAG_SAVE_FOR_GRAD) != 0, grid, st);
  } else if (p.dtype == SIL_BF16) {
    launch_main_bf16(m, p.DPX, p.metric, p.products, grid, st);
  } else {
    launch_main_fp8(m, p.DPX, p.metric, p.products, grid, st);
  }
  return hipGetLastError();
}

void reduce_split(int64_t nblocks, int64_t* chunk, int32_t* n1) {
  *chunk = ceil_div(nblocks, 1024) < 4096 ? 4096 : ceil_div(nblocks, 1024);
  *n1 = static_cast<int32_t>(ceil_div(nblocks, *chunk));
}

hipError_t launch_reduce(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st) {
  (void)L;
  int64_t chunk;
  int32_t n1;
  const int64_t nred = p.nred ? p.nred : p.nblocks * kMainWaves;  // one partial per wave
  reduce_split(nred, &chunk, &n1);
  k_reduce1<<<static_cast<unsigned>(n1), 1024, 0, st>>>(w.bpart, nred, chunk, w.bpart2);
  const double* extra =
      p.screen ? reinterpret_cast<const double*>(w.hdr + kHdrFallbackSumWord) : nullptr;
  k_reduce2<<<1, 1024, 0, st>>>(w.bpart2, n1, p.N, w.hdr, p.S, (p.assign || p.reduce_sum) ? 0 : 1,
                                extra);
  if (p.s) k_poison<<<1024, 256, 0, st>>>(w.hdr, p.s, p.N);
  if (p.labels_out) k_poison_labels<<<1024, 256, 0, st>>>(w.hdr, p.labels_out, p.N);
  return hipGetLastError();
}


// ------------------------------------------------------------------------------------------
// batched reduction of S (work item blockIdx.x of the phase)

__device__ __forceinline__ const BatchProblem& batch_item_red(const BatchDev& b, int phase,
                                                              int64_t* local) {
  const int32_t* pre = b.prefix + phase * (b.n + 1);
  const int32_t item = static_cast<int32_t>(blockIdx.x);
  const int j = batch_locate(pre, b.n, item);
  *local = item - pre[j];
  return b.prob[j];
}

__global__ __launch_bounds__(1024) void kb_red1(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item_red(b, BP_RED1, &it);
  reduce1_body(q.bpart, q.nblocks * kMainWaves, q.red_chunk, q.bpart2, it);
}

__global__ __launch_bounds__(1024) void kb_red2(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item_red(b, BP_RED2, &it);
  reduce2_body(q.bpart2, q.red_n1, q.N, q.hdr, q.S, 1);
}

__global__ __launch_bounds__(256) void kb_poison(BatchDev b) {
  int64_t it;
  const BatchProblem& q = batch_item_red(b, BP_POISON, &it);
  if (!q.s) return;
  const int64_t i0 = it * kPoisonPerItem;
  const int64_t n = q.N - i0 < kPoisonPerItem ? q.N - i0 : kPoisonPerItem;
  poison_body(q.hdr, q.s + i0, n, 0, 1);
}

hipError_t launch_reduce_batched(const BatchLaunch& b, hipStream_t st) {
  kb_red1<<<static_cast<unsigned>(b.items[BP_RED1]), 1024, 0, st>>>(b.dev);
  kb_red2<<<static_cast<unsigned>(b.items[BP_RED2]), 1024, 0, st>>>(b.dev);
  if (b.items[BP_POISON] > 0)
    kb_poison<<<static_cast<unsigned>(b.items[BP_POISON]), 256, 0, st>>>(b.dev);
  return hipGetLastError();
}

}  // namespace sil
