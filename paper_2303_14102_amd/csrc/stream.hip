// Out-of-core evaluation: X and labels stay in host memory and pass through two device chunk
// buffers, twice.
//
// The method needs every cluster's statistics before any point can be scored (Section III: the
// statistics pass, then the per-point pass over the same data), so a data set larger than device
// memory is read twice:
//   pass 1  per chunk: the statistics pass on the chunk, then its sums added in chunk order into
//           FP64 global sums (deterministic: the chunk order is fixed);
//   between the global sums copied into the chunk layout, the checks of the whole data set, the
//           tables;
//   pass 2  per chunk: the counting sort alone, the fused kernel against the global tables, the
//           chunk's sum of s_i, s_i copied back to the host;
//   end     S = sum of the chunk sums / N in a fixed order.
// Uploads run on a copy stream of the library's own, at the default priority: the upload of chunk
// j + 1 overlaps the kernels of chunk j, and an upload into a buffer waits for the kernels that
// last read it.  Everything else runs on the caller's stream, so the caller's stream holds the
// whole call.
#include <mutex>

#include "sil_internal.h"

namespace sil {

static size_t align256s(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct StreamLayout {
  WsLayout L;  // the layout of one chunk's problem, at offset 0
  int64_t chunk, nchunks;
  size_t xbuf[2], lbuf[2], sbuf[2];
  size_t gcount, gV, gpsi, gstat, gsum, gend;
  size_t total;
};

static StreamLayout stream_layout(int64_t N, int64_t chunk, int32_t D, int32_t K, int32_t metric,
                                  int32_t dtype, int32_t flags) {
  StreamLayout S{};
  S.chunk = chunk < N ? chunk : N;
  S.nchunks = ceil_div(N, S.chunk);
  S.L = make_layout(S.chunk, D, K, metric, dtype, flags);
  size_t o = S.L.total;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256s(o + bytes);
    return at;
  };
  const size_t esz = dtype == SIL_F32 ? 4 : dtype == SIL_BF16 ? 2 : 1;
  for (int b = 0; b < 2; ++b) {
    S.xbuf[b] = take(static_cast<size_t>(S.chunk) * D * esz);
    S.lbuf[b] = take(static_cast<size_t>(S.chunk) * 4);
    S.sbuf[b] = take(static_cast<size_t>(S.chunk) * 4);
  }
  // global accumulators, contiguous so that one fill clears them
  S.gcount = take(static_cast<size_t>(K) * 4);
  S.gV = take(static_cast<size_t>(K) * D * 8);
  S.gpsi = take(static_cast<size_t>(K) * 8);
  S.gstat = take(256);
  S.gsum = take(static_cast<size_t>(S.nchunks) * 8);
  S.gend = o;
  S.total = o;
  return S;
}

__global__ void k_stream_zero(uint32_t* __restrict__ p, int64_t n_words) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_words;
       i += stride)
    p[i] = 0u;
}

// global sums += this chunk's sums; the chunk's first error into the global status
__global__ void k_stream_accum(const int32_t* __restrict__ count, const double* __restrict__ V,
                               const double* __restrict__ psi, const int32_t* __restrict__ hdr,
                               int32_t K, int32_t D, int32_t* __restrict__ gcount,
                               double* __restrict__ gV, double* __restrict__ gpsi,
                               int32_t* __restrict__ gstat) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < static_cast<int64_t>(K) * D) gV[i] += V[i];
  if (i < K) {
    gcount[i] += count[i];
    gpsi[i] += psi[i];
  }
  if (i == 0 && hdr[0] != 0) atomicCAS(gstat, 0, hdr[0]);
}

// The global sums into the chunk layout (where the table kernels read them), the header of the
// whole data set (hdr[1] = N for the centring vector), and the check for enough non-empty
// clusters, whose failure becomes the global status.
__global__ __launch_bounds__(256) void k_stream_global(
    const int32_t* __restrict__ gcount, const double* __restrict__ gV,
    const double* __restrict__ gpsi, int32_t* __restrict__ gstat, int32_t K, int32_t D,
    int64_t N, int min_nonempty, int32_t* __restrict__ count, double* __restrict__ V,
    double* __restrict__ psi, int32_t* __restrict__ hdr) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < static_cast<int64_t>(K) * D) V[i] = gV[i];
  if (i < K) {
    count[i] = gcount[i];
    psi[i] = gpsi[i];
  }
  if (blockIdx.x != 0) return;
  __shared__ int32_t nz[256];
  int32_t n = 0;
  for (int32_t k = threadIdx.x; k < K; k += blockDim.x) n += gcount[k] > 0;
  nz[threadIdx.x] = n;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) nz[threadIdx.x] += nz[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (nz[0] < min_nonempty) atomicCAS(gstat, 0, static_cast<int32_t>(SIL_E_FEW_CLUSTERS));
    hdr[0] = 0;
    hdr[1] = static_cast<int32_t>(N);
    hdr[2] = nz[0];
  }
}

// chunk outputs become NaN once the whole data set has an error
__global__ void k_stream_poison(const int32_t* __restrict__ gstat, float* __restrict__ s,
                                int64_t n) {
  if (gstat[0] == 0) return;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    s[i] = __builtin_nanf("");
}

// S = sum of the chunk sums / N (fixed order: strided per thread, then a fixed tree); the global
// status goes to hdr[0], where silhouette_status reads it.
__global__ __launch_bounds__(1024) void k_stream_final(const double* __restrict__ gsum,
                                                       int64_t nchunks,
                                                       const int32_t* __restrict__ gstat,
                                                       int64_t N, double* __restrict__ S,
                                                       int32_t* __restrict__ hdr) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  double v = 0.0;
  for (int64_t c = t; c < nchunks; c += 1024) v += gsum[c];
  sh[t] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) {
    *S = gstat[0] != 0 ? __builtin_nan("") : sh[0] / static_cast<double>(N);
    hdr[0] = gstat[0];
  }
}

// The library's copy stream and events, one set per device, created on first use and kept until
// the process ends.  Calls on one device are serialised while they enqueue (the events are
// shared).
struct StreamRes {
  std::mutex mu;
  bool ready = false;
  hipStream_t cs = nullptr;
  hipEvent_t start = nullptr;
  hipEvent_t up[2] = {nullptr, nullptr};    // chunk in buffer b uploaded
  hipEvent_t done[2] = {nullptr, nullptr};  // kernels reading buffer b finished
};
constexpr int kMaxDevices = 64;
static StreamRes g_sres[kMaxDevices];

static bool stream_res_init(StreamRes& r) {
  if (r.ready) return true;
  if (hipStreamCreateWithFlags(&r.cs, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&r.start, hipEventDisableTiming) != hipSuccess) return false;
  for (int b = 0; b < 2; ++b) {
    if (hipEventCreateWithFlags(&r.up[b], hipEventDisableTiming) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&r.done[b], hipEventDisableTiming) != hipSuccess) return false;
  }
  r.ready = true;
  return true;
}

static int stream_forward(int32_t metric, const void* Xh, int32_t dtype, const float* col_scale,
                          const int32_t* labh, int64_t N, int32_t D, int32_t K, int32_t products,
                          int32_t flags, float* s_host, double* S, int64_t chunk_rows, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!shape_ok(N, D, K) || !Xh || !labh || !S || chunk_rows < 1) return SIL_E_ARG;
  if (metric != SIL_SQEUCLID && metric != SIL_COSINE) return SIL_E_ARG;
  if (flags & ~(SIL_FLAG_NO_CENTRE | SIL_FLAG_EUCLID_APPROX)) return SIL_E_ARG;
  if ((flags & SIL_FLAG_EUCLID_APPROX) && metric != SIL_SQEUCLID) return SIL_E_ARG;
  if (metric == SIL_COSINE) flags &= ~SIL_FLAG_NO_CENTRE;
  if (dtype != SIL_F32 && dtype != SIL_BF16 && dtype != SIL_FP8_E4M3) return SIL_E_DTYPE;
  if (dtype == SIL_FP8_E4M3 && !col_scale) return SIL_E_DTYPE;
  if (products == 0) products = 3;
  if (products < 1 || products > 3) return SIL_E_ARG;
  products = run_products(metric, dtype, flags, products);
  const StreamLayout SL = stream_layout(N, chunk_rows, D, K, metric, dtype, flags);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || ws_bytes < SL.total)
    return SIL_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SIL_E_HIP;
  StreamRes& R = g_sres[dev];
  std::lock_guard<std::mutex> lock(R.mu);
  if (!stream_res_init(R)) return SIL_E_HIP;

  char* base = static_cast<char*>(ws);
  const WsLayout& L = SL.L;
  const WsPtrs w = carve(L, ws);
  int32_t* gcount = reinterpret_cast<int32_t*>(base + SL.gcount);
  double* gV = reinterpret_cast<double*>(base + SL.gV);
  double* gpsi = reinterpret_cast<double*>(base + SL.gpsi);
  int32_t* gstat = reinterpret_cast<int32_t*>(base + SL.gstat);
  double* gsum = reinterpret_cast<double*>(base + SL.gsum);
  const size_t esz = dtype == SIL_F32 ? 4 : dtype == SIL_BF16 ? 2 : 1;
  const size_t row_bytes = static_cast<size_t>(D) * esz;
  const int rows_per_block = main_rows_per_block(dtype, L.DPX, products);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t KD = static_cast<int64_t>(K) * D;
  const unsigned kd_blocks = static_cast<unsigned>(ceil_div(KD > K ? KD : K, 256));

  // clear the global accumulators; uploads start once the caller's earlier work is done (it may
  // still read the chunk buffers of a previous call on this workspace)
  const int64_t gwords = static_cast<int64_t>((SL.gend - SL.gcount) / 4);
  k_stream_zero<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(gwords, 256), 1024)), 256, 0,
                  st>>>(reinterpret_cast<uint32_t*>(gcount), gwords);
  if (hipEventRecord(R.start, st) != hipSuccess) return SIL_E_HIP;
  if (hipStreamWaitEvent(R.cs, R.start, 0) != hipSuccess) return SIL_E_HIP;

  const int64_t nch = SL.nchunks;
  for (int64_t j = 0; j < 2 * nch; ++j) {
    const int pass = j < nch ? 0 : 1;
    const int64_t c = j % nch;
    const int b = static_cast<int>(j & 1);
    const int64_t r0 = c * SL.chunk;
    const int64_t n = std::min<int64_t>(SL.chunk, N - r0);
    void* xb = base + SL.xbuf[b];
    int32_t* lb = reinterpret_cast<int32_t*>(base + SL.lbuf[b]);
    float* sb = reinterpret_cast<float*>(base + SL.sbuf[b]);
    // upload on the copy stream once the kernels of job j - 2 (same buffer) are done
    if (j >= 2 && hipStreamWaitEvent(R.cs, R.done[b], 0) != hipSuccess) return SIL_E_HIP;
    if (hipMemcpyAsync(xb, static_cast<const char*>(Xh) + static_cast<size_t>(r0) * row_bytes,
                       static_cast<size_t>(n) * row_bytes, hipMemcpyHostToDevice, R.cs) != hipSuccess)
      return SIL_E_HIP;
    if (hipMemcpyAsync(lb, labh + r0, static_cast<size_t>(n) * 4, hipMemcpyHostToDevice, R.cs) !=
        hipSuccess)
      return SIL_E_HIP;
    if (hipEventRecord(R.up[b], R.cs) != hipSuccess) return SIL_E_HIP;
    if (hipStreamWaitEvent(st, R.up[b], 0) != hipSuccess) return SIL_E_HIP;

    Problem p{xb, col_scale, lb, n, D, L.DPX, K, L.Kpad, dtype, metric, products, flags,
              s_host ? sb : nullptr, gsum + c, ceil_div(n, rows_per_block)};
    p.min_nonempty = 0;  // a chunk may hold a single cluster; the whole data set is checked
    if (pass == 0) {
      if (launch_stats(p, L, w, st) != hipSuccess) return SIL_E_HIP;
      k_stream_accum<<<kd_blocks, 256, 0, st>>>(w.count, w.V, w.psi, w.hdr, K, D, gcount, gV, gpsi,
                                                gstat);
      if (j == nch - 1) {  // all statistics in: the tables of the whole data set
        k_stream_global<<<kd_blocks, 256, 0, st>>>(gcount, gV, gpsi, gstat, K, D, N, 2, w.count,
                                                   w.V, w.psi, w.hdr);
        if (launch_finalize(p, L, w, st) != hipSuccess) return SIL_E_HIP;
      }
    } else {
      p.reduce_sum = 1;
      if (launch_sort(p, L, w, st) != hipSuccess) return SIL_E_HIP;
      if (launch_main(p, L, w, st) != hipSuccess) return SIL_E_HIP;
      if (launch_reduce(p, L, w, st) != hipSuccess) return SIL_E_HIP;
      if (s_host) {
        k_stream_poison<<<256, 256, 0, st>>>(gstat, sb, n);
        if (hipMemcpyAsync(s_host + r0, sb, static_cast<size_t>(n) * 4, hipMemcpyDeviceToHost,
                           st) != hipSuccess)
          return SIL_E_HIP;
      }
    }
    if (hipEventRecord(R.done[b], st) != hipSuccess) return SIL_E_HIP;
  }
  k_stream_final<<<1, 1024, 0, st>>>(gsum, nch, gstat, N, S, w.hdr);
  return hipGetLastError() == hipSuccess ? SIL_OK : SIL_E_HIP;
}

}  // namespace sil

using namespace sil;

extern "C" {

size_t silhouette_stream_workspace_bytes(int64_t N, int64_t chunk_rows, int32_t D, int32_t K,
                                         int32_t metric, int32_t dtype, int32_t flags) {
  if (!shape_ok(N, D, K) || chunk_rows < 1) return 0;
  if (dtype != SIL_F32 && dtype != SIL_BF16 && dtype != SIL_FP8_E4M3) return 0;
  return stream_layout(N, chunk_rows, D, K, metric, dtype, flags).total;
}

int silhouette_stream(int32_t metric, const void* X_host, int32_t dtype, const float* col_scale,
                      const int32_t* labels_host, int64_t N, int32_t D, int32_t K,
                      int32_t products, int32_t flags, float* s_host, double* S,
                      int64_t chunk_rows, void* ws, size_t ws_bytes, void* stream) {
  return stream_forward(metric, X_host, dtype, col_scale, labels_host, N, D, K, products, flags,
                        s_host, S, chunk_rows, ws, ws_bytes, stream);
}

}  // extern "C"
