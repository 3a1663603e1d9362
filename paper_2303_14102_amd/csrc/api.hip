// C ABI entry points: argument checks, workspace carving, the stream-ordered launch sequence.
#include <algorithm>

#include "sil_internal.h"

namespace sil {

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

WsLayout make_layout(int64_t N, int32_t D, int32_t K, int32_t metric, int32_t dtype,
                     int32_t flags) {
  WsLayout L{};
  L.N = N;
  L.D = D;
  L.DPX = gemm_depth(D, dtype);
  L.K = K;
  L.Kpad = static_cast<int32_t>(round_up(K, kColTile));
  L.nseg = ceil_div(N, kSegLen);
  L.nblocks = ceil_div(N, kMainWaves * 32);  // upper bound over all kernel families
  L.dtype = dtype;
  L.metric = metric;
  L.flags = flags;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  // hdr .. segpart are zeroed together by the statistics pass: keep them first and contiguous
  L.hdr = take(64 * 4);
  L.count = take(static_cast<size_t>(K) * 4);
  L.offset = take(static_cast<size_t>(K + 1) * 4);
  L.cursor = take(static_cast<size_t>(K) * 4);
  L.V = take(static_cast<size_t>(K) * D * 8);
  L.psi = take(static_cast<size_t>(K) * 8);
  L.segpart = take(static_cast<size_t>(L.nseg) * 2 * (D + 1) * 8);
  L.perm = take(static_cast<size_t>(N) * 4);
  L.lsorted = take(static_cast<size_t>(N) * 4);
  L.gmean = take(static_cast<size_t>(L.DPX) * 8);
  L.mvec = take(static_cast<size_t>(L.DPX) * 4);
  const size_t bt_elem = dtype == SIL_F32 ? 4 : 2 * 2;  // fp32, or bf16 hi + lo
  L.btab = take(static_cast<size_t>(L.Kpad) * table_stride(L.DPX, dtype) * bt_elem);
  L.ctab = take(static_cast<size_t>(L.Kpad) * 4);
  L.atab = take(static_cast<size_t>(K) * L.DPX * 4);
  L.avec = take(static_cast<size_t>(K) * 4);
  L.ascale = take(static_cast<size_t>(K) * 4);
  // the one-product screen's regions whenever a call with this shape may take it
  const bool scr = screen_applies(metric, dtype, L.DPX, 2, flags);
  L.nsblk = scr ? ceil_div(N, screen_rows_per_block()) : 0;
  // block partials of S: one per wave of the fused kernel (kMainWaves per row block)
  L.bpart = take(static_cast<size_t>(std::max(L.nblocks, L.nsblk)) * kMainWaves * 8);
  L.bpart2 = take(1024 * 8);
  const bool save = (flags & SIL_FLAG_SAVE_FOR_GRAD) != 0;
  L.save_a = take(save ? static_cast<size_t>(N) * 4 : 0);
  L.save_b = take(save ? static_cast<size_t>(N) * 4 : 0);
  L.save_n = take(save ? static_cast<size_t>(N) * 4 : 0);
  const size_t KW = static_cast<size_t>(K) * (D + 1);
  L.gpart = take(save && (bwd_fits_lds(K, D) || bwd_fits_slices(K))
                     ? static_cast<size_t>(bwd_accum_workgroups(N)) * KW * 8
                     : 0);
  L.gAB = take(save ? KW * 8 : 0);
  L.galpha = take(save ? static_cast<size_t>(N) * 16 : 0);
  L.gtab = take(save ? (static_cast<size_t>(K) * L.DPX + K) * 4 : 0);
  L.stab = take(scr ? static_cast<size_t>(L.Kpad) * screen_stride(L.DPX) * 2 : 0);
  L.c64 = take(scr ? static_cast<size_t>(L.Kpad) * 8 : 0);
  L.rtab = take(scr && dtype == SIL_FP8_E4M3 ? static_cast<size_t>(K) * L.DPX * 4 : 0);
  L.fblist = take(scr ? static_cast<size_t>(N) * 4 : 0);
  // fallback workgroups take at least 128 list entries each
  L.fbpart = take(scr ? static_cast<size_t>(ceil_div(N, kMainWaves * 32)) * kMainWaves * 8 : 0);
  L.total = o;
  return L;
}

WsPtrs carve(const WsLayout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  WsPtrs w;
  w.hdr = reinterpret_cast<int32_t*>(b + L.hdr);
  w.count = reinterpret_cast<int32_t*>(b + L.count);
  w.offset = reinterpret_cast<int32_t*>(b + L.offset);
  w.cursor = reinterpret_cast<int32_t*>(b + L.cursor);
  w.V = reinterpret_cast<double*>(b + L.V);
  w.psi = reinterpret_cast<double*>(b + L.psi);
  w.segpart = reinterpret_cast<double*>(b + L.segpart);
  w.perm = reinterpret_cast<int32_t*>(b + L.perm);
  w.lsorted = reinterpret_cast<int32_t*>(b + L.lsorted);
  w.gmean = reinterpret_cast<double*>(b + L.gmean);
  w.mvec = reinterpret_cast<float*>(b + L.mvec);
  w.btab = b + L.btab;
  w.ctab = reinterpret_cast<float*>(b + L.ctab);
  w.atab = reinterpret_cast<float*>(b + L.atab);
  w.avec = reinterpret_cast<float*>(b + L.avec);
  w.ascale = reinterpret_cast<float*>(b + L.ascale);
  w.bpart = reinterpret_cast<double*>(b + L.bpart);
  w.bpart2 = reinterpret_cast<double*>(b + L.bpart2);
  w.save_a = reinterpret_cast<float*>(b + L.save_a);
  w.save_b = reinterpret_cast<float*>(b + L.save_b);
  w.save_n = reinterpret_cast<int32_t*>(b + L.save_n);
  w.gpart = reinterpret_cast<double*>(b + L.gpart);
  w.gAB = reinterpret_cast<double*>(b + L.gAB);
  w.galpha = b + L.galpha;
  w.gtab = reinterpret_cast<float*>(b + L.gtab);
  w.stab = b + L.stab;
  w.c64 = reinterpret_cast<double*>(b + L.c64);
  w.rtab = reinterpret_cast<float*>(b + L.rtab);
  w.fblist = reinterpret_cast<int32_t*>(b + L.fblist);
  w.fbpart = reinterpret_cast<double*>(b + L.fbpart);
  return w;
}

bool shape_ok(int64_t N, int32_t D, int32_t K) {
  return N >= 1 && N <= INT32_MAX && D >= 1 && D <= kMaxD && K >= 2 && K <= kMaxK;
}

static int check_common(const void* X, int32_t dtype, const float* col_scale,
                        const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t metric,
                        const void* ws, size_t ws_bytes, int32_t flags, WsLayout* L) {
  if (!shape_ok(N, D, K) || !X || !labels) return SIL_E_ARG;
  if (reinterpret_cast<uintptr_t>(X) & 15u) return SIL_E_ARG;  // rows are read as 16-byte vectors
  if (metric != SIL_SQEUCLID && metric != SIL_COSINE && metric != SIL_KL) return SIL_E_ARG;
  if (dtype != SIL_F32 && dtype != SIL_BF16 && dtype != SIL_FP8_E4M3) return SIL_E_DTYPE;
  if (dtype == SIL_FP8_E4M3 && !col_scale) return SIL_E_DTYPE;
  *L = make_layout(N, D, K, metric, dtype, flags);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || ws_bytes < L->total) return SIL_E_WORKSPACE;
  return SIL_OK;
}

// ------------------------------------------------------------------------------------------
// phase timing (benchmarks)

struct Profile {
  bool on = false;
  int cap = 0, used = 0;
  hipEvent_t* ev = nullptr;  // 5 events per call
};
static Profile g_prof;

static void prof_record(int call, int point, hipStream_t st) {
  // a failed record surfaces in silhouette_profile_end (elapsed time of that event)
  if (g_prof.on && call >= 0) (void)hipEventRecord(g_prof.ev[call * 5 + point], st);
}

int run_forward(int32_t metric, const void* X, int32_t dtype, const float* col_scale,
                const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t products,
                int32_t flags, float* s, double* S, void* ws, size_t ws_bytes, void* stream) {
  WsLayout L;
  int rc = check_common(X, dtype, col_scale, labels, N, D, K, metric, ws, ws_bytes, flags, &L);
  if (rc) return rc;
  if (!S) return SIL_E_ARG;
  if (products == 0) products = 3;
  if (products < 1 || products > 3) return SIL_E_ARG;
  if ((flags & SIL_FLAG_EUCLID_APPROX) &&
      (metric != SIL_SQEUCLID || (flags & SIL_FLAG_SAVE_FOR_GRAD)))
    return SIL_E_ARG;
  if (metric == SIL_KL) {  // no backward; fp32 or bf16 storage
    if (flags & (SIL_FLAG_SAVE_FOR_GRAD | SIL_FLAG_EUCLID_APPROX)) return SIL_E_ARG;
    if (dtype == SIL_FP8_E4M3) return SIL_E_DTYPE;
  }
  const WsPtrs w = carve(L, ws);
  if ((flags & SIL_FLAG_SAVE_FOR_GRAD) && dtype != SIL_F32) return SIL_E_DTYPE;
  products = run_products(metric, dtype, flags, products);
  // fp8: the screen's prologue reads whole 8-code chunks and 16-byte aligned column scales
  const bool fp8_vec = dtype != SIL_FP8_E4M3 ||
                       (D % 8 == 0 && (reinterpret_cast<uintptr_t>(col_scale) & 15u) == 0);
  const int screen = screen_applies(metric, dtype, L.DPX, products, flags) && fp8_vec ? 1 : 0;
  const int64_t nblocks =
      screen ? L.nsblk : ceil_div(N, main_rows_per_block(dtype, L.DPX, products));
  Problem p{X, col_scale, labels, N, D, L.DPX, K, L.Kpad, dtype, metric, products, flags, s, S,
            nblocks};
  p.screen = screen;
  p.nred = screen ? L.nsblk * kMainWaves : 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int call = g_prof.on && g_prof.used < g_prof.cap ? g_prof.used++ : -1;
  prof_record(call, 0, st);
  if (launch_stats(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 1, st);
  if (launch_finalize(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 2, st);
  if (launch_main(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 3, st);
  if (launch_reduce(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 4, st);
  return SIL_OK;
}

// One K-means (Lloyd) step on the same passes: the statistics and tables of the given labels
// (the means), then the fused kernel with the argmin over every cluster.  Phases are recorded
// like a forward call's.
static int kmeans(const void* X, int32_t dtype, const float* col_scale, const int32_t* labels,
                  int64_t N, int32_t D, int32_t K, int32_t products, int32_t flags,
                  int32_t* labels_out, double* inertia, void* ws, size_t ws_bytes, void* stream) {
  if (flags & ~SIL_FLAG_NO_CENTRE) return SIL_E_ARG;
  WsLayout L;
  int rc = check_common(X, dtype, col_scale, labels, N, D, K, SIL_SQEUCLID, ws, ws_bytes, flags,
                        &L);
  if (rc) return rc;
  if (!labels_out || !inertia) return SIL_E_ARG;
  if (products == 0) products = 3;
  if (products != 3 && !(products == 2 && dtype == SIL_BF16)) return SIL_E_ARG;
  const WsPtrs w = carve(L, ws);
  // one row block per wave (the argmin kernels), whatever the product count
  const int64_t nblocks = ceil_div(N, main_rows_per_block(dtype, L.DPX, 3));
  Problem p{X, col_scale, labels, N, D, L.DPX, K, L.Kpad, dtype, SIL_SQEUCLID, products, flags,
            nullptr, inertia, nblocks};
  p.labels_out = labels_out;
  p.assign = 1;
  p.min_nonempty = 1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int call = g_prof.on && g_prof.used < g_prof.cap ? g_prof.used++ : -1;
  prof_record(call, 0, st);
  if (launch_stats(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 1, st);
  if (launch_finalize(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 2, st);
  if (launch_main(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 3, st);
  if (launch_reduce(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  prof_record(call, 4, st);
  return SIL_OK;
}

static int backward(int32_t metric, const void* X, int32_t dtype, const float* col_scale,
                    const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t flags,
                    const double* gS, float* dX, void* ws, size_t ws_bytes, void* stream) {
  WsLayout L;
  if (flags & SIL_FLAG_EUCLID_APPROX) return SIL_E_ARG;
  flags |= SIL_FLAG_SAVE_FOR_GRAD;
  int rc = check_common(X, dtype, col_scale, labels, N, D, K, metric, ws, ws_bytes, flags, &L);
  if (rc) return rc;
  if (dtype != SIL_F32) return SIL_E_DTYPE;
  if (!gS || !dX) return SIL_E_ARG;
  const WsPtrs w = carve(L, ws);
  Problem p{X, col_scale, labels, N, D, L.DPX, K, L.Kpad, dtype, metric, 0, flags, nullptr,
            nullptr, 0};
  if (launch_backward(p, L, w, gS, dX, static_cast<hipStream_t>(stream)) != hipSuccess)
    return SIL_E_HIP;
  return SIL_OK;
}

// 16-byte-or-less device-to-device copies of the statistics (kernels, so that the call stays
// capturable and never touches the host)
__global__ void k_copy_stats(const int32_t* __restrict__ cnt_in, const double* __restrict__ V_in,
                             const double* __restrict__ psi_in, int32_t K, int32_t D,
                             int32_t* __restrict__ cnt, double* __restrict__ V,
                             double* __restrict__ psi) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t KD = static_cast<int64_t>(K) * D;
  if (V && i < KD) V[i] = V_in[i];
  if (i < K) {
    if (cnt) cnt[i] = cnt_in[i];
    if (psi) psi[i] = psi_in[i];
  }
}

hipError_t launch_copy_stats(const Problem& p, const WsLayout& L, const WsPtrs& w, int32_t* count,
                             double* V, double* psi, hipStream_t st) {
  (void)L;
  const int64_t n = static_cast<int64_t>(p.K) * p.D > p.K ? static_cast<int64_t>(p.K) * p.D : p.K;
  k_copy_stats<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, st>>>(w.count, w.V, w.psi, p.K,
                                                                        p.D, count, V, psi);
  return hipGetLastError();
}

}  // namespace sil

using namespace sil;

extern "C" {

size_t silhouette_workspace_bytes(int64_t N, int32_t D, int32_t K, int32_t metric, int32_t dtype,
                                  int32_t flags) {
  if (!shape_ok(N, D, K)) return 0;
  return make_layout(N, D, K, metric, dtype, flags).total;
}

int silhouette_sqeuclid(const void* X, int32_t dtype, const float* col_scale,
                        const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t products,
                        int32_t flags, float* s, double* S, void* ws, size_t ws_bytes,
                        void* stream) {
  return run_forward(SIL_SQEUCLID, X, dtype, col_scale, labels, N, D, K, products, flags, s, S, ws,
                 ws_bytes, stream);
}

int silhouette_kl(const void* X, int32_t dtype, const float* col_scale, const int32_t* labels,
                  int64_t N, int32_t D, int32_t K, int32_t products, int32_t flags, float* s,
                  double* S, void* ws, size_t ws_bytes, void* stream) {
  return run_forward(SIL_KL, X, dtype, col_scale, labels, N, D, K, products,
                 flags & ~SIL_FLAG_NO_CENTRE, s, S, ws, ws_bytes, stream);
}

int silhouette_cosine(const void* X, int32_t dtype, const float* col_scale, const int32_t* labels,
                      int64_t N, int32_t D, int32_t K, int32_t products, int32_t flags, float* s,
                      double* S, void* ws, size_t ws_bytes, void* stream) {
  return run_forward(SIL_COSINE, X, dtype, col_scale, labels, N, D, K, products,
                 flags & ~SIL_FLAG_NO_CENTRE, s, S, ws, ws_bytes, stream);
}

int silhouette_sqeuclid_backward(const void* X, int32_t dtype, const float* col_scale,
                                 const int32_t* labels, int64_t N, int32_t D, int32_t K,
                                 int32_t flags, const double* gS, float* dX, void* ws,
                                 size_t ws_bytes, void* stream) {
  return backward(SIL_SQEUCLID, X, dtype, col_scale, labels, N, D, K, flags, gS, dX, ws, ws_bytes,
                  stream);
}

int silhouette_cosine_backward(const void* X, int32_t dtype, const float* col_scale,
                               const int32_t* labels, int64_t N, int32_t D, int32_t K,
                               int32_t flags, const double* gS, float* dX, void* ws,
                               size_t ws_bytes, void* stream) {
  return backward(SIL_COSINE, X, dtype, col_scale, labels, N, D, K, flags & ~SIL_FLAG_NO_CENTRE,
                  gS, dX, ws, ws_bytes, stream);
}

int silhouette_kmeans_step(const void* X, int32_t dtype, const float* col_scale,
                           const int32_t* labels, int64_t N, int32_t D, int32_t K,
                           int32_t products, int32_t flags, int32_t* labels_out, double* inertia,
                           void* ws, size_t ws_bytes, void* stream) {
  return kmeans(X, dtype, col_scale, labels, N, D, K, products, flags, labels_out, inertia, ws,
                ws_bytes, stream);
}

int silhouette_cluster_stats(const void* X, int32_t dtype, const float* col_scale,
                             const int32_t* labels, int64_t N, int32_t D, int32_t K,
                             int32_t metric, int32_t* count, double* V, double* psi, void* ws,
                             size_t ws_bytes, void* stream) {
  WsLayout L;
  int rc = check_common(X, dtype, col_scale, labels, N, D, K, metric, ws, ws_bytes, 0, &L);
  if (rc) return rc;
  const WsPtrs w = carve(L, ws);
  Problem p{X, col_scale, labels, N, D, L.DPX, K, L.Kpad, dtype, metric, 3, 0, nullptr, nullptr, 0};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (launch_stats(p, L, w, st) != hipSuccess) return SIL_E_HIP;
  if (launch_copy_stats(p, L, w, count, V, psi, st) != hipSuccess) return SIL_E_HIP;
  return SIL_OK;
}

int silhouette_profile_begin(int32_t max_calls) {
  if (max_calls < 1 || max_calls > 4096) return SIL_E_ARG;
  if (g_prof.cap < max_calls) {
    for (int i = 0; i < g_prof.cap * 5; ++i) (void)hipEventDestroy(g_prof.ev[i]);
    delete[] g_prof.ev;
    g_prof.ev = new hipEvent_t[static_cast<size_t>(max_calls) * 5];
    for (int i = 0; i < max_calls * 5; ++i)
      if (hipEventCreate(&g_prof.ev[i]) != hipSuccess) {
        g_prof.cap = i / 5;
        return SIL_E_HIP;
      }
    g_prof.cap = max_calls;
  }
  g_prof.used = 0;
  g_prof.on = true;
  return SIL_OK;
}

int silhouette_profile_end(float* ms_sum, int32_t* ncalls) {
  g_prof.on = false;
  if (!ms_sum || !ncalls) return SIL_E_ARG;
  for (int k = 0; k < 4; ++k) ms_sum[k] = 0.0f;
  *ncalls = g_prof.used;
  if (g_prof.used == 0) return SIL_OK;
  if (hipEventSynchronize(g_prof.ev[g_prof.used * 5 - 1]) != hipSuccess) return SIL_E_HIP;
  for (int c = 0; c < g_prof.used; ++c)
    for (int k = 0; k < 4; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, g_prof.ev[c * 5 + k], g_prof.ev[c * 5 + k + 1]) != hipSuccess)
        return SIL_E_HIP;
      ms_sum[k] += ms;
    }
  return SIL_OK;
}

int silhouette_status(const void* ws, void* stream) {
  if (!ws) return SIL_E_WORKSPACE;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return SIL_E_HIP;
  int32_t v = 0;
  if (hipMemcpy(&v, ws, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return SIL_E_HIP;
  return v;
}

const char* silhouette_strerror(int status) {
  switch (status) {
    case SIL_OK: return "ok";
    case SIL_E_ARG: return "argument out of range or NULL pointer";
    case SIL_E_DTYPE: return "unsupported storage type (or fp8 without col_scale)";
    case SIL_E_LABEL: return "a label lies outside [0, K)";
    case SIL_E_FEW_CLUSTERS: return "fewer than two non-empty clusters";
    case SIL_E_ZERO_NORM: return "a point has zero norm under the cosine distance";
    case SIL_E_NONFINITE: return "X holds a NaN or an infinity";
    case SIL_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case SIL_E_HIP: return "a HIP runtime call failed";
    case SIL_E_DOMAIN: return "an entry lies outside the distance's domain (KL needs positive entries)";
    case SIL_E_SCRATCH: return "problem needs more than the static scratch of the no-allocation entry point";
    default: return "unknown status";
  }
}

}  // extern "C"
