// Fixed-matrix Mahalanobis distance d(x, y) = (x - y)^T M (x - y), M = L^T L.
//
// The paper's Section V notes that a similar approach serves other metrics.  This one is the
// squared Euclidean distance between z = L x and L y, so its mean distance to a cluster follows
// Eq.11 on the transformed points: the data are transformed once, Z = X L^T (a dense contraction,
// on fp32 MFMA), into the workspace, and the squared Euclidean path runs on Z in fp32.
#include "main_kernels.h"

namespace sil {

// Elements c and c + 1 of row `row` as float (c + 1 may be past D: then 0).
template <int DT>
__device__ __forceinline__ void load_pair(const void* __restrict__ X,
                                          const float* __restrict__ col_scale, int64_t row,
                                          int32_t D, int32_t c, float& v0, float& v1) {
  v0 = 0.0f;
  v1 = 0.0f;
  if (c >= D) return;
  const int64_t base = row * static_cast<int64_t>(D) + c;
  const bool two = c + 1 < D;
  if constexpr (DT == SIL_F32) {
    const float* p = static_cast<const float*>(X) + base;
    v0 = p[0];
    if (two) v1 = p[1];
  } else if constexpr (DT == SIL_BF16) {
    const uint16_t* p = static_cast<const uint16_t*>(X) + base;
    v0 = bf16_bits_f32(p[0]);
    if (two) v1 = bf16_bits_f32(p[1]);
  } else {
    const uint8_t* p = static_cast<const uint8_t*>(X) + base;
    v0 = e4m3_f32(p[0]) * col_scale[c];
    if (two) v1 = e4m3_f32(p[1]) * col_scale[c + 1];
  }
}

// Z = X L^T with v_mfma_f32_32x32x2f32.  A wave owns 32 rows and keeps them in registers; for
// each 32-column tile of Z it runs the depth in pairs of MFMA steps: at step q the lanes of half h
// supply features 4q + 2h and 4q + 2h + 1 of their row (A) and of row c of L (B, column c of
// L^T).  The workgroup stages the tile's 32 rows of L in LDS first (row stride D + 2 floats, so
// the 8-byte reads of the 32 lanes of a half fall in distinct banks), so that the B operands
// are LDS reads rather than dependent global loads.  Rows past N and columns past D are zero
// and never stored.  DQ = ceil(D / 4).
template <int DT, int DQ>
__global__ __launch_bounds__(256) void k_mahal_transform(const void* __restrict__ X,
                                                         const float* __restrict__ col_scale,
                                                         const float* __restrict__ L, int64_t N,
                                                         int32_t D, float* __restrict__ Z) {
  constexpr int LS = 4 * DQ + 2;  // LDS row stride (floats), >= D + 2
  __shared__ __attribute__((aligned(16))) float lt[32 * LS];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const int64_t row0 = (static_cast<int64_t>(blockIdx.x) * kMainWaves + wave) * 32;
  const bool active = row0 < N;  // wave-uniform; idle waves still help stage L
  const bool rok = active && row0 + r < N;
  const int64_t row = rok ? row0 + r : 0;
  float a[DQ][2];
#pragma unroll
  for (int q = 0; q < DQ; ++q) {
    float v0 = 0.0f, v1 = 0.0f;
    if (rok) load_pair<DT>(X, col_scale, row, D, 4 * q + 2 * h, v0, v1);
    a[q][0] = v0;
    a[q][1] = v1;
  }
  const int ntile = (D + 31) / 32;
  for (int t = 0; t < ntile; ++t) {
    __syncthreads();  // the previous tile's reads of lt are done
    for (int i = threadIdx.x; i < 32 * LS; i += 256) {
      const int lr = i / LS, lc = i % LS;
      const int c = 32 * t + lr;
      lt[i] = (c < D && lc < D) ? L[static_cast<int64_t>(c) * D + lc] : 0.0f;
    }
    __syncthreads();
    if (!active) continue;
    const float* lrow = lt + r * LS + 2 * h;
    f32x16_t acc = f32x16_t{};
#pragma unroll
    for (int q = 0; q < DQ; ++q) {
      const float2 bv = *reinterpret_cast<const float2*>(lrow + 4 * q);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q][0], bv.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q][1], bv.y, acc, 0, 0, 0);
    }
    const int c = 32 * t + r;
    if (c < D) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t orow = row0 + out_row(j, h);
        if (orow < N) Z[orow * D + c] = acc[j];
      }
    }
  }
}

template <int DT>
static void launch_transform_dt(const void* X, const float* col_scale, const float* L, int64_t N,
                                int32_t D, float* Z, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(ceil_div(N, kMainWaves * 32));
  const int dq = (D + 3) / 4;
  if (dq <= 4)
    k_mahal_transform<DT, 4><<<grid, 256, 0, st>>>(X, col_scale, L, N, D, Z);
  else if (dq <= 8)
    k_mahal_transform<DT, 8><<<grid, 256, 0, st>>>(X, col_scale, L, N, D, Z);
  else if (dq <= 16)
    k_mahal_transform<DT, 16><<<grid, 256, 0, st>>>(X, col_scale, L, N, D, Z);
  else if (dq <= 32)
    k_mahal_transform<DT, 32><<<grid, 256, 0, st>>>(X, col_scale, L, N, D, Z);
  else
    k_mahal_transform<DT, 64><<<grid, 256, 0, st>>>(X, col_scale, L, N, D, Z);
}

static size_t z_bytes(int64_t N, int32_t D) {
  return (static_cast<size_t>(N) * D * 4 + 255) & ~static_cast<size_t>(255);
}

}  // namespace sil

using namespace sil;

extern "C" {

size_t silhouette_mahalanobis_workspace_bytes(int64_t N, int32_t D, int32_t K, int32_t flags) {
  if (!shape_ok(N, D, K)) return 0;
  return z_bytes(N, D) + make_layout(N, D, K, SIL_SQEUCLID, SIL_F32, flags).total;
}

int silhouette_mahalanobis(const void* X, int32_t dtype, const float* col_scale, const float* L,
                           const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t flags,
                           float* s, double* S, void* ws, size_t ws_bytes, void* stream) {
  if (!shape_ok(N, D, K) || !X || !L || !labels || !S) return SIL_E_ARG;
  if (reinterpret_cast<uintptr_t>(X) & 15u) return SIL_E_ARG;
  if (flags & ~SIL_FLAG_NO_CENTRE) return SIL_E_ARG;
  if (dtype != SIL_F32 && dtype != SIL_BF16 && dtype != SIL_FP8_E4M3) return SIL_E_DTYPE;
  if (dtype == SIL_FP8_E4M3 && !col_scale) return SIL_E_DTYPE;
  const size_t zb = z_bytes(N, D);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) ||
      ws_bytes < zb + make_layout(N, D, K, SIL_SQEUCLID, SIL_F32, flags).total)
    return SIL_E_WORKSPACE;
  float* Z = static_cast<float*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == SIL_F32)
    launch_transform_dt<SIL_F32>(X, col_scale, L, N, D, Z, st);
  else if (dtype == SIL_BF16)
    launch_transform_dt<SIL_BF16>(X, col_scale, L, N, D, Z, st);
  else
    launch_transform_dt<SIL_FP8_E4M3>(X, col_scale, L, N, D, Z, st);
  if (hipGetLastError() != hipSuccess) return SIL_E_HIP;
  return silhouette_sqeuclid(Z, SIL_F32, nullptr, labels, N, D, K, 0, flags, s, S,
                             static_cast<char*>(ws) + zb, ws_bytes - zb, stream);
}

}  // extern "C"
