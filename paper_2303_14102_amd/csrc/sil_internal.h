// Internal declarations shared by the HIP translation units of the Silhouette library.
// Not part of the public ABI (that is include/silhouette.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/silhouette.h"

namespace sil {

// ------------------------------------------------------------------------------------------
// limits and tiling constants

constexpr int kMaxD = 256;
constexpr int kMaxK = 65536;
constexpr int kColTile = 32;        // MFMA output columns per tile (one 32x32 block)
constexpr int kSegLen = 4096;       // sorted positions per wave in the statistics reduction
constexpr int kChunk = 16384;       // labels per workgroup in the histogram / scatter passes
constexpr int kLdsHistMaxK = 16384; // histogram bins kept in LDS (int32)
constexpr int kMainWaves = 4;       // waves per workgroup in the fused GEMM+epilogue kernel

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// D rounded up to the GEMM depth the MFMA kernels are instantiated for: 16, 32, 64, 128, 256.
__host__ __device__ inline int padded_depth(int D) {
  int p = 16;
  while (p < D) p *= 2;
  return p;
}

// ------------------------------------------------------------------------------------------
// workspace layout (byte offsets from the workspace base; every region 256-byte aligned)

struct WsLayout {
  size_t hdr;      // int32[64]: [0] status, [1] valid points, [2] non-empty clusters
  size_t count;    // int32[K]       N_k
  size_t offset;   // int32[K+1]     exclusive prefix of N_k (cluster start in sorted order)
  size_t cursor;   // int32[K]       scatter cursors
  size_t V;        // f64[K*D]       Y_k or Omega_k
  size_t psi;      // f64[K]         Psi_k
  size_t segpart;  // f64[nseg*2*(D+1)] partial sums of runs cut by segment borders
  size_t perm;     // int32[N]       row ids sorted by label
  size_t gmean;    // f64[DP]        global mean (centring)
  size_t mvec;     // f32[DP]        global mean as float (centring)
  size_t btab;     // GEMM operand: f32[Kpad*DP] or bf16[2][Kpad*DP] (hi, lo)
  size_t cvec;     // f32[Kpad]      per-cluster constant of the b-path (+inf if empty/pad)
  size_t atab;     // f32[K*DP]      cluster means (centred) for the a-path
  size_t avec;     // f32[K]         sigma_k^2 (sq. Euclidean) or 1-||mu_k||^2 (cosine)
  size_t ascale;   // f32[K]         N_k/(N_k-1), 0 for singletons
  size_t bpart;    // f64[nblocks]   per-workgroup sums of s_i
  size_t save_a;   // f32[N]         a_i            (SIL_FLAG_SAVE_FOR_GRAD)
  size_t save_b;   // f32[N]         b_i
  size_t save_n;   // int32[N]       neighbouring cluster id
  size_t total;
  // shape
  int64_t N;
  int32_t D, DP, K, Kpad;
  int64_t nseg, nblocks;
  int dtype, metric, flags;
};

WsLayout make_layout(int64_t N, int32_t D, int32_t K, int32_t metric, int32_t dtype,
                     int32_t flags);

// Device pointers into one workspace.
struct WsPtrs {
  int32_t* hdr;
  int32_t* count;
  int32_t* offset;
  int32_t* cursor;
  double* V;
  double* psi;
  double* segpart;
  int32_t* perm;
  double* gmean;
  float* mvec;
  void* btab;
  float* cvec;
  float* atab;
  float* avec;
  float* ascale;
  double* bpart;
  float* save_a;
  float* save_b;
  int32_t* save_n;
};

WsPtrs carve(const WsLayout& L, void* ws);

// Status codes written into hdr[0] by kernels (first error wins).
__device__ inline void set_status(int32_t* hdr, int32_t code) { atomicCAS(hdr, 0, code); }

// ------------------------------------------------------------------------------------------
// launchers (one per translation unit)

struct Problem {
  const void* X;
  const float* col_scale;
  const int32_t* labels;
  int64_t N;
  int32_t D, DP, K, Kpad;
  int dtype, metric, products, flags;
  float* s;
  double* S;
  int64_t nblocks;  // workgroups of the fused kernel for this call
};

// zero the small workspace regions; histogram, scan, scatter, segmented reduction, combine
hipError_t launch_stats(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// global mean, per-cluster tables
hipError_t launch_finalize(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// fused GEMM + epilogue, then the fixed-order reduction of S
hipError_t launch_main(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
hipError_t launch_reduce(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// copy statistics out of the workspace
hipError_t launch_copy_stats(const Problem& p, const WsLayout& L, const WsPtrs& w, int32_t* count,
                             double* V, double* psi, hipStream_t st);

// rows per workgroup of the fused kernel for this problem (host and workspace sizing)
int main_rows_per_block(int dtype, int DP, int products);

}  // namespace sil
