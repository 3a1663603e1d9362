// Internal declarations shared by the HIP translation units of the Silhouette library.
// Not part of the public ABI (that is include/silhouette.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/silhouette.h"

namespace sil {

// ------------------------------------------------------------------------------------------
// limits and tiling constants

constexpr int kMaxD = 256;
constexpr int kMaxK = 65536;
constexpr int kColTile = 64;        // clusters per LDS tile of the fused kernel (two 32x32 blocks)
constexpr int kSegLen = 4096;       // sorted positions per wave in the statistics reduction
constexpr int kChunk = 16384;       // labels per workgroup in the histogram / scatter passes
constexpr int kLdsHistMaxK = 16384; // histogram bins kept in LDS (int32)
constexpr int kMainWaves = 4;       // waves per workgroup in the fused GEMM+epilogue kernel

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// GEMM depth of the fused kernels: D rounded up to an instantiated depth class (the
// per-cluster constant is added in the epilogue, not carried in the depth).  A bf16 k-step is 16
// deep, an fp32 one 8 (two halves of 4), so every multiple of 16 up to 64 is its own class and D
// of 16, 32, 64, 128 or 256 runs with no padded columns.
template <int... Ds>
struct DepthList {};
using DepthsBf16 = DepthList<16, 32, 48, 64, 96, 128, 256>;
using DepthsF32 = DepthList<16, 24, 32, 48, 64, 96, 128, 256>;

template <int... Ds>
constexpr int first_depth_at_least(DepthList<Ds...>, int D) {
  int r = 0;
  (void)((D <= Ds ? (r = Ds, true) : false) || ...);
  return r;
}
inline int gemm_depth(int D, int dtype) {
  return dtype == SIL_F32 ? first_depth_at_least(DepthsF32{}, D)
                          : first_depth_at_least(DepthsBf16{}, D);
}
// Calls f(std::integral_constant<int, DPX>{}) for the class equal to DPX (host launchers).
template <int... Ds, typename F>
inline void with_depth(DepthList<Ds...>, int DPX, F&& f) {
  (void)((DPX == Ds ? (f(std::integral_constant<int, Ds>{}), true) : false) || ...);
}

// One-product screen (squared Euclidean, bf16 storage, two-product request): an fp16 MFMA sweep
// finds each row's nearest other cluster, which the epilogue then scores exactly; rows whose two
// best screened values are too close for the screen's error bound go to the two-product kernel.
// Its table row: the fp16 table entries (DPX) and one 16-byte chunk of padding (the odd chunk
// count of table_stride); the per-cluster constant enters as the accumulators' initial value.
constexpr int screen_stride(int DPX) { return DPX + 8; }
constexpr int kScreenMaxDPX = 128;
// Header slots of the screen: 64-bit words from int32 word 16, each the bit pattern of a
// non-negative double raised with integer atomicMax (for such patterns the largest pattern is
// that of the largest value, whatever the order of the updates).
enum ScreenSlot {
  SC_TMAX = 0,  // max |table entry|
  SC_CMAX,      // max |c_k|
  SC_L1,        // max_k || fp16 table row - exact table row ||
  SC_L2,        // max_k || fp16 table row ||
  SC_L3,        // max_k |fl32(c_k)|, the constant the accumulation starts from
  SC_EC,        // max_k |fl32(c_k) - c_k|
  SC_MNORM,     // || centring vector (fp32, as the kernels use it) ||
  SC_COUNT
};
constexpr int kHdrScreenWord = 16;
constexpr int kHdrFallbackWord = 40;  // rows the screen left to the fallback (int32)
constexpr int kHdrFallbackSumWord = 48;  // sum of their s_i (double)
// fp16 scale exponent of the screen table: entries are stored times 2^-f so that the largest lies
// in (2^13, 2^14] (f = 0 for an all-zero table)
__host__ __device__ inline int screen_exponent(double amax) {
  if (!(amax > 0.0)) return 0;
  int e = 0;
  (void)frexp(amax, &e);  // amax = m 2^e, m in [0.5, 1)
  return e - 14;
}

// Row stride of the GEMM table in elements: DPX plus one 16-byte chunk, so that a row spans an
// odd number of 16-byte chunks and the 16 lanes of one LDS read phase hit 16 different bank
// groups.  (Every instantiated DPX spans an even number of chunks.)
constexpr int table_stride(int DPX, int dtype) { return dtype == SIL_F32 ? DPX + 4 : DPX + 8; }

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
  size_t lsorted;  // int32[N]       labels in sorted order
  size_t gmean;    // f64[DPX]       global mean (centring)
  size_t mvec;     // f32[DPX]       global mean as float (centring)
  size_t btab;     // GEMM operand: f32[Kpad*RS] or bf16[2][Kpad*RS] (hi, lo), RS the row stride:
                   //   row k = [alpha mu'_k (D), 0 ...]
  size_t ctab;     // f32[Kpad]      per-cluster constant c_k of the GEMM form (1e30: empty)
  size_t atab;     // f32[K*DPX]     cluster means (centred) for the a-path
  size_t avec;     // f32[K]         sigma_k^2 (sq. Euclidean) or 1-||mu_k||^2 (cosine)
  size_t ascale;   // f32[K]         N_k/(N_k-1), 0 for singletons
  size_t bpart;    // f64[4 max(nblocks, nsblk)] per-wave sums of s_i
  size_t bpart2;   // f64[1024]      first-stage sums of bpart
  size_t save_a;   // f32[N]         a_i            (SIL_FLAG_SAVE_FOR_GRAD)
  size_t save_b;   // f32[N]         b_i
  size_t save_n;   // int32[N]       neighbouring cluster id
  size_t gpart;    // f64[nwg*K*(D+1)] backward: per-workgroup partial A_k, B_k
  size_t gAB;      // f64[K*(D+1)]   backward: A_k (column D) and B_k
  size_t galpha;   // 16 B [N]       backward: per row {own, neighbour, alpha_own, alpha_nbr}
  size_t gtab;     // f32[K*DPX + K] backward: per-cluster terms of dX
  // one-product screen (squared Euclidean with bf16 storage; empty otherwise)
  size_t stab;     // f16[Kpad*screen_stride(DPX)]  screen table
  size_t c64;      // f64[Kpad]      c_k in binary64
  size_t rtab;     // f32[K*DPX]     fp8: the column scales times mu'_k (the exact score's table)
  size_t fblist;   // i32[N]         sorted positions of the rows left to the fallback
  size_t fbpart;   // f64[4 N/128]   per-wave sums of s_i of the fallback rows
  size_t total;
  // shape
  int64_t N;
  int32_t D, DPX, K, Kpad;
  int64_t nseg, nblocks;
  int64_t nsblk;   // screen workgroups; 0 without a screen region
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
  int32_t* lsorted;
  double* gmean;
  float* mvec;
  void* btab;
  float* ctab;
  float* atab;
  float* avec;
  float* ascale;
  double* bpart;
  double* bpart2;
  float* save_a;
  float* save_b;
  int32_t* save_n;
  double* gpart;
  double* gAB;
  void* galpha;
  float* gtab;
  void* stab;
  double* c64;
  float* rtab;
  int32_t* fblist;
  double* fbpart;
};

WsPtrs carve(const WsLayout& L, void* ws);
bool shape_ok(int64_t N, int32_t D, int32_t K);

// Status codes written into hdr[0] by kernels (first error wins).
__device__ inline void set_status(int32_t* hdr, int32_t code) { atomicCAS(hdr, 0, code); }

// ------------------------------------------------------------------------------------------
// launchers (one per translation unit)

struct Problem {
  const void* X;
  const float* col_scale;
  const int32_t* labels;
  int64_t N;
  int32_t D, DPX, K, Kpad;
  int dtype, metric, products, flags;
  float* s;
  double* S;
  int64_t nblocks;  // workgroups of the fused kernel for this call
  int64_t nred = 0; // partials of S for the reduction (0: one per wave of nblocks workgroups)
  // K-means step: the nearest mean of every row over all non-empty clusters goes to labels_out,
  // and S receives the sum of the squared distances to it
  int32_t* labels_out = nullptr;
  int assign = 0;
  // fewer non-empty clusters than this is an error of the statistics pass (0: never)
  int min_nonempty = 2;
  // the reduction returns the sum of the block partials rather than their mean
  int reduce_sum = 0;
  // squared Euclidean, bf16 storage, two products: the one-product screen with exact rescoring
  // and the two-product kernel for the rows it leaves (run_forward sets it)
  int screen = 0;
};

// zero the small workspace regions; histogram, scan, scatter, segmented reduction, combine
hipError_t launch_stats(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// the counting sort alone (zero, histogram, scan, scatter): perm and sorted labels, no sums
hipError_t launch_sort(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// global mean, per-cluster tables
hipError_t launch_finalize(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// fused GEMM + epilogue, then the fixed-order reduction of S
hipError_t launch_main(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
hipError_t launch_reduce(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
// copy statistics out of the workspace
hipError_t launch_copy_stats(const Problem& p, const WsLayout& L, const WsPtrs& w, int32_t* count,
                             double* V, double* psi, hipStream_t st);

// The forward entry points' common body: argument checks against the workspace, then the four
// phases (statistics, tables, fused GEMM + epilogue, reduction) on `stream`.
int run_forward(int32_t metric, const void* X, int32_t dtype, const float* col_scale,
                const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t products,
                int32_t flags, float* s, double* S, void* ws, size_t ws_bytes, void* stream);

// rows per workgroup of the fused kernel for this problem (host and workspace sizing)
int main_rows_per_block(int dtype, int DPX, int products);
// whether a forward call takes the one-product screen
bool screen_applies(int metric, int dtype, int DPX, int products, int flags);
// rows per workgroup of the screen kernel (its workgroups and per-workgroup sums)
int screen_rows_per_block();
// screen tables and bounds after launch_finalize; the screen kernel, the fallback list, the
// two-product kernel over it (launch_main with p.screen); the reduction adds the fallback sums
hipError_t launch_screen_table(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);
hipError_t launch_screen_main(const Problem& p, const WsLayout& L, const WsPtrs& w, hipStream_t st);

// Folded centring.  The two-product bf16 kernels for the squared Euclidean distance take x
// itself (exact in bf16 storage) into the GEMM rather than x' = x - m, and the constant carries
// the centring instead: -2 x'.mu'_k = -2 x.mu'_k + 2 m.mu'_k.  Both products then multiply an
// exact x, so only the split of mu'_k limits the cross term: relative 2^-16 of |x| |mu'_k|,
// where the three-product form on x' reaches 2^-16 of |x'| |mu'_k|.  m is the fp32 centring
// vector the row term uses, so the two agree.
//
// The cosine form does the same with the normalisation: the GEMM multiplies x rather than
// z = x / |x|, and the finish scales the row's minimum by 1 / |x|, since
// min_k (1 - z.mu_k) = 1 + (1 / |x|) min_k (-x.mu_k).  The cross term is then accurate to 2^-16
// of |mu_k| as for BF16x3 on z.
//
// With fp8 storage the GEMM multiplies the e4m3 codes themselves (exact in bf16 whatever the
// column scales) and the tables carry the scales: x.mu = sum_l code_l (s_l mu_l).
template <int DT, int P, int METRIC>
inline constexpr bool kRawX = (DT == SIL_BF16 || DT == SIL_FP8_E4M3) && P == 2 &&
                              (METRIC == SIL_SQEUCLID || METRIC == SIL_COSINE);
inline bool raw_x(int dtype, int products, int metric) {
  return (dtype == SIL_BF16 || dtype == SIL_FP8_E4M3) && products == 2 &&
         (metric == SIL_SQEUCLID || metric == SIL_COSINE);
}
inline bool fold_centre(int dtype, int products, int metric) {
  return raw_x(dtype, products, metric) && metric == SIL_SQEUCLID;
}

// Split products the bf16 kernel runs for a requested count.  When X is stored bf16 and x' = x
// (squared Euclidean without centring, KL) the low bf16 half of x' is zero, so the third product
// adds only zeros: the two-product kernel gives the same sums with a third less MFMA work.
inline int run_products(int metric, int dtype, int flags, int products) {
  const bool exact = dtype == SIL_BF16 && (metric == SIL_KL || (metric == SIL_SQEUCLID &&
                                                                (flags & SIL_FLAG_NO_CENTRE)));
  return exact && products == 3 ? 2 : products;
}

// backward (dS/dX) from the a_i, b_i, neighbour ids kept by a forward call
hipError_t launch_backward(const Problem& p, const WsLayout& L, const WsPtrs& w, const double* gS,
                           float* dX, hipStream_t st);
int bwd_accum_workgroups(int64_t N);
bool bwd_fits_lds(int32_t K, int32_t D);
bool bwd_fits_slices(int32_t K);

// ------------------------------------------------------------------------------------------
// batched evaluation: many problems (labelings of one or several data sets) per launch

constexpr int kBatchMaxProblems = 1024;
constexpr int kBatchMaxD = 128;  // fp32 storage, GEMM depth <= 128
// GEMM depths of the persistent kernel that may run two 32-row blocks per wave (the tuner's
// and silhouette_batched_config's rows-per-item classes, in this order)
constexpr int kShallowDepths[3] = {16, 24, 32};

// One problem of a batch as the kernels see it (device memory, written by the plan).
struct BatchProblem {
  const void* X;
  const float* col_scale;
  const int32_t* labels;
  float* s;
  double* S;
  int64_t N;
  int32_t D, DPX, K, Kpad;
  int32_t dtype, metric, flags, nb;  // nb: 32-row blocks per wave of the fused kernel
  // problems that share their X (the same rows, D and metric: labelings of one data set) form a
  // group led by its first problem: the fused kernel's items of the group are the leader's, in
  // the rows' original order, and run every member over the same loaded rows.  grp_n: members
  // (on the leader; 1 when not grouped), grp_next: the next member (-1 after the last).
  int32_t grp_n, grp_next;
  int64_t nseg, nblocks, zero_words;
  int32_t Gv;        // lanes per row of the 16-byte statistics reduction, 0 for the generic one
  int32_t rowch;     // bytes per lane of the whole-wave row reduction, 0 when not used
  int32_t G, E;      // lanes per row and columns per lane of the generic reduction
  int32_t red_n1;    // first-stage workgroups of the S reduction
  int64_t red_chunk; // partials per first-stage workgroup
  int32_t* hdr;
  int32_t* count;
  int32_t* offset;
  int32_t* cursor;
  double* V;
  double* psi;
  double* segpart;
  int32_t* perm;
  int32_t* lsorted;
  double* gmean;
  float* mvec;
  void* btab;
  float* ctab;
  float* atab;
  float* avec;
  float* ascale;
  double* bpart;
  double* bpart2;
};

// Phases of a batched run; each is one launch over the work items of every problem.
enum BatchPhase {
  BP_ZERO = 0,  // clear the per-problem counters and sums (4096 words per item)
  BP_HIST,      // label histogram and scatter (kChunk labels per item)
  BP_SCAN,      // cluster offsets (one item)
  BP_SEG,       // segmented reduction (4 segments per item)
  BP_COMBINE,   // runs across segments (256 (cluster, column) pairs per item)
  BP_GMEAN,     // centring vector (one item per GEMM depth column)
  BP_FIN,       // tables (4 clusters per item)
  BP_MAIN,      // fused GEMM + epilogue (one 128*nb-row block per item), queue order
  BP_RED1,      // first stage of the S reduction
  BP_RED2,      // second stage (one item)
  BP_POISON,    // NaN outputs of failed problems (65536 points per item)
  BP_COUNT
};
constexpr int kZeroWordsPerItem = 4096;
constexpr int kPoisonPerItem = 65536;

struct BatchDev {
  const BatchProblem* prob;  // [n]
  const int32_t* prefix;     // [BP_COUNT][n + 1] first work item of each problem, per phase
  const int32_t* order;      // [n] problem at each queue position of BP_MAIN
  int32_t* queue;            // [64] work counter of the persistent kernel (word 0)
  int32_t n;
};

// Work-item position -> (problem index into the phase's order, item within the problem).
__device__ __forceinline__ int batch_locate(const int32_t* __restrict__ pre, int n, int32_t item) {
  int lo = 0, hi = n;  // pre[lo] <= item < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

struct BatchLaunch {
  BatchDev dev;
  int64_t items[BP_COUNT];  // total work items per phase
  int32_t maxK;
  int32_t main_grid;        // workgroups of the persistent kernel
  int32_t main_grab;        // work items taken per queue access
  int32_t metric_mask;      // bit m set when some problem uses metric m
};

// lanes per row of the statistics reduction: Gv for 16-byte chunks (0 when D does not split into
// a power-of-two number of them), else G lanes of E columns each
void stats_lanes(int32_t D, int32_t dtype, int32_t* Gv, int32_t* G, int32_t* E);
// bytes per lane when a whole wave reads one row of the statistics pass (0: not that kernel)
int row_chunk(int32_t D, int32_t dtype);
hipError_t launch_stats_batched(const BatchLaunch& b, hipStream_t st);
hipError_t launch_finalize_batched(const BatchLaunch& b, hipStream_t st);
hipError_t launch_main_batched(const BatchLaunch& b, hipStream_t st);
hipError_t launch_reduce_batched(const BatchLaunch& b, hipStream_t st);
// first-stage split of the S reduction over nblocks partials
void reduce_split(int64_t nblocks, int64_t* chunk, int32_t* n1);

}  // namespace sil
