// Persistent fused GEMM + epilogue over a batch of problems (fp32 storage, D <= 128).
//
// One launch covers the row blocks of every problem.  A fixed grid of workgroups takes work
// items from a queue (an integer counter in the workspace, advanced by `grab` items at a time);
// item i of the queue is row block i - prefix[j] of problem order[j], where prefix is the
// per-problem start of its items in queue order.  Every workgroup leaves the loop once the
// counter passes the number of items, so the grid always drains.
//
// Each problem runs the same per-row-block body as the single-problem kernel, picked by its GEMM
// depth, metric and rows per block.  The next item's row ids and labels are loaded while the
// current item runs (within a batch of queue items).  The LDS is laid out for the deepest depth (128) with a
// two-stage table ring, so that two workgroups fit one CU for every depth.  The queue position
// of the next batch of items is fetched while the current batch is computed.
#include "main_kernels.h"

namespace sil {

static constexpr int kBatchDPXMax = 128;
constexpr int kBatchRS = table_stride(kBatchDPXMax, SIL_F32);
using RingMax = Ring<1, kBatchRS * 4, 2>;
constexpr int kBatchNBMax = 2;

// Values read back from LDS are the same in every lane; say so, so that the problem's fields are
// fetched with scalar loads into scalar registers.
static __device__ __forceinline__ int32_t uniform(int32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}

static __device__ __forceinline__ MainArgs batch_args(const BatchProblem& q) {
  MainArgs a;
  a.X = q.X;
  a.col_scale = q.col_scale;
  a.perm = q.perm;
  a.lsorted = q.lsorted;
  a.hdr = q.hdr;
  a.N = q.N;
  a.D = q.D;
  a.K = q.K;
  a.btab = q.btab;
  a.piece = static_cast<int64_t>(q.Kpad) * table_stride(q.DPX, SIL_F32);
  a.ctab = q.ctab;
  a.atab = q.atab;
  a.avec = q.avec;
  a.ascale = q.ascale;
  a.mvec = q.mvec;
  a.ntiles = q.Kpad / kColTile;
  a.root = (q.metric == SIL_SQEUCLID && (q.flags & SIL_FLAG_EUCLID_APPROX)) ? 1 : 0;
  a.s = q.s;
  a.bpart = q.bpart;
  a.save_a = nullptr;
  a.save_b = nullptr;
  a.save_n = nullptr;
  return a;
}

// Row ids and labels of block wb of problem q for this wave (q.nb blocks of 32 rows).
static __device__ __forceinline__ RowPre<kBatchNBMax> batch_rows(const BatchProblem& q, int64_t wb,
                                                                 int wave, int lane) {
  MainArgs a;
  a.perm = q.perm;
  a.lsorted = q.lsorted;
  a.N = q.N;
  const int64_t p0 = wb * (kMainWaves * 32 * q.nb) + wave * 32 * q.nb;
  RowPre<kBatchNBMax> pre;
  const RowPre<1> r0 = fetch_rows<1>(a, p0, lane);
  pre.row[0] = r0.row[0];
  pre.lab[0] = r0.lab[0];
  pre.row[1] = 0;
  pre.lab[1] = -1;
  if (q.nb == 2) {
    const RowPre<1> r1 = fetch_rows<1>(a, p0 + 32, lane);
    pre.row[1] = r1.row[0];
    pre.lab[1] = r1.lab[0];
  }
  return pre;
}

// First table tiles of the block, then the block body, for the problem's depth and rows.
template <int METRIC>
__device__ __forceinline__ void batch_body(const MainArgs& a, int DPX, int nb, int64_t wb,
                                           const RowPre<kBatchNBMax>& pre, uint8_t* r0,
                                           uint8_t* r1, float* lmin, int32_t* larg, int32_t* llab,
                                           double* lbsum, int tid) {
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
#define SIL_BODY(DP, NB)                                                                      \
  do {                                                                                        \
    issue_first<f32_ring<DP, 2>>(static_cast<const char*>(a.btab), a.piece * 4, a.ntiles, r0,  \
                                 r1, wave, lane);                                             \
    RowPre<NB> p;                                                                             \
    for (int i = 0; i < NB; ++i) {                                                            \
      p.row[i] = pre.row[i];                                                                  \
      p.lab[i] = pre.lab[i];                                                                  \
    }                                                                                         \
    main_f32_body<DP, NB, METRIC, false, 2>(a, wb, p, r0, r1, r1, lmin, larg, llab, lbsum, tid); \
  } while (0)
  switch (DPX) {
    case 16:
      if (nb == 2) SIL_BODY(16, 2);
      else SIL_BODY(16, 1);
      break;
    case 24:
      if (nb == 2) SIL_BODY(24, 2);
      else SIL_BODY(24, 1);
      break;
    case 32:
      if (nb == 2) SIL_BODY(32, 2);
      else SIL_BODY(32, 1);
      break;
    case 48:
      SIL_BODY(48, 1);
      break;
    case 64:
      SIL_BODY(64, 1);
      break;
    case 96:
      SIL_BODY(96, 1);
      break;
    default:
      SIL_BODY(128, 1);
      break;
  }
#undef SIL_BODY
}

__global__ __launch_bounds__(256, 2) void k_main_f32_batched(BatchDev b, int32_t total,
                                                             int32_t grab) {
  __shared__ __attribute__((aligned(16))) uint8_t ring0[RingMax::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[RingMax::STAGE_BYTES];
  __shared__ float lds_min[kMainWaves * kBatchNBMax * 32];
  __shared__ int32_t lds_arg[kMainWaves];
  __shared__ __attribute__((aligned(16))) int32_t lds_lab[kMainWaves * kBatchNBMax * 32];
  __shared__ double lds_bsum[kMainWaves];
  __shared__ int32_t pre_items[kBatchMaxProblems + 1];
  __shared__ int32_t next_base;

  const int n = b.n;
  const int32_t* gpre = b.prefix + BP_MAIN * (n + 1);
  for (int i = threadIdx.x; i <= n; i += blockDim.x) pre_items[i] = gpre[i];
  if (threadIdx.x == 0) next_base = atomicAdd(b.queue, grab);
  __syncthreads();
  int32_t base = uniform(next_base);
  while (base < total) {
    // fetch the next batch of items now; its value is needed only after this batch
    int32_t nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(b.queue, grab);
    const int32_t end = base + grab < total ? base + grab : total;
    const int wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane0 = threadIdx.x & 63;
    int jc = uniform(batch_locate(pre_items, n, base));
    RowPre<kBatchNBMax> rows = batch_rows(b.prob[b.order[jc]], base - pre_items[jc], wave0, lane0);
    for (int32_t it = base; it < end; ++it) {
      const BatchProblem& q = b.prob[b.order[jc]];
      const int64_t wb = it - uniform(pre_items[jc]);
      // the next item's row ids and labels load while this item runs
      RowPre<kBatchNBMax> nrows = rows;
      int jn = jc;
      if (it + 1 < end) {
        jn = uniform(batch_locate(pre_items, n, it + 1));
        nrows = batch_rows(b.prob[b.order[jn]], it + 1 - pre_items[jn], wave0, lane0);
      }
      const MainArgs a = batch_args(q);
      // an opaque copy of the thread index: keeps the body's lane-dependent addresses out of
      // the loop (hoisting them would exceed the register budget)
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      if (q.metric == SIL_SQEUCLID)
        batch_body<SIL_SQEUCLID>(a, q.DPX, q.nb, wb, rows, ring0, ring1, lds_min, lds_arg,
                                 lds_lab, lds_bsum, tid);
      else
        batch_body<SIL_COSINE>(a, q.DPX, q.nb, wb, rows, ring0, ring1, lds_min, lds_arg, lds_lab,
                               lds_bsum, tid);
      rows = nrows;
      jc = jn;
    }
    if (threadIdx.x == 0) next_base = nxt;
    __syncthreads();
    base = uniform(next_base);
    __syncthreads();  // next_base is rewritten by the next iteration
  }
}

__global__ void k_queue_reset(int32_t* queue) {
  if (threadIdx.x == 0) queue[0] = 0;
}

hipError_t launch_main_batched(const BatchLaunch& b, hipStream_t st) {
  k_queue_reset<<<1, 64, 0, st>>>(b.dev.queue);
  k_main_f32_batched<<<static_cast<unsigned>(b.main_grid), 256, 0, st>>>(
      b.dev, static_cast<int32_t>(b.items[BP_MAIN]), b.main_grab);
  return hipGetLastError();
}

}  // namespace sil
