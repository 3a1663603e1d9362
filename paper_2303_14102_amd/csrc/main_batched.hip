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

// Rows p0 + 32 nb + lane%32 of a group, in their original order, with the labels of problem q.
static __device__ __forceinline__ RowPre<kBatchNBMax> group_rows(const BatchProblem& q, int64_t wb,
                                                                 int wave, int lane) {
  const int64_t p0 = wb * (kMainWaves * 32 * q.nb) + wave * 32 * q.nb;
  RowPre<kBatchNBMax> pre;
#pragma unroll
  for (int nb = 0; nb < kBatchNBMax; ++nb) {
    const int64_t pos = p0 + nb * 32 + (lane & 31);
    const bool ok = nb < q.nb && pos < q.N;
    pre.row[nb] = ok ? static_cast<int32_t>(pos) : 0;
    pre.lab[nb] = ok ? q.labels[pos] : -1;
  }
  return pre;
}

// The a-path term of each row for the labels in B (the prologue's, for another problem of the
// group): ||v - mu'_o||^2 from the rows' transformed chunks v (areg) and the own cluster's mean.
template <int NB, int NQ, int METRIC>
__device__ __forceinline__ void group_apath(const MainArgs& a, const Blocks<NB>& B, int lane,
                                            const f32x4_t (&areg)[NB][NQ], float (&arow)[NB]) {
  constexpr int DPX = 8 * NQ;
  const int h = lane >> 5;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int32_t o = B.lab[nb];
    const int64_t orow = static_cast<int64_t>(o >= 0 ? o : 0) * DPX;
    float ad = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float at[4];
      load_f32w<4>(a.atab + orow + (2 * q + h) * 4, at);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float dd = areg[nb][q][e] - at[e];
        ad = fmaf(dd, dd, ad);
      }
    }
    ad += __shfl_xor(ad, 32, 64);
    if (o >= 0) {
      const float sc = a.ascale[o];
      arow[nb] = METRIC == SIL_SQEUCLID ? sc * (ad + a.avec[o]) : sc * 0.5f * (a.avec[o] + ad);
    } else {
      arow[nb] = 0.0f;
    }
  }
}

// One item of a group: a block of rows in their original order, loaded, centred (with the
// leader's centring vector, which every member's tables use) and split into MFMA operands once;
// then each member in turn sweeps its own cluster tiles over them (the rows' own clusters differ
// within a block, so every block takes the per-element own-cluster test) and writes its s_i and
// block sum.  The next member's first tiles and labels load while the current one finishes.
template <int DPX, int NB, int METRIC>
__device__ __forceinline__ void group_body(const BatchDev& b, int lead, int64_t wb,
                                           const RowPre<kBatchNBMax>& pre0, uint8_t* ring0,
                                           uint8_t* ring1, float* lds_min, int32_t* lds_arg,
                                           int32_t* lds_lab, int tid) {
  constexpr int NQ = DPX / 8;
  constexpr int RS = table_stride(DPX, SIL_F32);
  using R = f32_ring<DPX, 2>;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int col = lane & 31, h = lane >> 5;
  const int64_t p0 = wb * (kMainWaves * NB * 32) + wave * NB * 32;
  int32_t* lab_w = lds_lab + wave * NB * 32;

  int j = lead;
  MainArgs a = batch_args(b.prob[j]);
  RowPre<NB> pre;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    pre.row[nb] = pre0.row[nb];
    pre.lab[nb] = pre0.lab[nb];
  }
  Blocks<NB> B;
  make_blocks<NB>(a, pre, p0, lane, B, lab_w);
  f32x4_t areg[NB][NQ];
  float nrow[NB], arow[NB];
  prologue<SIL_F32, 4, NQ, NB, METRIC, false>(
      a, B, lane, nrow, arow, [&](int nb, int q, const float* v) __attribute__((always_inline)) {
        areg[nb][q] = f32x4_t{v[0], v[1], v[2], v[3]};
      });

  auto bfrag = [&](const uint8_t* st, int cb, int q) __attribute__((always_inline)) {
    return *reinterpret_cast<const f32x4_t*>(st + ((cb * 32 + col) * RS + 4 * (2 * q + h)) * 4);
  };
  for (;;) {
    float mn[NB][16];
    int32_t arg[NB][16];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        mn[nb][e] = __builtin_inff();
        arg[nb][e] = -1;
      }
    auto gemm = [&](const uint8_t* st, int cb, f32x16_t (&acc)[NB], auto&& after_first_read)
        __attribute__((always_inline)) {
      f32x4_t bv[2];
      bv[0] = bfrag(st, cb, 0);
      after_first_read();
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q + 1 < NQ) bv[(q + 1) & 1] = bfrag(st, cb, q + 1);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            if (q == 0 && e == 0)
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(areg[nb][0][0], bv[0][0], f32x16_t{},
                                                             0, 0, 0);
            else
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(areg[nb][q][e], bv[q & 1][e],
                                                             acc[nb], 0, 0, 0);
          }
      }
    };
    auto epi = [&](const f32x16_t (&acc)[NB], int blk, float cv) __attribute__((always_inline)) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        tile_min<false>(acc[nb], mn[nb], arg[nb], B.mixed[nb], blk == B.town[nb], col,
                        B.cown[nb], 32 * blk, lab_w + nb * 32, h, cv);
    };
    f32x16_t acc0[NB], acc1[NB];
    float c1p = 0.0f;
    const bool last_b1 = 64 * (a.ntiles - 1) + 32 < a.K;
    sweep<R>(static_cast<const char*>(a.btab), a.piece * 4, a.ntiles, ring0, ring1, ring1, wave,
             lane, [&](int t, const uint8_t* st, auto&& prefetch) __attribute__((always_inline)) {
               const float c0 = a.ctab[64 * t + col], c1 = a.ctab[64 * t + 32 + col];
               gemm(st, 0, acc0, prefetch);
               if (t > 0) epi(acc1, 2 * t - 1, c1p);
               if (t + 1 < a.ntiles || last_b1) gemm(st, 1, acc1, [] {});
               epi(acc0, 2 * t, c0);
               c1p = c1;
             });
    if (last_b1) epi(acc1, 2 * a.ntiles - 1, c1p);
    __syncthreads();  // every wave is done with the ring and with lab_w
    const int jn = __builtin_amdgcn_readfirstlane(b.prob[j].grp_next);
    RowPre<kBatchNBMax> pn{};
    if (jn >= 0) {
      const BatchProblem& qn = b.prob[jn];
      issue_first<R>(static_cast<const char*>(qn.btab),
                     static_cast<int64_t>(qn.Kpad) * RS * 4, qn.Kpad / kColTile, ring0, ring1,
                     wave, lane);
      pn = group_rows(qn, wb, wave, lane);
    }
    finish<NB, METRIC, false>(a, wb, B, wave, lane, mn, arg, nrow, arow, lds_min + wave * NB * 32,
                              lds_arg + wave);
    if (jn < 0) break;
    j = jn;
    a = batch_args(b.prob[j]);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      pre.row[nb] = pn.row[nb];
      pre.lab[nb] = pn.lab[nb];
    }
    make_blocks<NB>(a, pre, p0, lane, B, lab_w);
    group_apath<NB, NQ, METRIC>(a, B, lane, areg, arow);
  }
}

// First table tiles of the block, then the block body, for the problem's depth and rows.
template <int METRIC>
__device__ __forceinline__ void batch_body(const MainArgs& a, int DPX, int nb, int64_t wb,
                                           const RowPre<kBatchNBMax>& pre, uint8_t* r0,
                                           uint8_t* r1, float* lmin, int32_t* larg, int32_t* llab, int tid) {
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
    main_f32_body<DP, NB, METRIC, false, 2>(a, wb, p, r0, r1, r1, lmin, larg, llab, tid); \
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

template <int METRIC>
__device__ __forceinline__ void batch_group(const BatchDev& b, int lead, int DPX, int nb, int64_t wb,
                                            const RowPre<kBatchNBMax>& pre, uint8_t* r0,
                                            uint8_t* r1, float* lmin, int32_t* larg, int32_t* llab, int tid) {
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const BatchProblem& q = b.prob[lead];
#define SIL_GROUP(DP, NB)                                                                      \
  do {                                                                                         \
    issue_first<f32_ring<DP, 2>>(static_cast<const char*>(q.btab),                              \
                                 static_cast<int64_t>(q.Kpad) * table_stride(DP, SIL_F32) * 4,  \
                                 q.Kpad / kColTile, r0, r1, wave, lane);                        \
    group_body<DP, NB, METRIC>(b, lead, wb, pre, r0, r1, lmin, larg, llab, tid);         \
  } while (0)
  switch (DPX) {
    case 16:
      if (nb == 2) SIL_GROUP(16, 2);
      else SIL_GROUP(16, 1);
      break;
    case 24:
      if (nb == 2) SIL_GROUP(24, 2);
      else SIL_GROUP(24, 1);
      break;
    case 32:
      if (nb == 2) SIL_GROUP(32, 2);
      else SIL_GROUP(32, 1);
      break;
    case 48:
      SIL_GROUP(48, 1);
      break;
    case 64:
      SIL_GROUP(64, 1);
      break;
    case 96:
      SIL_GROUP(96, 1);
      break;
    default:
      SIL_GROUP(128, 1);
      break;
  }
#undef SIL_GROUP
}

__global__ __launch_bounds__(256, 2) void k_main_f32_batched(BatchDev b, int32_t total,
                                                             int32_t grab) {
  __shared__ __attribute__((aligned(16))) uint8_t ring0[RingMax::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[RingMax::STAGE_BYTES];
  __shared__ float lds_min[kMainWaves * kBatchNBMax * 32];
  __shared__ int32_t lds_arg[kMainWaves];
  __shared__ __attribute__((aligned(16))) int32_t lds_lab[kMainWaves * kBatchNBMax * 32];
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
    auto item_rows = [&](int jq, int32_t item) __attribute__((always_inline)) {
      const BatchProblem& qq = b.prob[b.order[jq]];
      const int64_t w = item - pre_items[jq];
      return qq.grp_n > 1 ? group_rows(qq, w, wave0, lane0) : batch_rows(qq, w, wave0, lane0);
    };
    RowPre<kBatchNBMax> rows = item_rows(jc, base);
    for (int32_t it = base; it < end; ++it) {
      const BatchProblem& q = b.prob[b.order[jc]];
      const int64_t wb = it - uniform(pre_items[jc]);
      // the next item's row ids and labels load while this item runs
      RowPre<kBatchNBMax> nrows = rows;
      int jn = jc;
      if (it + 1 < end) {
        jn = uniform(batch_locate(pre_items, n, it + 1));
        nrows = item_rows(jn, it + 1);
      }
      const MainArgs a = batch_args(q);
      // an opaque copy of the thread index: keeps the body's lane-dependent addresses out of
      // the loop (hoisting them would exceed the register budget)
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      if (q.grp_n > 1) {
        const int lead = uniform(b.order[jc]);
        if (q.metric == SIL_SQEUCLID)
          batch_group<SIL_SQEUCLID>(b, lead, q.DPX, q.nb, wb, rows, ring0, ring1, lds_min,
                                    lds_arg, lds_lab, tid);
        else
          batch_group<SIL_COSINE>(b, lead, q.DPX, q.nb, wb, rows, ring0, ring1, lds_min, lds_arg,
                                  lds_lab, tid);
      } else if (q.metric == SIL_SQEUCLID) {
        batch_body<SIL_SQEUCLID>(a, q.DPX, q.nb, wb, rows, ring0, ring1, lds_min, lds_arg,
                                 lds_lab, tid);
      } else {
        batch_body<SIL_COSINE>(a, q.DPX, q.nb, wb, rows, ring0, ring1, lds_min, lds_arg, lds_lab, tid);
      }
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
