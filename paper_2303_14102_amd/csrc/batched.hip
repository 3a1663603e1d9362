// Batched evaluation: many Silhouette problems (for instance the labelings of a k-sweep over one
// or several data sets) in a fixed number of launches, the fused GEMM + epilogue of all of them
// in one persistent launch.
//
// A plan (host object) validates the problem descriptors, lays out one workspace holding every
// problem's own region plus a batch header (device descriptors, the per-phase work-item
// prefixes, the queue order of the persistent kernel and its counter), and keeps the launch
// configuration.  The autotuner times the persistent launch over the plan's own problems for a
// few configurations (rows per work item for shallow GEMM depths, grid size, items per queue
// access, queue order) and keeps the fastest.  A run can be captured once into a hipGraph and
// replayed: the graph holds only kernels (counters are cleared by kernels, not memsets); the
// descriptors it reads are uploaded to the workspace before the capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "sil_internal.h"

using namespace sil;

struct sil_plan {
  std::vector<sil_problem> prob;
  std::vector<WsLayout> L;
  std::vector<size_t> off;      // per-problem region in the workspace
  std::vector<int32_t> nb;      // 32-row blocks per wave in the fused kernel, per problem
  int32_t flags = 0;
  int32_t grid = 0, grab = 1, order_mode = 0;
  int32_t share_x = 1;          // group problems that share X (see BatchProblem::grp_n)
  int32_t cus = 0;
  size_t hdr_bytes = 0, total = 0;
  // batch header layout (offsets from the workspace base)
  size_t o_prob = 0, o_prefix = 0, o_order = 0, o_queue = 0;
  // host staging of the header (pinned); the workspace it was last uploaded to
  uint8_t* staging = nullptr;
  const void* uploaded_ws = nullptr;
  BatchLaunch launch{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// cost of one work item of the persistent kernel (table elements swept x rows)
double item_cost(const WsLayout& L, int nb) {
  return static_cast<double>(L.Kpad) * static_cast<double>(L.DPX) * nb;
}

// Group leader of every problem: the first problem with the same X, N, D, metric, flags and row
// blocks per wave when X is shared, else the problem itself.
std::vector<int> group_leaders(const sil_plan* P) {
  const int n = static_cast<int>(P->prob.size());
  std::vector<int> lead(n);
  for (int i = 0; i < n; ++i) {
    lead[i] = i;
    if (!P->share_x) continue;
    const sil_problem& u = P->prob[i];
    for (int j = 0; j < i; ++j) {
      const sil_problem& v = P->prob[j];
      if (lead[j] == j && v.X == u.X && v.N == u.N && v.D == u.D && v.metric == u.metric &&
          P->nb[j] == P->nb[i]) {
        lead[i] = j;
        break;
      }
    }
  }
  return lead;
}

// Build the header (descriptors, prefixes, queue order) for workspace `ws` into the staging
// buffer and the launch description; returns the bytes to upload.
size_t build_header(sil_plan* P, void* ws) {
  const int n = static_cast<int>(P->prob.size());
  const std::vector<int> lead = group_leaders(P);
  uint8_t* base = static_cast<uint8_t*>(ws);
  std::memset(P->staging, 0, P->hdr_bytes);
  BatchProblem* bp = reinterpret_cast<BatchProblem*>(P->staging + P->o_prob);
  int32_t* prefix = reinterpret_cast<int32_t*>(P->staging + P->o_prefix);
  int32_t* order = reinterpret_cast<int32_t*>(P->staging + P->o_order);
  std::vector<int64_t> cnt(static_cast<size_t>(BP_COUNT) * n, 0);
  int32_t maxK = 0;
  for (int i = 0; i < n; ++i) {
    const sil_problem& u = P->prob[i];
    const WsLayout& L = P->L[i];
    const WsPtrs w = carve(L, base + P->off[i]);
    BatchProblem& q = bp[i];
    q.X = u.X;
    q.col_scale = nullptr;
    q.labels = u.labels;
    q.s = u.s;
    q.S = u.S;
    q.N = L.N;
    q.D = L.D;
    q.DPX = L.DPX;
    q.K = L.K;
    q.Kpad = L.Kpad;
    q.dtype = SIL_F32;
    q.metric = u.metric;
    q.flags = u.metric == SIL_COSINE ? (P->flags & ~SIL_FLAG_EUCLID_APPROX) : P->flags;
    q.nb = P->nb[i];
    q.nseg = L.nseg;
    q.nblocks = ceil_div(L.N, kMainWaves * 32 * q.nb);
    q.zero_words = static_cast<int64_t>((L.perm - L.hdr) / 4);
    stats_lanes(L.D, SIL_F32, &q.Gv, &q.G, &q.E);
    q.rowch = u.metric == SIL_SQEUCLID ? row_chunk(L.D, SIL_F32) : 0;
    reduce_split(q.nblocks * kMainWaves, &q.red_chunk, &q.red_n1);  // one partial per wave
    q.hdr = w.hdr;
    q.count = w.count;
    q.offset = w.offset;
    q.cursor = w.cursor;
    q.V = w.V;
    q.psi = w.psi;
    q.segpart = w.segpart;
    q.perm = w.perm;
    q.lsorted = w.lsorted;
    q.gmean = w.gmean;
    q.mvec = w.mvec;
    q.btab = w.btab;
    q.ctab = w.ctab;
    q.atab = w.atab;
    q.avec = w.avec;
    q.ascale = w.ascale;
    q.bpart = w.bpart;
    q.bpart2 = w.bpart2;
    maxK = std::max(maxK, L.K);
    int64_t* c = &cnt[static_cast<size_t>(i) * BP_COUNT];
    c[BP_ZERO] = ceil_div(q.zero_words, kZeroWordsPerItem);
    c[BP_HIST] = ceil_div(L.N, kChunk);
    c[BP_SCAN] = 1;
    c[BP_SEG] = ceil_div(L.nseg, 4);
    c[BP_COMBINE] = ceil_div(static_cast<int64_t>(L.K) * (L.D + 1), 256);
    c[BP_GMEAN] = L.DPX;
    c[BP_FIN] = ceil_div(L.Kpad, 4);
    c[BP_MAIN] = q.nblocks;
    c[BP_RED1] = q.red_n1;
    c[BP_RED2] = 1;
    c[BP_POISON] = q.s ? ceil_div(L.N, kPoisonPerItem) : 0;
    q.grp_n = 1;
    q.grp_next = -1;
  }
  // groups: members take the leader's centring vector (so that every member's tables fit the
  // rows as the leader centres them) and leave their fused-kernel items to the leader
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) cost[i] = item_cost(P->L[i], P->nb[i]);
  std::vector<int> last(n);
  for (int i = 0; i < n; ++i) last[i] = i;
  for (int i = 0; i < n; ++i) {
    const int l = lead[i];
    if (l == i) continue;
    const WsPtrs wl = carve(P->L[l], base + P->off[l]);
    bp[i].gmean = wl.gmean;
    bp[i].mvec = wl.mvec;
    cnt[static_cast<size_t>(i) * BP_COUNT + BP_GMEAN] = 0;
    cnt[static_cast<size_t>(i) * BP_COUNT + BP_MAIN] = 0;
    bp[last[l]].grp_next = i;
    last[l] = i;
    bp[l].grp_n += 1;
    cost[l] += cost[i];
  }
  // queue order of the persistent kernel: costliest items first, or problem order
  std::vector<int32_t> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  if (P->order_mode == 0)
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  for (int j = 0; j < n; ++j) order[j] = ord[j];
  BatchLaunch& B = P->launch;
  for (int ph = 0; ph < BP_COUNT; ++ph) {
    int32_t* pre = prefix + ph * (n + 1);
    int64_t run = 0;
    for (int j = 0; j < n; ++j) {
      pre[j] = static_cast<int32_t>(run);
      const int i = ph == BP_MAIN ? ord[j] : j;
      run += cnt[static_cast<size_t>(i) * BP_COUNT + ph];
    }
    pre[n] = static_cast<int32_t>(run);
    B.items[ph] = run;
  }
  B.dev.prob = reinterpret_cast<const BatchProblem*>(base + P->o_prob);
  B.dev.prefix = reinterpret_cast<const int32_t*>(base + P->o_prefix);
  B.dev.order = reinterpret_cast<const int32_t*>(base + P->o_order);
  B.dev.queue = reinterpret_cast<int32_t*>(base + P->o_queue);
  B.dev.n = n;
  B.maxK = maxK;
  B.main_grid = P->grid;
  B.main_grab = P->grab;
  return P->hdr_bytes;
}

// Upload the header unless this workspace already holds it for the current configuration.
int upload(sil_plan* P, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || ws_bytes < P->total) return SIL_E_WORKSPACE;
  if (P->uploaded_ws == ws) return SIL_OK;
  const size_t bytes = build_header(P, ws);
  if (hipMemcpyAsync(ws, P->staging, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return SIL_E_HIP;
  // the staging buffer is rewritten by the next upload: wait for this copy
  if (hipStreamSynchronize(st) != hipSuccess) return SIL_E_HIP;
  P->uploaded_ws = ws;
  return SIL_OK;
}

int launch_all(sil_plan* P, hipStream_t st) {
  const BatchLaunch& B = P->launch;
  if (launch_stats_batched(B, st) != hipSuccess) return SIL_E_HIP;
  if (launch_finalize_batched(B, st) != hipSuccess) return SIL_E_HIP;
  if (launch_main_batched(B, st) != hipSuccess) return SIL_E_HIP;
  if (launch_reduce_batched(B, st) != hipSuccess) return SIL_E_HIP;
  return SIL_OK;
}

void drop_graph(sil_plan* P) {
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->exec = nullptr;
  P->graph = nullptr;
}

// mean time of `reps` persistent launches with the current configuration (after one warm-up)
int time_main(sil_plan* P, void* ws, size_t ws_bytes, hipStream_t st, int reps, float* ms) {
  int rc = upload(P, ws, ws_bytes, st);
  if (rc) return rc;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SIL_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SIL_E_HIP;
  }
  rc = SIL_OK;
  if (launch_main_batched(P->launch, st) != hipSuccess) rc = SIL_E_HIP;
  if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = SIL_E_HIP;
  for (int r = 0; r < reps && !rc; ++r)
    if (launch_main_batched(P->launch, st) != hipSuccess) rc = SIL_E_HIP;
  if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = SIL_E_HIP;
  if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = SIL_E_HIP;
  float t = 0.0f;
  if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = SIL_E_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return rc;
}

}  // namespace

extern "C" {

int silhouette_batched_plan(const sil_problem* problems, int32_t count, int32_t flags,
                            sil_plan** plan) {
  if (!plan) return SIL_E_ARG;
  *plan = nullptr;
  if (!problems || count < 1 || count > kBatchMaxProblems) return SIL_E_ARG;
  if (flags & ~(SIL_FLAG_NO_CENTRE | SIL_FLAG_EUCLID_APPROX)) return SIL_E_ARG;
  for (int i = 0; i < count; ++i) {
    const sil_problem& u = problems[i];
    if (!u.X || !u.labels || !u.S || (reinterpret_cast<uintptr_t>(u.X) & 15u)) return SIL_E_ARG;
    if (u.N < 1 || u.N > INT32_MAX || u.D < 1 || u.D > kBatchMaxD || u.K < 2 ||
        u.K > kLdsHistMaxK)
      return SIL_E_ARG;
    if (u.metric != SIL_SQEUCLID && u.metric != SIL_COSINE) return SIL_E_ARG;
    if (u.dtype != SIL_F32) return SIL_E_DTYPE;
  }
  sil_plan* P = new (std::nothrow) sil_plan;
  if (!P) return SIL_E_ARG;
  P->prob.assign(problems, problems + count);
  P->flags = flags;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete P;
    return SIL_E_HIP;
  }
  P->cus = prop.multiProcessorCount;
  P->grid = 2 * P->cus;
  P->grab = 1;
  P->order_mode = 0;
  // header: descriptors, prefixes, order, queue
  size_t o = 0;
  P->o_prob = o;
  o = align256(o + sizeof(BatchProblem) * count);
  P->o_prefix = o;
  o = align256(o + sizeof(int32_t) * BP_COUNT * (count + 1));
  P->o_order = o;
  o = align256(o + sizeof(int32_t) * count);
  P->o_queue = o;
  o = align256(o + 256);
  P->hdr_bytes = o;
  for (int i = 0; i < count; ++i) {
    const sil_problem& u = problems[i];
    const int32_t fl = u.metric == SIL_COSINE ? 0 : (flags & (SIL_FLAG_NO_CENTRE | SIL_FLAG_EUCLID_APPROX));
    P->L.push_back(make_layout(u.N, u.D, u.K, u.metric, SIL_F32, fl));
    P->off.push_back(o);
    o = align256(o + P->L.back().total);
    P->nb.push_back(1);
  }
  P->total = o;
  if (hipHostMalloc(reinterpret_cast<void**>(&P->staging), P->hdr_bytes, hipHostMallocDefault) !=
      hipSuccess) {
    delete P;
    return SIL_E_HIP;
  }
  *plan = P;
  return SIL_OK;
}

size_t silhouette_batched_workspace_bytes(const sil_plan* plan) { return plan ? plan->total : 0; }

int silhouette_batched_run(sil_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return SIL_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = upload(plan, ws, ws_bytes, st);
  if (rc) return rc;
  return launch_all(plan, st);
}

int silhouette_batched_tune(sil_plan* plan, void* ws, size_t ws_bytes, void* stream,
                            float* best_ms) {
  if (!plan) return SIL_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  drop_graph(plan);
  plan->uploaded_ws = nullptr;
  // statistics and tables once: the persistent kernel only reads them
  int rc = silhouette_batched_run(plan, ws, ws_bytes, stream);
  if (rc) return rc;
  const int reps = 3;
  float best = 0.0f;
  rc = time_main(plan, ws, ws_bytes, st, reps, &best);
  if (rc) return rc;
  auto consider = [&](auto&& apply, auto&& undo) -> int {
    apply();
    plan->uploaded_ws = nullptr;
    float t = 0.0f;
    const int r = time_main(plan, ws, ws_bytes, st, reps, &t);
    if (r) return r;
    if (t < best) {
      best = t;
    } else {
      undo();
      plan->uploaded_ws = nullptr;
    }
    return SIL_OK;
  };
  // rows per work item, one depth class at a time
  for (int dpx : kShallowDepths) {
    std::vector<int> idx;
    for (size_t i = 0; i < plan->prob.size(); ++i)
      if (plan->L[i].DPX == dpx) idx.push_back(static_cast<int>(i));
    if (idx.empty()) continue;
    rc = consider([&] { for (int i : idx) plan->nb[i] = 2; },
                  [&] { for (int i : idx) plan->nb[i] = 1; });
    if (rc) return rc;
  }
  // workgroups of the persistent grid
  for (int g : {1, 3}) {
    const int old = plan->grid;
    rc = consider([&] { plan->grid = g * plan->cus; }, [&] { plan->grid = old; });
    if (rc) return rc;
  }
  // items per queue access
  for (int gr : {2, 4}) {
    const int old = plan->grab;
    rc = consider([&] { plan->grab = gr; }, [&] { plan->grab = old; });
    if (rc) return rc;
  }
  // queue order
  {
    const int old = plan->order_mode;
    rc = consider([&] { plan->order_mode = 1; }, [&] { plan->order_mode = old; });
    if (rc) return rc;
  }
  // problems that share X: one pass over the rows for all of them, or one per problem
  {
    const int old = plan->share_x;
    rc = consider([&] { plan->share_x = !old; }, [&] { plan->share_x = old; });
    if (rc) return rc;
  }
  if (best_ms) *best_ms = best;
  // leave the workspace consistent with the chosen configuration
  plan->uploaded_ws = nullptr;
  return silhouette_batched_run(plan, ws, ws_bytes, stream);
}

int silhouette_batched_config(const sil_plan* plan, int32_t* out, int32_t len) {
  if (!plan || !out || len < 6) return SIL_E_ARG;
  out[0] = plan->grid;
  out[1] = plan->grab;
  out[2] = plan->order_mode;
  for (int c = 0; c < 3; ++c) out[3 + c] = 1;
  for (size_t i = 0; i < plan->prob.size(); ++i)
    for (int c = 0; c < 3; ++c)
      if (plan->L[i].DPX == kShallowDepths[c]) out[3 + c] = plan->nb[i];
  if (len >= 7) out[6] = plan->share_x;
  return SIL_OK;
}

int silhouette_batched_set_config(sil_plan* plan, const int32_t* cfg, int32_t len) {
  if (!plan || !cfg || len < 6) return SIL_E_ARG;
  if (cfg[0] < 1 || cfg[0] > 65536 || cfg[1] < 1 || cfg[1] > 64 || cfg[2] < 0 || cfg[2] > 1)
    return SIL_E_ARG;
  for (int c = 0; c < 3; ++c)
    if (cfg[3 + c] < 1 || cfg[3 + c] > 2) return SIL_E_ARG;
  if (len >= 7 && (cfg[6] < 0 || cfg[6] > 1)) return SIL_E_ARG;
  plan->grid = cfg[0];
  plan->grab = cfg[1];
  plan->order_mode = cfg[2];
  if (len >= 7) plan->share_x = cfg[6];
  for (size_t i = 0; i < plan->prob.size(); ++i) {
    plan->nb[i] = 1;
    for (int c = 0; c < 3; ++c)
      if (plan->L[i].DPX == kShallowDepths[c]) plan->nb[i] = cfg[3 + c];
  }
  plan->uploaded_ws = nullptr;
  drop_graph(plan);
  return SIL_OK;
}

int silhouette_batched_capture(sil_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !stream) return SIL_E_ARG;  // the legacy default stream cannot be captured
  hipStream_t st = static_cast<hipStream_t>(stream);
  drop_graph(plan);
  int rc = upload(plan, ws, ws_bytes, st);
  if (rc) return rc;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SIL_E_HIP;
  rc = launch_all(plan, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : SIL_E_HIP;
  }
  plan->graph = g;
  if (hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(plan);
    return SIL_E_HIP;
  }
  return SIL_OK;
}

int silhouette_batched_replay(sil_plan* plan, void* stream) {
  if (!plan || !plan->exec) return SIL_E_ARG;
  return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? SIL_OK
                                                                                     : SIL_E_HIP;
}

int silhouette_batched_status(const sil_plan* plan, const void* ws, int32_t* status,
                              void* stream) {
  if (!plan || !ws || !status) return SIL_E_ARG;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return SIL_E_HIP;
  const uint8_t* base = static_cast<const uint8_t*>(ws);
  int first = SIL_OK;
  for (size_t i = 0; i < plan->prob.size(); ++i) {
    int32_t v = 0;
    if (hipMemcpy(&v, base + plan->off[i] + plan->L[i].hdr, sizeof v, hipMemcpyDeviceToHost) !=
        hipSuccess)
      return SIL_E_HIP;
    status[i] = v;
    if (v && !first) first = v;
  }
  return first;
}

void silhouette_batched_free(sil_plan* plan) {
  if (!plan) return;
  drop_graph(plan);
  if (plan->staging) (void)hipHostFree(plan->staging);
  delete plan;
}

}  // extern "C"
