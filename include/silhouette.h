/*
 * silhouette.h — C ABI of the MI355X (gfx950) linear-complexity Silhouette library.
 *
 * Method: M. Gaido, "Distributed Silhouette Algorithm: Evaluating Clustering on Big Data"
 * (arXiv 2303.14102).  For points X[N,D] with cluster labels, the Silhouette of point i is
 * s_i = (b_i - a_i) / max(a_i, b_i) (Section II, Eq.1/Eq.2), where a_i is the mean distance to
 * the other members of its own cluster and b_i the mean distance to the closest other cluster;
 * the overall score is S = sum_i s_i / N.  The mean distance from a point to a whole cluster is
 * obtained from per-cluster statistics in linear time: Eq.11 (squared Euclidean: N_k, Y_k,
 * Psi_k) and Eq.18 (cosine: N_k, Omega_k).
 *
 * Conventions for every entry point
 *  - Pointers named "device" are HIP device pointers; host pointers are marked "host".
 *  - X is row-major [N, D] in the storage given by `dtype` (sil_dtype), at a 16-byte aligned
 *    device address (rows are read as 16-byte vectors; SIL_E_ARG otherwise).  labels is int32
 *    [N] with values in [0, K) (0-based cluster ids; ids may be unused).
 *  - s (optional, may be NULL) receives s_i as float32 [N]; S receives the mean as one float64.
 *  - The caller owns every buffer, including the workspace `ws` (device, at least
 *    silhouette_workspace_bytes(...) bytes, 256-byte aligned).  The library never allocates or
 *    frees device memory.  Calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *    stream) and do not synchronise it.  Calls are re-entrant when they use distinct workspaces.
 *  - Problems visible on the host (sizes, NULL pointers, dtype, workspace too small) return a
 *    negative sil_status at once and launch nothing.  Problems in the data (a label outside
 *    [0, K), a non-finite value, a zero row under the cosine distance, fewer than two non-empty
 *    clusters) are found on the device: the call still returns SIL_OK, S becomes NaN, s becomes
 *    NaN, and silhouette_status() reports the first such error.
 *  - Readings of the paper: a point alone in its cluster has s_i = 0 and counts in N; s_i = 0
 *    when max(a_i, b_i) = 0; a_i and b_i are clamped at 0; b_i ranges over non-empty clusters.
 *  - Limits: 1 <= N <= 2^31 - 1, 1 <= D <= 256, 2 <= K <= 65536.
 */
#ifndef PAPER_2303_14102_AMD_SILHOUETTE_H
#define PAPER_2303_14102_AMD_SILHOUETTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SIL_OK = 0,
  SIL_E_ARG = -1,          /* size out of range or NULL pointer */
  SIL_E_DTYPE = -2,        /* unknown storage type, or fp8 without col_scale */
  SIL_E_LABEL = -3,        /* (device) a label outside [0, K) */
  SIL_E_FEW_CLUSTERS = -4, /* (device) fewer than two non-empty clusters */
  SIL_E_ZERO_NORM = -5,    /* (device) a zero row under the cosine distance */
  SIL_E_NONFINITE = -6,    /* (device) NaN or infinity in X */
  SIL_E_WORKSPACE = -7,    /* workspace NULL, misaligned or smaller than required */
  SIL_E_HIP = -8,          /* a HIP runtime call failed */
  SIL_E_DOMAIN = -9,       /* (device) an entry outside the distance's domain (KL: not > 0) */
  SIL_E_SCRATCH = -10      /* the problem's workspace exceeds SIL_NOALLOC_SCRATCH_BYTES */
} sil_status;

/* Storage of X.  SIL_BF16: bfloat16 values.  SIL_FP8_E4M3: OCP e4m3fn codes, element (i,l)
 * worth code * col_scale[l]. */
typedef enum { SIL_F32 = 0, SIL_BF16 = 1, SIL_FP8_E4M3 = 2 } sil_dtype;

/* SIL_KL: the generalized Kullback-Leibler divergence of positive vectors (silhouette_kl). */
typedef enum { SIL_SQEUCLID = 0, SIL_COSINE = 1, SIL_KL = 2 } sil_metric;

/* Option bits for `flags`. */
enum {
  /* Squared Euclidean only: do not subtract the global mean before the cross term.  Centring is
   * exact for this distance (it is translation invariant) and is on by default. */
  SIL_FLAG_NO_CENTRE = 1 << 0,
  /* Keep a_i, b_i and the neighbouring cluster id of every point in the workspace, as the
   * backward entry points need them (fp32 storage only; SIL_E_DTYPE otherwise). */
  SIL_FLAG_SAVE_FOR_GRAD = 1 << 1,
  /* Squared Euclidean only: the approximate Euclidean Silhouette that the paper names among its
   * limitations (Section V) -- each point-to-cluster mean distance is taken as the square root of
   * the mean squared distance, so a_i and b_i become their square roots before Eq.1.  This is
   * not the exact Euclidean Silhouette (by Jensen's inequality each root is at least the mean
   * Euclidean distance; they agree when all of a point's distances to a cluster are equal).
   * SIL_E_ARG with the cosine entry point or with SIL_FLAG_SAVE_FOR_GRAD. */
  SIL_FLAG_EUCLID_APPROX = 1 << 2,
  /* Squared Euclidean with bf16 storage and two products: run the plain two-product sweep for
   * every point instead of the one-product screen (see silhouette_sqeuclid). */
  SIL_FLAG_NO_SCREEN = 1 << 3
};

/*
 * Device workspace needed by the forward (and backward) calls for this problem shape.
 * `products` as in silhouette_sqeuclid; metric a sil_metric.  Returns 0 for arguments outside
 * the limits.
 */
size_t silhouette_workspace_bytes(int64_t N, int32_t D, int32_t K, int32_t metric, int32_t dtype,
                                  int32_t flags);

/*
 * Silhouette with the squared Euclidean distance (Section III-A, Eq.4-11).
 *   X          device, [N, D] row-major, storage `dtype`
 *   col_scale  device, float32 [D]; required for SIL_FP8_E4M3, ignored otherwise
 *   labels     device, int32 [N]
 *   products   number of bf16 MFMA products for the point-to-cluster-mean cross term when X is
 *              bf16 or fp8: 1 (hi x hi), 2 (adds x x mean_lo), 3 (adds x_lo x mean_hi); 0 picks
 *              the default (3).  Ignored for SIL_F32, which uses fp32 MFMA.  With bf16 storage,
 *              2 multiplies the stored x itself (exact in bf16; with fp8 storage its e4m3 codes,
 *              the column scales going into the cluster-side table): the centring moves into the
 *              per-cluster constant (cosine: 1/|x| scales the row's minimum), and the cross term
 *              is accurate to 2^-16 of |x| |mean| rather than of |x - m| |mean|, m the global
 *              mean.  That matches 3 while |m| is small against the data's spread, at two
 *              thirds of the MFMA work.  For the uncentred squared Euclidean distance and for
 *              KL, 3 runs as 2: x has no low half, so the results are the same.
 *              Squared Euclidean with bf16 storage and 2 (D <= 128): a one-product screen finds
 *              each point's closest other cluster first.  x is exact in fp16 and the cluster-side
 *              table is rounded to fp16, so an fp16 MFMA sweep gives every point-to-cluster
 *              value with a known per-point error bound; when the best value is ahead of the
 *              second by more than twice that bound, the closest cluster is known exactly and
 *              b_i is scored for it alone in fp32; every other point (and every point whose
 *              values fp16 cannot hold exactly) gets the two-product sweep above.  The results
 *              stay within the two-product form's accuracy at about half its MFMA work.
 *              SIL_FLAG_NO_SCREEN runs the two-product sweep for every point.
 *   flags      SIL_FLAG_* bits
 *   s          device, float32 [N], or NULL
 *   S          device, float64 [1]
 *   ws         device workspace, ws_bytes >= silhouette_workspace_bytes(...)
 *   stream     hipStream_t or NULL
 * Returns a sil_status.
 */
int silhouette_sqeuclid(const void* X, int32_t dtype, const float* col_scale,
                        const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t products,
                        int32_t flags, float* s, double* S, void* ws, size_t ws_bytes,
                        void* stream);

/*
 * Silhouette with the cosine distance 1 - x.y/(||x|| ||y||) (Section III-B, Eq.12-18).
 * Arguments as silhouette_sqeuclid; SIL_FLAG_NO_CENTRE is ignored (cosine is never centred).
 */
int silhouette_cosine(const void* X, int32_t dtype, const float* col_scale, const int32_t* labels,
                      int64_t N, int32_t D, int32_t K, int32_t products, int32_t flags, float* s,
                      double* S, void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): silhouette_sqeuclid without a caller workspace.  The
 * library keeps a static device array of SIL_NOALLOC_SCRATCH_BYTES bytes on every GPU it runs
 * on (held until the process ends) and uses it as the workspace; this call allocates and frees
 * nothing.
 *   status   device, int32 [1], or NULL: receives the first device-detected error (SIL_OK if
 *            none), as silhouette_status would report it for a workspace call
 * Other arguments, results and errors as silhouette_sqeuclid.  A problem whose workspace
 * (silhouette_workspace_bytes with the same arguments) exceeds SIL_NOALLOC_SCRATCH_BYTES returns
 * SIL_E_SCRATCH at once and launches nothing; SIL_FLAG_SAVE_FOR_GRAD returns SIL_E_ARG (the
 * backward needs the forward's workspace).  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one GPU (different streams, or host threads) race and must be
 * serialised by the caller; calls in one stream are ordered.  Each call clears the parts of the
 * scratch that must start at zero.  The first call on a device looks up that device's scratch
 * address (a host-side query, no allocation): make it outside graph capture.
 */
#define SIL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int silhouette_sqeuclid_noalloc(const void* X, int32_t dtype, const float* col_scale,
                                const int32_t* labels, int64_t N, int32_t D, int32_t K,
                                int32_t products, int32_t flags, float* s, double* S,
                                int32_t* status, void* stream);

/*
 * Gradient dS/dX of the squared-Euclidean Silhouette with the labels held fixed (not in the
 * paper; derived from Eq.11 by the chain rule through a_i, b_i and the cluster means):
 *   gS   device, float64 [1]   upstream gradient dL/dS
 *   dX   device, float32 [N, D] receives gS * dS/dX
 * Requires X stored fp32 (SIL_E_DTYPE otherwise) and `ws` as left by a silhouette_sqeuclid call
 * on the same X, labels, K and flags with SIL_FLAG_SAVE_FOR_GRAD set (the workspace sized with
 * that flag); the call reuses its statistics, a_i, b_i and neighbour ids.  At a kink (a_i = b_i,
 * or two clusters tying for b_i) it returns one subgradient: the branch a <= b of Eq.2 and the
 * lowest tied cluster id.  Rows of a forward call that reported a device error get NaN.
 * Other arguments as silhouette_sqeuclid.
 */
int silhouette_sqeuclid_backward(const void* X, int32_t dtype, const float* col_scale,
                                 const int32_t* labels, int64_t N, int32_t D, int32_t K,
                                 int32_t flags, const double* gS, float* dX, void* ws,
                                 size_t ws_bytes, void* stream);

/* The same for the cosine distance (derived from Eq.18); requires a silhouette_cosine forward. */
int silhouette_cosine_backward(const void* X, int32_t dtype, const float* col_scale,
                               const int32_t* labels, int64_t N, int32_t D, int32_t K,
                               int32_t flags, const double* gS, float* dX, void* ws,
                               size_t ws_bytes, void* stream);

/*
 * One K-means (Lloyd) step, the producer of the labels that the Silhouette evaluates (the paper's
 * Introduction names K-Means among the clustering methods whose output it scores).  It runs on the
 * same passes as silhouette_sqeuclid:
 *   update   the mean of every non-empty cluster of `labels`, mu_k = Y_k / N_k (Eq.8 sums);
 *   assign   labels_out[i] = the non-empty cluster whose mean is nearest to x_i in squared
 *            Euclidean distance, the lowest id on ties (empty clusters stay empty);
 *   inertia  *inertia = sum_i ||x_i - mu_{labels_out[i]}||^2, reduced in FP64 in a fixed order.
 *   labels_out  device, int32 [N]; may be the same buffer as `labels` (the labels are read only
 *               by the statistics pass, before any label is written)
 *   inertia     device, float64 [1]
 *   products    0 or 3: the BF16x3 form for bf16 / fp8 storage; 2 (bf16 storage only): the
 *               stored x itself with the centring folded into the per-cluster constant, as in
 *               silhouette_sqeuclid.  With fp32 storage only 0 and 3 are accepted (both mean
 *               fp32 MFMA).
 *   flags       0 or SIL_FLAG_NO_CENTRE
 * The distances are formed like the forward call's (centred, split products, fp32 accumulation),
 * so a point whose two nearest means lie within that rounding of each other may take either.
 * Workspace: silhouette_workspace_bytes(N, D, K, SIL_SQEUCLID, dtype, flags).  Errors: as
 * silhouette_sqeuclid, except that one non-empty cluster suffices; on a device-detected error
 * every labels_out[i] becomes -1 and the inertia NaN.
 */
int silhouette_kmeans_step(const void* X, int32_t dtype, const float* col_scale,
                           const int32_t* labels, int64_t N, int32_t D, int32_t K,
                           int32_t products, int32_t flags, int32_t* labels_out, double* inertia,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * Silhouette under the generalized Kullback-Leibler divergence of positive vectors,
 *   d(x, y) = sum_l (x_l log(x_l / y_l) - x_l + y_l),
 * the Bregman divergence of phi(x) = sum_l (x_l log x_l - x_l) (Section V notes that a similar
 * approach serves other metrics).  The distance from point i to point j is d(x_i, x_j), point
 * first.  Its mean over cluster k needs only sum_{y in k} log y and sum_{y in k} sum_l y_l:
 *   m(x, k) = phi(x) + (sum_y sum_l y_l) / N_k - x . (sum_y log y) / N_k,
 * which the statistics pass and the fused kernel form like Eq.11.  Every entry of X must be
 * positive: otherwise the device reports SIL_E_DOMAIN (S and s become NaN).  Storage: fp32 or
 * bf16 (SIL_E_DTYPE for fp8).  flags: 0 (SIL_E_ARG for SIL_FLAG_SAVE_FOR_GRAD or
 * SIL_FLAG_EUCLID_APPROX; SIL_FLAG_NO_CENTRE is ignored, nothing is centred).  Workspace:
 * silhouette_workspace_bytes(N, D, K, SIL_KL, dtype, 0).  Other arguments as silhouette_sqeuclid.
 */
int silhouette_kl(const void* X, int32_t dtype, const float* col_scale, const int32_t* labels,
                  int64_t N, int32_t D, int32_t K, int32_t products, int32_t flags, float* s,
                  double* S, void* ws, size_t ws_bytes, void* stream);

/*
 * Silhouette under a fixed-matrix Mahalanobis distance d(x, y) = (x - y)^T M (x - y), M = L^T L
 * (Section V notes that a similar approach serves other metrics).  The distance is the squared
 * Euclidean distance between L x and L y, so Eq.11 applies to the transformed points: the call
 * forms Z = X L^T once in fp32 (MFMA) inside the workspace, then runs the squared Euclidean
 * Silhouette on Z in fp32.
 *   L      device, float32 [D, D] row-major (any real matrix; M = L^T L is positive
 *          semi-definite, rank-deficient allowed)
 *   flags  0 or SIL_FLAG_NO_CENTRE
 *   ws     device, silhouette_mahalanobis_workspace_bytes(N, D, K, flags) bytes: Z, then a
 *          squared Euclidean fp32 workspace
 * Other arguments, outputs and errors as silhouette_sqeuclid (a non-finite L shows as a
 * non-finite value of the data).
 */
size_t silhouette_mahalanobis_workspace_bytes(int64_t N, int32_t D, int32_t K, int32_t flags);
int silhouette_mahalanobis(const void* X, int32_t dtype, const float* col_scale, const float* L,
                           const int32_t* labels, int64_t N, int32_t D, int32_t K, int32_t flags,
                           float* s, double* S, void* ws, size_t ws_bytes, void* stream);

/*
 * Out-of-core evaluation for data sets larger than device memory.  Section II notes that the
 * quadratic method needs the whole data set on every machine; Section III-A computes the cluster
 * statistics first and then scores every point independently, so a device need only hold a share
 * of the points plus the statistics.  X and labels stay in host memory and are streamed through
 * two device chunk buffers of `chunk_rows` rows, twice: pass 1 accumulates every chunk's
 * statistics into FP64 global sums (in chunk order), pass 2 scores every chunk against the
 * tables of the whole data set.  The result equals silhouette_sqeuclid / silhouette_cosine on
 * the same data up to the order of the FP64 cluster sums (with bf16 storage and two products,
 * the chunks run the plain two-product sweep: SIL_FLAG_NO_SCREEN's result).
 *   metric       SIL_SQEUCLID or SIL_COSINE
 *   X_host       host, [N, D] in `dtype`; pinned (hipHostMalloc) for the uploads to overlap the
 *                kernels, pageable memory works but serialises them
 *   col_scale    device, float32 [D] (fp8 only)
 *   labels_host  host, int32 [N]
 *   s_host       host, float32 [N], or NULL
 *   S            device, float64 [1]
 *   chunk_rows   rows per chunk (>= 1; clamped to N)
 *   flags        SIL_FLAG_NO_CENTRE, SIL_FLAG_EUCLID_APPROX (squared Euclidean only)
 *   ws           device, silhouette_stream_workspace_bytes(...) bytes, 256-byte aligned: one
 *                chunk's workspace, the two chunk buffers and the global sums
 * The call enqueues the work and returns: the host buffers must stay valid and unchanged (and
 * s_host unread) until `stream` has completed.  Uploads run on a copy stream the library creates
 * once per device (default priority, kept until the process ends); events order it against
 * `stream`.  Concurrent calls on one device are serialised while they enqueue.  Errors: as
 * silhouette_sqeuclid (silhouette_status reads the whole data set's status from `ws`).
 */
size_t silhouette_stream_workspace_bytes(int64_t N, int64_t chunk_rows, int32_t D, int32_t K,
                                         int32_t metric, int32_t dtype, int32_t flags);
int silhouette_stream(int32_t metric, const void* X_host, int32_t dtype, const float* col_scale,
                      const int32_t* labels_host, int64_t N, int32_t D, int32_t K,
                      int32_t products, int32_t flags, float* s_host, double* S,
                      int64_t chunk_rows, void* ws, size_t ws_bytes, void* stream);

/*
 * Only the per-cluster statistics pass (one pass over X; Eq.5, Eq.6, Eq.8 for the squared
 * Euclidean distance, Eq.15-16 for cosine), copied out of the workspace:
 *   count  device, int32 [K]        N_k
 *   V      device, float64 [K, D]   Y_k (squared Euclidean) or Omega_k (cosine)
 *   psi    device, float64 [K]      Psi_k (squared Euclidean; zeros for cosine)
 * Any of count/V/psi may be NULL.  Same error behaviour as the forward calls.
 */
int silhouette_cluster_stats(const void* X, int32_t dtype, const float* col_scale,
                             const int32_t* labels, int64_t N, int32_t D, int32_t K,
                             int32_t metric, int32_t* count, double* V, double* psi, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Waits for `stream`, then returns the first device-detected error recorded in `ws` by the last
 * call that used it (SIL_OK if none), or SIL_E_HIP if the wait failed.
 */
int silhouette_status(const void* ws, void* stream);

/* Static English text for a sil_status value. */
const char* silhouette_strerror(int status);

/*
 * Phase timing for benchmarks (not needed for results).  After silhouette_profile_begin(n), the
 * next n forward calls (either metric) record HIP events on their own stream around their four
 * phases: cluster statistics, table finalisation, fused GEMM+epilogue, reduction of S.
 * silhouette_profile_end waits for the last recorded event, writes the summed milliseconds of
 * each phase into ms_sum[4] (host) and the number of recorded calls into *ncalls (host), and
 * stops recording.  Process-wide state: not for concurrent use from several host threads.
 * Returns a sil_status (SIL_E_HIP if an event call failed, SIL_E_ARG for n outside 1..4096).
 */
int silhouette_profile_begin(int32_t max_calls);
int silhouette_profile_end(float* ms_sum, int32_t* ncalls);

/* ---------------------------------------------------------------------------------------------
 * Batched evaluation (a k-sweep: many labelings of one or several data sets).
 *
 * Each problem is the forward above (Section II, Eq.11 / Eq.18) on its own X, labels and K.  A
 * batch runs every problem's statistics, tables, fused GEMM+epilogue and reduction in a fixed
 * number of launches whatever the number of problems; the fused GEMM+epilogue of all problems is
 * one persistent launch whose workgroups take row blocks of any problem from a work queue.
 * Results are those of the single-problem entry points on the same inputs (fp32 storage).
 *
 * Limits per problem: dtype SIL_F32 only (SIL_E_DTYPE otherwise), 1 <= N <= 2^31 - 1,
 * 1 <= D <= 128, 2 <= K <= 16384; 1 <= count <= 1024 problems.
 * -------------------------------------------------------------------------------------------*/
typedef struct sil_problem {
  const void* X;          /* device, [N, D] row-major, storage `dtype` */
  const int32_t* labels;  /* device, int32 [N] in [0, K) */
  int64_t N;
  int32_t D;
  int32_t K;
  int32_t dtype;          /* sil_dtype: SIL_F32 */
  int32_t metric;         /* sil_metric */
  float* s;               /* device, float32 [N], or NULL */
  double* S;              /* device, one float64 */
} sil_problem;

/* Opaque host object: the problems, the workspace layout, the launch configuration chosen by
 * the tuner, and an optional captured hipGraph.  It owns host memory only (a pinned staging
 * buffer for the descriptors it uploads) and the graph. */
typedef struct sil_plan sil_plan;

/*
 * Validates `count` problem descriptors (host array, copied) and creates a plan on the current
 * device.  flags: SIL_FLAG_NO_CENTRE and SIL_FLAG_EUCLID_APPROX bits (both apply to the squared
 * Euclidean problems only).  Problems with the same X pointer, N, D and metric (the labelings of
 * one data set) are evaluated together by default: the fused kernel reads each block of rows
 * once for all of them, and they share the first one's centring vector.  On success *plan is set
 * (free it with silhouette_batched_free); otherwise *plan is NULL and a sil_status is returned.
 */
int silhouette_batched_plan(const sil_problem* problems, int32_t count, int32_t flags,
                            sil_plan** plan);

/* Device workspace bytes for the plan (256-byte aligned buffer owned by the caller; 0 if plan is
 * NULL).  Between calls the workspace belongs to the plan: it keeps the uploaded descriptors. */
size_t silhouette_batched_workspace_bytes(const sil_plan* plan);

/*
 * Runs every problem, asynchronously on `stream`.  The first call with a given workspace (and
 * the first after tuning) uploads the descriptors and waits for that copy; later calls only
 * launch kernels.  Device-detected data errors are per problem: that problem's S (and s) become
 * NaN and silhouette_batched_status reports it; the other problems are unaffected.
 */
int silhouette_batched_run(sil_plan* plan, void* ws, size_t ws_bytes, void* stream);

/*
 * Autotuner: runs the batch once, then times the persistent launch (events on `stream`, which it
 * synchronises) over the plan's own problems while it varies, one at a time, the rows per work
 * item of the shallow GEMM depths (128 or 256), the persistent grid (1, 2 or 3 workgroups per
 * CU), the items taken per queue access (1, 2, 4), the queue order (costliest first, or
 * problem order) and whether problems sharing X read their rows together, keeping each change
 * that is faster.  Ends with a run in the chosen
 * configuration; *best_ms (host, may be NULL) receives the persistent launch's time.  Drops a
 * captured graph.
 */
int silhouette_batched_tune(sil_plan* plan, void* ws, size_t ws_bytes, void* stream,
                            float* best_ms);

/* The chosen configuration into out[0..5] (host): workgroups of the persistent grid, items per
 * queue access, queue order (0 costliest first, 1 problem order), and 32-row blocks per wave
 * for GEMM depths 16, 24, 32 (D up to 16, 17..24, 25..32); with len >= 7 also out[6], 1 when
 * problems that share their X (same pointer, N, D and metric: the labelings of one data set) are
 * evaluated together, reading the rows once for all of them (the default), 0 when each problem
 * reads its own.  len must be >= 6. */
int silhouette_batched_config(const sil_plan* plan, int32_t* out, int32_t len);

/* Sets the configuration from cfg[0..5] (and cfg[6] when len >= 7; host, same layout as
 * silhouette_batched_config), for instance one saved from an earlier tuning: grid 1..65536,
 * items per access 1..64, order 0 or 1, blocks per wave 1 or 2, shared rows 0 or 1.  SIL_E_ARG
 * for values out of range.  Drops a captured graph; the next run uploads the descriptors again. */
int silhouette_batched_set_config(sil_plan* plan, const int32_t* cfg, int32_t len);

/*
 * Captures one run into a hipGraph held by the plan (replacing an earlier one).  `stream` must
 * not be the legacy default stream (NULL): SIL_E_ARG.  The descriptors are uploaded before the
 * capture; the graph contains kernels only.  The graph is bound to `ws`: replay it only while
 * the same workspace and the same X, labels, s, S buffers stay valid.
 */
int silhouette_batched_capture(sil_plan* plan, void* ws, size_t ws_bytes, void* stream);

/* Launches the captured graph on `stream` (SIL_E_ARG if nothing was captured). */
int silhouette_batched_replay(sil_plan* plan, void* stream);

/*
 * Waits for `stream`, then writes each problem's first device-detected error (SIL_OK if none)
 * into status[count] (host) and returns the first non-zero one (SIL_OK if none, SIL_E_HIP if a
 * copy failed).
 */
int silhouette_batched_status(const sil_plan* plan, const void* ws, int32_t* status,
                              void* stream);

/* Releases the plan, its graph and its staging buffer (NULL is ignored). */
void silhouette_batched_free(sil_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2303_14102_AMD_SILHOUETTE_H */
