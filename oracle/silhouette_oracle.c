/*
 * FP64 CPU oracle for the linear-complexity Silhouette (squared Euclidean and cosine distance).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call this file:
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Reference: M. Gaido, "Distributed Silhouette Algorithm: Evaluating Clustering on Big Data"
 * (arXiv 2303.14102).  Every function cites the passage it follows.  All arithmetic is IEEE
 * binary64 in the order the loops state (build with -O2, no fast-math), one point at a time.
 *
 * Readings where the paper is silent or garbled (each one is also listed in the design notes):
 *  - a_i is the mean distance to the OTHER members of the own cluster (Section II, Definition):
 *    the own-cluster mean of Eq.3 includes the point itself at distance 0, so
 *    a_i = m_io * N_o / (N_o - 1).
 *  - a point alone in its cluster has s_i = 0 and still counts in N.
 *  - s_i = 0 when max(a_i, b_i) = 0 (Eq.1 is 0/0 there).
 *  - a_i and b_i are clamped at 0 (rounding can make the expanded forms slightly negative).
 *  - b_i is the minimum over non-empty clusters other than the own one; fewer than two non-empty
 *    clusters is an error.  For the gradient a tie picks the lowest cluster id.
 *  - cosine: Eq.15 writes ||X||; read ||X_i||.  A zero row is an error (Eq.12 divides by it).
 *  - labels are 0-based ids in [0, K).
 *  - generalized Kullback-Leibler divergence (Section V names other metrics): the distance from
 *    point i to point j is d(x_i, x_j), point first (the divergence is not symmetric); every entry
 *    must be positive.
 *
 * Input storage: X is float32 [N,D] row-major, or float64, or bf16 bit patterns (uint16), or
 * fp8 e4m3fn codes (uint8) with a float32 per-column scale.  The oracle decodes the stored
 * values exactly into binary64 itself (the decoders follow the published format definitions).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_F32 = 0, ORC_BF16 = 1, ORC_FP8_E4M3 = 2, ORC_F64 = 3 };
enum { ORC_SQEUCLID = 0, ORC_COSINE = 1, ORC_EUCLID_APPROX = 2, ORC_KL = 3 };
enum {
  ORC_OK = 0,
  ORC_E_ARG = -1,
  ORC_E_LABEL = -3,
  ORC_E_FEW_CLUSTERS = -4,
  ORC_E_ZERO_NORM = -5,
  ORC_E_NONFINITE = -6,
  ORC_E_NOMEM = -9,
  ORC_E_DOMAIN = -10
};

/* ---------------------------------------------------------------------------------------- */
/* storage decoding                                                                          */

/* bfloat16: the upper 16 bits of an IEEE binary32. */
static double orc_bf16_to_f64(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, sizeof f);
  return (double)f;
}

/* OCP 8-bit float E4M3 ("fn" flavour): 1 sign bit, 4 exponent bits with bias 7, 3 mantissa
 * bits; exponent field 0 is subnormal (m/8 * 2^-6); S.1111.111 is NaN; there is no infinity. */
static double orc_e4m3_to_f64(uint8_t q) {
  int sign = (q >> 7) & 1;
  int e = (q >> 3) & 15;
  int m = q & 7;
  double v;
  if (e == 15 && m == 7) return NAN;
  if (e == 0)
    v = ldexp((double)m / 8.0, -6);
  else
    v = ldexp(1.0 + (double)m / 8.0, e - 7);
  return sign ? -v : v;
}

double orc_decode_bf16(uint16_t h) { return orc_bf16_to_f64(h); }
double orc_decode_e4m3(uint8_t q) { return orc_e4m3_to_f64(q); }

/* Row i of X as binary64 into out[0..D). */
static void orc_row(const void* X, int dtype, const float* col_scale, int64_t i, int32_t D,
                    double* out) {
  int32_t l;
  switch (dtype) {
    case ORC_F32: {
      const float* p = (const float*)X + i * (int64_t)D;
      for (l = 0; l < D; ++l) out[l] = (double)p[l];
      break;
    }
    case ORC_F64: {
      const double* p = (const double*)X + i * (int64_t)D;
      for (l = 0; l < D; ++l) out[l] = p[l];
      break;
    }
    case ORC_BF16: {
      const uint16_t* p = (const uint16_t*)X + i * (int64_t)D;
      for (l = 0; l < D; ++l) out[l] = orc_bf16_to_f64(p[l]);
      break;
    }
    case ORC_FP8_E4M3: {
      const uint8_t* p = (const uint8_t*)X + i * (int64_t)D;
      for (l = 0; l < D; ++l) out[l] = orc_e4m3_to_f64(p[l]) * (double)col_scale[l];
      break;
    }
  }
}

static int orc_check_args(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                          int64_t N, int32_t D, int32_t K, int metric) {
  if (!X || !labels || N < 1 || D < 1 || K < 1) return ORC_E_ARG;
  if (dtype < ORC_F32 || dtype > ORC_F64) return ORC_E_ARG;
  if (dtype == ORC_FP8_E4M3 && !col_scale) return ORC_E_ARG;
  if (metric != ORC_SQEUCLID && metric != ORC_COSINE && metric != ORC_EUCLID_APPROX &&
      metric != ORC_KL)
    return ORC_E_ARG;
  return ORC_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* pass 1: per-cluster statistics                                                            */

/*
 * One pass over the data (footnotes to Eq.6 and Eq.9: the sums are accumulated together).
 *   count[k] = N_{Gamma_k}
 *   squared Euclidean:  V[k][l] = Y_{Gamma_k l} = sum_{j in k} c_jl           (Eq.8)
 *                       psi[k]  = Psi_{Gamma_k} = sum_{j in k} xi_{C_j}         (Eq.6),
 *                       xi_{X} = sum_l x_l^2                                    (Eq.5)
 *   cosine:             V[k][l] = Omega_{Gamma_k l} = sum_{j in k} c_jl/||C_j|| (Eq.15, Eq.16)
 *                       psi[k]  = 0
 *   generalized KL:     V[k][l] = sum_{j in k} log c_jl,  psi[k] = sum_{j in k} sum_l c_jl
 *                       (the Bregman statistics below; every entry must be positive)
 * Sums run over j in increasing row order.
 */
int orc_cluster_stats(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                      int64_t N, int32_t D, int32_t K, int metric, int64_t* count, double* V,
                      double* psi) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, metric);
  if (rc) return rc;
  double* x = (double*)malloc(sizeof(double) * (size_t)D);
  if (!x) return ORC_E_NOMEM;
  memset(count, 0, sizeof(int64_t) * (size_t)K);
  memset(V, 0, sizeof(double) * (size_t)K * (size_t)D);
  memset(psi, 0, sizeof(double) * (size_t)K);
  for (int64_t i = 0; i < N; ++i) {
    int32_t k = labels[i];
    if (k < 0 || k >= K) { rc = ORC_E_LABEL; break; }
    orc_row(X, dtype, col_scale, i, D, x);
    double xi = 0.0;
    for (int32_t l = 0; l < D; ++l) {
      if (!isfinite(x[l])) { rc = ORC_E_NONFINITE; break; }
      xi += x[l] * x[l];
    }
    if (rc) break;
    count[k] += 1;
    if (metric == ORC_KL) {
      double sx = 0.0;
      for (int32_t l = 0; l < D; ++l) {
        if (!(x[l] > 0.0)) { rc = ORC_E_DOMAIN; break; }
        V[(int64_t)k * D + l] += log(x[l]);
        sx += x[l];
      }
      if (rc) break;
      psi[k] += sx;
    } else if (metric != ORC_COSINE) {
      for (int32_t l = 0; l < D; ++l) V[(int64_t)k * D + l] += x[l];
      psi[k] += xi;
    } else {
      double norm = sqrt(xi);
      if (norm == 0.0) { rc = ORC_E_ZERO_NORM; break; }
      for (int32_t l = 0; l < D; ++l) V[(int64_t)k * D + l] += x[l] / norm;
    }
  }
  free(x);
  return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* pass 2: mean distance from a point to every cluster, then s_i                             */

/*
 * The generalized Kullback-Leibler divergence of positive vectors, the Bregman divergence of
 * phi(x) = sum_l (x_l log x_l - x_l):
 *   d(x, y) = phi(x) - phi(y) - grad phi(y).(x - y) = sum_l (x_l log(x_l / y_l) - x_l + y_l).
 * It is not symmetric; the Silhouette of point i uses d(x_i, x_j) with x_i first.  Section V notes
 * that a similar approach serves other metrics: averaging over y in cluster k needs only
 * sum_y log y (a vector) and sum_y sum_l y_l (a scalar), since grad phi(y).y - phi(y) = sum_l y_l.
 * d(x, x) = 0, so the readings of the squared Euclidean distance (self-exclusion included) apply.
 */
static double orc_kl_distance(const double* x, const double* y, int32_t D) {
  double d = 0.0;
  for (int32_t l = 0; l < D; ++l) d += x[l] * log(x[l] / y[l]) - x[l] + y[l];
  return d;
}

/*
 * m[k] = d(X_i, Gamma_k), the mean distance from point i to the members of cluster k, self
 * included (Eq.3), from the cluster statistics alone:
 *   squared Euclidean (Eq.11): m_k = xi_{X_i} + Psi_k / N_k - 2 * (sum_l Y_kl x_il) / N_k
 *   cosine (Eq.18):            m_k = 1 - (sum_l xi_{X_i l} Omega_kl) / N_k,
 *                              xi_{X_i l} = x_il / ||X_i||                      (Eq.15)
 * Empty clusters get m_k = NaN (they have no mean distance).
 */
static void orc_point_means(const double* x, int32_t D, int32_t K, int metric,
                            const int64_t* count, const double* V, const double* psi,
                            double* m) {
  if (metric == ORC_KL) {
    /* Bregman form of the generalized KL divergence (see orc_kl_distance):
     *   m_k = phi(x) + psi_k / N_k - sum_l x_l V_kl / N_k,  phi(x) = sum_l (x_l log x_l - x_l) */
    double phi = 0.0;
    for (int32_t l = 0; l < D; ++l) phi += x[l] * log(x[l]) - x[l];
    for (int32_t k = 0; k < K; ++k) {
      if (count[k] == 0) { m[k] = NAN; continue; }
      double dot = 0.0;
      for (int32_t l = 0; l < D; ++l) dot += x[l] * V[(int64_t)k * D + l];
      const double nk = (double)count[k];
      m[k] = phi + psi[k] / nk - dot / nk;
    }
    return;
  }
  double xi = 0.0;
  for (int32_t l = 0; l < D; ++l) xi += x[l] * x[l];
  double norm = sqrt(xi);
  for (int32_t k = 0; k < K; ++k) {
    if (count[k] == 0) { m[k] = NAN; continue; }
    double nk = (double)count[k];
    double dot = 0.0;
    if (metric != ORC_COSINE) {
      for (int32_t l = 0; l < D; ++l) dot += V[(int64_t)k * D + l] * x[l];
      m[k] = xi + psi[k] / nk - 2.0 * dot / nk;
    } else {
      for (int32_t l = 0; l < D; ++l) dot += (x[l] / norm) * V[(int64_t)k * D + l];
      m[k] = 1.0 - dot / nk;
    }
  }
}

/*
 * s_i from the mean distances of point i (own cluster o):
 *   a_i = max(0, m_o * N_o / (N_o - 1))                 (own cluster, other members only)
 *   b_i = max(0, min_{k != o, N_k >= 1} m_k)            (neighbouring cluster, Section II)
 *   s_i = (b_i - a_i) / max(a_i, b_i)                   (Eq.1; equal to Eq.2)
 * with s_i = 0 for a singleton own cluster or when max(a_i, b_i) = 0.  With root set (the
 * approximate Euclidean form of Section V: the square root of each point-to-cluster mean squared
 * distance) a_i and b_i are replaced by their square roots before Eq.1.  nbr receives the lowest
 * cluster id attaining b_i.  Returns s_i.
 */
static double orc_point_score(const double* m, int32_t K, int32_t o, const int64_t* count,
                              int root, double* a_out, double* b_out, int32_t* nbr_out) {
  double b = INFINITY;
  int32_t nbr = -1;
  for (int32_t k = 0; k < K; ++k) {
    if (k == o || count[k] == 0) continue;
    if (m[k] < b) { b = m[k]; nbr = k; }
  }
  if (b < 0.0) b = 0.0;
  double a = 0.0, s = 0.0;
  if (root) b = sqrt(b);
  if (count[o] >= 2) {
    a = m[o] * (double)count[o] / (double)(count[o] - 1);
    if (a < 0.0) a = 0.0;
    if (root) a = sqrt(a);
    double mx = a > b ? a : b;
    s = mx > 0.0 ? (b - a) / mx : 0.0;
  }
  if (a_out) *a_out = a;
  if (b_out) *b_out = b;
  if (nbr_out) *nbr_out = nbr;
  return s;
}

static int orc_nonempty(const int64_t* count, int32_t K) {
  int n = 0;
  for (int32_t k = 0; k < K; ++k) n += count[k] > 0;
  return n;
}

/*
 * s_i for the listed points, given cluster statistics from orc_cluster_stats.  Points are
 * independent (Section III-A: "every point can be analyzed independently"), so the loop over
 * them may run on several threads; each point's arithmetic is sequential.
 * a, b, nbr may be NULL.
 */
int orc_scores_at(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                  int64_t N, int32_t D, int32_t K, int metric, const int64_t* count,
                  const double* V, const double* psi, const int64_t* idx, int64_t n_idx,
                  double* s, double* a, double* b, int32_t* nbr) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, metric);
  if (rc) return rc;
  if (orc_nonempty(count, K) < 2) return ORC_E_FEW_CLUSTERS;
  for (int64_t t = 0; t < n_idx; ++t)
    if (idx[t] < 0 || idx[t] >= N) return ORC_E_ARG;
  int bad = 0;
#pragma omp parallel
  {
    double* x = (double*)malloc(sizeof(double) * (size_t)D);
    double* m = (double*)malloc(sizeof(double) * (size_t)K);
    if (!x || !m) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t t = 0; t < n_idx; ++t) {
        int64_t i = idx[t];
        orc_row(X, dtype, col_scale, i, D, x);
        orc_point_means(x, D, K, metric, count, V, psi, m);
        s[t] = orc_point_score(m, K, labels[i], count, metric == ORC_EUCLID_APPROX,
                               a ? a + t : NULL, b ? b + t : NULL, nbr ? nbr + t : NULL);
      }
    }
    free(x);
    free(m);
  }
  return bad ? ORC_E_NOMEM : ORC_OK;
}

/*
 * The whole method: cluster statistics (pass 1), s_i for every point (pass 2), and the overall
 * score S = sum_i s_i / N (Section II), summed in index order.  s, a, b, nbr may be NULL.
 */
int orc_silhouette(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                   int64_t N, int32_t D, int32_t K, int metric, double* s, double* S, double* a,
                   double* b, int32_t* nbr) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, metric);
  if (rc) return rc;
  int64_t* count = (int64_t*)malloc(sizeof(int64_t) * (size_t)K);
  double* V = (double*)malloc(sizeof(double) * (size_t)K * (size_t)D);
  double* psi = (double*)malloc(sizeof(double) * (size_t)K);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  double* s_loc = s ? s : (double*)malloc(sizeof(double) * (size_t)N);
  if (!count || !V || !psi || !idx || !s_loc) { rc = ORC_E_NOMEM; goto done; }
  rc = orc_cluster_stats(X, dtype, col_scale, labels, N, D, K, metric, count, V, psi);
  if (rc) goto done;
  for (int64_t i = 0; i < N; ++i) idx[i] = i;
  rc = orc_scores_at(X, dtype, col_scale, labels, N, D, K, metric, count, V, psi, idx, N, s_loc,
                     a, b, nbr);
  if (rc) goto done;
  {
    double tot = 0.0;
    for (int64_t i = 0; i < N; ++i) tot += s_loc[i];
    *S = tot / (double)N;
  }
done:
  free(count);
  free(V);
  free(psi);
  free(idx);
  if (!s) free(s_loc);
  return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* the quadratic definition                                                                  */

/*
 * The standard O(N^2 D) Silhouette (Section II, Computational Complexity): for each point, the
 * distance to every other point, averaged per cluster; then a_i, b_i, s_i and S exactly as
 * above.  Distances: ||x_i - x_j||^2, or 1 - x_i.x_j / (||x_i|| ||x_j||) (Eq.12).
 */
int orc_brute_silhouette(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                         int64_t N, int32_t D, int32_t K, int metric, double* s, double* S) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, metric);
  if (rc) return rc;
  double* all = (double*)malloc(sizeof(double) * (size_t)N * (size_t)D);
  int64_t* count = (int64_t*)calloc((size_t)K, sizeof(int64_t));
  if (!all || !count) { free(all); free(count); return ORC_E_NOMEM; }
  for (int64_t i = 0; i < N; ++i) {
    if (labels[i] < 0 || labels[i] >= K) { rc = ORC_E_LABEL; goto done; }
    orc_row(X, dtype, col_scale, i, D, all + i * (int64_t)D);
    for (int32_t l = 0; l < D; ++l)
      if (!isfinite(all[i * (int64_t)D + l])) { rc = ORC_E_NONFINITE; goto done; }
    count[labels[i]] += 1;
  }
  if (metric == ORC_KL)
    for (int64_t e = 0; e < N * (int64_t)D; ++e)
      if (!(all[e] > 0.0)) { rc = ORC_E_DOMAIN; goto done; }
  if (orc_nonempty(count, K) < 2) { rc = ORC_E_FEW_CLUSTERS; goto done; }
  if (metric == ORC_COSINE)
    for (int64_t i = 0; i < N; ++i) {
      double n2 = 0.0;
      for (int32_t l = 0; l < D; ++l) n2 += all[i * (int64_t)D + l] * all[i * (int64_t)D + l];
      if (n2 == 0.0) { rc = ORC_E_ZERO_NORM; goto done; }
    }
  {
    int bad = 0;
#pragma omp parallel
    {
      double* sum = (double*)malloc(sizeof(double) * (size_t)K);
      if (!sum) {
#pragma omp atomic write
        bad = 1;
      } else {
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
          const double* xi = all + i * (int64_t)D;
          for (int32_t k = 0; k < K; ++k) sum[k] = 0.0;
          for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            const double* xj = all + j * (int64_t)D;
            double d = 0.0;
            if (metric == ORC_KL) {
              d = orc_kl_distance(xi, xj, D);
            } else if (metric != ORC_COSINE) {
              for (int32_t l = 0; l < D; ++l) d += (xi[l] - xj[l]) * (xi[l] - xj[l]);
            } else {
              double dot = 0.0, ni = 0.0, nj = 0.0;
              for (int32_t l = 0; l < D; ++l) {
                dot += xi[l] * xj[l];
                ni += xi[l] * xi[l];
                nj += xj[l] * xj[l];
              }
              d = 1.0 - dot / (sqrt(ni) * sqrt(nj));
            }
            sum[labels[j]] += d;
          }
          int32_t o = labels[i];
          double si = 0.0;
          if (count[o] >= 2) {
            double a = sum[o] / (double)(count[o] - 1);
            double b = INFINITY;
            for (int32_t k = 0; k < K; ++k)
              if (k != o && count[k] > 0 && sum[k] / (double)count[k] < b) b = sum[k] / (double)count[k];
            if (metric == ORC_EUCLID_APPROX) {  /* roots of the mean squared distances */
              a = sqrt(a);
              b = sqrt(b);
            }
            double mx = a > b ? a : b;
            si = mx > 0.0 ? (b - a) / mx : 0.0;
          }
          s[i] = si;
        }
      }
      free(sum);
    }
    if (bad) { rc = ORC_E_NOMEM; goto done; }
    double tot = 0.0;
    for (int64_t i = 0; i < N; ++i) tot += s[i];
    *S = tot / (double)N;
  }
done:
  free(all);
  free(count);
  return rc;
}

/*
 * The quadratic definition for listed points only: for each listed point i, its distance to
 * every other point j (Section II, Definition; cosine distance as in Eq.12), summed per cluster,
 * then a_i, b_i and s_i exactly as in orc_brute_silhouette.  Rows are decoded on the fly, so the
 * cost is O(n_idx * N * D) time and O(threads * K) memory: this checks single points of
 * workloads too large for the full quadratic form.  The sum over j is split into one contiguous
 * range per thread and the per-thread sums are added in thread order.  a, b may be NULL.
 */
int orc_brute_scores_at(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                        int64_t N, int32_t D, int32_t K, int metric, const int64_t* idx,
                        int64_t n_idx, double* s, double* a, double* b) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, metric);
  if (rc) return rc;
  for (int64_t t = 0; t < n_idx; ++t)
    if (idx[t] < 0 || idx[t] >= N) return ORC_E_ARG;
  int64_t* count = (int64_t*)calloc((size_t)K, sizeof(int64_t));
  if (!count) return ORC_E_NOMEM;
  for (int64_t j = 0; j < N; ++j) {
    if (labels[j] < 0 || labels[j] >= K) { free(count); return ORC_E_LABEL; }
    count[labels[j]] += 1;
  }
  if (orc_nonempty(count, K) < 2) { free(count); return ORC_E_FEW_CLUSTERS; }
  int nthr = 1;
#ifdef _OPENMP
  nthr = omp_get_max_threads();
#endif
  double* part = (double*)malloc(sizeof(double) * (size_t)nthr * (size_t)K);
  double* xi = (double*)malloc(sizeof(double) * (size_t)D);
  if (!part || !xi) { free(count); free(part); free(xi); return ORC_E_NOMEM; }
  for (int64_t t = 0; t < n_idx && rc == ORC_OK; ++t) {
    const int64_t i = idx[t];
    orc_row(X, dtype, col_scale, i, D, xi);
    double ni = 0.0;
    for (int32_t l = 0; l < D; ++l) ni += xi[l] * xi[l];
    if (!isfinite(ni)) { rc = ORC_E_NONFINITE; break; }
    if (metric == ORC_COSINE && ni == 0.0) { rc = ORC_E_ZERO_NORM; break; }
    if (metric == ORC_KL)
      for (int32_t l = 0; l < D; ++l)
        if (!(xi[l] > 0.0)) rc = ORC_E_DOMAIN;
    if (rc) break;
    int bad = ORC_OK;
    memset(part, 0, sizeof(double) * (size_t)nthr * (size_t)K);
#pragma omp parallel num_threads(nthr)
    {
      int tid = 0, nt = 1;
#ifdef _OPENMP
      tid = omp_get_thread_num();
      nt = omp_get_num_threads();
#endif
      double* sum = part + (size_t)tid * (size_t)K;
      double* xj = (double*)malloc(sizeof(double) * (size_t)D);
      if (!xj) {
#pragma omp atomic write
        bad = ORC_E_NOMEM;
      } else {
        const int64_t lo = N * tid / nt, hi = N * (tid + 1) / nt;
        for (int64_t j = lo; j < hi; ++j) {
          if (j == i) continue;
          orc_row(X, dtype, col_scale, j, D, xj);
          double d = 0.0;
          if (metric == ORC_KL) {
            for (int32_t l = 0; l < D; ++l)
              if (!(xj[l] > 0.0)) {
#pragma omp atomic write
                bad = ORC_E_DOMAIN;
              }
            d = orc_kl_distance(xi, xj, D);
          } else if (metric != ORC_COSINE) {
            for (int32_t l = 0; l < D; ++l) d += (xi[l] - xj[l]) * (xi[l] - xj[l]);
          } else {
            double dot = 0.0, nj = 0.0;
            for (int32_t l = 0; l < D; ++l) {
              dot += xi[l] * xj[l];
              nj += xj[l] * xj[l];
            }
            if (nj == 0.0) {
#pragma omp atomic write
              bad = ORC_E_ZERO_NORM;
            }
            d = 1.0 - dot / (sqrt(ni) * sqrt(nj));
          }
          if (!isfinite(d)) {
#pragma omp atomic write
            bad = ORC_E_NONFINITE;
          }
          sum[labels[j]] += d;
        }
      }
      free(xj);
    }
    if (bad) { rc = bad; break; }
    for (int th = 1; th < nthr; ++th)
      for (int32_t k = 0; k < K; ++k) part[k] += part[(size_t)th * (size_t)K + k];
    const int32_t o = labels[i];
    double si = 0.0, ai = 0.0, bi = 0.0;
    if (count[o] >= 2) {
      ai = part[o] / (double)(count[o] - 1);
      bi = INFINITY;
      for (int32_t k = 0; k < K; ++k)
        if (k != o && count[k] > 0 && part[k] / (double)count[k] < bi) bi = part[k] / (double)count[k];
      if (metric == ORC_EUCLID_APPROX) {  /* roots of the mean squared distances */
        ai = sqrt(ai);
        bi = sqrt(bi);
      }
      const double mx = ai > bi ? ai : bi;
      si = mx > 0.0 ? (bi - ai) / mx : 0.0;
    }
    s[t] = si;
    if (a) a[t] = ai;
    if (b) b[t] = bi;
  }
  free(count);
  free(part);
  free(xi);
  return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* gradient of S with respect to X (labels held fixed); not in the paper, derived from Eq.11  */
/* and Eq.18                                                                                 */

/*
 * S = (1/N) sum_i s_i(a_i, b_i).  With alpha_ik = dS/dm_ik:
 *   alpha_io = (1/N) ds_i/da_i * N_o/(N_o-1),  alpha_in = (1/N) ds_i/db_i  (n = neighbour id),
 *   ds/da = -1/b, ds/db = a/b^2 when a <= b (Eq.2 first branch); -b/a^2 and 1/a when a > b;
 *   all zero for singletons or when max(a, b) = 0.
 * Squared Euclidean, m_ik = mean_{j in k} ||x_i - x_j||^2, mu_k = Y_k/N_k:
 *   dS/dx_j = 2 sum_k alpha_jk (x_j - mu_k) + (2/N_c)(A_c x_j - B_c),   c = label of j,
 *   A_k = sum_i alpha_ik,  B_k = sum_i alpha_ik x_i.
 * Cosine, m_ik = 1 - z_i . Omega_k / N_k with z = x/||x||, mu_k = Omega_k/N_k:
 *   g_j = -sum_k alpha_jk mu_k - B_c/N_c (B with z_i in place of x_i),
 *   dS/dx_j = (g_j - (g_j . z_j) z_j) / ||x_j||.
 * dX is binary64 [N,D].
 */
int orc_gradient(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                 int64_t N, int32_t D, int32_t K, int metric, double* dX) {
  if (metric == ORC_EUCLID_APPROX || metric == ORC_KL) return ORC_E_ARG;
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, metric);
  if (rc) return rc;
  int64_t* count = (int64_t*)malloc(sizeof(int64_t) * (size_t)K);
  double* V = (double*)malloc(sizeof(double) * (size_t)K * (size_t)D);
  double* psi = (double*)malloc(sizeof(double) * (size_t)K);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  double* s = (double*)malloc(sizeof(double) * (size_t)N);
  double* a = (double*)malloc(sizeof(double) * (size_t)N);
  double* b = (double*)malloc(sizeof(double) * (size_t)N);
  int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  double* al_own = (double*)malloc(sizeof(double) * (size_t)N);
  double* al_nbr = (double*)malloc(sizeof(double) * (size_t)N);
  double* A = (double*)calloc((size_t)K, sizeof(double));
  double* B = (double*)calloc((size_t)K * (size_t)D, sizeof(double));
  double* x = (double*)malloc(sizeof(double) * (size_t)D);
  double* g = (double*)malloc(sizeof(double) * (size_t)D);
  if (!count || !V || !psi || !idx || !s || !a || !b || !nbr || !al_own || !al_nbr || !A || !B ||
      !x || !g) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  rc = orc_cluster_stats(X, dtype, col_scale, labels, N, D, K, metric, count, V, psi);
  if (rc) goto done;
  for (int64_t i = 0; i < N; ++i) idx[i] = i;
  rc = orc_scores_at(X, dtype, col_scale, labels, N, D, K, metric, count, V, psi, idx, N, s, a, b,
                     nbr);
  if (rc) goto done;
  for (int64_t i = 0; i < N; ++i) {
    int32_t o = labels[i];
    double dsa = 0.0, dsb = 0.0;
    double mx = a[i] > b[i] ? a[i] : b[i];
    if (count[o] >= 2 && mx > 0.0) {
      if (a[i] <= b[i]) {
        dsa = -1.0 / b[i];
        dsb = a[i] / (b[i] * b[i]);
      } else {
        dsa = -b[i] / (a[i] * a[i]);
        dsb = 1.0 / a[i];
      }
    }
    al_own[i] = count[o] >= 2 ? dsa * (double)count[o] / (double)(count[o] - 1) / (double)N : 0.0;
    al_nbr[i] = dsb / (double)N;
  }
  /* A_k, B_k over rows in index order */
  for (int64_t i = 0; i < N; ++i) {
    int32_t o = labels[i], n = nbr[i];
    orc_row(X, dtype, col_scale, i, D, x);
    if (metric == ORC_COSINE) {
      double n2 = 0.0;
      for (int32_t l = 0; l < D; ++l) n2 += x[l] * x[l];
      double nr = sqrt(n2);
      for (int32_t l = 0; l < D; ++l) x[l] = x[l] / nr;
    }
    A[o] += al_own[i];
    for (int32_t l = 0; l < D; ++l) B[(int64_t)o * D + l] += al_own[i] * x[l];
    if (n >= 0) {
      A[n] += al_nbr[i];
      for (int32_t l = 0; l < D; ++l) B[(int64_t)n * D + l] += al_nbr[i] * x[l];
    }
  }
  for (int64_t j = 0; j < N; ++j) {
    int32_t c = labels[j], n = nbr[j];
    double nc = (double)count[c];
    orc_row(X, dtype, col_scale, j, D, x);
    double* out = dX + j * (int64_t)D;
    if (metric == ORC_SQEUCLID) {
      for (int32_t l = 0; l < D; ++l) {
        double mu_c = V[(int64_t)c * D + l] / nc;
        double v = 2.0 * al_own[j] * (x[l] - mu_c);
        if (n >= 0) v += 2.0 * al_nbr[j] * (x[l] - V[(int64_t)n * D + l] / (double)count[n]);
        v += 2.0 / nc * (A[c] * x[l] - B[(int64_t)c * D + l]);
        out[l] = v;
      }
    } else {
      double n2 = 0.0;
      for (int32_t l = 0; l < D; ++l) n2 += x[l] * x[l];
      double nr = sqrt(n2);
      double gz = 0.0;
      for (int32_t l = 0; l < D; ++l) {
        double v = -al_own[j] * V[(int64_t)c * D + l] / nc;
        if (n >= 0) v -= al_nbr[j] * V[(int64_t)n * D + l] / (double)count[n];
        v -= B[(int64_t)c * D + l] / nc;
        g[l] = v;
        gz += v * (x[l] / nr);
      }
      for (int32_t l = 0; l < D; ++l) out[l] = (g[l] - gz * (x[l] / nr)) / nr;
    }
  }
done:
  free(count); free(V); free(psi); free(idx); free(s); free(a); free(b); free(nbr);
  free(al_own); free(al_nbr); free(A); free(B); free(x); free(g);
  return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* fixed-matrix Mahalanobis distance                                                         */

/*
 * Section V notes that a similar approach may serve other metrics.  For
 *   d(x, y) = (x - y)^T M (x - y),   M [D, D] fixed, symmetric positive semi-definite,
 * expanding the quadratic form as Eq.9-11 expand the squared Euclidean distance gives the mean
 * distance from x to cluster k (self included, Eq.3) from per-cluster statistics alone:
 *   m(x, k) = x^T M x + PsiM_k / N_k - 2 x^T M Y_k / N_k,   PsiM_k = sum_{y in k} y^T M y,
 * with Y_k the plain vector sums of Eq.8.  a_i, b_i and s_i then follow orc_point_score with the
 * readings of the squared Euclidean distance (M = I gives exactly that distance).
 */
static double orc_quad(const double* M, const double* x, int32_t D) {
  double q = 0.0;
  for (int32_t r = 0; r < D; ++r) {
    double t = 0.0;
    for (int32_t c = 0; c < D; ++c) t += M[(int64_t)r * D + c] * x[c];
    q += x[r] * t;
  }
  return q;
}

int orc_silhouette_mahalanobis(const void* X, int dtype, const float* col_scale, const double* M,
                               const int32_t* labels, int64_t N, int32_t D, int32_t K, double* s,
                               double* S, double* a, double* b) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, ORC_SQEUCLID);
  if (rc) return rc;
  if (!M || !s || !S) return ORC_E_ARG;
  int64_t* count = (int64_t*)calloc((size_t)K, sizeof(int64_t));
  double* Y = (double*)calloc((size_t)K * (size_t)D, sizeof(double));
  double* psi = (double*)calloc((size_t)K, sizeof(double));
  double* x = (double*)malloc(sizeof(double) * (size_t)D);
  if (!count || !Y || !psi || !x) { rc = ORC_E_NOMEM; goto done; }
  /* statistics: N_k, Y_k (Eq.8) and PsiM_k, one pass in increasing row order */
  for (int64_t i = 0; i < N; ++i) {
    int32_t k = labels[i];
    if (k < 0 || k >= K) { rc = ORC_E_LABEL; goto done; }
    orc_row(X, dtype, col_scale, i, D, x);
    for (int32_t l = 0; l < D; ++l)
      if (!isfinite(x[l])) { rc = ORC_E_NONFINITE; goto done; }
    count[k] += 1;
    for (int32_t l = 0; l < D; ++l) Y[(int64_t)k * D + l] += x[l];
    psi[k] += orc_quad(M, x, D);
  }
  if (orc_nonempty(count, K) < 2) { rc = ORC_E_FEW_CLUSTERS; goto done; }
  int bad = 0;
#pragma omp parallel
  {
    double* xl = (double*)malloc(sizeof(double) * (size_t)D);
    double* Mx = (double*)malloc(sizeof(double) * (size_t)D);
    double* m = (double*)malloc(sizeof(double) * (size_t)K);
    if (!xl || !Mx || !m) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        orc_row(X, dtype, col_scale, i, D, xl);
        double xmx = 0.0;
        for (int32_t r = 0; r < D; ++r) {
          double t = 0.0;
          for (int32_t c = 0; c < D; ++c) t += M[(int64_t)r * D + c] * xl[c];
          Mx[r] = t;
          xmx += xl[r] * t;
        }
        for (int32_t k = 0; k < K; ++k) {
          if (count[k] == 0) { m[k] = NAN; continue; }
          double dot = 0.0;
          for (int32_t l = 0; l < D; ++l) dot += Mx[l] * Y[(int64_t)k * D + l];
          const double nk = (double)count[k];
          m[k] = xmx + psi[k] / nk - 2.0 * dot / nk;
        }
        s[i] = orc_point_score(m, K, labels[i], count, 0, a ? &a[i] : NULL, b ? &b[i] : NULL, NULL);
      }
    }
    free(xl); free(Mx); free(m);
  }
  if (bad) { rc = ORC_E_NOMEM; goto done; }
  {
    double tot = 0.0;
    for (int64_t i = 0; i < N; ++i) tot += s[i];
    *S = tot / (double)N;
  }
done:
  free(count); free(Y); free(psi); free(x);
  return rc;
}

/* The quadratic definition under the same distance: every pair's (x_i - x_j)^T M (x_i - x_j). */
int orc_brute_silhouette_mahalanobis(const void* X, int dtype, const float* col_scale,
                                     const double* M, const int32_t* labels, int64_t N, int32_t D,
                                     int32_t K, double* s, double* S) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, ORC_SQEUCLID);
  if (rc) return rc;
  if (!M || !s || !S) return ORC_E_ARG;
  double* Xd = (double*)malloc(sizeof(double) * (size_t)N * (size_t)D);
  int64_t* count = (int64_t*)calloc((size_t)K, sizeof(int64_t));
  if (!Xd || !count) { rc = ORC_E_NOMEM; goto done; }
  for (int64_t i = 0; i < N; ++i) {
    if (labels[i] < 0 || labels[i] >= K) { rc = ORC_E_LABEL; goto done; }
    orc_row(X, dtype, col_scale, i, D, Xd + i * (int64_t)D);
    count[labels[i]] += 1;
  }
  if (orc_nonempty(count, K) < 2) { rc = ORC_E_FEW_CLUSTERS; goto done; }
  int bad = 0;
#pragma omp parallel
  {
    double* sum = (double*)malloc(sizeof(double) * (size_t)K);
    double* diff = (double*)malloc(sizeof(double) * (size_t)D);
    double* m = (double*)malloc(sizeof(double) * (size_t)K);
    if (!sum || !diff || !m) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        for (int32_t k = 0; k < K; ++k) sum[k] = 0.0;
        for (int64_t j = 0; j < N; ++j) {
          for (int32_t l = 0; l < D; ++l) diff[l] = Xd[i * D + l] - Xd[j * D + l];
          sum[labels[j]] += orc_quad(M, diff, D);
        }
        for (int32_t k = 0; k < K; ++k) m[k] = count[k] ? sum[k] / (double)count[k] : NAN;
        s[i] = orc_point_score(m, K, labels[i], count, 0, NULL, NULL, NULL);
      }
    }
    free(sum); free(diff); free(m);
  }
  if (bad) { rc = ORC_E_NOMEM; goto done; }
  {
    double tot = 0.0;
    for (int64_t i = 0; i < N; ++i) tot += s[i];
    *S = tot / (double)N;
  }
done:
  free(Xd); free(count);
  return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* K-means (Lloyd) step                                                                      */

/*
 * The Introduction names K-Means among the clustering methods whose output the Silhouette
 * evaluates.  One Lloyd step on given labels, written out from its textbook definition:
 *   update:  mu_k = Y_k / N_k for every non-empty cluster, Y_k and N_k as in Eq.8;
 *   assign:  each point goes to the non-empty cluster with the smallest squared Euclidean
 *            distance sum_l (x_l - mu_kl)^2, the lowest id on ties; empty clusters stay empty.
 * d1[i] is the distance to the chosen mean, d2[i] the next smallest one over the other
 * non-empty clusters (+inf when there is none); *inertia = sum_i d1[i] in increasing i.
 * d1 and d2 may be NULL.  At least one cluster must be non-empty (always true for N >= 1).
 */
int orc_kmeans_step(const void* X, int dtype, const float* col_scale, const int32_t* labels,
                    int64_t N, int32_t D, int32_t K, int32_t* labels_out, double* inertia,
                    double* d1, double* d2) {
  int rc = orc_check_args(X, dtype, col_scale, labels, N, D, K, ORC_SQEUCLID);
  if (rc) return rc;
  if (!labels_out || !inertia) return ORC_E_ARG;
  int64_t* count = (int64_t*)malloc(sizeof(int64_t) * (size_t)K);
  double* V = (double*)malloc(sizeof(double) * (size_t)K * (size_t)D);
  double* psi = (double*)malloc(sizeof(double) * (size_t)K);
  double* dist = (double*)malloc(sizeof(double) * (size_t)N);
  if (!count || !V || !psi || !dist) { rc = ORC_E_NOMEM; goto done; }
  rc = orc_cluster_stats(X, dtype, col_scale, labels, N, D, K, ORC_SQEUCLID, count, V, psi);
  if (rc) goto done;
  for (int32_t k = 0; k < K; ++k)  /* the means replace the sums in place */
    if (count[k] > 0)
      for (int32_t l = 0; l < D; ++l) V[(int64_t)k * D + l] /= (double)count[k];
  int bad = 0;
#pragma omp parallel
  {
    double* x = (double*)malloc(sizeof(double) * (size_t)D);
    if (!x) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        orc_row(X, dtype, col_scale, i, D, x);
        double best = INFINITY, second = INFINITY;
        int32_t arg = -1;
        for (int32_t k = 0; k < K; ++k) {
          if (count[k] == 0) continue;
          double d = 0.0;
          for (int32_t l = 0; l < D; ++l) {
            const double t = x[l] - V[(int64_t)k * D + l];
            d += t * t;
          }
          if (d < best) {
            second = best;
            best = d;
            arg = k;
          } else if (d < second) {
            second = d;
          }
        }
        labels_out[i] = arg;
        dist[i] = best;
        if (d1) d1[i] = best;
        if (d2) d2[i] = second;
      }
      free(x);
    }
  }
  if (bad) { rc = ORC_E_NOMEM; goto done; }
  double tot = 0.0;
  for (int64_t i = 0; i < N; ++i) tot += dist[i];
  *inertia = tot;
done:
  free(count); free(V); free(psi); free(dist);
  return rc;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
