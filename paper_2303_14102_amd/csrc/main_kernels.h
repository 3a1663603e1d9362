// Pass 2 of the method, fused: for every point the mean distance to every cluster from the
// cluster statistics (Eq.11 / Eq.18), a_i, b_i, s_i (Eq.1) and a per-workgroup sum of s_i;
// then the fixed-order reduction of S (Section II).
//
// The point-to-cluster-mean cross term x'.mu'_k over all (i, k) is a dense [N x D] x [D x K]
// product and runs on MFMA; the [N x K] result never leaves registers.
//
// Workgroup: 4 waves; each wave owns NB blocks of 32 rows whose MFMA A-fragments stay in
// registers for the whole sweep over the clusters.  The cluster-mean table is streamed through
// LDS in tiles of 32 clusters (double-buffered, one barrier per tile).  Per tile every wave runs
// the 32x32 MFMA blocks and the epilogue
//     v = c_k + alpha * acc          (alpha = -2 squared Euclidean, -1 cosine)
//     v = +inf for the own cluster   (the column equal to the row's label)
//     running minimum over the tiles (and its column when the backward needs it)
// so b_i = ||x'_i||^2 + min_k v (squared Euclidean) or min_k v (cosine).  Empty and padding
// clusters carry c_k = +inf.
//
// a_i uses the difference form ||x' - mu'_o||^2 + sigma_o^2 (cosine: (1 - ||mu_o||^2 +
// ||z - mu_o||^2)/2) in fp32 from the unrounded point, so the own-cluster term has no
// cancellation; it is computed in the prologue while the point is loaded.
//
// bf16 / fp8 storage: the point is decoded to fp32, centred (squared Euclidean), normalised
// (cosine), then split x' = hi + lo into two bf16; the cluster means are split the same way in
// the table.  products = 1: hi.hi; 2: hi.hi + hi.lo; 3: hi.hi + hi.lo + lo.hi.  fp32 storage
// runs fp32 MFMA on the unsplit values.
#pragma once
#include "sil_internal.h"

namespace sil {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

struct MainArgs {
  const void* X;
  const float* col_scale;
  const int32_t* labels;
  int64_t N;
  int32_t D;
  int32_t K;
  const void* btab;
  const float* cvec;
  const float* atab;
  const float* avec;
  const float* ascale;
  const float* mvec;
  int32_t Kpad;
  int32_t ntiles;
  float* s;
  double* bpart;
  float* save_a;
  float* save_b;
  int32_t* save_n;
};

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (inputs are finite here)
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ float e4m3_f32(uint32_t q) {
  const uint32_t sign = (q & 0x80u) << 24;
  const uint32_t e = (q >> 3) & 15u;
  const uint32_t m = q & 7u;
  if (e == 15u && m == 7u) return __uint_as_float(0x7fc00000u);
  if (e == 0u) {
    const float v = static_cast<float>(m) * 0.001953125f;
    return sign ? -v : v;
  }
  return __uint_as_float(sign | ((e + 120u) << 23) | (m << 20));
}

// W consecutive stored elements of row `row` starting at column c0, decoded to fp32; zero
// outside [0, D) and for rows outside [0, N).
template <int DT, int W>
__device__ __forceinline__ void load_chunk(const void* __restrict__ X,
                                           const float* __restrict__ col_scale, int64_t row,
                                           bool row_ok, int32_t D, int32_t c0, float* out) {
  if (!row_ok || c0 >= D) {
#pragma unroll
    for (int e = 0; e < W; ++e) out[e] = 0.0f;
    return;
  }
  const int64_t base = row * static_cast<int64_t>(D) + c0;
  const bool vec = (D % W) == 0;  // then the whole chunk is inside the row and aligned
  if constexpr (DT == SIL_F32) {
    static_assert(W == 4, "fp32 chunks are 4 wide");
    const float* p = static_cast<const float*>(X) + base;
    if (vec) {
      const f32x4_t v = *reinterpret_cast<const f32x4_t*>(p);
      out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) out[e] = (c0 + e < D) ? p[e] : 0.0f;
    }
  } else if constexpr (DT == SIL_BF16) {
    static_assert(W == 8, "bf16 chunks are 8 wide");
    const uint16_t* p = static_cast<const uint16_t*>(X) + base;
    if (vec) {
      const u32x4_t v = *reinterpret_cast<const u32x4_t*>(p);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        out[2 * e] = bf16_bits_f32(v[e] & 0xffffu);
        out[2 * e + 1] = bf16_bits_f32(v[e] >> 16);
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) out[e] = (c0 + e < D) ? bf16_bits_f32(p[e]) : 0.0f;
    }
  } else {
    static_assert(W == 8, "fp8 chunks are 8 wide");
    const uint8_t* p = static_cast<const uint8_t*>(X) + base;
    if (vec) {
      const u32x2_t v = *reinterpret_cast<const u32x2_t*>(p);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        out[e] = e4m3_f32((v[0] >> (8 * e)) & 0xffu);
        out[4 + e] = e4m3_f32((v[1] >> (8 * e)) & 0xffu);
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) out[e] = (c0 + e < D) ? e4m3_f32(p[e]) : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < W; ++e) out[e] *= (c0 + e < D) ? col_scale[c0 + e] : 0.0f;
  }
}

// Output row (within a 32-row block) held by accumulator register j of a lane in half h of the
// 32x32 MFMA result.
__device__ __forceinline__ int out_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

// ------------------------------------------------------------------------------------------
// Prologue shared by both kernel families.  Lane (r = lane%32, h = lane/32) holds, for each of
// its NB row blocks, the chunks c = 2q + h (q < NQ) of W elements of row r: it decodes them,
// centres / normalises, computes its halves of ||x'||^2 and of the a-path sum, and hands each
// transformed chunk to `emit(nb, q, vals)`.
template <int DT, int W, int NQ, int NB, int METRIC, typename Emit>
__device__ __forceinline__ void prologue(const MainArgs& a, int64_t wrow0, int lane,
                                         float (&nrow)[NB], float (&arow)[NB],
                                         int32_t (&orow)[NB], Emit&& emit) {
  const int r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t row = wrow0 + nb * 32 + r;
    const bool ok = row < a.N;
    int32_t o = ok ? a.labels[row] : -1;
    if (o < 0 || o >= a.K) o = -1;
    float inv = 1.0f;
    if constexpr (METRIC == SIL_COSINE) {
      float n2 = 0.0f;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        float v[W];
        load_chunk<DT, W>(a.X, a.col_scale, row, ok, a.D, (2 * q + h) * W, v);
#pragma unroll
        for (int e = 0; e < W; ++e) n2 = fmaf(v[e], v[e], n2);
      }
      n2 += __shfl_xor(n2, 32, 64);
      inv = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    }
    float nx = 0.0f, ad = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c0 = (2 * q + h) * W;
      float v[W];
      load_chunk<DT, W>(a.X, a.col_scale, row, ok, a.D, c0, v);
#pragma unroll
      for (int e = 0; e < W; ++e) {
        if constexpr (METRIC == SIL_COSINE) {
          v[e] *= inv;
        } else {
          v[e] = ok ? v[e] - a.mvec[c0 + e] : 0.0f;  // mvec is zero when not centring
        }
        nx = fmaf(v[e], v[e], nx);
        if (o >= 0) {
          const float dd = v[e] - a.atab[static_cast<int64_t>(o) * (2 * NQ * W) + c0 + e];
          ad = fmaf(dd, dd, ad);
        }
      }
      emit(nb, q, v);
    }
    nx += __shfl_xor(nx, 32, 64);
    ad += __shfl_xor(ad, 32, 64);
    nrow[nb] = nx;
    orow[nb] = o;
    if (o >= 0) {
      const float sc = a.ascale[o];
      arow[nb] = METRIC == SIL_SQEUCLID ? sc * (ad + a.avec[o]) : sc * 0.5f * (a.avec[o] + ad);
    } else {
      arow[nb] = 0.0f;
    }
  }
}

// Epilogue after the sweep: row minima across the 32 lanes of each half, then s_i per row and
// the workgroup's sum of s_i.
template <int NB, int METRIC, bool SAVE>
__device__ __forceinline__ void finish(const MainArgs& a, int64_t wrow0, int wave, int lane,
                                       float (&mn)[NB][16], int32_t (&arg)[NB][16],
                                       const float (&nrow)[NB], const float (&arow)[NB],
                                       const int32_t (&orow)[NB], float* lds_min,
                                       int32_t* lds_arg, double* lds_bsum) {
  const int h = lane >> 5, col = lane & 31;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        const float ov = __shfl_xor(mn[nb][j], off, 64);
        if constexpr (SAVE) {
          const int32_t oa = __shfl_xor(arg[nb][j], off, 64);
          if (ov < mn[nb][j] || (ov == mn[nb][j] && oa < arg[nb][j])) {
            mn[nb][j] = ov;
            arg[nb][j] = oa;
          }
        } else {
          mn[nb][j] = fminf(mn[nb][j], ov);
        }
      }
      if (col == 0) {
        lds_min[nb * 32 + out_row(j, h)] = mn[nb][j];
        if constexpr (SAVE) lds_arg[nb * 32 + out_row(j, h)] = arg[nb][j];
      }
    }
  __syncthreads();
  double bsum = 0.0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if ((nb & 1) != h) continue;  // lanes of half h finish the blocks nb = h, h+2, ...
    const int r = lane & 31;
    const int64_t row = wrow0 + nb * 32 + r;
    if (row >= a.N) continue;
    const int32_t o = orow[nb];
    float b = lds_min[nb * 32 + r];
    if constexpr (METRIC == SIL_SQEUCLID) b += nrow[nb];
    b = fmaxf(b, 0.0f);
    const float av = fmaxf(arow[nb], 0.0f);
    float s = 0.0f;
    if (o >= 0 && a.ascale[o] > 0.0f) {
      const float mx = fmaxf(av, b);
      s = mx > 0.0f ? (b - av) / mx : 0.0f;
    }
    if (a.s) a.s[row] = s;
    if constexpr (SAVE) {
      a.save_a[row] = av;
      a.save_b[row] = b;
      a.save_n[row] = lds_arg[nb * 32 + r];
    }
    bsum += static_cast<double>(s);
  }
  for (int off = 1; off < 64; off <<= 1) bsum += __shfl_xor(bsum, off, 64);
  if (lane == 0) lds_bsum[wave] = bsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kMainWaves; ++w) t += lds_bsum[w];
    a.bpart[blockIdx.x] = t;
  }
}

// ------------------------------------------------------------------------------------------
// Staging of one 32-cluster tile of the mean table: global (L2) -> registers -> LDS.  Every
// thread loads a valid 16-byte chunk (small tiles wrap around) so that the staging registers
// are written unconditionally; only threads with a chunk index below CHUNKS store to LDS.

template <int DP, int NPC, int CPT>
__device__ __forceinline__ void stage_load_bf16(u32x4_t (&stg)[NPC][CPT],
                                                const uint16_t* __restrict__ bt, int64_t piece,
                                                int t, int tid) {
  constexpr int CHUNKS = 32 * DP / 8;
#pragma unroll
  for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = (tid + 256 * i) % CHUNKS;
      const int rr = q / (DP / 8), cc = q % (DP / 8);
      stg[pc][i] = *reinterpret_cast<const u32x4_t*>(bt + pc * piece +
                                                    static_cast<int64_t>(32 * t + rr) * DP + 8 * cc);
    }
}

template <int DP, int NPC, int CPT, int LROW>
__device__ __forceinline__ void stage_store_bf16(const u32x4_t (&stg)[NPC][CPT], uint16_t* lds,
                                                 int tile_elems, int tid) {
  constexpr int CHUNKS = 32 * DP / 8;
#pragma unroll
  for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = tid + 256 * i;
      if (CHUNKS % 256 == 0 || q < CHUNKS) {
        const int rr = q / (DP / 8), cc = q % (DP / 8);
        *reinterpret_cast<u32x4_t*>(lds + pc * tile_elems + rr * LROW + 8 * cc) = stg[pc][i];
      }
    }
}

template <int DP, int CPT>
__device__ __forceinline__ void stage_load_f32(f32x4_t (&stg)[CPT], const float* __restrict__ bt,
                                               int t, int tid) {
  constexpr int CHUNKS = 32 * DP / 4;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int q = (tid + 256 * i) % CHUNKS;
    const int rr = q / (DP / 4), cc = q % (DP / 4);
    stg[i] = *reinterpret_cast<const f32x4_t*>(bt + static_cast<int64_t>(32 * t + rr) * DP + 4 * cc);
  }
}

template <int DP, int CPT, int LROW>
__device__ __forceinline__ void stage_store_f32(const f32x4_t (&stg)[CPT], float* lds, int tid) {
  constexpr int CHUNKS = 32 * DP / 4;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int q = tid + 256 * i;
    if (CHUNKS % 256 == 0 || q < CHUNKS) {
      const int rr = q / (DP / 4), cc = q % (DP / 4);
      *reinterpret_cast<f32x4_t*>(lds + rr * LROW + 4 * cc) = stg[i];
    }
  }
}

// ------------------------------------------------------------------------------------------
// bf16 MFMA family (X stored bf16 or fp8).  v_mfma_f32_32x32x16_bf16: lane (r, h) supplies
// A[row r][16s + 8h .. +8] and B[col r][16s + 8h .. +8] for k-step s.

template <int DP, int NB, int P, int DT, int METRIC, bool SAVE>
__global__ __launch_bounds__(256, DP >= 256 ? 1 : 2) void k_main_bf16(MainArgs a) {
  constexpr int S = DP / 16;
  constexpr int NPC = P >= 2 ? 2 : 1;
  constexpr int LROW = DP + 8;  // padded LDS row (bf16 elements)
  constexpr int TILE = 32 * LROW;
  constexpr int CHUNKS = 32 * DP / 8;  // 16-byte chunks per piece per tile
  constexpr int CPT = (CHUNKS + 255) / 256;
  constexpr float ALPHA = METRIC == SIL_SQEUCLID ? -2.0f : -1.0f;
  __shared__ __attribute__((aligned(16))) uint16_t lds_b[2][NPC][TILE];
  __shared__ float lds_min[kMainWaves][NB * 32];
  __shared__ int32_t lds_arg[kMainWaves][SAVE ? NB * 32 : 1];
  __shared__ double lds_bsum[kMainWaves];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = lane & 31, h = lane >> 5;
  const int64_t wrow0 = static_cast<int64_t>(blockIdx.x) * (kMainWaves * NB * 32) + wave * NB * 32;

  // ---- A fragments
  u32x4_t ahi[NB][S];
  u32x4_t alo[NB][P == 3 ? S : 1];
  float nrow[NB], arow[NB];
  int32_t orow[NB];
  prologue<DT, 8, S, NB, METRIC>(
      a, wrow0, lane, nrow, arow, orow, [&](int nb, int q, const float* v) __attribute__((always_inline)) {
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint16_t h0 = f32_to_bf16_bits(v[2 * e]);
          const uint16_t h1 = f32_to_bf16_bits(v[2 * e + 1]);
          hw[e] = static_cast<uint32_t>(h0) | (static_cast<uint32_t>(h1) << 16);
          if constexpr (P == 3) {
            const uint16_t l0 = f32_to_bf16_bits(v[2 * e] - bf16_bits_f32(h0));
            const uint16_t l1 = f32_to_bf16_bits(v[2 * e + 1] - bf16_bits_f32(h1));
            lw[e] = static_cast<uint32_t>(l0) | (static_cast<uint32_t>(l1) << 16);
          }
        }
        ahi[nb][q] = u32x4_t{hw[0], hw[1], hw[2], hw[3]};
        if constexpr (P == 3) alo[nb][q] = u32x4_t{lw[0], lw[1], lw[2], lw[3]};
      });

  // own-cluster test: label(row of accumulator j) - col == 32 t
  int32_t dlab[NB][16];
  float mn[NB][16];
  int32_t arg[NB][16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int32_t o = __shfl(orow[nb], out_row(j, h), 64);
      dlab[nb][j] = o >= 0 ? o - col : -1;
      mn[nb][j] = __builtin_inff();
      arg[nb][j] = -1;
    }

  // ---- sweep over cluster tiles
  const uint16_t* bt = static_cast<const uint16_t*>(a.btab);
  const int64_t piece = static_cast<int64_t>(a.Kpad) * DP;
  u32x4_t stg[NPC][CPT];
  stage_load_bf16<DP, NPC, CPT>(stg, bt, piece, 0, tid);
  stage_store_bf16<DP, NPC, CPT, LROW>(stg, &lds_b[0][0][0], TILE, tid);
  float cv_next = a.cvec[col];
  __syncthreads();

  for (int t = 0; t < a.ntiles; ++t) {
    const int buf = t & 1;
    const float cv = cv_next;
    if (t + 1 < a.ntiles) {
      stage_load_bf16<DP, NPC, CPT>(stg, bt, piece, t + 1, tid);
      cv_next = a.cvec[32 * (t + 1) + col];
    }
    f32x16_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[nb][j] = 0.0f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const u32x4_t bh = *reinterpret_cast<const u32x4_t*>(&lds_b[buf][0][col * LROW + 16 * s + 8 * h]);
      const bf16x8_t bhv = __builtin_bit_cast(bf16x8_t, bh);
      bf16x8_t blv;
      if constexpr (P >= 2) {
        const u32x4_t bl = *reinterpret_cast<const u32x4_t*>(&lds_b[buf][NPC - 1][col * LROW + 16 * s + 8 * h]);
        blv = __builtin_bit_cast(bf16x8_t, bl);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, ahi[nb][s]);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bhv, acc[nb], 0, 0, 0);
        if constexpr (P >= 2) acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, blv, acc[nb], 0, 0, 0);
        if constexpr (P == 3) {
          const bf16x8_t al = __builtin_bit_cast(bf16x8_t, alo[nb][s]);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bhv, acc[nb], 0, 0, 0);
        }
      }
    }
    const int32_t t32 = 32 * t;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        float v = fmaf(ALPHA, acc[nb][j], cv);
        v = dlab[nb][j] == t32 ? __builtin_inff() : v;
        if constexpr (SAVE) {
          if (v < mn[nb][j]) {
            mn[nb][j] = v;
            arg[nb][j] = t32 + col;
          }
        } else {
          mn[nb][j] = fminf(mn[nb][j], v);
        }
      }
    if (t + 1 < a.ntiles) stage_store_bf16<DP, NPC, CPT, LROW>(stg, &lds_b[buf ^ 1][0][0], TILE, tid);
    __syncthreads();
  }

  finish<NB, METRIC, SAVE>(a, wrow0, wave, lane, mn, arg, nrow, arow, orow, lds_min[wave],
                           lds_arg[wave], lds_bsum);
}

// ------------------------------------------------------------------------------------------
// fp32 MFMA family.  v_mfma_f32_32x32x2f32: at k-step s lane (r, h) supplies A[row r][k(s,h)]
// and B[col r][k(s,h)] with k(s,h) = 8(s/4) + 4h + s%4, so each lane's operands are whole
// float4 chunks c = 2q + h.

template <int DP, int NB, int METRIC, bool SAVE>
__global__ __launch_bounds__(256, DP >= 256 ? 1 : 2) void k_main_f32(MainArgs a) {
  constexpr int NQ = DP / 8;   // float4 chunks per lane per row
  constexpr int LROW = DP + 4; // padded LDS row (floats)
  constexpr int TILE = 32 * LROW;
  constexpr int CHUNKS = 32 * DP / 4;
  constexpr int CPT = (CHUNKS + 255) / 256;
  constexpr float ALPHA = METRIC == SIL_SQEUCLID ? -2.0f : -1.0f;
  __shared__ __attribute__((aligned(16))) float lds_b[2][TILE];
  __shared__ float lds_min[kMainWaves][NB * 32];
  __shared__ int32_t lds_arg[kMainWaves][SAVE ? NB * 32 : 1];
  __shared__ double lds_bsum[kMainWaves];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = lane & 31, h = lane >> 5;
  const int64_t wrow0 = static_cast<int64_t>(blockIdx.x) * (kMainWaves * NB * 32) + wave * NB * 32;

  f32x4_t areg[NB][NQ];
  float nrow[NB], arow[NB];
  int32_t orow[NB];
  prologue<SIL_F32, 4, NQ, NB, METRIC>(
      a, wrow0, lane, nrow, arow, orow, [&](int nb, int q, const float* v) __attribute__((always_inline)) {
        areg[nb][q] = f32x4_t{v[0], v[1], v[2], v[3]};
      });

  int32_t dlab[NB][16];
  float mn[NB][16];
  int32_t arg[NB][16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int32_t o = __shfl(orow[nb], out_row(j, h), 64);
      dlab[nb][j] = o >= 0 ? o - col : -1;
      mn[nb][j] = __builtin_inff();
      arg[nb][j] = -1;
    }

  const float* bt = static_cast<const float*>(a.btab);
  f32x4_t stg[CPT];
  stage_load_f32<DP, CPT>(stg, bt, 0, tid);
  stage_store_f32<DP, CPT, LROW>(stg, &lds_b[0][0], tid);
  float cv_next = a.cvec[col];
  __syncthreads();

  for (int t = 0; t < a.ntiles; ++t) {
    const int buf = t & 1;
    const float cv = cv_next;
    if (t + 1 < a.ntiles) {
      stage_load_f32<DP, CPT>(stg, bt, t + 1, tid);
      cv_next = a.cvec[32 * (t + 1) + col];
    }
    f32x16_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[nb][j] = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const f32x4_t bv = *reinterpret_cast<const f32x4_t*>(&lds_b[buf][col * LROW + 4 * (2 * q + h)]);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(areg[nb][q][e], bv[e], acc[nb], 0, 0, 0);
        }
    }
    const int32_t t32 = 32 * t;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        float v = fmaf(ALPHA, acc[nb][j], cv);
        v = dlab[nb][j] == t32 ? __builtin_inff() : v;
        if constexpr (SAVE) {
          if (v < mn[nb][j]) {
            mn[nb][j] = v;
            arg[nb][j] = t32 + col;
          }
        } else {
          mn[nb][j] = fminf(mn[nb][j], v);
        }
      }
    if (t + 1 < a.ntiles) stage_store_f32<DP, CPT, LROW>(stg, &lds_b[buf ^ 1][0], tid);
    __syncthreads();
  }

  finish<NB, METRIC, SAVE>(a, wrow0, wave, lane, mn, arg, nrow, arow, orow, lds_min[wave],
                           lds_arg[wave], lds_bsum);
}

}  // namespace sil

namespace sil {

// Per-family launchers (one translation unit each, compiled in parallel).
void launch_main_f32(const MainArgs& m, int DP, int metric, bool save, unsigned grid,
                     hipStream_t st);
void launch_main_bf16(const MainArgs& m, int DP, int metric, int products, unsigned grid,
                      hipStream_t st);
void launch_main_fp8(const MainArgs& m, int DP, int metric, int products, unsigned grid,
                     hipStream_t st);

// Row blocks of 32 per wave for the bf16 family: two unless the split operands of three
// products (or a 256-deep row) would not fit the register budget of two waves per SIMD.
constexpr int bf16_nb(int DP, int P) { return (P == 3 || DP > 128) ? 1 : 2; }

}  // namespace sil
