// Pass 2 of the method, fused: for every point the mean distance to every cluster from the
// cluster statistics (Eq.11 / Eq.18), a_i, b_i, s_i (Eq.1) and a per-workgroup sum of s_i.
//
// The point-to-cluster-mean term over all (i, k) is a dense [N x D] x [D x K] product and runs
// on MFMA; the [N x K] result never leaves registers.  The table row of cluster k is
// alpha * mu'_k (alpha = -2 squared Euclidean, -1 cosine) and the point supplies x', so the
// accumulator holds alpha x'_i.mu'_k; the epilogue adds the per-cluster constant c_k (one fp32
// value per lane, since every accumulator of a lane lies in one cluster column) and keeps a
// running minimum:
//     v_ik = c_k + alpha x'_i.mu'_k,
// b_i = ||x'_i||^2 + min_{k != own} v_ik (squared Euclidean) or 1 + min_{k != own} v_ik (cosine,
// c_k = 0, the 1 added after the minimum).  Empty and padding clusters carry a huge finite c_k.
//
// Rows are visited in label-sorted order (the permutation of the statistics pass), so a block
// of 32 rows almost always belongs to one cluster: its own-cluster column is then excluded by a
// lane mask in a single tile instead of a test per element.  Blocks that straddle a cluster
// boundary take a per-element test against labels staged in LDS.
//
// Workgroup: 4 waves; each wave owns NB blocks of 32 sorted rows whose MFMA A-fragments stay in
// registers for the whole sweep over the clusters.  The table is streamed in tiles of 64
// clusters through an LDS ring of NSTAGE stages filled by direct global->LDS loads, NSTAGE-1
// tiles ahead, one barrier per tile.  Within a tile the two 32-cluster blocks alternate between
// two accumulator sets, so that the minimum over one block runs while the MFMAs of the next are
// in flight, and each k-step's table fragments are read one step ahead.
//
// a_i uses the difference form ||x' - mu'_o||^2 + sigma_o^2 (cosine: (1 - ||mu_o||^2 +
// ||z - mu_o||^2)/2) in fp32 from the unrounded point, so the own-cluster term has no
// cancellation; it is computed in the prologue while the point is loaded.
//
// bf16 / fp8 storage: the point is decoded to fp32, centred (squared Euclidean), normalised
// (cosine), then split x' = hi + lo into two bf16; the table holds the same split of
// alpha mu'.  products = 1: hi.hi; 2: hi.hi + hi.lo; 3: hi.hi + hi.lo + lo.hi.  fp32 storage
// runs fp32 MFMA on unsplit values.
#pragma once
#include "sil_internal.h"

namespace sil {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

struct MainArgs {
  const void* X;
  const float* col_scale;
  const int32_t* perm;     // sorted position -> row
  const int32_t* lsorted;  // sorted position -> label
  const int32_t* hdr;      // [1] = number of valid (sorted) positions
  int64_t N;
  int32_t D;
  int32_t K;
  const void* btab;        // [pieces][Kpad][RS], RS = table_stride(DPX)
  int64_t piece;           // elements per piece (Kpad * RS)
  const float* ctab;       // [Kpad] c_k, added to the cross term in the epilogue
  const float* atab;       // [K][DPX] mu' (a-path)
  const float* avec;
  const float* ascale;
  const float* mvec;       // [DPX] centring vector (zeros when not centring)
  int32_t ntiles;
  int32_t root;            // approximate Euclidean form: square roots of a_i and b_i
  float* s;
  double* bpart;
  float* save_a;
  float* save_b;
  int32_t* save_n;
  // K-means assignment (kernels with the argmin, SAVE): no own-cluster exclusion, the nearest
  // mean's id goes to labels_out[row] and the squared distance to it into the block sum
  int32_t* labels_out = nullptr;
  int32_t assign = 0;
  // rows of X when the positions (N) index a list of them rather than the sorted order (the
  // screen's fallback); 0: N
  int64_t nrows = 0;
};

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (inputs are finite here)
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_f32(uint32_t h) { return __uint_as_float(h << 16); }

// OCP FP8 E4M3 codes by the hardware conversion (gfx950's v_cvt_[pk_]f32_fp8 decode the OCP
// encoding exactly, NaN codes included)
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float e4m3_f32(uint32_t q) {
  return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(q & 0xffu), 0);
}
// the four codes of a 32-bit word, lowest byte first
__device__ __forceinline__ void e4m3x4_f32(uint32_t w, float* out) {
  const f32x2_t lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), false);
  const f32x2_t hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), true);
  out[0] = lo[0];
  out[1] = lo[1];
  out[2] = hi[0];
  out[3] = hi[1];
}

// W consecutive stored elements of row `row` starting at column c0, decoded to fp32; zero
// outside [0, D) and for invalid rows.  SCALE = false leaves fp8 codes unscaled.
template <int DT, int W, bool SCALE = true>
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
      e4m3x4_f32(v[0], out);
      e4m3x4_f32(v[1], out + 4);
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) out[e] = (c0 + e < D) ? e4m3_f32(p[e]) : 0.0f;
    }
    if constexpr (SCALE) {
#pragma unroll
      for (int e = 0; e < W; ++e) out[e] *= (c0 + e < D) ? col_scale[c0 + e] : 0.0f;
    }
  }
}

// Output row (within a 32-row block) held by accumulator register j of a lane in half h of the
// 32x32 MFMA result.
__device__ __forceinline__ int out_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

// ------------------------------------------------------------------------------------------
// Per-block bookkeeping: sorted positions, rows, labels.

template <int NB>
struct Blocks {
  int64_t p0;          // first sorted position of the wave's blocks
  int64_t row[NB];     // row id of this lane's A-layout row (lane % 32) in block nb
  bool ok[NB];         // position valid
  int32_t lab[NB];     // label of that row (-1 if invalid)
  bool mixed[NB];      // block straddles a cluster boundary (wave-uniform)
  int32_t town[NB];    // uniform block: tile holding the own cluster (wave-uniform)
  int32_t cown[NB];    // uniform block: lane column of the own cluster (wave-uniform)
};

// Row ids and labels of a wave's row blocks, loaded ahead of the block that uses them.
template <int NB>
struct RowPre {
  int32_t row[NB];
  int32_t lab[NB];
};

// Loads the row ids and labels of sorted positions p0 + 32 nb + lane%32.  Positions are
// valid below N: when every label is in range the sort covers all N rows; otherwise the
// result is replaced by NaN and only the addresses must stay in bounds, so row ids are
// clamped to [0, N) and labels outside [0, K) become -1.
template <int NB>
__device__ __forceinline__ RowPre<NB> fetch_rows(const MainArgs& a, int64_t p0, int lane) {
  RowPre<NB> pre;
  const int r = lane & 31;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t pos = p0 + nb * 32 + r;
    const bool ok = pos < a.N;
    pre.row[nb] = ok ? a.perm[pos] : 0;
    pre.lab[nb] = ok ? a.lsorted[pos] : -1;
  }
  return pre;
}

template <int NB>
__device__ __forceinline__ void make_blocks(const MainArgs& a, const RowPre<NB>& pre, int64_t p0,
                                            int lane, Blocks<NB>& B, int32_t* lds_lab) {
  const int r = lane & 31;
  B.p0 = p0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t pos = p0 + nb * 32 + r;
    B.ok[nb] = pos < a.N;
    const int32_t rw = pre.row[nb];
    B.row[nb] = (rw >= 0 && rw < (a.nrows ? a.nrows : a.N)) ? rw : 0;
    int32_t o = B.ok[nb] ? pre.lab[nb] : -1;
    if (o < 0 || o >= a.K) o = -1;
    B.lab[nb] = o;
    const int32_t o0 = __shfl(o, 0, 64);
    B.mixed[nb] = !__all(o == o0 || o < 0);
    B.town[nb] = o0 >> 5;
    B.cown[nb] = o0 & 31;
    if (a.assign) {  // the minimum runs over every cluster, the own one included
      B.mixed[nb] = false;
      B.town[nb] = -1;
    }
    if (lane < 32) lds_lab[nb * 32 + r] = o;  // labels of the block for the mixed-block path
  }
}

// ------------------------------------------------------------------------------------------
// Prologue shared by both kernel families.  Lane (r = lane%32, h = lane/32) holds, for each of
// its NB row blocks, the chunks c = 2q + h (q < NQ) of W elements of row r: it decodes them,
// centres / normalises, computes its halves of ||x'||^2 (phi(x) for KL) and of the a-path sum,
// and hands each transformed chunk (zero past D) to emit(nb, q, vals).
// When D is a multiple of W every chunk is one aligned vector load, issued for the whole row
// before any is used (addresses clamped in range, values masked afterwards).
// RAW: emit hands over x itself rather than x' = x - m (squared Euclidean: the tables fold the
// centring into c_k) or z = x / |x| (cosine: the finish scales by 1 / |x|); the row and a-path
// terms still use x' or z.  For fp8 storage it hands over the e4m3 codes, unscaled (the tables
// carry the column scales).  For cosine, nrow holds the finish's scale: 1 / |x| (RAW) or 1.

template <int DT>
struct RawChunk;
template <>
struct RawChunk<SIL_F32> { typedef f32x4_t T; };
template <>
struct RawChunk<SIL_BF16> { typedef u32x4_t T; };
template <>
struct RawChunk<SIL_FP8_E4M3> { typedef u32x2_t T; };

template <int DT, int W>
__device__ __forceinline__ typename RawChunk<DT>::T load_raw(const void* __restrict__ X,
                                                              int64_t row, int32_t D, int32_t c0) {
  const int64_t base = row * static_cast<int64_t>(D) + c0;
  if constexpr (DT == SIL_F32)
    return *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(X) + base);
  else if constexpr (DT == SIL_BF16)
    return *reinterpret_cast<const u32x4_t*>(static_cast<const uint16_t*>(X) + base);
  else
    return *reinterpret_cast<const u32x2_t*>(static_cast<const uint8_t*>(X) + base);
}

template <int DT, int W, bool SCALE = true>
__device__ __forceinline__ void decode_raw(typename RawChunk<DT>::T raw,
                                           const float* __restrict__ col_scale, int32_t c0,
                                           bool valid, float* out) {
  if constexpr (DT == SIL_F32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = raw[e];
  } else if constexpr (DT == SIL_BF16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      out[2 * e] = bf16_bits_f32(raw[e] & 0xffffu);
      out[2 * e + 1] = bf16_bits_f32(raw[e] >> 16);
    }
  } else {
    e4m3x4_f32(raw[0], out);
    e4m3x4_f32(raw[1], out + 4);
    if constexpr (SCALE) {
#pragma unroll
      for (int e = 0; e < 8; ++e) out[e] *= col_scale[c0 + e];
    }
  }
#pragma unroll
  for (int e = 0; e < W; ++e) out[e] = valid ? out[e] : 0.0f;
}

// W consecutive floats from a 16-byte aligned address.
template <int W>
__device__ __forceinline__ void load_f32w(const float* __restrict__ p, float* out) {
#pragma unroll
  for (int i = 0; i < W / 4; ++i) {
    const f32x4_t v = *reinterpret_cast<const f32x4_t*>(p + 4 * i);
    out[4 * i] = v[0];
    out[4 * i + 1] = v[1];
    out[4 * i + 2] = v[2];
    out[4 * i + 3] = v[3];
  }
}

// VEC_ONLY: the caller guarantees D % W == 0 and 16-byte aligned column scales, so only the
// whole-vector paths are compiled.
// ROWTERMS = false: only the emitted chunks; nrow and arow are left to the caller.
// WHOLE: the caller guarantees D == DPX (no chunk past D) and discards every result of a row
// past N, so those rows (which read row 0's values) are not zeroed.
template <int DT, int W, int NQ, int NB, int METRIC, bool RAW, bool VEC_ONLY = false,
          bool ROWTERMS = true, bool WHOLE = false, typename Emit>
__device__ __forceinline__ void prologue(const MainArgs& a, const Blocks<NB>& B, int lane,
                                         float (&nrow)[NB], float (&arow)[NB], Emit&& emit) {
  constexpr int DPX = 2 * NQ * W;
  constexpr bool CODES = RAW && DT == SIL_FP8_E4M3;  // xv holds unscaled fp8 codes
  const int h = lane >> 5;
  const bool vec = VEC_ONLY || WHOLE || (a.D % W) == 0;  // wave-uniform
  // chunk c0 lies inside the row
  auto inside = [&](int c0) __attribute__((always_inline)) { return WHOLE || c0 < a.D; };
  // the column scales of chunk c0 (fp8 codes), zero past D: whole-vector loads when every chunk
  // lies inside the row and the scales are 16-byte aligned
  const bool svec =
      VEC_ONLY || (vec && (reinterpret_cast<uintptr_t>(a.col_scale) & 15u) == 0);
  const float* colsc = a.col_scale;
  auto scales = [&](int c0, float* sc) __attribute__((always_inline)) {
    if (svec) {
      if (inside(c0)) {
        load_f32w<W>(colsc + c0, sc);
      } else {
#pragma unroll
        for (int e = 0; e < W; ++e) sc[e] = 0.0f;
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) sc[e] = c0 + e < a.D ? colsc[c0 + e] : 0.0f;
    }
  };
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const bool ok = WHOLE || B.ok[nb];  // zero the row's values unless it lies below N
    const int64_t row = B.ok[nb] ? B.row[nb] : 0;
    const int32_t o = B.lab[nb];
    const int64_t orow = static_cast<int64_t>(o >= 0 ? o : 0) * DPX;
    float xv[NQ][W];
    if (vec) {
      typename RawChunk<DT>::T raw[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c0 = (2 * q + h) * W;
        raw[q] = load_raw<DT, W>(a.X, row, a.D, inside(c0) ? c0 : 0);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c0 = (2 * q + h) * W;
        decode_raw<DT, W, !CODES>(raw[q], a.col_scale, inside(c0) ? c0 : 0, ok && inside(c0),
                                  xv[q]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        load_chunk<DT, W, !CODES>(a.X, a.col_scale, row, ok, a.D, (2 * q + h) * W, xv[q]);
    }
    float inv = 1.0f;
    if constexpr (METRIC == SIL_COSINE) {
      float n2 = 0.0f;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        float sc[W];
        if constexpr (CODES) scales((2 * q + h) * W, sc);
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const float x = CODES ? xv[q][e] * sc[e] : xv[q][e];
          n2 = fmaf(x, x, n2);
        }
      }
      n2 += __shfl_xor(n2, 32, 64);
      inv = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    }
    if constexpr (!ROWTERMS) {
      static_assert(RAW, "without the row terms the prologue only hands over raw chunks");
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        float u[W];
#pragma unroll
        for (int e = 0; e < W; ++e) u[e] = ok ? xv[q][e] : 0.0f;
        emit(nb, q, u);
      }
      continue;
    }
    float nx = 0.0f, ad = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c0 = (2 * q + h) * W;
      // the chunk's centring values and own-cluster mean: W consecutive floats at a multiple of
      // W (mvec and atab rows hold DPX floats, 256-byte aligned regions), so whole-vector loads
      float mv[W], at[W];
      if constexpr (METRIC == SIL_SQEUCLID) load_f32w<W>(a.mvec + c0, mv);
      load_f32w<W>(a.atab + orow + c0, at);
      float x[W];  // the stored values (fp8 codes times their column scales)
      if constexpr (CODES) {
        float sc[W];
        scales(c0, sc);
#pragma unroll
        for (int e = 0; e < W; ++e) x[e] = xv[q][e] * sc[e];
      } else {
#pragma unroll
        for (int e = 0; e < W; ++e) x[e] = xv[q][e];
      }
      float v[W];
#pragma unroll
      for (int e = 0; e < W; ++e) {
        if constexpr (METRIC == SIL_KL) {
          // phi(x) = sum x log x - x for the row term, x . (mean log y) of the own cluster for
          // the a-path; x is not centred (the divergence is not translation invariant)
          v[e] = ok ? x[e] : 0.0f;
          nx += v[e] > 0.0f ? v[e] * logf(v[e]) - v[e] : 0.0f;
          ad = fmaf(v[e], at[e], ad);
        } else {
          if constexpr (METRIC == SIL_COSINE)
            v[e] = x[e] * inv;
          else
            v[e] = ok ? x[e] - mv[e] : 0.0f;  // mvec is zero when not centring
          nx = fmaf(v[e], v[e], nx);
          const float dd = v[e] - at[e];
          ad = fmaf(dd, dd, ad);
        }
      }
      if constexpr (RAW) {
        static_assert(METRIC == SIL_SQEUCLID || METRIC == SIL_COSINE, "raw x: squared Euclidean or cosine");
        float u[W];
#pragma unroll
        for (int e = 0; e < W; ++e) u[e] = ok ? xv[q][e] : 0.0f;
        emit(nb, q, u);
      } else {
        emit(nb, q, v);
      }
    }
    nx += __shfl_xor(nx, 32, 64);
    ad += __shfl_xor(ad, 32, 64);
    if constexpr (METRIC == SIL_COSINE)
      nrow[nb] = RAW ? inv : 1.0f;
    else
      nrow[nb] = nx;
    if (o >= 0) {
      const float sc = a.ascale[o];
      if constexpr (METRIC == SIL_SQEUCLID)
        arow[nb] = sc * (ad + a.avec[o]);
      else if constexpr (METRIC == SIL_COSINE)
        arow[nb] = sc * 0.5f * (a.avec[o] + ad);
      else  // m_io = phi(x) + c_o - x . (mean log y)_o
        arow[nb] = sc * (nx + a.avec[o] - ad);
    } else {
      arow[nb] = 0.0f;
    }
  }
}

// Running minimum over one tile of the accumulators of block nb.  cv is c_k of the lane's
// column (every accumulator of a lane lies in that column): m = cross term + c_k.
template <bool SAVE>
__device__ __forceinline__ void tile_min(const f32x16_t& acc, float (&mn)[16], int32_t (&arg)[16],
                                         bool mixed, bool own_tile, int col, int cown, int t32,
                                         const int32_t* lab_block, int h, float cv) {
  constexpr float BIG = 3.0e38f;
  if (mixed) {  // per-element own-cluster test against the block's labels
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const i32x4_t l4 = *reinterpret_cast<const i32x4_t*>(lab_block + 8 * q + 4 * h);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * q + e;
        const float v = (l4[e] == t32 + col) ? BIG : acc[j] + cv;
        if constexpr (SAVE) {
          if (v < mn[j]) { mn[j] = v; arg[j] = t32 + col; }
        } else {
          mn[j] = fminf(mn[j], v);
        }
      }
    }
  } else if (own_tile) {  // the own cluster is column cown of this tile for every row
    const bool me = col == cown;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float v = me ? BIG : acc[j] + cv;
      if constexpr (SAVE) {
        if (v < mn[j]) { mn[j] = v; arg[j] = t32 + col; }
      } else {
        mn[j] = fminf(mn[j], v);
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float v = acc[j] + cv;
      if constexpr (SAVE) {
        if (v < mn[j]) { mn[j] = v; arg[j] = t32 + col; }
      } else {
        mn[j] = fminf(mn[j], v);
      }
    }
  }
}

// Minimum over the 32 lanes of each half of the wave, in every lane of that half: data-parallel
// lane moves fused into the min within 16-lane rows (swap neighbours, swap pairs, mirror
// within 8, mirror within 16), then a swizzle that exchanges lane i and i ^ 16.
template <int CTRL>
__device__ __forceinline__ float dpp_min(float v) {
  const int o = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xf, 0xf,
                                            false);
  return fminf(v, __int_as_float(o));
}

__device__ __forceinline__ float min_over_half(float v) {
  v = dpp_min<0xb1>(v);   // quad_perm [1,0,3,2]
  v = dpp_min<0x4e>(v);   // quad_perm [2,3,0,1]
  v = dpp_min<0x141>(v);  // row_half_mirror
  v = dpp_min<0x140>(v);  // row_mirror
  const int o = __builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401f);  // lane ^ 16 in 32
  return fminf(v, __int_as_float(o));
}

// min(keep, send of the partner lane) for a data-parallel lane move CTRL.
template <int CTRL>
__device__ __forceinline__ float dpp_min2(float keep, float send) {
  const int o = __builtin_amdgcn_update_dpp(__float_as_int(send), __float_as_int(send), CTRL, 0xf,
                                            0xf, false);
  return fminf(keep, __int_as_float(o));
}

// Minimum over the 32 lanes of each half of the wave for each of a lane's 16 values, spread over
// the lanes: lane c of a half ends with the minimum of value j = c >> 1 (lanes c and c ^ 1 both
// hold it).  Each step pairs lanes that differ in one lane bit (bit 4: lane ^ 16; bit 3: the
// mirror within 16 lanes; bit 2: the mirror within 8; bit 1: lane ^ 2), and each lane keeps the
// half of its values that its bit selects, taking the minimum with what its partner sends for
// that half; a last step with lane ^ 1 completes the minimum.  8 + 4 + 2 + 1 + 1 exchanges for
// the 16 values, against 5 per value when every lane reduces all 16.
__device__ __forceinline__ float min_scatter16(const float (&v)[16], int lane) {
  const bool b4 = (lane & 16) != 0, b3 = (lane & 8) != 0, b2 = (lane & 4) != 0,
             b1 = (lane & 2) != 0;
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float keep = b4 ? v[i + 8] : v[i], send = b4 ? v[i] : v[i + 8];
    const int o = __builtin_amdgcn_ds_swizzle(__float_as_int(send), 0x401f);  // lane ^ 16 in 32
    a[i] = fminf(keep, __int_as_float(o));
  }
  float b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    b[i] = dpp_min2<0x140>(b3 ? a[i + 4] : a[i], b3 ? a[i] : a[i + 4]);  // row_mirror
  float c[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
    c[i] = dpp_min2<0x141>(b2 ? b[i + 2] : b[i], b2 ? b[i] : b[i + 2]);  // row_half_mirror
  const float d = dpp_min2<0x4e>(b1 ? c[1] : c[0], b1 ? c[0] : c[1]);  // quad_perm [2,3,0,1]
  return dpp_min2<0xb1>(d, d);                                          // quad_perm [1,0,3,2]
}

// After the sweep: row minima across the 32 lanes of each half, then s_i per row (written to
// the row's original index) and each wave's sum of s_i (bpart[kMainWaves wb + wave]).
template <int NB, int METRIC, bool SAVE>
__device__ __forceinline__ void finish(const MainArgs& a, int64_t wb, const Blocks<NB>& B, int wave, int lane,
                                       float (&mn)[NB][16], int32_t (&arg)[NB][16],
                                       const float (&nrow)[NB], const float (&arow)[NB],
                                       float* lds_min, int32_t* lds_arg) {
  const int h = lane >> 5, col = lane & 31;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if constexpr (!SAVE) {
      const float m = min_scatter16(mn[nb], lane);
      if ((col & 1) == 0) lds_min[nb * 32 + out_row(col >> 1, h)] = m;
      continue;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if constexpr (SAVE) {  // minimum and its (lowest) cluster id
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) {
          const float ov = __shfl_xor(mn[nb][j], off, 64);
          const int32_t oa = __shfl_xor(arg[nb][j], off, 64);
          if (ov < mn[nb][j] || (ov == mn[nb][j] && oa < arg[nb][j])) {
            mn[nb][j] = ov;
            arg[nb][j] = oa;
          }
        }
      } else {
        mn[nb][j] = min_over_half(mn[nb][j]);
      }
      if (col == 0) {
        lds_min[nb * 32 + out_row(j, h)] = mn[nb][j];
        if constexpr (SAVE) lds_arg[nb * 32 + out_row(j, h)] = arg[nb][j];
      }
    }
  }
  // lds_min / lds_arg are this wave's own: the LDS completes one wave's operations in order, so
  // the reads below see the writes above without a workgroup barrier
  __builtin_amdgcn_wave_barrier();
  double bsum = 0.0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if ((nb & 1) != h) continue;  // lanes of half h finish the blocks nb = h, h+2, ...
    if (!B.ok[nb]) continue;
    const int r = lane & 31;
    const int64_t row = B.row[nb];
    const int32_t o = B.lab[nb];
    float b = lds_min[nb * 32 + r];
    if constexpr (METRIC == SIL_COSINE)
      b = fmaf(nrow[nb], b, 1.0f);  // 1 + min_k(-z.mu_k), or the raw form's 1 + min_k(-x.mu_k) / |x|
    else
      b += nrow[nb];  // ||x'||^2, or phi(x) for KL
    b = fmaxf(b, 0.0f);
    if constexpr (SAVE) {
      if (a.assign) {  // K-means assignment: nearest mean and the squared distance to it
        a.labels_out[row] = lds_arg[nb * 32 + r];
        bsum += static_cast<double>(b);
        continue;
      }
    }
    float av = fmaxf(arow[nb], 0.0f);
    if (METRIC == SIL_SQEUCLID && a.root) {  // the mean distances' square roots
      b = sqrtf(b);
      av = sqrtf(av);
    }
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
  // one partial sum per wave (kMainWaves per row block): no workgroup barrier in the finish
  for (int off = 1; off < 64; off <<= 1) bsum += __shfl_xor(bsum, off, 64);
  if (lane == 0) a.bpart[wb * kMainWaves + wave] = bsum;
}

// ------------------------------------------------------------------------------------------
// Tile ring: one tile is PIECES contiguous blocks of kColTile table rows x ROWBYTES in global memory;
// wave w moves 1 KB per instruction (lane l -> 16 bytes at LDS offset 16 l), IPW instructions
// per wave and tile.

template <int PIECES_, int ROWBYTES, int NS_MAX = 3, int COLS = kColTile>
struct Ring {
  static constexpr int PIECES = PIECES_;
  static constexpr int SLOTS_PER_PIECE = COLS * ROWBYTES / 16;
  static constexpr int TOT = PIECES * SLOTS_PER_PIECE;  // 16-byte slots per tile
  static constexpr int IPW = (TOT + 64 * kMainWaves - 1) / (64 * kMainWaves);
  // fewest instructions any wave issues per tile: waiting until at most this many are in
  // flight guarantees that every older tile has landed
  static constexpr int IPW_MIN = TOT / (64 * kMainWaves);
  static constexpr int STAGE_BYTES = TOT * 16;
  // three stages while two workgroups per CU still fit the 160 KB of LDS, else two
  static constexpr int NSTAGE = NS_MAX >= 3 && 3 * STAGE_BYTES <= 52 * 1024 ? 3 : 2;
};

// Tile t into an LDS stage; piece_bytes is the byte size of one piece of the table (every piece
// holds all ntiles tiles).  The table is read through a buffer resource (the buffer form of
// the global -> LDS load): unlike the flat-encoded global form, it leaves the compiler's count
// of outstanding LDS reads exact, so that fragment reads are waited for one by one instead of
// all at once.  The resource spans the table's PIECES pieces (at most 2^31 bytes).
template <typename R>
__device__ __forceinline__ void issue_tile(const char* __restrict__ base, int64_t piece_bytes,
                                           int t, uint8_t* stage, int wave, int lane) {
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(base), 0, static_cast<int>(piece_bytes * R::PIECES), 0x00020000);
#pragma unroll
  for (int i = 0; i < R::IPW; ++i) {
    const int blk = i * kMainWaves + wave;
    const int q = blk * 64 + lane;
    if (blk * 64 < R::TOT) {
      const int pc = q / R::SLOTS_PER_PIECE, w = q % R::SLOTS_PER_PIECE;
      const int off = static_cast<int>(pc * piece_bytes) + t * R::SLOTS_PER_PIECE * 16 + w * 16;
      if (q < R::TOT)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rsrc, (__attribute__((address_space(3))) void*)(stage + blk * 1024), 16, off, 0, 0, 0);
    }
  }
}

// s_waitcnt for the vector-memory counter only (expcnt and lgkmcnt left at their maximum);
// gfx9 encoding: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt_hi[15:14].
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Sweep over the tiles (the first NSTAGE-1 already issued by issue_first) with an LDS ring of
// NSTAGE (2 or 3) stages, each its own __shared__
// array and visited in a statically unrolled order, so that the compiler can tell the stage
// being read from the stages being filled.  body(t, stage_to_read, prefetch) must call
// prefetch() once, after its first LDS read; prefetch() issues tile t + NSTAGE - 1 into the stage
// read in the previous step.  Each step: wait for this wave's loads of tile t, barrier (without
// a memory fence: the loads of later tiles stay in flight), then the body.
// The first NSTAGE-1 tiles, issued before the row block's prologue so that their latency
// overlaps it (every wave must be done with the ring: call after a barrier).
template <typename R>
__device__ __forceinline__ void issue_first(const char* bt, int64_t piece_bytes, int ntiles,
                                            uint8_t* r0, uint8_t* r1, int wave, int lane) {
  for (int t = 0; t < R::NSTAGE - 1 && t < ntiles; ++t)
    issue_tile<R>(bt, piece_bytes, t, t == 0 ? r0 : r1, wave, lane);
}

template <typename R, typename Body>
__device__ __forceinline__ void sweep(const char* bt, int64_t piece_bytes, int ntiles,
                                      uint8_t* r0, uint8_t* r1, uint8_t* r2, int wave, int lane,
                                      Body&& body) {
  constexpr int NS = R::NSTAGE;
  auto step = [&](int t, uint8_t* rd, uint8_t* wr) __attribute__((always_inline)) {
    if (NS == 3 && t + 1 < ntiles)
      wait_vmcnt<R::IPW_MIN>();
    else
      wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    body(t, rd, [&]() __attribute__((always_inline)) {
      if (t + NS - 1 < ntiles) issue_tile<R>(bt, piece_bytes, t + NS - 1, wr, wave, lane);
    });
  };
  for (int t = 0; t < ntiles; t += NS) {
    if constexpr (NS == 3) {
      step(t, r0, r2);
      if (t + 1 < ntiles) step(t + 1, r1, r0);
      if (t + 2 < ntiles) step(t + 2, r2, r1);
    } else {
      step(t, r0, r1);
      if (t + 1 < ntiles) step(t + 1, r1, r0);
    }
  }
}

// ------------------------------------------------------------------------------------------
// bf16 MFMA family (X stored bf16 or fp8).  v_mfma_f32_32x32x16_bf16: lane (r, h) supplies
// A[row r][16s + 8h .. +8] and B[col r][16s + 8h .. +8] for k-step s.

// One row block (wb) of the bf16 kernel, given the wave's row ids and labels (pre) and with
// the block's first table tiles already issued into the ring.  LDS buffers and tid as in
// main_f32_body.
template <int DPX, int NB, int P, int DT, int METRIC, bool SAVE, int TC = kColTile>
__device__ __forceinline__ void main_bf16_body(const MainArgs& a, int64_t wb,
                                               const RowPre<NB>& pre, uint8_t* ring0,
                                               uint8_t* ring1, uint8_t* ring2, float* lds_min,
                                               int32_t* lds_arg, int32_t* lds_lab, int tid) {
  constexpr int S = DPX / 16;
  constexpr int NPC = P >= 2 ? 2 : 1;
  constexpr int RS = table_stride(DPX, SIL_BF16);
  using R = Ring<NPC, RS * 2, 3, TC>;
  constexpr int ARGW = SAVE ? NB * 32 : 1;

  // wave-uniform, so that per-wave addresses (LDS DMA destinations) live in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int col = lane & 31, h = lane >> 5;
  const int64_t wg0 = wb * (kMainWaves * NB * 32);
  int32_t* lab_w = lds_lab + wave * NB * 32;

  Blocks<NB> B;
  make_blocks<NB>(a, pre, wg0 + wave * NB * 32, lane, B, lab_w);

  u32x4_t ahi[NB][S];
  u32x4_t alo[NB][P == 3 ? S : 1];
  float nrow[NB], arow[NB];
  prologue<DT, 8, S, NB, METRIC, kRawX<DT, P, METRIC>>(
      a, B, lane, nrow, arow, [&](int nb, int q, const float* v) __attribute__((always_inline)) {
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

  float mn[NB][16];
  int32_t arg[NB][16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      mn[nb][j] = __builtin_inff();
      arg[nb][j] = -1;
    }

  // B fragments of k-step s of one 32-cluster block: [piece]
  struct Frag { bf16x8_t v[2]; };
  auto bfrag = [&](const uint8_t* st, int cb, int s) __attribute__((always_inline)) {
    Frag f;
    const int off = ((cb * 32 + col) * RS + 16 * s + 8 * h) * 2;
    f.v[0] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(st + off));
    if constexpr (P >= 2)
      f.v[1] = __builtin_bit_cast(bf16x8_t,
                                  *reinterpret_cast<const u32x4_t*>(st + R::SLOTS_PER_PIECE * 16 + off));
    return f;
  };
  constexpr int LA = S >= 3 ? 2 : 1;  // k-steps of table fragments read ahead

  // All k-steps of one 32-cluster block into acc: hi.hi (+ hi.lo) (+ lo.hi) per step.
  auto gemm = [&](const uint8_t* st, int cb, f32x16_t (&acc)[NB], auto&& after_first_read)
      __attribute__((always_inline)) {
    Frag f[LA + 1];
    f[0] = bfrag(st, cb, 0);
    after_first_read();
#pragma unroll
    for (int s = 1; s < LA; ++s) f[s] = bfrag(st, cb, s);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (s + LA < S) f[(s + LA) % (LA + 1)] = bfrag(st, cb, s + LA);
      // keep the read-ahead ahead: the scheduler would otherwise sink the reads next to
      // their first use and wait for them there
      __builtin_amdgcn_sched_barrier(0);
      const Frag& g = f[s % (LA + 1)];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, ahi[nb][s]);
        if (s == 0)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, g.v[0], f32x16_t{}, 0, 0, 0);
        else
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, g.v[0], acc[nb], 0, 0, 0);
        if constexpr (P >= 2)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, g.v[1], acc[nb], 0, 0, 0);
        if constexpr (P == 3) {
          const bf16x8_t al = __builtin_bit_cast(bf16x8_t, alo[nb][s]);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, g.v[0], acc[nb], 0, 0, 0);
        }
      }
    }
  };
  // Running minimum over 32-cluster block blk (global index) of the tile sweep; cv = c_k of
  // the lane's column, loaded ahead of the block's MFMAs.
  auto epi = [&](const f32x16_t (&acc)[NB], int blk, float cv) __attribute__((always_inline)) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      tile_min<SAVE>(acc[nb], mn[nb], arg[nb], B.mixed[nb], blk == B.town[nb], col, B.cown[nb],
                     32 * blk, lab_w + nb * 32, h, cv);
  };

  if constexpr (TC == 64) {
    // Per tile: block 0's MFMAs, the previous block 1's minimum (under them), block 1's MFMAs,
    // block 0's minimum (under them).  Block 1 of the last tile is skipped when it holds only
    // padding clusters (K mod 64 in 1 .. 32): they never win the minimum.
    f32x16_t acc0[NB], acc1[NB];
    float c1p = 0.0f;  // c_k of block 1 of the previous tile
    const bool last_b1 = 64 * (a.ntiles - 1) + 32 < a.K;
    sweep<R>(static_cast<const char*>(a.btab), a.piece * 2, a.ntiles, ring0, ring1, ring2, wave,
             lane, [&](int t, const uint8_t* st, auto&& prefetch) __attribute__((always_inline)) {
      const float c0 = a.ctab[64 * t + col], c1 = a.ctab[64 * t + 32 + col];
      gemm(st, 0, acc0, prefetch);
      if (t > 0) epi(acc1, 2 * t - 1, c1p);
      if (t + 1 < a.ntiles || last_b1) gemm(st, 1, acc1, [] {});
      epi(acc0, 2 * t, c0);
      c1p = c1;
    });
    if (last_b1) epi(acc1, 2 * a.ntiles - 1, c1p);
  } else {
    // 32-cluster tiles (one block each): the other workgroups' waves on the SIMD fill the gap
    // of each minimum
    static_assert(TC == 32, "tiles of 32 or 64 clusters");
    f32x16_t acc0[NB];
    // the last tile is skipped when it holds only padding clusters (its prefetch issues nothing)
    const bool last_real = 32 * (a.ntiles - 1) < a.K;
    sweep<R>(static_cast<const char*>(a.btab), a.piece * 2, a.ntiles, ring0, ring1, ring2, wave,
             lane, [&](int t, const uint8_t* st, auto&& prefetch) __attribute__((always_inline)) {
      if (t + 1 < a.ntiles || last_real) {
        const float c0 = a.ctab[32 * t + col];
        gemm(st, 0, acc0, prefetch);
        epi(acc0, t, c0);
      }
    });
  }

  __syncthreads();
  finish<NB, METRIC, SAVE>(a, wb, B, wave, lane, mn, arg, nrow, arow, lds_min + wave * NB * 32,
                           lds_arg + wave * ARGW);
}

// One row block per workgroup; two workgroups share a CU, so that one's prologue and finish
// run under the other's sweep.
// TC: clusters per table tile, 64 (two workgroups per CU) or 32 (three per CU: the ring is half
// as large and the kernel fits 168 registers; a.ntiles counts tiles of TC clusters).
template <int DPX, int NB, int P, int DT, int METRIC, bool SAVE, int TC = kColTile>
__global__ __launch_bounds__(256, DPX > 128 ? 1 : (TC == 32 ? 3 : 2)) void k_main_bf16(MainArgs a) {
  constexpr int NPC = P >= 2 ? 2 : 1;
  constexpr int RS = table_stride(DPX, SIL_BF16);
  using R = Ring<NPC, RS * 2, 3, TC>;
  __shared__ __attribute__((aligned(16))) uint8_t ring0[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring2[R::NSTAGE == 3 ? R::STAGE_BYTES : 16];
  __shared__ float lds_min[kMainWaves * NB * 32];
  __shared__ int32_t lds_arg[kMainWaves * (SAVE ? NB * 32 : 1)];
  __shared__ __attribute__((aligned(16))) int32_t lds_lab[kMainWaves * NB * 32];

  constexpr int64_t ROWS = kMainWaves * NB * 32;
  const int64_t wb = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // the first tiles' latency overlaps the prologue
  issue_first<R>(static_cast<const char*>(a.btab), a.piece * 2, a.ntiles, ring0, ring1, wave, lane);
  const RowPre<NB> pre = fetch_rows<NB>(a, wb * ROWS + wave * NB * 32, lane);
  main_bf16_body<DPX, NB, P, DT, METRIC, SAVE, TC>(a, wb, pre, ring0, ring1, ring2, lds_min,
                                                   lds_arg, lds_lab, threadIdx.x);
}

// ------------------------------------------------------------------------------------------
// fp32 MFMA family.  v_mfma_f32_32x32x2f32: at k-step s lane (r, h) supplies A[row r][k(s,h)]
// and B[col r][k(s,h)] with k(s,h) = 8(s/4) + 4h + s%4, so each lane's operands are whole
// float4 chunks c = 2q + h.

// One row block (wb) of the fp32 kernel, given the wave's row ids and labels (pre) and with
// the block's first table tiles already issued into the ring (f32_ring<DPX, NS_MAX>).  The LDS
// buffers come from the caller: ring0..2 the table stages (ring2 unused with two stages),
// lds_min/lds_lab [kMainWaves][NB*32], lds_arg [kMainWaves][SAVE ? NB*32 : 1].  NS_MAX caps the ring at two stages where the caller provides only two.  tid
// is the thread's index in the workgroup; a caller that runs the body in a loop passes it
// through an opaque copy, so that the lane-dependent addresses are recomputed per block
// instead of being kept live across the loop.
template <int DPX, int NS_MAX>
using f32_ring = Ring<1, table_stride(DPX, SIL_F32) * 4, NS_MAX>;

template <int DPX, int NB, int METRIC, bool SAVE, int NS_MAX>
__device__ __forceinline__ void main_f32_body(const MainArgs& a, int64_t wb, const RowPre<NB>& pre,
                                              uint8_t* ring0, uint8_t* ring1, uint8_t* ring2,
                                              float* lds_min, int32_t* lds_arg, int32_t* lds_lab, int tid) {
  constexpr int NQ = DPX / 8;
  constexpr int RS = table_stride(DPX, SIL_F32);
  using R = f32_ring<DPX, NS_MAX>;
  constexpr int ARGW = SAVE ? NB * 32 : 1;

  // wave-uniform, so that per-wave addresses (LDS DMA destinations) live in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int col = lane & 31, h = lane >> 5;
  const int64_t wg0 = wb * (kMainWaves * NB * 32);

  int32_t* lab_w = lds_lab + wave * NB * 32;
  Blocks<NB> B;
  make_blocks<NB>(a, pre, wg0 + wave * NB * 32, lane, B, lab_w);

  f32x4_t areg[NB][NQ];
  float nrow[NB], arow[NB];
  prologue<SIL_F32, 4, NQ, NB, METRIC, false>(
      a, B, lane, nrow, arow, [&](int nb, int q, const float* v) __attribute__((always_inline)) {
        areg[nb][q] = f32x4_t{v[0], v[1], v[2], v[3]};
      });

  float mn[NB][16];
  int32_t arg[NB][16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      mn[nb][j] = __builtin_inff();
      arg[nb][j] = -1;
    }

  auto bfrag = [&](const uint8_t* st, int cb, int q) __attribute__((always_inline)) {
    return *reinterpret_cast<const f32x4_t*>(st + ((cb * 32 + col) * RS + 4 * (2 * q + h)) * 4);
  };
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
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(areg[nb][0][0], bv[0][0], f32x16_t{}, 0, 0, 0);
          else
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(areg[nb][q][e], bv[q & 1][e], acc[nb], 0, 0, 0);
        }
    }
  };
  auto epi = [&](const f32x16_t (&acc)[NB], int blk, float cv) __attribute__((always_inline)) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      tile_min<SAVE>(acc[nb], mn[nb], arg[nb], B.mixed[nb], blk == B.town[nb], col, B.cown[nb],
                     32 * blk, lab_w + nb * 32, h, cv);
  };

  // block 1 of the last tile is skipped when it holds only padding clusters (as in the bf16 body)
  f32x16_t acc0[NB], acc1[NB];
  float c1p = 0.0f;  // c_k of block 1 of the previous tile
  const bool last_b1 = 64 * (a.ntiles - 1) + 32 < a.K;
  sweep<R>(static_cast<const char*>(a.btab), a.piece * 4, a.ntiles, ring0, ring1, ring2, wave, lane,
           [&](int t, const uint8_t* st, auto&& prefetch) __attribute__((always_inline)) {
    const float c0 = a.ctab[64 * t + col], c1 = a.ctab[64 * t + 32 + col];
    gemm(st, 0, acc0, prefetch);
    if (t > 0) epi(acc1, 2 * t - 1, c1p);
    if (t + 1 < a.ntiles || last_b1) gemm(st, 1, acc1, [] {});
    epi(acc0, 2 * t, c0);
    c1p = c1;
  });
  if (last_b1) epi(acc1, 2 * a.ntiles - 1, c1p);

  __syncthreads();
  finish<NB, METRIC, SAVE>(a, wb, B, wave, lane, mn, arg, nrow, arow, lds_min + wave * NB * 32,
                           lds_arg + wave * ARGW);
}

template <int DPX, int NB, int METRIC, bool SAVE>
__global__ __launch_bounds__(256, DPX > 128 ? 1 : 2) void k_main_f32(MainArgs a) {
  constexpr int RS = table_stride(DPX, SIL_F32);
  using R = Ring<1, RS * 4>;
  __shared__ __attribute__((aligned(16))) uint8_t ring0[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring2[R::NSTAGE == 3 ? R::STAGE_BYTES : 16];
  __shared__ float lds_min[kMainWaves * NB * 32];
  __shared__ int32_t lds_arg[kMainWaves * (SAVE ? NB * 32 : 1)];
  __shared__ __attribute__((aligned(16))) int32_t lds_lab[kMainWaves * NB * 32];
  constexpr int64_t ROWS = kMainWaves * NB * 32;
  const int64_t wb = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // the first tiles' latency overlaps the prologue
  issue_first<R>(static_cast<const char*>(a.btab), a.piece * 4, a.ntiles, ring0, ring1, wave, lane);
  const RowPre<NB> pre = fetch_rows<NB>(a, wb * ROWS + wave * NB * 32, lane);
  main_f32_body<DPX, NB, METRIC, SAVE, 3>(a, wb, pre, ring0, ring1, ring2, lds_min, lds_arg,
                                          lds_lab, threadIdx.x);
}

}  // namespace sil

namespace sil {

// Per-family launchers (one translation unit each, compiled in parallel).
void launch_main_f32(const MainArgs& m, int DPX, int metric, bool save, unsigned grid,
                     hipStream_t st);
void launch_main_bf16(const MainArgs& m, int DPX, int metric, int products, unsigned grid,
                      hipStream_t st);
// K-means assignment with bf16 MFMA (X stored bf16 or fp8), squared Euclidean: three products,
// or two with folded centring for bf16 storage; one row block per wave
void launch_main_assign(const MainArgs& m, int DPX, int dtype, int products, unsigned grid,
                        hipStream_t st);
void launch_main_fp8(const MainArgs& m, int DPX, int metric, int products, unsigned grid,
                     hipStream_t st);

// Row blocks of 32 per wave for the bf16 family: two unless the split operands of three
// products (or a deep row) would not fit the register budget of two waves per SIMD.  Two row
// blocks read each table fragment from LDS once for 64 rows, which halves the LDS traffic per
// MFMA: at depth 128 with two products it is as large as the MFMA time with one block.  fp8
// storage stops at depth 64 (its decode would spill at 128).
constexpr int bf16_nb(int DPX, int P, int DT) {
  return (P == 3 || DPX > (DT == SIL_BF16 ? 128 : 64)) ? 1 : 2;
}

}  // namespace sil
