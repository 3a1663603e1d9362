// Fused pass 2 with a one-product screen (squared Euclidean, X stored bf16 or fp8, Eq.11).
//
// The two-product kernel spends half its MFMA work on the low half of the cluster means, which
// only matters for the few clusters that can be a row's closest other cluster.  Here one fp16
// product finds that cluster and the epilogue scores it exactly:
//   1. screen: x in fp16 (exact for bf16 values of magnitude 2^-14 .. 65504, off by less than
//      2^-24 below that; rows with larger values go to the fallback) times the fp16 table
//      T16_k ~ -2 mu'_k, accumulated onto the fp32 constant c_k (the first MFMA's accumulator
//      input, so the epilogue has no add and no k-step carries the constant); every value is
//      known to within the row's bound E (see screen.hip).  Each lane keeps, per row, the smallest and second smallest value over its
//      columns (v_med3 + v_min); the 32-cluster block index rides in the low mantissa bits of
//      the smallest, so that the lane and those bits name the cluster.
//   2. the finish takes both minima across the 32 lanes of a row.  When the second exceeds the
//      first by more than 2 E (plus the perturbation of the index bits), the smallest names the
//      row's closest other cluster n exactly, and b_i = ||x'||^2 + c_n - 2 x . mu'_n is formed
//      for n alone in fp32 (x exact, mu'_n and c_n as the two-product form rounds them).
//   3. the other rows are appended to a list (one atomic per wave reserves its entries), and
//      the two-product kernel runs over that list (fallback), adding its own partial sums of
//      s_i.  S = (sum over screened rows + sum over fallback rows) / N; the fallback's sums
//      follow the list's order, which depends on the schedule (as the order of rows within a
//      cluster does in the statistics pass), so S is reproducible to binary64 rounding, not
//      bitwise.
// When the clusters are large (N >= 512 K, so at most one row in 16 lies in a 32-row block that
// straddles a cluster boundary), such blocks are deferred whole to the fallback and the sweep
// excludes only a uniform block's own cluster, with selects and no branches; otherwise the sweep
// tests every row of a straddling block against its own cluster.
// Rows are visited in label-sorted order as in the other fused kernels; 4 waves, two 32-row
// blocks per wave, 64-cluster tiles through the same LDS ring.
#include "main_kernels.h"

namespace sil {

typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

struct ScreenArgs {
  const void* stab;     // fp16 screen table [Kpad][screen_stride(DPX)]
  int64_t stab_bytes;   // its size
  int32_t* hdr;         // header: the screen's bound slots, the fallback count
  int32_t* fblist;      // [N] sorted positions of the rows left to the fallback
  const float* rtab;    // fp8: [K][DPX] column scales times mu'_k
  int32_t ibits;        // bits of the 32-cluster block index packed into the screen values
};

constexpr uint32_t kExcluded = 0x7f7fffffu;  // FLT_MAX: a column that never competes

__device__ __forceinline__ float slot_f(const int32_t* hdr, int slot) {
  const unsigned long long* p =
      reinterpret_cast<const unsigned long long*>(hdr + kHdrScreenWord) + slot;
  // rounded up, so that the bound stays a bound in fp32
  return static_cast<float>(__longlong_as_double(static_cast<long long>(*p)) * (1.0 + 0x1p-20));
}

// Running smallest (m1, with the block index in its low bits) and second smallest (m2) over one
// 32-cluster block of the accumulators of a row block.  keep / tag: AND and OR applied to each
// value's bits (keep = 0, tag = kExcluded for a column that does not compete).
__device__ __forceinline__ void screen_min(const f32x16_t& acc, float (&m1)[16], float (&m2)[16],
                                           uint32_t keep, uint32_t tag) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const float v = __uint_as_float((__float_as_uint(acc[j]) & keep) | tag);
    m2[j] = __builtin_amdgcn_fmed3f(v, m1[j], m2[j]);
    m1[j] = fminf(m1[j], v);
  }
}

// The same for a block that straddles a cluster boundary: the own column is excluded per row.
__device__ __forceinline__ void screen_min_mixed(const f32x16_t& acc, float (&m1)[16],
                                                 float (&m2)[16], uint32_t keep, uint32_t tag,
                                                 int32_t k, const int32_t* lab_block, int h) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const i32x4_t l4 = *reinterpret_cast<const i32x4_t*>(lab_block + 8 * q + 4 * h);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * q + e;
      const uint32_t bits = (__float_as_uint(acc[j]) & keep) | tag;
      const float v = __uint_as_float(l4[e] == k ? kExcluded : bits);
      m2[j] = __builtin_amdgcn_fmed3f(v, m1[j], m2[j]);
      m1[j] = fminf(m1[j], v);
    }
  }
}

// Smallest and second smallest over the 32 lanes of each half of the wave, for each of a lane's
// 16 rows, with the lane (column) of the smallest: the reduce-scatter of min_scatter16, each
// exchange merging two partial results (first = the smaller first, second = the smaller of the
// larger first and both seconds, column of the smaller first).  Lane c of a half ends with row
// j = c >> 1 (lanes c and c ^ 1 hold the same result up to the column of an exact tie, where the
// two firsts are equal and the row fails the screen's test anyway).
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ void top2_merge(float& k1, float& k2, int& kw, float r1, float r2,
                                           int rw) {
  const bool take = r1 < k1;
  k2 = fminf(fmaxf(k1, r1), fminf(k2, r2));
  kw = take ? rw : kw;
  k1 = fminf(k1, r1);
}

template <int CTRL>
__device__ __forceinline__ void top2_step(float& k1, float& k2, int& kw, float s1, float s2, int sw) {
  top2_merge(k1, k2, kw, __int_as_float(dpp_mov<CTRL>(__float_as_int(s1))),
             __int_as_float(dpp_mov<CTRL>(__float_as_int(s2))), dpp_mov<CTRL>(sw));
}

__device__ __forceinline__ void top2_scatter16(const float (&m1)[16], const float (&m2)[16], int lane,
                                               float& g1, float& g2, int& win) {
  const int col = lane & 31;
  const bool b4 = (lane & 16) != 0, b3 = (lane & 8) != 0, b2 = (lane & 4) != 0,
             b1 = (lane & 2) != 0;
  float a1[8], a2[8];
  int aw[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {  // partner lane ^ 16: its column is known
    a1[i] = b4 ? m1[i + 8] : m1[i];
    a2[i] = b4 ? m2[i + 8] : m2[i];
    aw[i] = col;
    const float s1 = b4 ? m1[i] : m1[i + 8], s2 = b4 ? m2[i] : m2[i + 8];
    top2_merge(a1[i], a2[i], aw[i],
               __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(s1), 0x401f)),
               __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(s2), 0x401f)),
               col ^ 16);
  }
  float c1[4], c2[4];
  int cw[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {  // row_mirror
    c1[i] = b3 ? a1[i + 4] : a1[i];
    c2[i] = b3 ? a2[i + 4] : a2[i];
    cw[i] = b3 ? aw[i + 4] : aw[i];
    top2_step<0x140>(c1[i], c2[i], cw[i], b3 ? a1[i] : a1[i + 4], b3 ? a2[i] : a2[i + 4],
                     b3 ? aw[i] : aw[i + 4]);
  }
  float d1[2], d2[2];
  int dw[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {  // row_half_mirror
    d1[i] = b2 ? c1[i + 2] : c1[i];
    d2[i] = b2 ? c2[i + 2] : c2[i];
    dw[i] = b2 ? cw[i + 2] : cw[i];
    top2_step<0x141>(d1[i], d2[i], dw[i], b2 ? c1[i] : c1[i + 2], b2 ? c2[i] : c2[i + 2],
                     b2 ? cw[i] : cw[i + 2]);
  }
  g1 = b1 ? d1[1] : d1[0];  // quad_perm [2,3,0,1]
  g2 = b1 ? d2[1] : d2[0];
  win = b1 ? dw[1] : dw[0];
  top2_step<0x4e>(g1, g2, win, b1 ? d1[0] : d1[1], b1 ? d2[0] : d2[1], b1 ? dw[0] : dw[1]);
  const float e1 = g1, e2 = g2;  // quad_perm [1,0,3,2]
  const int ew = win;
  top2_step<0xb1>(g1, g2, win, e1, e2, ew);
}

// fp8 codes: ||x'||^2 (x' = codes times column scales, centred) and the a-path term of each row,
// from the rows' fp16 code fragments, formed after the sweep.  In the prologue, every chunk's
// scales, centring values and own-cluster means would be loaded together beside the fragments
// and spill; here the registers of the running minima are free.  Same arithmetic as the
// prologue's row terms.
template <int S, int NB, bool WHOLE>
__device__ __forceinline__ void code_row_terms(const MainArgs& a, const Blocks<NB>& B, int lane,
                                               const u32x4_t (&xf)[NB][S], float (&nrow)[NB],
                                               float (&arow)[NB]) {
  constexpr int DPX = 16 * S;
  const int h = lane >> 5;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const bool ok = WHOLE || B.ok[nb];  // as in the prologue
    const int32_t o = B.lab[nb];
    const int64_t orow = static_cast<int64_t>(o >= 0 ? o : 0) * DPX;
    float nx = 0.0f, ad = 0.0f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int c0 = 16 * s + 8 * h;  // the chunk the prologue handed over as q = s
      float sc[8], mv[8], at[8];
      if (WHOLE || c0 < a.D) {
        load_f32w<8>(a.col_scale + c0, sc);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) sc[e] = 0.0f;
      }
      load_f32w<8>(a.mvec + c0, mv);
      load_f32w<8>(a.atab + orow + c0, at);
      const f16x8_t cf = __builtin_bit_cast(f16x8_t, xf[nb][s]);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = static_cast<float>(cf[e]) * sc[e];
        const float v = ok ? x - mv[e] : 0.0f;
        nx = fmaf(v, v, nx);
        const float dd = v - at[e];
        ad = fmaf(dd, dd, ad);
      }
      if (s % 2 == 1) __builtin_amdgcn_sched_barrier(0);  // at most two chunks' loads in flight
    }
    nx += __shfl_xor(nx, 32, 64);
    ad += __shfl_xor(ad, 32, 64);
    nrow[nb] = nx;
    arow[nb] = o >= 0 ? a.ascale[o] * (ad + a.avec[o]) : 0.0f;
  }
}

// TC: clusters per table tile (64 or 128; a tile is one barrier and one ring stage).  NB: 32-row
// blocks per wave: 2 (two workgroups per CU, one accumulator set) or 1 (three workgroups per CU,
// two accumulator sets alternating between the tile's two 32-cluster blocks, TC = 64).
// DT: X stored bf16 (x itself in the GEMM) or fp8 e4m3 (its codes in the GEMM, the column scales
// in the table); both are exact in fp16 (fp8 always, bf16 for magnitudes 2^-14 .. 65504).
// WHOLE: D == DPX, so no chunk lies past D, and the rows past N are not zeroed (the finish
// discards them).  DEFER: the rows of a block that straddles a cluster boundary go to the
// fallback (the sweep has no per-row exclusion).
template <int DPX, int TC, int NB, int DT, bool WHOLE, bool DEFER>
__global__ __launch_bounds__(256, NB == 2 ? 2 : 3) void k_main_screen(MainArgs a, ScreenArgs sa) {
  static_assert(NB == 2 || (NB == 1 && TC == 64), "screen configurations");
  static_assert(DT == SIL_BF16 || DT == SIL_FP8_E4M3, "bf16 or fp8 storage");
  constexpr bool CODES = DT == SIL_FP8_E4M3;
  constexpr int S = DPX / 16;  // k-steps over the coordinates
  constexpr int RSS = screen_stride(DPX);
  constexpr int BPT = TC / 32;  // 32-cluster blocks per tile
  using R = Ring<1, RSS * 2, TC == 64 ? 3 : 2, TC>;
  constexpr int64_t ROWS = kMainWaves * NB * 32;
  // the ring's stages (separate arrays, so that the compiler tells the stage being read from the
  // stages being filled); the row minima have arrays of their own, so that a wave that is done
  // with the sweep goes on to its finish while the others still read the ring
  __shared__ __attribute__((aligned(16))) uint8_t ring0[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring2[R::NSTAGE == 3 ? R::STAGE_BYTES : 16];
  __shared__ float lds_m1[kMainWaves * NB * 32];
  __shared__ float lds_m2[kMainWaves * NB * 32];
  __shared__ int32_t lds_win[kMainWaves * NB * 32];
  __shared__ __attribute__((aligned(16))) int32_t lds_lab[kMainWaves * NB * 32];

  const int64_t wb = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int col = lane & 31, h = lane >> 5;
  const char* tab = static_cast<const char*>(sa.stab);
  const int64_t piece_bytes = sa.stab_bytes;
  const int ntiles = static_cast<int>(ceil_div(a.K, TC));  // tiles holding real clusters
  issue_first<R>(tab, piece_bytes, ntiles, ring0, ring1, wave, lane);
  const RowPre<NB> pre = fetch_rows<NB>(a, wb * ROWS + wave * NB * 32, lane);
  int32_t* lab_w = lds_lab + wave * NB * 32;
  Blocks<NB> B;
  make_blocks<NB>(a, pre, wb * ROWS + wave * NB * 32, lane, B, lab_w);

  // Prologue: the row term ||x'||^2 and the a-path as in the other kernels; the GEMM operand (x,
  // or the fp8 codes) goes into fp16 fragments (round toward zero: exact for bf16 values of
  // magnitude 2^-14 .. 65504, within 2^-24 below; exact for every e4m3 code), with the row's
  // largest magnitude (bf16 rows at or above 65504 are not screened) and, for fp8, the squared
  // norm of the codes.
  u32x4_t xf[NB][S];
  float nrow[NB], arow[NB], amax[NB], ncode[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    amax[nb] = 0.0f;
    ncode[nb] = 0.0f;
  }
  prologue<DT, 8, S, NB, SIL_SQEUCLID, true, CODES, !CODES, WHOLE>(
      a, B, lane, nrow, arow, [&](int nb, int q, const float* v) __attribute__((always_inline)) {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          w[e] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(v[2 * e], v[2 * e + 1]));
          if constexpr (CODES) {
            ncode[nb] = fmaf(v[2 * e], v[2 * e], ncode[nb]);
            ncode[nb] = fmaf(v[2 * e + 1], v[2 * e + 1], ncode[nb]);
          } else {
            amax[nb] = fmaxf(amax[nb], fmaxf(fabsf(v[2 * e]), fabsf(v[2 * e + 1])));
          }
        }
        xf[nb][q] = u32x4_t{w[0], w[1], w[2], w[3]};
      });
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    amax[nb] = fmaxf(amax[nb], __shfl_xor(amax[nb], 32, 64));
    ncode[nb] += __shfl_xor(ncode[nb], 32, 64);
  }
  // the table's scale 2^-f (see screen.hip), for the constant the accumulations start from
  const float inv_scale = ldexpf(1.0f, -screen_exponent(
      fmax(__longlong_as_double(static_cast<long long>(
               reinterpret_cast<const unsigned long long*>(sa.hdr + kHdrScreenWord)[SC_TMAX])),
           __longlong_as_double(static_cast<long long>(
               reinterpret_cast<const unsigned long long*>(sa.hdr + kHdrScreenWord)[SC_CMAX])))));

  float m1[NB][16], m2[NB][16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      m1[nb][j] = __builtin_inff();
      m2[nb][j] = __builtin_inff();
    }

  auto bfrag = [&](const uint8_t* st, int cb, int s) __attribute__((always_inline)) {
    const int off = ((cb * 32 + col) * RSS + 16 * s + 8 * h) * 2;
    return __builtin_bit_cast(f16x8_t, *reinterpret_cast<const u32x4_t*>(st + off));
  };
  constexpr int LA = 2;  // k-steps of table fragments read ahead
  // cv: c_k of the lane's column (fp32, unscaled); every accumulator of a lane lies in that
  // column, so the block's accumulations of both row blocks start from cv 2^-f
  auto gemm = [&](const uint8_t* st, int cb, f32x16_t (&acc)[NB], auto&& after_first_read,
                  float cv) __attribute__((always_inline)) {
    f16x8_t f[LA + 1];
    f[0] = bfrag(st, cb, 0);
    after_first_read();
#pragma unroll
    for (int s = 1; s < LA; ++s) f[s] = bfrag(st, cb, s);
    const float c = cv * inv_scale;
    const f32x16_t cinit = {c, c, c, c, c, c, c, c, c, c, c, c, c, c, c, c};
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (s + LA < S) f[(s + LA) % (LA + 1)] = bfrag(st, cb, s + LA);
      __builtin_amdgcn_sched_barrier(0);
      const f16x8_t g = f[s % (LA + 1)];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const f16x8_t x = __builtin_bit_cast(f16x8_t, xf[nb][s]);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(x, g, s == 0 ? cinit : acc[nb], 0, 0, 0);
      }
    }
  };
  const uint32_t keep_in = ~((1u << sa.ibits) - 1u);
  int town_x[NB];  // DEFER: the 32-cluster block holding the own cluster (-1: none excluded)
  bool mycol[NB];  // DEFER: the lane's column is the own cluster's
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    town_x[nb] = __builtin_amdgcn_readfirstlane(B.mixed[nb] ? -1 : B.town[nb]);
    mycol[nb] = col == B.cown[nb];
  }
  // minima over 32-cluster block blk; cv = c_k of the lane's column (1e30: empty or padding)
  auto epi = [&](const f32x16_t (&acc)[NB], int blk_in, float cv) __attribute__((always_inline)) {
    const bool empty = cv >= 1.0e29f;
    if constexpr (DEFER) {
      const int blk = __builtin_amdgcn_readfirstlane(blk_in);  // wave-uniform
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        // selects, not branches: excluded are empty (or padding) columns and the own cluster
        const bool out = empty | ((blk == town_x[nb]) & mycol[nb]);
        const uint32_t keep = out ? 0u : keep_in;
        const uint32_t tag = out ? kExcluded : static_cast<uint32_t>(blk);
        screen_min(acc[nb], m1[nb], m2[nb], keep, tag);
      }
      return;
    }
    const int blk = blk_in;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bool out = empty || (!B.mixed[nb] && blk == B.town[nb] && col == B.cown[nb]);
      const uint32_t keep = out ? 0u : keep_in;
      const uint32_t tag = out ? kExcluded : static_cast<uint32_t>(blk);
      if (B.mixed[nb])
        screen_min_mixed(acc[nb], m1[nb], m2[nb], keep, tag, 32 * blk + col, lab_w + nb * 32, h);
      else
        screen_min(acc[nb], m1[nb], m2[nb], keep, tag);
    }
  };

  // One accumulator set (two would not fit the registers of two workgroups per CU beside the
  // second minimum): the other waves on the SIMD fill each block's minimum with their MFMAs.
  // Blocks past the last real cluster (padding only) are skipped; table rows past Kpad read as
  // zeros (the buffer resource ends at the table).
  const int nblk = static_cast<int>(ceil_div(a.K, 32));
  if constexpr (NB == 2) {
    f32x16_t acc[NB];
    sweep<R>(tab, piece_bytes, ntiles, ring0, ring1, ring2, wave, lane,
             [&](int t, const uint8_t* st, auto&& prefetch) __attribute__((always_inline)) {
      float cv[BPT];
#pragma unroll
      for (int cb = 0; cb < BPT; ++cb)
        cv[cb] = BPT * t + cb < nblk ? a.ctab[TC * t + 32 * cb + col] : 0.0f;
      gemm(st, 0, acc, prefetch, cv[0]);
      epi(acc, BPT * t, cv[0]);
#pragma unroll
      for (int cb = 1; cb < BPT; ++cb) {
        if (BPT * t + cb < nblk) {
          gemm(st, cb, acc, [] {}, cv[cb]);
          epi(acc, BPT * t + cb, cv[cb]);
        }
      }
    });
  } else {
    // block 0's MFMAs, the previous tile's block 1 minimum under them, block 1's MFMAs, block 0's
    // minimum under them
    f32x16_t acc0[NB], acc1[NB];
    float c1p = 0.0f;
    const bool last_b1 = 2 * (ntiles - 1) + 1 < nblk;
    sweep<R>(tab, piece_bytes, ntiles, ring0, ring1, ring2, wave, lane,
             [&](int t, const uint8_t* st, auto&& prefetch) __attribute__((always_inline)) {
      const float c0 = a.ctab[64 * t + col];
      const float c1 = 2 * t + 1 < nblk ? a.ctab[64 * t + 32 + col] : 0.0f;
      gemm(st, 0, acc0, prefetch, c0);
      if (t > 0) epi(acc1, 2 * t - 1, c1p);
      if (t + 1 < ntiles || last_b1) gemm(st, 1, acc1, [] {}, c1);
      epi(acc0, 2 * t, c0);
      c1p = c1;
    });
    if (last_b1) epi(acc1, 2 * ntiles - 1, c1p);
  }

  // ---- finish: both minima across the row's 32 lanes (no workgroup barrier from here on)
  float* lm1 = lds_m1 + wave * NB * 32;
  float* lm2 = lds_m2 + wave * NB * 32;
  int32_t* lwin = lds_win + wave * NB * 32;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    float g1, g2;
    int win;
    top2_scatter16(m1[nb], m2[nb], lane, g1, g2, win);
    if ((col & 1) == 0) {
      lm1[nb * 32 + out_row(col >> 1, h)] = g1;
      lm2[nb * 32 + out_row(col >> 1, h)] = g2;
      lwin[nb * 32 + out_row(col >> 1, h)] = win;
    }
  }
  if constexpr (CODES) code_row_terms<S, NB, WHOLE>(a, B, lane, xf, nrow, arow);
  // lm1 / lm2 / lwin are this wave's own (the LDS completes one wave's operations in order)
  __builtin_amdgcn_wave_barrier();

  const float L1 = slot_f(sa.hdr, SC_L1), L2 = slot_f(sa.hdr, SC_L2);
  const float L3 = slot_f(sa.hdr, SC_L3), EC = slot_f(sa.hdr, SC_EC);
  const float MN = slot_f(sa.hdr, SC_MNORM);
  constexpr float acc_eps = (DPX + 16) * 0x1p-23f;
  // ||x - x16|| < sqrt(DPX) 2^-24 (values below fp16's normal range), times ||T16_k|| <= L2
  const float xq_err = sqrtf(static_cast<float>(DPX)) * 0x1p-24f * L2;
  const float tiny_row = sqrtf(static_cast<float>(DPX)) * 0x1p-8f;
  const float pert = ldexpf(1.0f, sa.ibits - 21);
  const uint32_t idx_mask = (1u << sa.ibits) - 1u;
  const int r = lane & 31;
  double bsum = 0.0;
  uint64_t fmask[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const float g1 = lm1[nb * 32 + r], g2 = lm2[nb * 32 + r];
    const int32_t n = static_cast<int32_t>(__float_as_uint(g1) & idx_mask) * 32 + lwin[nb * 32 + r];
    const int32_t o = B.lab[nb];
    const bool valid = B.ok[nb] && o >= 0;
    const bool single = valid && !(a.ascale[o] > 0.0f);
    // the GEMM operand's norm: ||x|| <= ||x'|| + ||m|| (x' = x - m) for bf16, the codes' for fp8
    const float nx = CODES ? sqrtf(ncode[nb]) : sqrtf(fmaxf(nrow[nb], 0.0f)) + MN;
    const float E = (nx * L1 + EC + acc_eps * (nx * L2 + L3) + xq_err) * inv_scale * 1.001f;
    const float P = pert * (fabsf(g1) + fabsf(g2)) + 1.0e-30f;
    // rows beyond fp16's range, and rows so small (max |x| < sqrt(DPX) 2^-8, hence ||x|| too)
    // that the fp16 rounding of their smallest values could reach the two-product form's error
    // in the exact score, are not screened
    const bool fits = CODES || (amax[nb] < 65504.0f && amax[nb] >= tiny_row);
    const bool unique = valid && !single && !(DEFER && B.mixed[nb]) && fits && n < a.K &&
                        (g2 - g1) > 2.0f * E + P;
    const bool flag = valid && !single && !unique;
    // the exact score of cluster n: this lane's half of x . mu'_n (x from its fp16 fragments;
    // fp8: the codes against the column scales times mu'_n)
    float dot = 0.0f;
    if (unique) {
      const float* mu = (CODES ? sa.rtab : a.atab) + static_cast<int64_t>(n) * DPX + 8 * h;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        float mv[8];
        load_f32w<8>(mu + 16 * s, mv);
        const f16x8_t xv = __builtin_bit_cast(f16x8_t, xf[nb][s]);
#pragma unroll
        for (int e = 0; e < 8; ++e) dot = fmaf(static_cast<float>(xv[e]), mv[e], dot);
      }
    }
    dot += __shfl_xor(dot, 32, 64);
    const bool owner = h == (nb & 1);
    if (owner && valid && !flag) {
      float s_i = 0.0f;
      if (!single) {
        float b = fmaxf(nrow[nb] + a.ctab[n] - 2.0f * dot, 0.0f);
        float av = fmaxf(arow[nb], 0.0f);
        if (a.root) {
          b = sqrtf(b);
          av = sqrtf(av);
        }
        const float mx = fmaxf(av, b);
        s_i = mx > 0.0f ? (b - av) / mx : 0.0f;
      }
      if (a.s) a.s[B.row[nb]] = s_i;
      bsum += static_cast<double>(s_i);
    }
    fmask[nb] = __ballot(owner && flag);
  }
  int nflag = 0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) nflag += __popcll(fmask[nb]);
  // one partial sum per wave (kMainWaves per workgroup), and each wave reserves its own list
  // entries: no workgroup barrier after the sweep's
  for (int off = 1; off < 64; off <<= 1) bsum += __shfl_xor(bsum, off, 64);
  if (lane == 0) a.bpart[wb * kMainWaves + wave] = bsum;
  if (nflag > 0) {  // wave-uniform: the wave's marked rows, in position order
    int base = 0;
    if (lane == 0) base = atomicAdd(sa.hdr + kHdrFallbackWord, nflag);
    int at = __shfl(base, 0, 64);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const uint64_t m = fmask[nb];
      if ((m >> lane) & 1u) {
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        sa.fblist[at + before] = static_cast<int32_t>(wb * ROWS + wave * NB * 32 + nb * 32 + r);
      }
      at += __popcll(m);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Fallback: the two-product kernel over the listed rows (a persistent grid; each workgroup takes
// 256 list entries at a time until the list is exhausted).

template <int DPX, int DT>
__global__ __launch_bounds__(256, 2) void k_main_fallback(MainArgs a, const int32_t* fblist,
                                                          const int32_t* hdr) {
  constexpr int NB = bf16_nb(DPX, 2, DT);
  constexpr int RS = table_stride(DPX, SIL_BF16);
  using R = Ring<2, RS * 2, 3, kColTile>;
  constexpr int64_t ROWS = kMainWaves * NB * 32;
  __shared__ __attribute__((aligned(16))) uint8_t ring0[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[R::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t ring2[R::NSTAGE == 3 ? R::STAGE_BYTES : 16];
  __shared__ float lds_min[kMainWaves * NB * 32];
  __shared__ int32_t lds_arg[kMainWaves];
  __shared__ __attribute__((aligned(16))) int32_t lds_lab[kMainWaves * NB * 32];

  const int32_t total = hdr[kHdrFallbackWord];
  MainArgs b = a;
  b.nrows = a.N;
  b.N = total;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int64_t lb = blockIdx.x; lb * ROWS < total; lb += gridDim.x) {
    issue_first<R>(static_cast<const char*>(a.btab), a.piece * 2, a.ntiles, ring0, ring1, wave, lane);
    RowPre<NB> pre;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t p = lb * ROWS + wave * NB * 32 + nb * 32 + (lane & 31);
      pre.row[nb] = 0;
      pre.lab[nb] = -1;
      if (p < total) {
        int64_t pos = fblist[p];
        pos = pos < 0 ? 0 : (pos >= a.N ? a.N - 1 : pos);
        pre.row[nb] = a.perm[pos];
        pre.lab[nb] = a.lsorted[pos];
      }
    }
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));  // keep the body's lane addresses inside the loop
    main_bf16_body<DPX, NB, 2, DT, SIL_SQEUCLID, false, kColTile>(
        b, lb, pre, ring0, ring1, ring2, lds_min, lds_arg, lds_lab, tid);
  }
}

hipError_t launch_fb_sum(const WsPtrs& w, int rows_per_wg, hipStream_t st);

constexpr int kScreenTile = 64;
constexpr int kScreenNB = 2;
int screen_rows_per_block() { return kMainWaves * kScreenNB * 32; }

template <int DPX, int DT>
static void run_screen(const MainArgs& m, const ScreenArgs& sa, const WsLayout& L,
                       const WsPtrs& w, hipStream_t st) {
  // large clusters: at most 32 (K - 1) rows lie in blocks that straddle a boundary
  const bool defer = m.N >= int64_t{512} * m.K;
  const unsigned g = static_cast<unsigned>(L.nsblk);
  if (m.D == DPX) {
    if (defer)
      k_main_screen<DPX, kScreenTile, kScreenNB, DT, true, true><<<g, 256, 0, st>>>(m, sa);
    else
      k_main_screen<DPX, kScreenTile, kScreenNB, DT, true, false><<<g, 256, 0, st>>>(m, sa);
  } else {
    if (defer)
      k_main_screen<DPX, kScreenTile, kScreenNB, DT, false, true><<<g, 256, 0, st>>>(m, sa);
    else
      k_main_screen<DPX, kScreenTile, kScreenNB, DT, false, false><<<g, 256, 0, st>>>(m, sa);
  }
  MainArgs f = m;
  f.bpart = w.fbpart;
  constexpr int rows = kMainWaves * bf16_nb(DPX, 2, DT) * 32;
  const int64_t flb = ceil_div(m.N, rows);
  const unsigned fgrid = static_cast<unsigned>(flb < 512 ? flb : 512);
  k_main_fallback<DPX, DT><<<fgrid, 256, 0, st>>>(f, w.fblist, w.hdr);
  (void)launch_fb_sum(w, rows, st);
}

hipError_t launch_screen_main(const Problem& p, const WsLayout& L, const WsPtrs& w,
                              hipStream_t st) {
  MainArgs m;
  m.X = p.X;
  m.col_scale = p.col_scale;
  m.perm = w.perm;
  m.lsorted = w.lsorted;
  m.hdr = w.hdr;
  m.N = p.N;
  m.D = p.D;
  m.K = p.K;
  m.btab = w.btab;
  m.piece = static_cast<int64_t>(p.Kpad) * table_stride(p.DPX, p.dtype);
  m.ctab = w.ctab;
  m.atab = w.atab;
  m.avec = w.avec;
  m.ascale = w.ascale;
  m.mvec = w.mvec;
  m.ntiles = p.Kpad / kColTile;
  m.root = (p.flags & SIL_FLAG_EUCLID_APPROX) ? 1 : 0;
  m.s = p.s;
  m.bpart = w.bpart;
  m.save_a = nullptr;
  m.save_b = nullptr;
  m.save_n = nullptr;
  ScreenArgs sa;
  sa.stab = w.stab;
  sa.stab_bytes = static_cast<int64_t>(p.Kpad) * screen_stride(p.DPX) * 2;
  sa.hdr = w.hdr;
  sa.fblist = w.fblist;
  sa.rtab = w.rtab;
  int bits = 1;
  while ((1 << bits) < p.Kpad / 32) ++bits;
  sa.ibits = bits;
  with_depth(DepthsBf16{}, p.DPX, [&](auto dp) {
    constexpr int D_ = decltype(dp)::value;
    if constexpr (D_ <= kScreenMaxDPX) {
      if (p.dtype == SIL_FP8_E4M3)
        run_screen<D_, SIL_FP8_E4M3>(m, sa, L, w, st);
      else
        run_screen<D_, SIL_BF16>(m, sa, L, w, st);
    }
  });
  return hipGetLastError();
}

}  // namespace sil
