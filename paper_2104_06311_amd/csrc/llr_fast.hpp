// Fast MFMA kernel of the exact and max-log demappers (template shared by the two
// translation units that instantiate it).  See llr.hip for the method.
#pragma once

#include <cmath>
#include <cstdlib>

#include "common.hpp"

namespace md {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace fastk {

constexpr float kLn2 = 0.69314718055994530942f;

__device__ __forceinline__ half8 as_half8(uint4 v) {
  half8 h;
  __builtin_memcpy(&h, &v, 16);
  return h;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// One K step of the score contraction.  SC 0 and 1 hold FP16 operands; SC 2 holds BF16
// bits in the same 16-byte registers (the one-pass BF16 layout of prep.hip).
template <int SC>
__device__ __forceinline__ floatx16 score_mfma(half8 a, half8 b, floatx16 c) {
  if constexpr (SC == 2) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
}

// ------------------------------------------------------------------ fast kernel
// e = 2^(t + kExpBias): with t <= 0 (up to rounding) every partial sum stays below
// 2^(16 + 1 + kExpBias) < 2^128, and a subset only loses FP32 range (sum < 2^-96, the
// fallback trigger) when its best point is more than 196 base-2 units below -c||y||^2.
constexpr float kExpBias = 100.0f;

template <int MB>
struct Geo {
  static constexpr int LOG2G = MB - 5 < 3 ? MB - 5 : 3;   // tile-index bits handled inside a group
  static constexpr int G = 1 << LOG2G;
  static constexpr int NH = MB - 5 - LOG2G;               // tile-index bits routed through H0/H1
  static constexpr int NHA = NH > 0 ? NH : 1;
};

template <int MB>
struct SymAcc {
  float E[16], Tg[Geo<MB>::G], H0[Geo<MB>::NHA], H1[Geo<MB>::NHA], GT;
};

// Bytes of LDS used to assemble the symbol-side (B) operand of one 32-symbol block.
template <int KS>
constexpr int bstage_bytes() { return 32 * 16 * KS * 2; }

// Symbol (B) operand of the score contraction for the wavefront's symbol n (lane % 32):
// the row of K slots [ w_hi (D), w_hi (D), w_lo (D), a, a, r_hi, r_lo, 0 ... ] with
// w = (2c/a) y and r = (bias - c ||y||^2)/a is assembled in the wave's LDS staging row
// (lane half 0 writes), then every lane reads its 8-slot fragments.  Returns true when
// an operand leaves the FP16 split range (the symbol then takes the fallback path).
//
// SC 1 and 2 (one-pass FP16 or BF16 scores): the row is [ w (D), a, a, r_hi, r_lo, 0 ... ]
// with every slot rounded once to the operand format.
template <int SC>
__device__ __forceinline__ _Float16 op_round(float v) {
  if constexpr (SC == 2) return __builtin_bit_cast(_Float16, static_cast<__bf16>(v));
  else return static_cast<_Float16>(v);
}

template <int KS, int SC = 0>
__device__ __forceinline__ bool build_symbol_operand(_Float16* row, const float* __restrict__ y, int64_t n,
                                                     bool live, int D, float cb, float cn, float alpha,
                                                     float bias, half8 (&bf)[KS]) {
  constexpr int S = 16 * KS;
  constexpr int DMAX = SC == 0 ? (S - 4) / 3 : S - 4;   // 3 D + 4 (or D + 4) slots fit in KS steps
  const int h = (threadIdx.x & 63) >> 5;
  float ysq = 0.0f;
  bool bad = false;
  // all loads first, so that their latency is paid once per symbol, not once per dimension
  float yv[DMAX];
#pragma unroll
  for (int d = 0; d < DMAX; ++d) yv[d] = (live && d < D) ? y[n * D + d] : 0.0f;
#pragma unroll
  for (int d = 0; d < DMAX; ++d) {
    if (d >= D) break;
    const float yd = yv[d];
    ysq = fmaf(yd, yd, ysq);
    const float w = cb * yd;
    bad |= !(fabsf(w) <= 30000.0f);
    if constexpr (SC == 0) {
      const _Float16 hi = static_cast<_Float16>(w);
      const _Float16 lo = static_cast<_Float16>(w - static_cast<float>(hi));
      if (h == 0) {
        row[d] = hi;
        row[D + d] = hi;
        row[2 * D + d] = lo;
      }
    } else {
      if (h == 0) row[d] = op_round<SC>(w);
    }
  }
  const float r = bias / alpha - cn * ysq;
  bad |= !(fabsf(r) <= 30000.0f);
  const _Float16 rhi = op_round<SC>(r);
  const float rhi_f = SC == 2 ? static_cast<float>(__builtin_bit_cast(__bf16, rhi)) : static_cast<float>(rhi);
  const _Float16 rlo = op_round<SC>(r - rhi_f);
  if (h == 0) {
    const _Float16 a16 = op_round<SC>(alpha);
    const int nb = SC == 0 ? 3 * D : D;
    row[nb] = a16;
    row[nb + 1] = a16;
    row[nb + 2] = rhi;
    row[nb + 3] = rlo;
    for (int k = nb + 4; k < S; ++k) row[k] = static_cast<_Float16>(0.0f);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const uint4 v = *reinterpret_cast<const uint4*>(row + 16 * ks + 8 * h);
    __builtin_memcpy(&bf[ks], &v, 16);
  }
  return bad;
}

// Tiles are visited in groups of G = 2^LOG2G consecutive tiles so that the low LOG2G
// bits of the tile index (label bits 5 .. 4+LOG2G) are compile-time inside a group:
// their tile sums go to Tg[i]; only the group sum is routed by the remaining label
// bits into H0/H1.  Each wavefront carries SB blocks of 32 symbols and reads the A
// fragments of a tile once for all blocks.  The MFMAs of tile t+1 are issued before the
// exponentials of tile t (hard scheduling fences keep that order), so a wavefront's
// matrix work runs underneath its own VALU work.
template <int MB, int SB, bool MAXLOG>
__device__ __forceinline__ void acc_init(SymAcc<MB> (&ac)[SB]) {
  const float ident = MAXLOG ? -INFINITY : 0.0f;
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) ac[sb].E[rr] = ident;
#pragma unroll
    for (int i = 0; i < Geo<MB>::G; ++i) ac[sb].Tg[i] = ident;
#pragma unroll
    for (int q = 0; q < Geo<MB>::NHA; ++q) {
      ac[sb].H0[q] = ident;
      ac[sb].H1[q] = ident;
    }
  }
}

// Copies `total` uint4 (a multiple of 64: whole 1 KiB blocks) from global memory straight
// into LDS: wavefront w issues the direct loads (global_load_lds_dwordx4, 16 bytes per
// lane) of blocks w, w + NT/64, ... with a wave-uniform LDS base, and waits for them, so
// that the whole chunk is in flight at once without passing through registers.  The
// caller's barrier then publishes it to the block.
template <int NT>
__device__ __forceinline__ void stage_chunk_direct(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                   int total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int wave_u = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int nblk = total >> 6;
  for (int b = wave_u; b < nblk; b += NW)
    __builtin_amdgcn_global_load_lds(src + b * 64 + lane, dst + b * 64, 16, 0, 0);
  __builtin_amdgcn_s_waitcnt(0);
}

// Stages one fragment chunk: a constellation whose fragments all fit in LDS beside the NB
// staging bytes is copied once per block by the plain loop; larger ones are re-copied for
// every symbol group by direct global-to-LDS loads.  The choice is made at compile time, so
// that the resident kernels keep their register allocation.
template <int KS, int MB, int NB>
constexpr bool fragments_resident() {
  return (MB >= 5) && ((1 << MB) / 32) * KS * 1024 + NB <= 160 * 1024;
}

template <int KS, int MB, int NT, int NB>
__device__ __forceinline__ void copy_chunk(uint4* __restrict__ dst, const uint4* __restrict__ src, int total) {
  if constexpr (fragments_resident<KS, MB, NB>()) {
    for (int i = threadIdx.x; i < total; i += NT) dst[i] = src[i];
  } else {
    stage_chunk_direct<NT>(dst, src, total);
  }
}

// Accumulates the tiles [t0, t0 + tn) of one LDS-resident chunk (tile t of the chunk is at
// lds[t * KS * 64 ...]; tn is a multiple of G) into the SB symbol blocks' partial sums.
template <int KS, int MB, int SB, bool MAXLOG, int SC = 0>
__device__ __forceinline__ void tile_loop(const uint4* __restrict__ lds, int t0, int tn, int lane,
                                          const half8 (&bf)[SB][KS], SymAcc<MB> (&ac)[SB]) {
  constexpr int LOG2G = Geo<MB>::LOG2G;
  constexpr int G = Geo<MB>::G;
  constexpr int nh = Geo<MB>::NH;
  // prologue: score block of the chunk's first tile, and the fragments of the second
  floatx16 cur[SB];
  half8 ah[KS];
  {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) ah[ks] = as_half8(lds[ks * 64 + lane]);
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) cur[sb][rr] = 0.0f;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) cur[sb] = score_mfma<SC>(ah[ks], bf[sb][ks], cur[sb]);
    }
    const int t1 = min(1, tn - 1);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) ah[ks] = as_half8(lds[(t1 * KS + ks) * 64 + lane]);
  }
  for (int tg = 0; tg < tn; tg += G) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      // issue the next tile's score blocks (the chunk's last tile recomputes itself) and
      // the LDS reads of the tile after it, which then have a whole tile of VALU work
      // to arrive
      floatx16 nxt[SB];
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) nxt[sb][rr] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) nxt[sb] = score_mfma<SC>(ah[ks], bf[sb][ks], nxt[sb]);
      }
      // At the chunk's end this reads up to two tiles past it, into the symbol staging rows
      // that follow every fragment buffer in LDS (at least 2 KS KiB); those products are
      // never used.  Unclamped, the address is one base per group plus an immediate offset.
      const int tpre = tg + i + 2;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) ah[ks] = as_half8(lds[(tpre * KS + ks) * 64 + lane]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        SymAcc<MB>& A = ac[sb];
        float v[16];
        if (MAXLOG) {
#pragma unroll
          for (int rr = 0; rr < 16; ++rr) {
            v[rr] = cur[sb][rr];
            A.E[rr] = fmaxf(A.E[rr], v[rr]);
          }
#pragma unroll
          for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
            for (int rr = 0; rr < w; ++rr) v[rr] = fmaxf(v[rr], v[rr + w]);
          A.Tg[i] = fmaxf(A.Tg[i], v[0]);
          A.GT = (i == 0) ? v[0] : fmaxf(A.GT, v[0]);
        } else {
#pragma unroll
          for (int rr = 0; rr < 16; ++rr) {
            v[rr] = __builtin_amdgcn_exp2f(cur[sb][rr]);
            A.E[rr] += v[rr];
          }
#pragma unroll
          for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
            for (int rr = 0; rr < w; ++rr) v[rr] += v[rr + w];
          A.Tg[i] += v[0];
          A.GT = (i == 0) ? v[0] : A.GT + v[0];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) cur[sb] = nxt[sb];
    }
    // route the group sums by the label bits above the group
    const int grp = (t0 + tg) >> LOG2G;
#pragma unroll
    for (int q = 0; q < nh; ++q) {
      const bool bit = (grp >> q) & 1;
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        SymAcc<MB>& A = ac[sb];
        if (MAXLOG) {
          A.H1[q] = bit ? fmaxf(A.H1[q], A.GT) : A.H1[q];
          A.H0[q] = bit ? A.H0[q] : fmaxf(A.H0[q], A.GT);
        } else {
          // selects, not GT - a: in the wide-range pass a near group's GT may be +inf
          A.H1[q] += bit ? A.GT : 0.0f;
          A.H0[q] += bit ? 0.0f : A.GT;
        }
      }
    }
  }
}

// Label-0 / label-1 subset sums (or maxima) of every label bit from one symbol block's
// partial sums: bits 0..3 are positions inside the lane, bit 4 the lane half, bits
// 5..4+LOG2G the in-group tile sums, higher bits the routed group sums.  Every lane of
// the wavefront must call it (cross-half shuffles); the result is valid in lane half 0.
// With half_tile (M = 16) the lane half 1 holds no labels and is ignored.
template <int MB, bool MAXLOG>
__device__ __forceinline__ void combine_subsets(const SymAcc<MB>& A, bool half_tile, float (&S0)[MB],
                                                float (&S1)[MB]) {
  constexpr int LOG2G = Geo<MB>::LOG2G;
  constexpr int G = Geo<MB>::G;
  constexpr int NHMAX = Geo<MB>::NHA;
  const float ident = MAXLOG ? -INFINITY : 0.0f;
  auto comb = [](float a, float b) { return MAXLOG ? fmaxf(a, b) : a + b; };
  float L0[4 + LOG2G], L1[4 + LOG2G];
  // position bits 0..3 of the 16 position sums by a shared tree: pairs P, quads Q
  // (36 operations instead of 4 x 14)
  {
    const float* E = A.E;
    float P[8], Q[4];
#pragma unroll
    for (int j = 0; j < 8; ++j) P[j] = comb(E[2 * j], E[2 * j + 1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) Q[k] = comb(P[2 * k], P[2 * k + 1]);
    L0[0] = comb(comb(comb(E[0], E[2]), comb(E[4], E[6])), comb(comb(E[8], E[10]), comb(E[12], E[14])));
    L1[0] = comb(comb(comb(E[1], E[3]), comb(E[5], E[7])), comb(comb(E[9], E[11]), comb(E[13], E[15])));
    L0[1] = comb(comb(P[0], P[2]), comb(P[4], P[6]));
    L1[1] = comb(comb(P[1], P[3]), comb(P[5], P[7]));
    L0[2] = comb(Q[0], Q[2]);
    L1[2] = comb(Q[1], Q[3]);
    L0[3] = comb(Q[0], Q[1]);
    L1[3] = comb(Q[2], Q[3]);
  }
  if (LOG2G == 3) {
    // in-group tile bits by the same tree over the 8 tile sums
    const float* T = A.Tg;
    float p[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) p[j] = comb(T[2 * j], T[2 * j + 1]);
    L0[4] = comb(comb(T[0], T[2]), comb(T[4], T[6]));
    L1[4] = comb(comb(T[1], T[3]), comb(T[5], T[7]));
    L0[5] = comb(p[0], p[2]);
    L1[5] = comb(p[1], p[3]);
    L0[6] = comb(p[0], p[1]);
    L1[6] = comb(p[2], p[3]);
  } else {
#pragma unroll
    for (int b = 0; b < LOG2G; ++b) {
      float a0 = ident, a1 = ident;
#pragma unroll
      for (int i = 0; i < G; ++i) {
        if ((i >> b) & 1) a1 = comb(a1, A.Tg[i]);
        else a0 = comb(a0, A.Tg[i]);
      }
      L0[4 + b] = a0;
      L1[4 + b] = a1;
    }
  }
  const float Th = MAXLOG ? fmaxf(L0[0], L1[0]) : L0[0] + L1[0];
  float pL0[4 + LOG2G], pL1[4 + LOG2G], pH0[NHMAX], pH1[NHMAX];
#pragma unroll
  for (int b = 0; b < 4 + LOG2G; ++b) {
    pL0[b] = half_tile ? ident : __shfl_xor(L0[b], 32, 64);
    pL1[b] = half_tile ? ident : __shfl_xor(L1[b], 32, 64);
  }
  const float pTh = __shfl_xor(Th, 32, 64);
#pragma unroll
  for (int q = 0; q < NHMAX; ++q) {
    pH0[q] = __shfl_xor(A.H0[q], 32, 64);
    pH1[q] = __shfl_xor(A.H1[q], 32, 64);
  }
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    float a0, a1;
    if (b < 4) {
      a0 = MAXLOG ? fmaxf(L0[b], pL0[b]) : L0[b] + pL0[b];
      a1 = MAXLOG ? fmaxf(L1[b], pL1[b]) : L1[b] + pL1[b];
    } else if (b == 4) {
      a0 = Th;
      a1 = pTh;
    } else if (b < 5 + LOG2G) {
      a0 = MAXLOG ? fmaxf(L0[b - 1], pL0[b - 1]) : L0[b - 1] + pL0[b - 1];
      a1 = MAXLOG ? fmaxf(L1[b - 1], pL1[b - 1]) : L1[b - 1] + pL1[b - 1];
    } else {
      const int q = b - 5 - LOG2G;
      a0 = MAXLOG ? fmaxf(A.H0[q], pH0[q]) : A.H0[q] + pH0[q];
      a1 = MAXLOG ? fmaxf(A.H1[q], pH1[q]) : A.H1[q] + pH1[q];
    }
    S0[b] = a0;
    S1[b] = a1;
  }
}

// log2 of a positive normal float: the hardware logarithm alone.  Every caller has
// checked that its argument lies in [2^-96, 2^127], where log2f would add only the
// scaling of denormal arguments around the same instruction.
__device__ __forceinline__ float log2_normal(float x) { return __builtin_amdgcn_logf(x); }

// Whether the FP32 subset sums of a symbol kept their range (exact path).
template <int MB>
__device__ __forceinline__ bool sums_in_range(const float (&S0)[MB], const float (&S1)[MB]) {
  float smin = INFINITY, smax = 0.0f;
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    smin = fminf(smin, fminf(S0[b], S1[b]));
    smax = fmaxf(smax, fmaxf(S0[b], S1[b]));
  }
  return smin >= 0x1p-96f && smax <= 0x1p+126f;
}

template <int KS, int WAVES, int MB, int SB, bool MAXLOG, int SC = 0, bool GMI = false>
__global__ void __launch_bounds__(WAVES * 64) llr_fast_kernel(const uint4* __restrict__ frag, int ntiles,
                                                              int chunk_tiles, int D,
                                                              const float* __restrict__ y, int64_t N, float cb,
                                                              float cn, float alpha, float* __restrict__ llr,
                                                              int* __restrict__ flags,
                                                              unsigned* __restrict__ fb_list,
                                                              const uint32_t* __restrict__ gmi_tx,
                                                              const uint32_t* __restrict__ gmi_labels,
                                                              float* __restrict__ gmi_terms) {
  constexpr int m = MB;
  constexpr int S = 16 * KS;                 // K slots per symbol
  extern __shared__ uint4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const bool invalid = flags[0] != 0;
  const bool range_bad = flags[2] != 0;
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32 * SB;
  const int64_t ngroups = (N + per_group - 1) / per_group;
  const int nchunks = (ntiles + chunk_tiles - 1) / chunk_tiles;
  const int frag_per_tile = KS * 64;
  // per-wave staging rows for the B operand: after the fragment chunk, or, when the
  // fragments pass through LDS in several chunks, over the chunk buffer's start (the rows
  // are read once per group, before its first chunk is copied), so that the chunks can be
  // larger; the launcher sizes the buffer for either layout
  constexpr bool kMayOverlay = !fragments_resident<KS, MB, WAVES * SB * bstage_bytes<KS>()>();
  const bool overlay = kMayOverlay && nchunks > 1;
  _Float16* bst = reinterpret_cast<_Float16*>(overlay ? lds : lds + chunk_tiles * frag_per_tile) + wave * SB * 32 * S;
  bool staged = false;

  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    // overlaid rows: every wavefront has left the previous group's last chunk
    if (overlay) __syncthreads();
    half8 bf[SB][KS];
    SymAcc<MB> ac[SB];
    bool bad[SB];
    int64_t nsym[SB];
    uint32_t lab_sent[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t n = g * per_group + (static_cast<int64_t>(wave) * SB + sb) * 32 + (lane & 31);
      nsym[sb] = n;
      const bool b = build_symbol_operand<KS, SC>(bst + (sb * 32 + (lane & 31)) * S, y, n, n < N, D, cb, cn,
                                                  alpha, MAXLOG ? 0.0f : kExpBias, bf[sb]);
      bad[sb] = b || range_bad;
      if constexpr (GMI) {
        // the sent label, fetched now so that the tile loop hides the two dependent loads
        const uint32_t u = (h == 0 && n < N) ? gmi_tx[n] : 0u;
        const bool ok = u < (1u << MB);
        lab_sent[sb] = ok ? gmi_labels[u] : 0xFFFFFFFFu;   // all ones: an index outside the labels
      }
    }
    acc_init<MB, SB, MAXLOG>(ac);
    for (int ch = 0; ch < nchunks; ++ch) {
      const int t0 = ch * chunk_tiles;
      const int tn = min(chunk_tiles, ntiles - t0);     // a multiple of G
      if (nchunks > 1 || !staged) {
        __syncthreads();
        const int total = tn * frag_per_tile;
        const uint4* src = frag + static_cast<int64_t>(t0) * frag_per_tile;
        copy_chunk<KS, MB, WAVES * 64, WAVES * SB * bstage_bytes<KS>()>(lds, src, total);
        __syncthreads();
        staged = true;
      }
      tile_loop<KS, MB, SB, MAXLOG, SC>(lds, t0, tn, lane, bf, ac);
    }
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t n = nsym[sb];
      float S0[MB], S1[MB];
      combine_subsets<MB, MAXLOG>(ac[sb], false, S0, S1);
      const bool badp = __shfl_xor(static_cast<int>(bad[sb]), 32, 64) != 0;
      if (h == 0 && n < N) {
        if (invalid) {
          for (int k = 0; k < m; ++k) llr[n * m + k] = __builtin_nanf("");
          if constexpr (GMI) gmi_terms[n] = __builtin_nanf("");
        } else if (bad[sb] || badp || (!MAXLOG && !sums_in_range<MB>(S0, S1))) {
          const int idx = atomicAdd(&flags[1], 1);
          fb_list[idx] = static_cast<unsigned>(n);
          if constexpr (GMI) gmi_terms[n] = __builtin_nanf("");   // taken from its final LLRs later
        } else {
          float l2s0[MB], l2s1[MB];
#pragma unroll
          for (int k = 0; k < m; ++k) {
            const int b = m - 1 - k;
            if (!MAXLOG) {
              l2s0[b] = log2_normal(S0[b]);
              l2s1[b] = log2_normal(S1[b]);
            }
            llr[n * m + k] = MAXLOG ? kLn2 * (S0[b] - S1[b]) : kLn2 * (l2s0[b] - l2s1[b]);
          }
          if constexpr (GMI) {
            // GMI loss of the symbol, sum over bits of log2((S0 + S1) / S_sent); S0 + S1 is
            // the sum over all points for every bit, so one logarithm serves all of them
            const uint32_t lab = lab_sent[sb];
            const float l2tot = log2_normal(S0[0] + S1[0]);
            float T = lab != 0xFFFFFFFFu ? 0.0f : __builtin_nanf("");
#pragma unroll
            for (int b = 0; b < MB; ++b) T += l2tot - (((lab >> b) & 1u) ? l2s1[b] : l2s0[b]);
            gmi_terms[n] = T;
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ streamed fragments
// Constellations whose fragments exceed LDS (the 16D M = 65536 workload: 2048 tiles, 8 MiB
// at four K steps) stream them through two LDS buffers of C tiles.  Before the tile loop
// over one buffer the wavefronts issue the direct global-to-LDS loads
// (global_load_lds_dwordx4, 1 KiB per wavefront instruction) of the next chunk into the
// other, so that the loads' latency hides behind a whole chunk of work and each chunk costs
// one barrier instead of a synchronous copy between two.  The buffers are two distinct
// arrays, used in a fixed alternation (the chunk loop is unrolled by two), so that the
// compiler can tell the reads of one buffer from the loads into the other and does not make
// them wait for each other.  Each buffer carries two spare tiles for the tile loop's
// prefetch past a chunk's end.  After the last chunk of a symbol group the first chunk of
// the block's next group is already on its way.  Same arithmetic and epilogue as
// llr_fast_kernel (no fused GMI: that path needs one or two K steps).  Used for max-log.
constexpr int kStreamTiles = 8;

template <int KS, int WAVES, int MB, int SB, bool MAXLOG>
__global__ void __launch_bounds__(WAVES * 64) llr_stream_kernel(const uint4* __restrict__ frag, int ntiles,
                                                                int ctiles, int D,
                                                                const float* __restrict__ y, int64_t N, float cb,
                                                                float cn, float alpha, float* __restrict__ llr,
                                                                int* __restrict__ flags,
                                                                unsigned* __restrict__ fb_list) {
  constexpr int C = kStreamTiles;
  constexpr int FPT = KS * 64;                      // uint4 per tile
  constexpr int S = 16 * KS;                        // K slots per symbol
  __shared__ uint4 bufA[(C + 2) * FPT];
  __shared__ uint4 bufB[(C + 2) * FPT];
  __shared__ _Float16 stage[WAVES * SB * 32 * S];
  constexpr int m = MB;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const bool invalid = flags[0] != 0;
  const bool range_bad = flags[2] != 0;
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32 * SB;
  const int64_t ngroups = (N + per_group - 1) / per_group;
  const int nchunks = ntiles / C;                   // even (checked by the launcher)
  _Float16* bst = stage + wave * SB * 32 * S;
  // wavefront w loads the 1 KiB blocks w, w + WAVES, ... of a chunk's C KS blocks: a
  // wave-uniform base (scalar registers) plus the lane's 16 bytes, so that the loads need
  // no address registers of their own
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  auto issue = [&](int c, uint4* dst) {
    const uint4* src = frag + static_cast<int64_t>(c) * (C * FPT) + wave_u * 64;
    uint4* d = dst + wave_u * 64;
#pragma unroll
    for (int k = 0; k < (C * KS + WAVES - 1) / WAVES; ++k)
      if (wave_u + k * WAVES < C * KS)
        __builtin_amdgcn_global_load_lds(src + k * WAVES * 64 + lane, d + k * WAVES * 64, 16, 0, 0);
  };
  if (static_cast<int64_t>(blockIdx.x) < ngroups) {
    issue(0, bufA);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const bool next_group = g + gridDim.x < ngroups;
    half8 bf[SB][KS];
    SymAcc<MB> ac[SB];
    bool bad[SB];
    int64_t nsym[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t n = g * per_group + (static_cast<int64_t>(wave) * SB + sb) * 32 + (lane & 31);
      nsym[sb] = n;
      const bool b = build_symbol_operand<KS, 0>(bst + (sb * 32 + (lane & 31)) * S, y, n, n < N, D, cb, cn, alpha,
                                                 MAXLOG ? 0.0f : kExpBias, bf[sb]);
      bad[sb] = b || range_bad;
    }
    acc_init<MB, SB, MAXLOG>(ac);
    for (int c = 0; c < nchunks; c += 2) {
      // bufA holds chunk c; chunk c + 1 goes to bufB meanwhile
      issue(c + 1, bufB);
      // ctiles = C, passed at run time: a compile-time trip count lets the compiler unroll
      // the whole chunk and hoist every tile's products, which spills
      tile_loop<KS, MB, SB, MAXLOG, 0>(bufA, c * C, ctiles, lane, bf, ac);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // bufB holds chunk c + 1; chunk c + 2 (or the next group's first) goes to bufA
      if (c + 2 < nchunks || next_group) issue(c + 2 < nchunks ? c + 2 : 0, bufA);
      tile_loop<KS, MB, SB, MAXLOG, 0>(bufB, (c + 1) * C, ctiles, lane, bf, ac);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t n = nsym[sb];
      float S0[MB], S1[MB];
      combine_subsets<MB, MAXLOG>(ac[sb], false, S0, S1);
      const bool badp = __shfl_xor(static_cast<int>(bad[sb]), 32, 64) != 0;
      if (h == 0 && n < N) {
        if (invalid) {
          for (int k = 0; k < m; ++k) llr[n * m + k] = __builtin_nanf("");
        } else if (bad[sb] || badp || (!MAXLOG && !sums_in_range<MB>(S0, S1))) {
          const int idx = atomicAdd(&flags[1], 1);
          fb_list[idx] = static_cast<unsigned>(n);
        } else {
#pragma unroll
          for (int k = 0; k < m; ++k) {
            const int b = m - 1 - k;
            llr[n * m + k] = MAXLOG ? kLn2 * (S0[b] - S1[b]) : kLn2 * (log2_normal(S0[b]) - log2_normal(S1[b]));
          }
        }
      }
    }
  }
}

template <int KS, int WAVES, int MB, int SB, bool MAXLOG>
int launch_stream_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr, hipStream_t stream) {
  const int ntiles = M / 32;
  auto kern = llr_stream_kernel<KS, WAVES, MB, SB, MAXLOG>;
  int dev = 0, ncu = 0, occ = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), WAVES * 64, 0));
  if (occ < 1) occ = 1;
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32 * SB;
  const int64_t ngroups = (N + per_group - 1) / per_group;
  int64_t grid = static_cast<int64_t>(ncu) * occ;
  if (grid > ngroups) grid = ngroups;
  const double c = P.c_over_alpha * static_cast<double>(P.alpha);
  const float cb = static_cast<float>(2.0 * c / P.alpha);
  const float cn = P.c_over_alpha;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(WAVES * 64), 0, stream, P.frag, ntiles,
                     kStreamTiles, D, d_y, N, cb, cn, P.alpha, d_llr, P.flags, P.fb_list);
  MD_LAUNCH_CHECK("llr_stream_kernel launch");
  return MD_OK;
}

template <int KS, int WAVES, int MB, int SB, bool MAXLOG, int SC = 0, bool GMI = false>
int launch_fast_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                  hipStream_t stream) {
  const int ntiles = M / 32;
  const int frag_tile_bytes = KS * 64 * 16;
  const int bstage = WAVES * SB * bstage_bytes<KS>();
  const int max_lds = 160 * 1024 - bstage;
  int chunk_tiles = max_lds / frag_tile_bytes;
  constexpr int G = Geo<MB>::G;
  chunk_tiles -= chunk_tiles % G;
  if (chunk_tiles > ntiles) chunk_tiles = ntiles;
  if (chunk_tiles < G) return fail(MD_EUNSUPPORTED, "constellation fragments do not fit in LDS");
  size_t lds_bytes = static_cast<size_t>(chunk_tiles) * frag_tile_bytes + bstage;
  if constexpr (!fragments_resident<KS, MB, WAVES * SB * bstage_bytes<KS>()>()) {
    // several chunks: the staging rows go over the chunk buffer's start (see the kernel)
    // and the buffer keeps two spare tiles for the tile loop's prefetch past its end
    int ov = (160 * 1024) / frag_tile_bytes - 2;
    ov -= ov % G;
    if (chunk_tiles < ntiles && ov < ntiles && ov > chunk_tiles && ov * frag_tile_bytes >= bstage) {
      chunk_tiles = ov;
      lds_bytes = static_cast<size_t>(ov + 2) * frag_tile_bytes;
    }
  }
  if constexpr (KS == 4 && WAVES == 16 && SB == 1 && SC == 0 && !GMI && MAXLOG && MB >= 10) {
    // max-log with fragments beyond LDS: stream them through two buffers (an even number of
    // chunks) with twelve wavefronts per block.  The exact path keeps the synchronous
    // chunks: its tile loop needs all 128 registers of four wavefronts per SIMD, and the
    // three of the streamed kernel cost it more than the hidden copies gain
    if (chunk_tiles < ntiles && ntiles % (2 * kStreamTiles) == 0)
      return launch_stream_t<KS, 12, MB, SB, MAXLOG>(P, M, D, d_y, N, d_llr, stream);
  }
  auto kern = llr_fast_kernel<KS, WAVES, MB, SB, MAXLOG, SC, GMI>;
  {
    const int st_attr = set_lds_limit(reinterpret_cast<const void*>(kern), 160 * 1024);
    if (st_attr != MD_OK) return st_attr;
  }
  int dev = 0, ncu = 0, occ = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), WAVES * 64,
                                                           lds_bytes));
  if (occ < 1) occ = 1;
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32 * SB;
  const int64_t ngroups = (N + per_group - 1) / per_group;
  int64_t grid = static_cast<int64_t>(ncu) * occ;
  if (grid > ngroups) grid = ngroups;
  const double c = P.c_over_alpha * static_cast<double>(P.alpha);
  const float cb = static_cast<float>(2.0 * c / P.alpha);
  const float cn = P.c_over_alpha;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(WAVES * 64), lds_bytes, stream, P.frag, ntiles,
                     chunk_tiles, D, d_y, N, cb, cn, P.alpha, d_llr, P.flags, P.fb_list, P.gmi_tx, P.gmi_labels,
                     P.gmi_terms);
  MD_LAUNCH_CHECK("llr_fast_kernel launch");
  return MD_OK;
}

template <int KS, int W, int SBV, bool MAXLOG, int SC = 0, bool GMI = false>
int launch_fast_m(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                  hipStream_t stream) {
  switch (ilog2_pow2(M)) {
    case 5: return launch_fast_t<KS, W, 5, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 6: return launch_fast_t<KS, W, 6, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 7: return launch_fast_t<KS, W, 7, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 8: return launch_fast_t<KS, W, 8, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 9: return launch_fast_t<KS, W, 9, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 10: return launch_fast_t<KS, W, 10, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 11: return launch_fast_t<KS, W, 11, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 12: return launch_fast_t<KS, W, 12, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 13: return launch_fast_t<KS, W, 13, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 14: return launch_fast_t<KS, W, 14, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 15: return launch_fast_t<KS, W, 15, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
    default: return launch_fast_t<KS, W, 16, SBV, MAXLOG, SC, GMI>(P, M, D, d_y, N, sigma2, d_llr, stream);
  }
}

// ------------------------------------------------------------------ wide-range passes
// Later passes of the exact path over the symbols an earlier pass listed.  Every symbol is
// evaluated in NW exponent windows at once, e_w = 2^(t + kExpBias + w kWideShift) for
// w < NW (the NW symbol blocks of tile_loop carry the same symbols with the NW biases).
// Every partial sum holds points of one label subset only, so each subset sum is taken
// from the first window in which it kept its range: window w covers subsets whose best
// point lies less than 196 + w kWideShift units below the bias (and not so close to it
// that the window overflows).  The second pass uses two windows (best points down to
// 386 units), the third three (576 units).  Symbols with a subset in no window (or
// operands outside the FP16 split range) go on through list_out.
constexpr float kWideShift = 190.0f;

template <int KS, int WAVES, int MB, int NW>
__global__ void __launch_bounds__(WAVES * 64) llr_wide_kernel(const uint4* __restrict__ frag, int ntiles,
                                                              int chunk_tiles, int D,
                                                              const float* __restrict__ y, float cb, float cn,
                                                              float alpha, float* __restrict__ llr,
                                                              int* __restrict__ flags, int slot_in, int slot_out,
                                                              const unsigned* __restrict__ list_in,
                                                              unsigned* __restrict__ list_out) {
  constexpr int m = MB;
  constexpr int S = 16 * KS;
  extern __shared__ uint4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const bool range_bad = flags[2] != 0;
  const int64_t count = flags[slot_in];
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32;
  const int64_t ngroups = (count + per_group - 1) / per_group;
  const int nchunks = (ntiles + chunk_tiles - 1) / chunk_tiles;
  const int frag_per_tile = KS * 64;
  _Float16* bst = reinterpret_cast<_Float16*>(lds + chunk_tiles * frag_per_tile) + wave * NW * 32 * S;
  bool staged = false;

  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int64_t item = g * per_group + static_cast<int64_t>(wave) * 32 + (lane & 31);
    const bool live = item < count;
    const int64_t n = live ? static_cast<int64_t>(list_in[item]) : 0;
    half8 bf[NW][KS];
    SymAcc<MB> ac[NW];
    bool bad = range_bad;
#pragma unroll
    for (int w = 0; w < NW; ++w)
      bad |= build_symbol_operand<KS>(bst + (w * 32 + (lane & 31)) * S, y, n, live, D, cb, cn, alpha,
                                      kExpBias + w * kWideShift, bf[w]);
    acc_init<MB, NW, false>(ac);
    for (int ch = 0; ch < nchunks; ++ch) {
      const int t0 = ch * chunk_tiles;
      const int tn = min(chunk_tiles, ntiles - t0);
      if (nchunks > 1 || !staged) {
        __syncthreads();
        const int total = tn * frag_per_tile;
        const uint4* src = frag + static_cast<int64_t>(t0) * frag_per_tile;
        copy_chunk<KS, MB, WAVES * 64, WAVES * NW * bstage_bytes<KS>()>(lds, src, total);
        __syncthreads();
        staged = true;
      }
      tile_loop<KS, MB, NW, false>(lds, t0, tn, lane, bf, ac);
    }
    float S0[NW][MB], S1[NW][MB];
#pragma unroll
    for (int w = 0; w < NW; ++w) combine_subsets<MB, false>(ac[w], false, S0[w], S1[w]);
    const bool badp = __shfl_xor(static_cast<int>(bad), 32, 64) != 0;
    if (h == 0 && live) {
      float l2[2][MB];
      bool ok = !(bad || badp);
#pragma unroll
      for (int b = 0; b < MB; ++b) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          // the first window (in order) that kept the subset sum in range
          bool found = false;
          float val = 0.0f;
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            const float a = v ? S1[w][b] : S0[w][b];
            const bool in = a >= 0x1p-96f && a <= 0x1p+126f;
            val = (!found && in) ? log2_normal(a) - w * kWideShift : val;
            found = found || in;
          }
          ok = ok && found;
          l2[v][b] = val;
        }
      }
      if (!ok) {
        const int idx = atomicAdd(&flags[slot_out], 1);
        list_out[idx] = static_cast<unsigned>(n);
      } else {
#pragma unroll
        for (int k = 0; k < m; ++k) {
          const int b = m - 1 - k;
          llr[n * m + k] = kLn2 * (l2[0][b] - l2[1][b]);
        }
      }
    }
  }
}

template <int KS, int WAVES, int MB, int NW>
int launch_wide_t(const Prepared& P, int M, const float* d_y, int D, float* d_llr, int slot_in, int slot_out,
                  const unsigned* list_in, unsigned* list_out, hipStream_t stream) {
  const int ntiles = M / 32;
  const int frag_tile_bytes = KS * 64 * 16;
  const int bstage = WAVES * NW * bstage_bytes<KS>();
  int chunk_tiles = (160 * 1024 - bstage) / frag_tile_bytes;
  constexpr int G = Geo<MB>::G;
  chunk_tiles -= chunk_tiles % G;
  if (chunk_tiles > ntiles) chunk_tiles = ntiles;
  if (chunk_tiles < G) return fail(MD_EUNSUPPORTED, "constellation fragments do not fit in LDS");
  const size_t lds_bytes = static_cast<size_t>(chunk_tiles) * frag_tile_bytes + bstage;
  auto kern = llr_wide_kernel<KS, WAVES, MB, NW>;
  {
    const int st_attr = set_lds_limit(reinterpret_cast<const void*>(kern), 160 * 1024);
    if (st_attr != MD_OK) return st_attr;
  }
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // the list length is only known on the device: one block per CU, each loops until
  // the list is exhausted
  const double c = P.c_over_alpha * static_cast<double>(P.alpha);
  const float cb = static_cast<float>(2.0 * c / P.alpha);
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(ncu)), dim3(WAVES * 64), lds_bytes, stream, P.frag, ntiles,
                     chunk_tiles, D, d_y, cb, P.c_over_alpha, P.alpha, d_llr, P.flags, slot_in, slot_out, list_in,
                     list_out);
  MD_LAUNCH_CHECK("llr_wide_kernel launch");
  return MD_OK;
}

template <int KS, int NW>
int launch_wide_m(const Prepared& P, int M, const float* d_y, int D, float* d_llr, int slot_in, int slot_out,
                  const unsigned* list_in, unsigned* list_out, hipStream_t stream) {
  // three windows need about 1.5 times the accumulators of two: four wavefronts per block
  // (one per SIMD) leave each wavefront the whole register file, so that what does not fit
  // in the 256 architectural registers spills to accumulation registers, not to memory
  constexpr int WAVES = NW > 2 ? 4 : 8;
#define MD_WIDE_CASE(MB_)                                                                                   \
  case MB_:                                                                                                 \
    return launch_wide_t<KS, WAVES, MB_, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
  switch (ilog2_pow2(M)) {
    MD_WIDE_CASE(5) MD_WIDE_CASE(6) MD_WIDE_CASE(7) MD_WIDE_CASE(8) MD_WIDE_CASE(9) MD_WIDE_CASE(10)
    MD_WIDE_CASE(11) MD_WIDE_CASE(12) MD_WIDE_CASE(13) MD_WIDE_CASE(14) MD_WIDE_CASE(15)
    default: MD_WIDE_CASE(16)
  }
#undef MD_WIDE_CASE
}

// NW = 2: the second pass (list 1 -> list 2); NW = 3: the third pass (list 2 -> list 3).
template <int NW>
int launch_wide(const Prepared& P, int M, int D, const float* d_y, float* d_llr, int slot_in, int slot_out,
                const unsigned* list_in, unsigned* list_out, hipStream_t stream) {
  switch (P.ks) {
    case 1: return launch_wide_m<1, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
    case 2: return launch_wide_m<2, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
    case 3: return launch_wide_m<3, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
    case 4: return launch_wide_m<4, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
    case 5: return launch_wide_m<5, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
    default: return launch_wide_m<6, NW>(P, M, d_y, D, d_llr, slot_in, slot_out, list_in, list_out, stream);
  }
}

// Launch shapes of the fast kernel: (wavefronts per block, 32-symbol blocks per wavefront)
// = (16, 1) for one to four K steps: four wavefronts per SIMD at <= 128 registers, which
// hides latency better than (8, 2) (measured 6 % faster at 8D M = 2048); more K steps use
// (8, 1).
template <bool MAXLOG>
int launch_fast(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                hipStream_t stream) {
  switch (P.ks) {
    case 1: return launch_fast_m<1, 16, 1, MAXLOG>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 2: return launch_fast_m<2, 16, 1, MAXLOG>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 3: return launch_fast_m<3, 16, 1, MAXLOG>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 4: return launch_fast_m<4, 16, 1, MAXLOG>(P, M, D, d_y, N, sigma2, d_llr, stream);
    case 5: return launch_fast_m<5, 8, 1, MAXLOG>(P, M, D, d_y, N, sigma2, d_llr, stream);
    default: return launch_fast_m<6, 8, 1, MAXLOG>(P, M, D, d_y, N, sigma2, d_llr, stream);
  }
}

// Exact LLRs with the fused GMI epilogue (P.gmi_terms set): split scores with one or two
// K steps (D <= 9), or one-pass scores (D <= 12).
inline bool fused_gmi_supported(int sc, int ks) { return sc == 0 ? ks <= 2 : ks == 1; }

template <int UNUSED = 0>
int launch_fast_gmi(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                    hipStream_t stream) {
  if (!fused_gmi_supported(P.sc, P.ks)) return fail(MD_EUNSUPPORTED, "no fused GMI epilogue for this shape");
  if (P.sc == 1) return launch_fast_m<1, 16, 1, false, 1, true>(P, M, D, d_y, N, sigma2, d_llr, stream);
  if (P.sc == 2) return launch_fast_m<1, 16, 1, false, 2, true>(P, M, D, d_y, N, sigma2, d_llr, stream);
  if (P.ks == 1) return launch_fast_m<1, 16, 1, false, 0, true>(P, M, D, d_y, N, sigma2, d_llr, stream);
  return launch_fast_m<2, 16, 1, false, 0, true>(P, M, D, d_y, N, sigma2, d_llr, stream);
}

// One-pass FP16 (SC 1) or BF16 (SC 2) scores, exact LLRs: one K step (D <= 12).
template <int SC>
int launch_fast_lowp(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                     hipStream_t stream) {
  if (P.ks != 1 || P.sc != SC) return fail(MD_EUNSUPPORTED, "reduced-precision scores need D <= 12");
  return launch_fast_m<1, 16, 1, false, SC>(P, M, D, d_y, N, sigma2, d_llr, stream);
}


// ------------------------------------------------------------------ BF16 subset-sum kernel
// Same scores as llr_fast_kernel; the exponentials are rounded to BF16 and the 2m subset
// sums are a second MFMA contraction, e (32 points x 32 symbols) against the 0/1 matrix
// R (32 rows x 32 points): row b < 16 selects the points whose label has bit b set, row
// 16 + b those with bit b clear.  Two v_mfma_f32_32x32x16_bf16 per tile accumulate the
// sums in FP32 over all tiles, so each pair costs one exponential and half a conversion
// instruction on the VALU.  R's columns follow the B-operand layout of the exponentials:
// K slot k of reduction step q is the point at tile offset 16 (k / 8) + 8 q + k % 8.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One step t (0 <= t <= tn) of the BF16 kernel's tile pipeline: score MFMAs of tile t + 1
// into nx, reduction MFMAs of tile t - 1 (operands Ap/Bp), then the reduction operands of
// tile t from the scores in cu.  Step tn only drains the last reduction.
template <int KS, int SB>
__device__ __forceinline__ void bf16_step(const uint4* __restrict__ lds, int t, int t0, int tn, int lane,
                                          bool r_high, int rb, uint32_t want, const uint32_t (&lowA)[2][4],
                                          const half8 (&bf)[SB][KS], const floatx16 (&cu)[SB],
                                          floatx16 (&nx)[SB], half8 (&ah)[KS], bf16x8 (&Ap)[2],
                                          bf16x8 (&Bp)[SB][2], floatx16 (&R0)[SB], floatx16 (&R1)[SB]) {
  constexpr uint32_t kOne = 0x3F80u;   // BF16 1.0
  const bool more = t < tn;
  if (more) {
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) nx[sb][rr] = 0.0f;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        nx[sb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[ks], bf[sb][ks], nx[sb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
    R0[sb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ap[0], Bp[sb][0], R0[sb], 0, 0, 0);
    R1[sb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ap[1], Bp[sb][1], R1[sb], 0, 0, 0);
  }
  if (!more) return;
  const int tpre = min(t + 2, tn - 1);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) ah[ks] = as_half8(lds[(tpre * KS + ks) * 64 + lane]);
  __builtin_amdgcn_sched_barrier(0);
  // reduction matrix of this tile: the rows of the tile-index bits select all or none
  const uint32_t tau = static_cast<uint32_t>(t0 + t);
  const uint32_t hv = (r_high && (((tau >> (rb - 5)) & 1u) == want)) ? (kOne | (kOne << 16)) : 0u;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t wv[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) wv[w] = lowA[q][w] | hv;
    __builtin_memcpy(&Ap[q], wv, 16);
  }
#pragma unroll
  for (int sb = 0; sb < SB; ++sb)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 8; ++v) Bp[sb][q][v] = static_cast<__bf16>(__builtin_amdgcn_exp2f(cu[sb][8 * q + v]));
  __builtin_amdgcn_sched_barrier(0);
}

template <int KS, int WAVES, int MB, int SB>
__global__ void __launch_bounds__(WAVES * 64) llr_bf16_kernel(const uint4* __restrict__ frag, int ntiles,
                                                              int chunk_tiles, int D,
                                                              const float* __restrict__ y, int64_t N, float cb,
                                                              float cn, float alpha, float* __restrict__ llr,
                                                              int* __restrict__ flags,
                                                              unsigned* __restrict__ fb_list) {
  constexpr int m = MB;
  constexpr int S = 16 * KS;
  extern __shared__ uint4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const bool invalid = flags[0] != 0;
  const bool range_bad = flags[2] != 0;
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32 * SB;
  const int64_t ngroups = (N + per_group - 1) / per_group;
  const int nchunks = (ntiles + chunk_tiles - 1) / chunk_tiles;
  const int frag_per_tile = KS * 64;
  _Float16* bst = reinterpret_cast<_Float16*>(lds + chunk_tiles * frag_per_tile) + wave * SB * 32 * S;
  // this lane's row of R: label bit rb, selecting label bit value want
  const int rrow = lane & 31;
  const int rb = rrow & 15;
  const uint32_t want = rrow < 16 ? 1u : 0u;
  const bool r_low = rb < 5 && rb < m;       // decided by the offset inside the tile
  const bool r_high = rb >= 5 && rb < m;     // decided by the tile index
  constexpr uint32_t kOne = 0x3F80u;         // BF16 1.0
  uint32_t lowA[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t word = 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint32_t off = 16u * h + 8u * q + 2u * w + e;
        const bool sel = r_low && (((off >> rb) & 1u) == want);
        word |= (sel ? kOne : 0u) << (16 * e);
      }
      lowA[q][w] = word;
    }
  bool staged = false;

  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    half8 bf[SB][KS];
    floatx16 R0[SB], R1[SB];   // subset sums: two accumulators break the MFMA dependency chain
    bool bad[SB];
    int64_t nsym[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t n = g * per_group + (static_cast<int64_t>(wave) * SB + sb) * 32 + (lane & 31);
      nsym[sb] = n;
      const bool b = build_symbol_operand<KS>(bst + (sb * 32 + (lane & 31)) * S, y, n, n < N, D, cb, cn, alpha,
                                              kExpBias, bf[sb]);
      bad[sb] = b || range_bad;
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        R0[sb][rr] = 0.0f;
        R1[sb][rr] = 0.0f;
      }
    }

    for (int ch = 0; ch < nchunks; ++ch) {
      const int t0 = ch * chunk_tiles;
      const int tn = min(chunk_tiles, ntiles - t0);
      if (nchunks > 1 || !staged) {
        __syncthreads();
        const int total = tn * frag_per_tile;
        const uint4* src = frag + static_cast<int64_t>(t0) * frag_per_tile;
        copy_chunk<KS, MB, WAVES * 64, WAVES * SB * bstage_bytes<KS>()>(lds, src, total);
        __syncthreads();
        staged = true;
      }
      // Software pipeline over the tiles: in step t the score MFMAs of tile t + 1 and
      // the reduction MFMAs of tile t - 1 are issued first; the exponentials of tile t
      // then run on the VALU while the matrix pipe works through them.
      floatx16 cur[SB];
      bf16x8 Bp[SB][2];
      half8 ah[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) ah[ks] = as_half8(lds[ks * 64 + lane]);
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) cur[sb][rr] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          cur[sb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[ks], bf[sb][ks], cur[sb], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int v = 0; v < 8; ++v) Bp[sb][q][v] = static_cast<__bf16>(0.0f);
      }
      {
        const int t1 = min(1, tn - 1);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) ah[ks] = as_half8(lds[(t1 * KS + ks) * 64 + lane]);
      }
      bf16x8 Ap[2];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 8; ++v) Ap[q][v] = static_cast<__bf16>(0.0f);
      floatx16 nxt[SB];
      // two steps per iteration with the score registers swapping roles, so that no
      // register copies are needed between steps
      for (int t = 0;; t += 2) {
        bf16_step<KS, SB>(lds, t, t0, tn, lane, r_high, rb, want, lowA, bf, cur, nxt, ah, Ap, Bp, R0, R1);
        if (t == tn) break;
        bf16_step<KS, SB>(lds, t + 1, t0, tn, lane, r_high, rb, want, lowA, bf, nxt, cur, ah, Ap, Bp, R0, R1);
        if (t + 1 == tn) break;
      }
    }

#pragma unroll
    for (int sb = 0; sb < SB; ++sb) R0[sb] += R1[sb];

#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t n = nsym[sb];
      // lane half h holds result rows 8 (r / 4) + 4 h + r % 4; gather all 32 rows in half 0
      float P[16];
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) P[rr] = __shfl_xor(R0[sb][rr], 32, 64);
      const bool badp = __shfl_xor(static_cast<int>(bad[sb]), 32, 64) != 0;
      if (h == 0 && n < N) {
        if (invalid) {
          for (int k = 0; k < m; ++k) llr[n * m + k] = __builtin_nanf("");
        } else {
          float rowv[32];
#pragma unroll
          for (int rr = 0; rr < 16; ++rr) {
            rowv[8 * (rr / 4) + (rr % 4)] = R0[sb][rr];
            rowv[8 * (rr / 4) + 4 + (rr % 4)] = P[rr];
          }
          float smin = INFINITY, smax = 0.0f;
#pragma unroll
          for (int b = 0; b < m; ++b) {
            smin = fminf(smin, fminf(rowv[b], rowv[16 + b]));
            smax = fmaxf(smax, fmaxf(rowv[b], rowv[16 + b]));
          }
          const bool range_lost = !(smin >= 0x1p-96f && smax <= 0x1p+126f);
          if (bad[sb] || badp || range_lost) {
            const int idx = atomicAdd(&flags[1], 1);
            fb_list[idx] = static_cast<unsigned>(n);
          } else {
#pragma unroll
            for (int k = 0; k < m; ++k) {
              const int b = m - 1 - k;
              llr[n * m + k] = kLn2 * (log2_normal(rowv[16 + b]) - log2_normal(rowv[b]));
            }
          }
        }
      }
    }
  }
}

template <int KS, int WAVES, int MB, int SB>
int launch_bf16_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr, hipStream_t stream) {
  const int ntiles = M / 32;
  const int frag_tile_bytes = KS * 64 * 16;
  const int bstage = WAVES * SB * bstage_bytes<KS>();
  int chunk_tiles = (160 * 1024 - bstage) / frag_tile_bytes;
  if (chunk_tiles > ntiles) chunk_tiles = ntiles;
  if (chunk_tiles < 1) return fail(MD_EUNSUPPORTED, "constellation fragments do not fit in LDS");
  const size_t lds_bytes = static_cast<size_t>(chunk_tiles) * frag_tile_bytes + bstage;
  auto kern = llr_bf16_kernel<KS, WAVES, MB, SB>;
  {
    const int st_attr = set_lds_limit(reinterpret_cast<const void*>(kern), 160 * 1024);
    if (st_attr != MD_OK) return st_attr;
  }
  int dev = 0, ncu = 0, occ = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), WAVES * 64,
                                                           lds_bytes));
  if (occ < 1) occ = 1;
  const int64_t per_group = static_cast<int64_t>(WAVES) * 32 * SB;
  const int64_t ngroups = (N + per_group - 1) / per_group;
  int64_t grid = static_cast<int64_t>(ncu) * occ;
  if (grid > ngroups) grid = ngroups;
  const double c = P.c_over_alpha * static_cast<double>(P.alpha);
  const float cb = static_cast<float>(2.0 * c / P.alpha);
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(WAVES * 64), lds_bytes, stream, P.frag, ntiles,
                     chunk_tiles, D, d_y, N, cb, P.c_over_alpha, P.alpha, d_llr, P.flags, P.fb_list);
  MD_LAUNCH_CHECK("llr_bf16_kernel launch");
  return MD_OK;
}

template <int KS, int W, int SB>
int launch_bf16_m(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr, hipStream_t stream) {
  switch (ilog2_pow2(M)) {
    case 5: return launch_bf16_t<KS, W, 5, SB>(P, M, D, d_y, N, d_llr, stream);
    case 6: return launch_bf16_t<KS, W, 6, SB>(P, M, D, d_y, N, d_llr, stream);
    case 7: return launch_bf16_t<KS, W, 7, SB>(P, M, D, d_y, N, d_llr, stream);
    case 8: return launch_bf16_t<KS, W, 8, SB>(P, M, D, d_y, N, d_llr, stream);
    case 9: return launch_bf16_t<KS, W, 9, SB>(P, M, D, d_y, N, d_llr, stream);
    case 10: return launch_bf16_t<KS, W, 10, SB>(P, M, D, d_y, N, d_llr, stream);
    case 11: return launch_bf16_t<KS, W, 11, SB>(P, M, D, d_y, N, d_llr, stream);
    case 12: return launch_bf16_t<KS, W, 12, SB>(P, M, D, d_y, N, d_llr, stream);
    case 13: return launch_bf16_t<KS, W, 13, SB>(P, M, D, d_y, N, d_llr, stream);
    case 14: return launch_bf16_t<KS, W, 14, SB>(P, M, D, d_y, N, d_llr, stream);
    case 15: return launch_bf16_t<KS, W, 15, SB>(P, M, D, d_y, N, d_llr, stream);
    default: return launch_bf16_t<KS, W, 16, SB>(P, M, D, d_y, N, d_llr, stream);
  }
}

template <int UNUSED = 0>
int launch_bf16(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr, hipStream_t stream) {
  // (16 wavefronts, 1 block) would need more than the 128 registers it allows
  switch (P.ks) {
    case 1: return launch_bf16_m<1, 8, 2>(P, M, D, d_y, N, d_llr, stream);
    case 2: return launch_bf16_m<2, 8, 2>(P, M, D, d_y, N, d_llr, stream);
    case 3: return launch_bf16_m<3, 8, 1>(P, M, D, d_y, N, d_llr, stream);
    case 4: return launch_bf16_m<4, 8, 1>(P, M, D, d_y, N, d_llr, stream);
    case 5: return launch_bf16_m<5, 8, 1>(P, M, D, d_y, N, d_llr, stream);
    default: return launch_bf16_m<6, 8, 1>(P, M, D, d_y, N, d_llr, stream);
  }
}

}  // namespace fastk

}  // namespace md
