// Batched sweep: channel draw, exact LLRs and GMI for many constellations (uneven M and
// D) at many noise levels, in persistent kernels (one per constellation class) launched
// together from one captured hipGraph.
//
// A plan holds one "problem" per (instance, noise level): its label-ordered constellation,
// its MFMA fragments (which depend on the noise level through the score scales), the
// channel stream and N.  Each problem is cut into work items of a fixed number of
// symbol groups; items are grouped by class (K steps and label bits: one tile-loop shape,
// one kernel instantiation) and ordered by cost (M times K steps, largest first), and the
// blocks of a class's persistent kernel claim its items dynamically so that they finish
// together.  For every item a block draws
// the channel uses itself (the awgn_sample definition at offset = noise index * N), forms
// the scores and subset sums with the same tile loop as llr_exact, and adds the item's
// GMI loss sum_n sum_k log2(S_all / S_sent) to a per-item FP64 slot -- LLRs and
// received symbols never touch HBM.  Symbols whose subset sums leave FP32 range are
// queued with their received vector and label and re-evaluated in FP64 by a second kernel,
// which adds its losses as 2^-40 fixed-point integers (order independent).  A final kernel
// adds the item slots of each problem in a fixed order: the result is deterministic.
// The graph: reset -> one persistent kernel per class -> fallback -> final (no memset nodes).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "llr_fast.hpp"
#include "llr_kernels.hpp"
#include "rng.hpp"

namespace md {
namespace {

using fastk::Geo;
using fastk::SymAcc;

constexpr int kMaxKS = 2;          // D <= 8
constexpr int kFbCap = 1 << 20;    // fallback records per run
constexpr int kDynLds = 159 * 1024;  // dynamic LDS of the persistent kernel

struct Problem {
  const uint4* frag;
  const float* xl;         // label order
  const float* vx;         // per-point score terms (M = 32, 64: 2c x_j, -c ||x_j||^2), or null
  const float* X;          // index order (for the channel)
  const uint32_t* labels;  // label of each index
  int M, m, D, ks, ntiles, chunk_tiles;
  float cb, cn, alpha;
  double sigma;
  uint32_t k0, k1;
  uint64_t offset;
  int64_t N;
  int item_begin, item_end;
};

struct Item {
  int prob;
  int count;       // symbols in this item
  int64_t start;   // first symbol
};

struct FbRecord {
  int prob;
  uint32_t label;
  float y[8];
};

// Every symbol of a group: lane half h of wave w owns symbol (w * SB + h) * 32 + lane % 32
// of the group when SB = 2 (with SB = 1 only half 0 owns symbols).
// Writes the symbol's K-slot row (see prep.hip); returns true when an operand leaves the
// FP16 split range.
template <int KS>
__device__ __forceinline__ bool write_symbol_row(_Float16* row, const float (&yv)[8], int D, float cb, float cn,
                                                 float alpha, float bias) {
  constexpr int S = 16 * KS;
  float ysq = 0.0f;
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    if (d < D) {
      ysq = fmaf(yv[d], yv[d], ysq);
      const float w = cb * yv[d];
      bad |= !(fabsf(w) <= 30000.0f);
      const _Float16 hi = static_cast<_Float16>(w);
      const _Float16 lo = static_cast<_Float16>(w - static_cast<float>(hi));
      row[d] = hi;
      row[D + d] = hi;
      row[2 * D + d] = lo;
    }
  }
  const float r = bias / alpha - cn * ysq;
  bad |= !(fabsf(r) <= 30000.0f);
  const _Float16 rhi = static_cast<_Float16>(r);
  const _Float16 rlo = static_cast<_Float16>(r - static_cast<float>(rhi));
  const _Float16 a16 = static_cast<_Float16>(alpha);
  row[3 * D] = a16;
  row[3 * D + 1] = a16;
  row[3 * D + 2] = rhi;
  row[3 * D + 3] = rlo;
  for (int k = 3 * D + 4; k < S; ++k) row[k] = static_cast<_Float16>(0.0f);
  return bad;
}

// The channel use of symbol `local` of item I: its received vector (yv[d] for d < D, zeros
// after) and its point index.
__device__ __forceinline__ uint32_t draw_symbol(const Problem& P, const Item& I, int64_t local, float (&yv)[8]) {
  const uint64_t g = P.offset + static_cast<uint64_t>(I.start + local);
  switch (P.D) {      // compile-time D: the received vector stays in registers
    case 1: return rng::channel_symbol_d<1>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    case 2: return rng::channel_symbol_d<2>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    case 3: return rng::channel_symbol_d<3>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    case 4: return rng::channel_symbol_d<4>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    case 5: return rng::channel_symbol_d<5>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    case 6: return rng::channel_symbol_d<6>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    case 7: return rng::channel_symbol_d<7>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
    default: return rng::channel_symbol_d<8>(P.X, P.m, P.k0, P.k1, g, P.sigma, yv);
  }
}

// Queues a symbol for the FP64 fallback kernel.
__device__ __forceinline__ void queue_fallback(const Item& I, uint32_t lab, const float (&yv)[8],
                                               int* __restrict__ counters, FbRecord* __restrict__ fb) {
  const int idx = atomicAdd(&counters[1], 1);
  if (idx < kFbCap) {
    FbRecord& r = fb[idx];
    r.prob = I.prob;
    r.label = lab;
#pragma unroll
    for (int d = 0; d < 8; ++d) r.y[d] = yv[d];
  } else {
    atomicOr(&counters[2], 1);
  }
}

template <int WAVES, int SB, int KS, int MB>
__device__ void process_item(const Problem& P, const Item& I, int it, uint4* lds, int& staged_prob,
                             double* __restrict__ item_sum, FbRecord* __restrict__ fb, int* __restrict__ counters,
                             float* __restrict__ wsum) {
  constexpr int S = 16 * KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
  const int frag_per_tile = KS * 64;
  const int per_group = WAVES * 32 * SB;
  const int ngroups = (I.count + per_group - 1) / per_group;
  const int nchunks = (P.ntiles + P.chunk_tiles - 1) / P.chunk_tiles;
  _Float16* bst = reinterpret_cast<_Float16*>(lds + P.chunk_tiles * frag_per_tile) + wave * SB * 32 * S;
  const bool half_tile = P.M < 32;
  float acc_loss = 0.0f;
  // Channel draw.  SB = 2: lane half h draws symbol block h of every group.  SB = 1: both
  // halves draw every other group, half 0 the symbols of group gi and half 1 those of group
  // gi + 1, whose staging rows it writes once the operands of group gi are read; the
  // (label, live, out-of-range) state of a symbol stays with the half that drew it.
  uint32_t lab_own = 0;
  bool live_own = false, bad_own = false;
  for (int gi = 0; gi < ngroups; ++gi) {
    const bool draw_now = SB == 2 || (gi & 1) == 0;
    // the lane half that holds this group's symbols (SB = 1) or block sb's (SB = 2: half sb)
    const int cur_half = SB == 2 ? 0 : (gi & 1);
    float yv_own[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) yv_own[d] = 0.0f;
    if (draw_now) {
      const int64_t local = SB == 2 ? static_cast<int64_t>(gi) * per_group + (wave * SB + h) * 32 + (lane & 31)
                                    : static_cast<int64_t>(gi + h) * per_group + wave * 32 + (lane & 31);
      live_own = local < I.count;
      lab_own = 0;
      if (live_own) lab_own = P.labels[draw_symbol(P, I, local, yv_own)];
      if (SB == 2 || h == 0) {
        _Float16* row = bst + ((SB == 2 ? h : 0) * 32 + (lane & 31)) * S;
        bad_own = write_symbol_row<KS>(row, yv_own, P.D, P.cb, P.cn, P.alpha, fastk::kExpBias);
        // operands outside the FP16 split range: straight to the FP64 fallback
        if (live_own && bad_own) queue_fallback(I, lab_own, yv_own, counters, fb);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    half8 bf[SB][KS];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const uint4 v = *reinterpret_cast<const uint4*>(bst + (sb * 32 + (lane & 31)) * S + 16 * ks + 8 * h);
        __builtin_memcpy(&bf[sb][ks], &v, 16);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if constexpr (SB == 1) {
      // the rows are consumed: half 1 stages the next group's symbols in them
      if (draw_now && h == 1) {
        _Float16* row = bst + (lane & 31) * S;
        bad_own = write_symbol_row<KS>(row, yv_own, P.D, P.cb, P.cn, P.alpha, fastk::kExpBias);
        if (live_own && bad_own) queue_fallback(I, lab_own, yv_own, counters, fb);
      }
    } else {
      // the owners park their received vectors there (8 floats <= 32 KS bytes) for the
      // rare symbol that needs the FP64 fallback after the tile loop
      float* yrow = reinterpret_cast<float*>(bst + (h * 32 + (lane & 31)) * S);
#pragma unroll
      for (int d = 0; d < 8; ++d) yrow[d] = yv_own[d];
    }
    SymAcc<MB> ac[SB];
    fastk::acc_init<MB, SB, false>(ac);
    for (int ch = 0; ch < nchunks; ++ch) {
      const int t0 = ch * P.chunk_tiles;
      const int tn = min(P.chunk_tiles, P.ntiles - t0);
      if (nchunks > 1 || staged_prob != I.prob) {
        __syncthreads();
        const int total = tn * frag_per_tile;
        const uint4* src = P.frag + static_cast<int64_t>(t0) * frag_per_tile;
        fastk::stage_chunk_direct<WAVES * 64>(lds, src, total);
        __syncthreads();
        staged_prob = (nchunks > 1) ? -1 : I.prob;
      }
      fastk::tile_loop<KS, MB, SB, false>(lds, t0, tn, lane, bf, ac);
    }
    // ---- GMI loss of every symbol: sum_k log2(S0_k + S1_k) - log2(S_sent,k)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      float S0[MB], S1[MB];
      fastk::combine_subsets<MB, false>(ac[sb], half_tile, S0, S1);
      // the owner of block sb is lane half sb (SB = 2) or the half that drew the group (SB = 1)
      const int src = 32 * (SB == 2 ? sb : cur_half);
      const uint32_t lab = __shfl(lab_own, src + (lane & 31), 64);
      const bool live = __shfl(static_cast<int>(live_own), src + (lane & 31), 64) != 0;
      const bool bad = __shfl(static_cast<int>(bad_own), src + (lane & 31), 64) != 0;
      if (h == 0 && live && !bad) {
        const int m = P.m;
        float smin = INFINITY, smax = 0.0f;
#pragma unroll
        for (int b = 0; b < MB; ++b)
          if (b < m) {
            smin = fminf(smin, fminf(S0[b], S1[b]));
            smax = fmaxf(smax, fmaxf(S0[b], S1[b]));
          }
        if (smin >= 0x1p-96f && smax <= 0x1p+126f) {
          // S0 + S1 is the sum over all points for every bit: one logarithm serves all
          const float l2tot = fastk::log2_normal(S0[0] + S1[0]);
          float T = 0.0f;
#pragma unroll
          for (int b = 0; b < MB; ++b)
            if (b < m) {
              const float sent = ((lab >> b) & 1u) ? S1[b] : S0[b];
              T += l2tot - fastk::log2_normal(sent);
            }
          acc_loss += T;
        } else {
          float yv[8];
#pragma unroll
          for (int d = 0; d < 8; ++d) yv[d] = 0.0f;
          if constexpr (SB == 2) {
            // the owner parked the received vector in the symbol's staging row
            const float* yrow = reinterpret_cast<const float*>(bst + (sb * 32 + (lane & 31)) * S);
#pragma unroll
            for (int d = 0; d < 8; ++d) yv[d] = yrow[d];
          } else {
            // the rows hold the next group's operands: draw the channel use again
            (void)draw_symbol(P, I, static_cast<int64_t>(gi) * per_group + wave * 32 + (lane & 31), yv);
          }
          queue_fallback(I, lab, yv, counters, fb);
        }
      }
    }
  }
  // ---- item sum: wave sums, then the block's waves in a fixed order
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc_loss += __shfl_xor(acc_loss, o, 64);
  __syncthreads();
  if (lane == 0) wsum[wave] = acc_loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < WAVES; ++w) s += static_cast<double>(wsum[w]);
    item_sum[it] = s;
  }
}

// One persistent kernel per class (K steps, label bits) of the plan: it claims the
// class's items [item_begin, item_end) through its own counter, so every instantiation
// carries the registers of one tile-loop shape only.
template <int WAVES, int SB, int KS, int MBK>
__global__ void __launch_bounds__(WAVES * 64) sweep_kernel(const Problem* __restrict__ probs,
                                                           const Item* __restrict__ items, int item_begin,
                                                           int item_end, int* __restrict__ claim,
                                                           int* __restrict__ counters, double* __restrict__ item_sum,
                                                           FbRecord* __restrict__ fb) {
  extern __shared__ uint4 lds[];
  __shared__ int next;
  __shared__ float wsum[WAVES];
  int staged_prob = -1;
  for (;;) {
    if (threadIdx.x == 0) next = item_begin + atomicAdd(claim, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next);     // uniform: scalar loads below
    __syncthreads();
    if (it >= item_end) break;
    const Item I = items[it];
    const Problem P = probs[I.prob];
    process_item<WAVES, SB, KS, MBK>(P, I, it, lds, staged_prob, item_sum, fb, counters, wsum);
  }
}

// ------------------------------------------------------------------ small constellations
// For M <= 64 the matrix-core path spends most of its time around the tile loop (operand
// staging, subset combine, and for M = 16 half of every 32-point tile is padding).  The
// vector path gives each thread whole symbols: the channel draw, all M squared distances
// ||y - x_j||^2 from differences (the constellation's label-order copy is read at uniform
// addresses, so through the scalar cache), one exponential per point with the same fixed
// bias as the tile loop, e_j = 2^(kExpBias - c ||y - x_j||^2), and the 2m subset sums by
// one pass per label bit over block sums (about 2.3 adds per point).  Range check, FP64
// fallback queue and loss term are those of the matrix-core kernel.
constexpr int kSmallThreads = 256;

template <int MB, int D>
__device__ __forceinline__ float small_item(const Problem& P, const Item& I, int lane, int* __restrict__ counters,
                                            FbRecord* __restrict__ fb) {
  constexpr int M = 1 << MB;
  const float cexp = static_cast<float>(static_cast<double>(P.cn) * static_cast<double>(P.alpha));
  // the label-order points, read-only during the kernel and at uniform addresses: through the
  // constant address space, so that they arrive by scalar loads into scalar registers
  typedef const __attribute__((address_space(4))) float ConstFloat;
  ConstFloat* xl = (ConstFloat*)P.xl;
  // M = 32 and 64: the score from the per-point terms, sum_d y_d (2c x_jd) - c ||x_j||^2 +
  // (bias - c ||y||^2), D + 1 operations per point as in llr_exact's one-thread-per-symbol
  // kernel; M = 16 from the differences y - x_j
  constexpr bool kTerms = MB == 5 || MB == 6;
  float acc = 0.0f;
  for (int local = lane; local < I.count; local += 64) {
    const uint64_t g = P.offset + static_cast<uint64_t>(I.start + local);
    float yv[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) yv[d] = 0.0f;
    const uint32_t u = rng::channel_symbol_d<D>(P.X, MB, P.k0, P.k1, g, P.sigma, yv);
    const uint32_t lab = P.labels[u];
    float v[M];
    if constexpr (kTerms) {
      // the table's address passes through an empty asm statement on every symbol, so that
      // its M (D + 1) terms are loaded as they are used rather than all hoisted
      uint64_t vaddr = reinterpret_cast<uint64_t>(P.vx);
      asm volatile("" : "+s"(vaddr));
      ConstFloat* vx = reinterpret_cast<ConstFloat*>(vaddr);
      float ysq = 0.0f;
#pragma unroll
      for (int d = 0; d < D; ++d) ysq = fmaf(yv[d], yv[d], ysq);
      const float r = fmaf(-cexp, ysq, fastk::kExpBias);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        float t = vx[j * (D + 1) + D] + r;
#pragma unroll
        for (int d = 0; d < D; ++d) t = fmaf(yv[d], vx[j * (D + 1) + d], t);
        v[j] = __builtin_amdgcn_exp2f(t);
      }
    } else {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        float d2 = 0.0f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const float df = yv[d] - xl[j * D + d];
          d2 = fmaf(df, df, d2);
        }
        v[j] = __builtin_amdgcn_exp2f(fmaf(-cexp, d2, fastk::kExpBias));
      }
    }
    // level b: v[k] is the sum over the 2^b consecutive labels of block k, so bit b of a
    // label is the parity of its block index
    float S0[MB], S1[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int n = M >> b;
      float a0 = v[0], a1 = v[1];
#pragma unroll
      for (int k = 2; k < n; k += 2) {
        a0 += v[k];
        a1 += v[k + 1];
      }
      S0[b] = a0;
      S1[b] = a1;
#pragma unroll
      for (int k = 0; k < n / 2; ++k) v[k] = v[2 * k] + v[2 * k + 1];
    }
    float smin = INFINITY, smax = 0.0f;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      smin = fminf(smin, fminf(S0[b], S1[b]));
      smax = fmaxf(smax, fmaxf(S0[b], S1[b]));
    }
    if (smin >= 0x1p-96f && smax <= 0x1p+126f) {
      const float l2tot = fastk::log2_normal(S0[0] + S1[0]);
      float T = 0.0f;
#pragma unroll
      for (int b = 0; b < MB; ++b) T += l2tot - fastk::log2_normal(((lab >> b) & 1u) ? S1[b] : S0[b]);
      acc += T;
    } else {
      const int idx = atomicAdd(&counters[1], 1);
      if (idx < kFbCap) {
        FbRecord& r = fb[idx];
        r.prob = I.prob;
        r.label = lab;
#pragma unroll
        for (int d = 0; d < 8; ++d) r.y[d] = yv[d];
      } else {
        atomicOr(&counters[2], 1);
      }
    }
  }
  return acc;
}

// Every wavefront claims work items on its own: no LDS, no block barriers, and no branch
// on the lane index around the claim (all lanes take part in one atomic that only lane 0
// increments, and all lanes store the item's sum).
template <int MB>
__global__ void __launch_bounds__(kSmallThreads) sweep_small_kernel(const Problem* __restrict__ probs,
                                                                    const Item* __restrict__ items, int item_begin,
                                                                    int item_end, int* __restrict__ claim,
                                                                    int* __restrict__ counters,
                                                                    double* __restrict__ item_sum,
                                                                    FbRecord* __restrict__ fb) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int c = atomicAdd(claim, lane == 0 ? 1 : 0);
    const int it = item_begin + __builtin_amdgcn_readfirstlane(c);
    if (it >= item_end) break;
    const Item I = items[it];
    const Problem P = probs[I.prob];
    float acc = 0.0f;
    switch (P.D) {
      case 1: acc = small_item<MB, 1>(P, I, lane, counters, fb); break;
      case 2: acc = small_item<MB, 2>(P, I, lane, counters, fb); break;
      case 3: acc = small_item<MB, 3>(P, I, lane, counters, fb); break;
      case 4: acc = small_item<MB, 4>(P, I, lane, counters, fb); break;
      case 5: acc = small_item<MB, 5>(P, I, lane, counters, fb); break;
      case 6: acc = small_item<MB, 6>(P, I, lane, counters, fb); break;
      case 7: acc = small_item<MB, 7>(P, I, lane, counters, fb); break;
      default: acc = small_item<MB, 8>(P, I, lane, counters, fb); break;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    item_sum[it] = static_cast<double>(acc);
  }
}

// Re-evaluates queued symbols in FP64 (one wavefront per record): per-subset maxima and
// log-sum-exp, then the loss sum_k log2(1 + e^{L_other - L_sent}) added to the problem's
// fixed-point accumulator.
__global__ void __launch_bounds__(256) sweep_fallback_kernel(const Problem* __restrict__ probs,
                                                             const FbRecord* __restrict__ fb,
                                                             const int* __restrict__ counters,
                                                             unsigned long long* __restrict__ fb_acc) {
  const int lane = threadIdx.x & 63;
  const int64_t wave_id = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  const int64_t count = min(counters[1], kFbCap);
  for (int64_t r = wave_id; r < count; r += nwaves) {
    const FbRecord R = fb[r];
    const Problem P = probs[R.prob];
    const double cnat = static_cast<double>(P.cn) * static_cast<double>(P.alpha) / 1.4426950408889634;
    double mx0[16], mx1[16];
    for (int k = 0; k < 16; ++k) {
      mx0[k] = -INFINITY;
      mx1[k] = -INFINITY;
    }
    for (int j = lane; j < P.M; j += 64) {
      double d2 = 0.0;
      for (int d = 0; d < P.D; ++d) {
        const double df = static_cast<double>(R.y[d]) - static_cast<double>(P.xl[static_cast<int64_t>(j) * P.D + d]);
        d2 = fma(df, df, d2);
      }
      const double q = -cnat * d2;
      for (int b = 0; b < P.m; ++b) {
        if ((j >> b) & 1) mx1[b] = fmax(mx1[b], q);
        else mx0[b] = fmax(mx0[b], q);
      }
    }
    for (int b = 0; b < P.m; ++b)
      for (int o = 32; o >= 1; o >>= 1) {
        mx0[b] = fmax(mx0[b], __shfl_xor(mx0[b], o, 64));
        mx1[b] = fmax(mx1[b], __shfl_xor(mx1[b], o, 64));
      }
    double s0[16], s1[16];
    for (int k = 0; k < 16; ++k) {
      s0[k] = 0.0;
      s1[k] = 0.0;
    }
    for (int j = lane; j < P.M; j += 64) {
      double d2 = 0.0;
      for (int d = 0; d < P.D; ++d) {
        const double df = static_cast<double>(R.y[d]) - static_cast<double>(P.xl[static_cast<int64_t>(j) * P.D + d]);
        d2 = fma(df, df, d2);
      }
      const double q = -cnat * d2;
      for (int b = 0; b < P.m; ++b) {
        if ((j >> b) & 1) s1[b] += exp(q - mx1[b]);
        else s0[b] += exp(q - mx0[b]);
      }
    }
    double T = 0.0;
    for (int b = 0; b < P.m; ++b) {
      double a0 = s0[b], a1 = s1[b];
      for (int o = 32; o >= 1; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
      }
      const double l0 = mx0[b] + log(a0), l1 = mx1[b] + log(a1);
      const bool one = (R.label >> b) & 1u;
      const double diff = one ? l0 - l1 : l1 - l0;          // other minus sent
      T += (fmax(diff, 0.0) + log1p(exp(-fabs(diff)))) / 0.69314718055994530942;
    }
    if (lane == 0) atomicAdd(&fb_acc[R.prob], static_cast<unsigned long long>(llround(T * 1099511627776.0)));
  }
}

__global__ void sweep_reset_kernel(int* __restrict__ counters, int ncounters, unsigned long long* __restrict__ fb_acc,
                                   int nprob) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncounters) counters[i] = 0;
  if (i < nprob) fb_acc[i] = 0ull;
}

__global__ void sweep_final_kernel(const Problem* __restrict__ probs, int nprob, const double* __restrict__ item_sum,
                                   const unsigned long long* __restrict__ fb_acc, const int* __restrict__ counters,
                                   double* __restrict__ gmi) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const Problem P = probs[p];
  double s = 0.0;
  for (int i = P.item_begin; i < P.item_end; ++i) s += item_sum[i];
  s += static_cast<double>(fb_acc[p]) * (1.0 / 1099511627776.0);
  const bool overflow = counters[2] != 0;
  gmi[p] = overflow ? __builtin_nan("") : static_cast<double>(P.m) - s / static_cast<double>(P.N);
}

}  // namespace

// ------------------------------------------------------------------ plan
struct SweepPlan {
  int n_inst = 0, n_snr = 0, nprob = 0, n_items = 0;
  int waves = 8, sb = 2, gpi = 1;
  int device = 0;
  std::vector<void*> allocs;
  Problem* d_probs = nullptr;
  Item* d_items = nullptr;
  int* d_counters = nullptr;
  double* d_item_sum = nullptr;
  FbRecord* d_fb = nullptr;
  unsigned long long* d_fb_acc = nullptr;
  double* d_gmi = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<Problem> h_probs;
  std::vector<int*> h_flags;
  size_t lds_bytes = 0;
  // classes of problems with one tile-loop shape: (K steps, label bits), their item ranges
  // and their launch shape (an index into kShapes)
  struct Class {
    int ks, m, begin, end, v;
    size_t lds;   // dynamic LDS of the class kernel: its largest fragment chunk + staging rows
  };
  std::vector<Class> classes;
  std::map<std::pair<int, int>, int> class_var;   // (K steps, label bits) -> launch shape
  std::map<std::pair<int, int>, int> tuned;       // the autotuner's choices for this plan
  std::map<std::pair<int, int>, float> tuned_ms;  // and the class kernel times they gave
};

// Launch shapes: wavefronts per block, 32-symbol blocks per wavefront, symbol groups per
// work item.  Shape 4 is the vector kernel of the small classes (M <= 64): blocks of four
// wavefronts, each claiming work items of 512 symbols on its own.
struct Shape {
  int waves, sb, gpi;
};
constexpr int kNumShapes = 5;
constexpr int kValuShape = 4;
constexpr int kValuMaxBits = 6;
constexpr Shape kShapes[kNumShapes] = {{8, 2, 1}, {8, 2, 4}, {16, 1, 1}, {16, 1, 4}, {4, 1, 4}};

// The shape a class of label bits m gets under plan variant v: the vector kernel only for
// small constellations (shape 0 elsewhere).
inline int class_shape(int v, int m) { return (v == kValuShape && m > kValuMaxBits) ? 0 : v; }

// Autotuner choices, per device and constellation class (K steps, label bits): measured
// once per process, reused by every later plan with the same classes.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;

constexpr int kCounterBase = 4;    // counters[0..3]: unused, fallback count, overflow, unused

namespace {

int dev_alloc(SweepPlan* p, size_t bytes, void** out) {
  void* q = nullptr;
  if (dev_malloc(&q, bytes > 0 ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MD_ENOMEM, "sweep plan allocation failed");
  }
  p->allocs.push_back(q);
  *out = q;
  return MD_OK;
}

void free_plan(SweepPlan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (void* q : p->allocs) (void)md::dev_free(q);
  delete p;
}

template <int WAVES, int SB, int KS, int MBK>
int launch_class(SweepPlan* p, const SweepPlan::Class& c, int ci, hipStream_t s) {
  auto kern = sweep_kernel<WAVES, SB, KS, MBK>;
  {
    const int st_attr = set_lds_limit(reinterpret_cast<const void*>(kern), kDynLds);
    if (st_attr != MD_OK) return st_attr;
  }
  int ncu = 0, occ = 0;
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  MD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), WAVES * 64,
                                                           c.lds));
  if (occ < 1) occ = 1;
  int64_t grid = static_cast<int64_t>(ncu) * occ;
  if (grid > c.end - c.begin) grid = c.end - c.begin;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(WAVES * 64), c.lds, s, p->d_probs,
                     p->d_items, c.begin, c.end, p->d_counters + kCounterBase + ci, p->d_counters, p->d_item_sum,
                     p->d_fb);
  MD_LAUNCH_CHECK("sweep_kernel launch");
  return MD_OK;
}

template <int WAVES, int SB>
int launch_class_shape(SweepPlan* p, const SweepPlan::Class& c, int ci, hipStream_t s) {
  const int key = (c.ks - 1) * 16 + c.m;
  switch (key) {
#define MD_SWEEP_CASE(KS_, MB_, MBK_) \
  case (KS_ - 1) * 16 + MB_:        \
    return launch_class<WAVES, SB, KS_, MBK_>(p, c, ci, s);
    MD_SWEEP_CASE(1, 4, 5) MD_SWEEP_CASE(1, 5, 5) MD_SWEEP_CASE(1, 6, 6) MD_SWEEP_CASE(1, 7, 7)
    MD_SWEEP_CASE(1, 8, 8) MD_SWEEP_CASE(1, 9, 9) MD_SWEEP_CASE(1, 10, 10) MD_SWEEP_CASE(1, 11, 11)
    MD_SWEEP_CASE(1, 12, 12) MD_SWEEP_CASE(1, 13, 13)
    MD_SWEEP_CASE(2, 4, 5) MD_SWEEP_CASE(2, 5, 5) MD_SWEEP_CASE(2, 6, 6) MD_SWEEP_CASE(2, 7, 7)
    MD_SWEEP_CASE(2, 8, 8) MD_SWEEP_CASE(2, 9, 9) MD_SWEEP_CASE(2, 10, 10) MD_SWEEP_CASE(2, 11, 11)
    MD_SWEEP_CASE(2, 12, 12) MD_SWEEP_CASE(2, 13, 13)
#undef MD_SWEEP_CASE
    default:
      return fail(MD_EUNSUPPORTED, "no sweep kernel for this constellation class");
  }
}

template <int MB>
int launch_small_class(SweepPlan* p, const SweepPlan::Class& c, int ci, hipStream_t s) {
  auto kern = sweep_small_kernel<MB>;
  int ncu = 0, occ = 0;
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  MD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), kSmallThreads,
                                                           0));
  if (occ < 1) occ = 1;
  int64_t grid = static_cast<int64_t>(ncu) * occ;
  if (grid > c.end - c.begin) grid = c.end - c.begin;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(kSmallThreads), 0, s, p->d_probs, p->d_items,
                     c.begin, c.end, p->d_counters + kCounterBase + ci, p->d_counters, p->d_item_sum, p->d_fb);
  MD_LAUNCH_CHECK("sweep_small_kernel launch");
  return MD_OK;
}

int launch_small(SweepPlan* p, const SweepPlan::Class& c, int ci, hipStream_t s) {
  switch (c.m) {
    case 4: return launch_small_class<4>(p, c, ci, s);
    case 5: return launch_small_class<5>(p, c, ci, s);
    case 6: return launch_small_class<6>(p, c, ci, s);
    default: return fail(MD_EUNSUPPORTED, "no vector sweep kernel for this constellation class");
  }
}

// ev: NULL, or two events per class recorded around that class's kernel (autotuning).
int enqueue(SweepPlan* p, hipStream_t s, const std::vector<hipEvent_t>* ev = nullptr) {
  const int ncounters = kCounterBase + static_cast<int>(p->classes.size());
  hipLaunchKernelGGL(sweep_reset_kernel, dim3((std::max(p->nprob, ncounters) + 255) / 256), dim3(256), 0, s,
                     p->d_counters, ncounters, p->d_fb_acc, p->nprob);
  MD_LAUNCH_CHECK("sweep_reset_kernel launch");
  for (size_t ci = 0; ci < p->classes.size(); ++ci) {
    const SweepPlan::Class& c = p->classes[ci];
    if (ev) MD_HIP_TRY(hipEventRecord((*ev)[2 * ci], s));
    const int st = c.v == kValuShape            ? launch_small(p, c, static_cast<int>(ci), s)
                   : kShapes[c.v].waves == 16 ? launch_class_shape<16, 1>(p, c, static_cast<int>(ci), s)
                                              : launch_class_shape<8, 2>(p, c, static_cast<int>(ci), s);
    if (st != MD_OK) return st;
    if (ev) MD_HIP_TRY(hipEventRecord((*ev)[2 * ci + 1], s));
  }
  int ncu = 0;
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  hipLaunchKernelGGL(sweep_fallback_kernel, dim3(ncu * 4), dim3(256), 0, s, p->d_probs, p->d_fb, p->d_counters,
                     p->d_fb_acc);
  MD_LAUNCH_CHECK("sweep_fallback_kernel launch");
  hipLaunchKernelGGL(sweep_final_kernel, dim3((p->nprob + 255) / 256), dim3(256), 0, s, p->d_probs, p->nprob,
                     p->d_item_sum, p->d_fb_acc, p->d_counters, p->d_gmi);
  MD_LAUNCH_CHECK("sweep_final_kernel launch");
  return MD_OK;
}

// Builds the item list for the launch shapes of the plan's classes (class_var; shape 0
// for a class without an entry) and every problem's LDS chunk size.
int build_items(SweepPlan* p) {
  std::vector<int> order(static_cast<size_t>(p->nprob));
  for (int i = 0; i < p->nprob; ++i) order[static_cast<size_t>(i)] = i;
  // by class (K steps, label bits), most expensive class first, then by N
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const Problem& A = p->h_probs[static_cast<size_t>(a)];
    const Problem& B = p->h_probs[static_cast<size_t>(b)];
    const int64_t ca = static_cast<int64_t>(A.M) * A.ks, cb = static_cast<int64_t>(B.M) * B.ks;
    if (ca != cb) return ca > cb;
    if (A.ks != B.ks) return A.ks > B.ks;
    return A.N > B.N;
  });
  std::vector<Item> items;
  p->classes.clear();
  for (int pi : order) {
    Problem& P = p->h_probs[static_cast<size_t>(pi)];
    const auto cv = p->class_var.find({P.ks, P.m});
    const int v = cv == p->class_var.end() ? 0 : cv->second;
    const Shape sh = kShapes[v];
    if (p->classes.empty() || p->classes.back().ks != P.ks || p->classes.back().m != P.m)
      p->classes.push_back(
          SweepPlan::Class{P.ks, P.m, static_cast<int>(items.size()), static_cast<int>(items.size()), v, 0});
    // dynamic LDS: fragment chunk (whole tile groups), then the symbol staging rows; a class
    // asks for no more than its largest chunk needs, so that small constellations run
    // several blocks per compute unit
    const int bstage = sh.waves * sh.sb * fastk::bstage_bytes<kMaxKS>();
    int ct = (kDynLds - bstage) / (P.ks * 64 * 16);
    ct -= ct % 8;
    P.chunk_tiles = std::min(ct, P.ntiles);
    // the tile loop's prefetch reads up to two tiles past a chunk's end (into the staging
    // rows that follow it), so the staging rows must span at least two tiles; the vector
    // kernel has no dynamic LDS
    const size_t need = v == kValuShape ? 0
                                        : static_cast<size_t>(P.chunk_tiles) * P.ks * 64 * 16 +
                                              std::max<size_t>(bstage, static_cast<size_t>(2) * P.ks * 64 * 16);
    p->classes.back().lds = std::max(p->classes.back().lds, need);
    const int per_item = sh.waves * 32 * sh.sb * sh.gpi;
    P.item_begin = static_cast<int>(items.size());
    for (int64_t s0 = 0; s0 < P.N; s0 += per_item) {
      Item it;
      it.prob = pi;
      it.start = s0;
      it.count = static_cast<int>(std::min<int64_t>(per_item, P.N - s0));
      items.push_back(it);
    }
    P.item_end = static_cast<int>(items.size());
    p->classes.back().end = P.item_end;
  }
  if (items.size() > static_cast<size_t>(1) << 30) return fail(MD_EINVAL, "too many work items");
  p->n_items = static_cast<int>(items.size());
  void* q = nullptr;
  int st = dev_alloc(p, sizeof(Item) * items.size(), &q);
  if (st != MD_OK) return st;
  p->d_items = static_cast<Item*>(q);
  st = dev_alloc(p, sizeof(double) * items.size(), &q);
  if (st != MD_OK) return st;
  p->d_item_sum = static_cast<double*>(q);
  MD_HIP_TRY(hipMemcpy(p->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
  MD_HIP_TRY(hipMemcpy(p->d_probs, p->h_probs.data(), sizeof(Problem) * p->h_probs.size(), hipMemcpyHostToDevice));
  return MD_OK;
}

int capture(SweepPlan* p) {
  if (p->exec) {
    MD_HIP_TRY(hipGraphExecDestroy(p->exec));
    p->exec = nullptr;
  }
  if (p->graph) {
    MD_HIP_TRY(hipGraphDestroy(p->graph));
    p->graph = nullptr;
  }
  MD_HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  int st = enqueue(p, p->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
  if (st != MD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  p->graph = g;
  MD_HIP_TRY(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
  return MD_OK;
}

}  // namespace
}  // namespace md

extern "C" {

int sweep_plan_create(const md_sweep_instance* inst, int n_inst, const double* sigma2, int n_snr, int variant,
                      void** out) {
  md::set_error("");
  if (!out || !inst || !sigma2) return md::fail(MD_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_inst < 1 || n_snr < 1 || static_cast<int64_t>(n_inst) * n_snr > (1 << 20))
    return md::fail(MD_EINVAL, "need 1 <= instances x noise levels <= 2^20");
  if (variant < -1 || variant > 4) return md::fail(MD_EINVAL, "variant outside [-1, 4]");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  for (int i = 0; i < n_inst; ++i) {
    const md_sweep_instance& I = inst[i];
    if (!I.d_X || !I.d_labels) return md::fail(MD_EINVAL, "instance " + std::to_string(i) + ": NULL pointer");
    if (I.M < 16 || I.M > 8192 || !md::is_pow2(I.M))
      return md::fail(MD_EUNSUPPORTED, "instance " + std::to_string(i) + ": the sweep takes M in {16 .. 8192}");
    if (I.D < 1 || I.D > 8)
      return md::fail(MD_EUNSUPPORTED, "instance " + std::to_string(i) + ": the sweep takes D in [1, 8]");
    if (I.N < 1) return md::fail(MD_EINVAL, "instance " + std::to_string(i) + ": N must be >= 1");
    st = md::check_labels_once(I.d_labels, I.M, nullptr);
    if (st != MD_OK) return st;
    for (int s = 0; s < n_snr; ++s) {
      const double v = sigma2[static_cast<size_t>(i) * n_snr + s];
      if (!(v > 0.0) || !std::isfinite(v)) return md::fail(MD_EINVAL, "sigma2 must be finite and > 0");
    }
  }
  md::SweepPlan* p = new md::SweepPlan();
  p->n_inst = n_inst;
  p->n_snr = n_snr;
  p->nprob = n_inst * n_snr;
  p->device = dev;
  auto bail = [&](int code) {
    md::free_plan(p);
    return code;
  };
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(md::hip_fail(hipGetLastError(), "hipStreamCreate"));
  void* q = nullptr;
  if ((st = md::dev_alloc(p, sizeof(md::Problem) * p->nprob, &q))) return bail(st);
  p->d_probs = static_cast<md::Problem*>(q);
  if ((st = md::dev_alloc(p, sizeof(int) * (md::kCounterBase + 2 * 16), &q))) return bail(st);
  p->d_counters = static_cast<int*>(q);
  if ((st = md::dev_alloc(p, sizeof(md::FbRecord) * md::kFbCap, &q))) return bail(st);
  p->d_fb = static_cast<md::FbRecord*>(q);
  if ((st = md::dev_alloc(p, sizeof(unsigned long long) * p->nprob, &q))) return bail(st);
  p->d_fb_acc = static_cast<unsigned long long*>(q);
  if ((st = md::dev_alloc(p, sizeof(double) * p->nprob, &q))) return bail(st);
  p->d_gmi = static_cast<double*>(q);
  // per (instance, noise level): label-order copy + fragments (prep kernels on cap_stream)
  int max_frag_bytes = 0;
  p->h_probs.resize(static_cast<size_t>(p->nprob));
  p->h_flags.resize(static_cast<size_t>(p->nprob));
  for (int i = 0; i < n_inst; ++i) {
    const md_sweep_instance& I = inst[i];
    const int ks = md::frag_ksteps(I.D);
    const int mpad = I.M < 32 ? 32 : I.M;
    max_frag_bytes = std::max(max_frag_bytes, mpad / 32 * ks * 64 * 16);
    for (int s = 0; s < n_snr; ++s) {
      const int pi = i * n_snr + s;
      const double s2 = sigma2[static_cast<size_t>(i) * n_snr + s];
      char* ws = nullptr;
      if ((st = md::dev_alloc(p, md::prep_bytes(I.M, I.D, 1), &q))) return bail(st);
      ws = static_cast<char*>(q);
      float alpha = 1.0f, c_over_alpha = 1.0f;
      md::score_scales(s2, &alpha, &c_over_alpha);
      md::Prepared prep;
      if ((st = md::prepare(I.d_X, I.d_labels, I.M, I.D, 1, alpha, c_over_alpha, ws, p->cap_stream, &prep)))
        return bail(st);
      p->h_flags[static_cast<size_t>(pi)] = prep.flags;
      md::Problem& P = p->h_probs[static_cast<size_t>(pi)];
      P.frag = prep.frag;
      P.xl = prep.xl;
      P.vx = prep.vx;
      P.X = I.d_X;
      P.labels = I.d_labels;
      P.M = I.M;
      P.m = md::ilog2_pow2(I.M);
      P.D = I.D;
      P.ks = ks;
      P.ntiles = mpad / 32;
      const double c = static_cast<double>(c_over_alpha) * alpha;
      P.cb = static_cast<float>(2.0 * c / alpha);
      P.cn = c_over_alpha;
      P.alpha = alpha;
      P.sigma = std::sqrt(s2);
      P.k0 = static_cast<uint32_t>(I.seed);
      P.k1 = static_cast<uint32_t>(I.seed >> 32);
      P.offset = static_cast<uint64_t>(s) * static_cast<uint64_t>(I.N);
      P.N = I.N;
    }
  }
  if (hipStreamSynchronize(p->cap_stream) != hipSuccess) return bail(md::hip_fail(hipGetLastError(), "prep"));
  for (int pi = 0; pi < p->nprob; ++pi) {
    // the prep flags sit right after the fragments' inverse-label table: read them back
    int fl[4] = {0, 0, 0, 0};
    if (hipMemcpy(fl, p->h_flags[static_cast<size_t>(pi)], sizeof(fl), hipMemcpyDeviceToHost) != hipSuccess)
      return bail(md::hip_fail(hipGetLastError(), "prep flags"));
    if (fl[0]) return bail(md::fail(MD_ELABEL, "labels of problem " + std::to_string(pi) + " are invalid"));
    if (fl[2])
      return bail(md::fail(MD_EUNSUPPORTED, "problem " + std::to_string(pi) +
                                                ": constellation outside the FP16 split range at this noise level"));
  }
  // launch shapes per class: fixed (variant >= 0), from the autotuner's cache, or measured
  p->lds_bytes = static_cast<size_t>(md::kDynLds);
  std::set<std::pair<int, int>> keys;
  for (const auto& P : p->h_probs) keys.insert({P.ks, P.m});
  bool cached = variant < 0;
  if (variant < 0) {
    std::lock_guard<std::mutex> lk(md::g_tune_mu);
    for (const auto& k : keys) {
      const auto it = md::g_tune.find({dev, k.first, k.second});
      if (it == md::g_tune.end()) {
        cached = false;
        break;
      }
      p->class_var[k] = it->second;
    }
  }
  if (variant >= 0) {
    for (const auto& k : keys) p->class_var[k] = md::class_shape(variant, k.second);
  } else if (!cached) {
    // run the whole plan once per shape, timing every class's kernel with events, and give
    // each class the shape under which its own kernel was fastest
    std::map<std::pair<int, int>, float> best;
    for (int v = 0; v < md::kNumShapes; ++v) {
      bool any = false;
      for (const auto& k : keys) {
        p->class_var[k] = md::class_shape(v, k.second);
        any |= p->class_var[k] == v;
      }
      if (!any) continue;
      if ((st = md::build_items(p))) return bail(st);
      const size_t nc = p->classes.size();
      std::vector<hipEvent_t> ev(2 * nc, nullptr);
      for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) st = md::hip_fail(hipGetLastError(), "autotune events");
      if (!st) st = md::enqueue(p, p->cap_stream);                 // warm-up
      if (!st) st = md::enqueue(p, p->cap_stream, &ev);
      if (!st && hipStreamSynchronize(p->cap_stream) != hipSuccess) st = md::hip_fail(hipGetLastError(), "autotune");
      for (size_t ci = 0; ci < nc && !st; ++ci) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[2 * ci], ev[2 * ci + 1]) != hipSuccess) {
          st = md::hip_fail(hipGetLastError(), "autotune timing");
          break;
        }
        const std::pair<int, int> k{p->classes[ci].ks, p->classes[ci].m};
        if (p->classes[ci].v != v) continue;        // a class measured under another pass
        const auto b = best.find(k);
        if (b == best.end() || ms < b->second) {
          best[k] = ms;
          p->tuned[k] = v;
          p->tuned_ms[k] = ms;
        }
      }
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
      if (st) return bail(st);
    }
    std::lock_guard<std::mutex> lk(md::g_tune_mu);
    for (const auto& kv : p->tuned) {
      p->class_var[kv.first] = kv.second;
      md::g_tune[{dev, kv.first.first, kv.first.second}] = kv.second;
    }
  }
  if ((st = md::build_items(p))) return bail(st);
  const md::Shape sh0 = md::kShapes[p->classes.front().v];
  p->waves = sh0.waves;
  p->sb = sh0.sb;
  p->gpi = sh0.gpi;
  if ((st = md::capture(p))) return bail(st);
  *out = p;
  return MD_OK;
}

int sweep_plan_info(const void* plan, int* variant_waves, int* variant_sb, int* groups_per_item, int* n_items) {
  const md::SweepPlan* p = static_cast<const md::SweepPlan*>(plan);
  if (!p) return md::fail(MD_EINVAL, "plan is NULL");
  if (variant_waves) *variant_waves = p->waves;
  if (variant_sb) *variant_sb = p->sb;
  if (groups_per_item) *groups_per_item = p->gpi;
  if (n_items) *n_items = p->n_items;
  return MD_OK;
}

int sweep_plan_class(const void* plan, int i, int* k_steps, int* label_bits, int* shape, int* n_items,
                     float* tuned_ms) {
  md::set_error("");
  const md::SweepPlan* p = static_cast<const md::SweepPlan*>(plan);
  if (!p) return md::fail(MD_EINVAL, "plan is NULL");
  if (i < 0 || i >= static_cast<int>(p->classes.size())) return md::fail(MD_EINVAL, "no such class");
  const md::SweepPlan::Class& c = p->classes[static_cast<size_t>(i)];
  if (k_steps) *k_steps = c.ks;
  if (label_bits) *label_bits = c.m;
  if (shape) *shape = c.v;
  if (n_items) *n_items = c.end - c.begin;
  if (tuned_ms) {
    const auto it = p->tuned_ms.find({c.ks, c.m});
    *tuned_ms = it == p->tuned_ms.end() ? -1.0f : it->second;
  }
  return MD_OK;
}

int sweep_tuning_clear(void) {
  md::set_error("");
  std::lock_guard<std::mutex> lk(md::g_tune_mu);
  md::g_tune.clear();
  return MD_OK;
}

int sweep_run(void* plan, double* d_gmi, int use_graph, void* stream) {
  md::set_error("");
  md::SweepPlan* p = static_cast<md::SweepPlan*>(plan);
  if (!p || !d_gmi) return md::fail(MD_EINVAL, "plan or gmi is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (use_graph) {
    MD_HIP_TRY(hipGraphLaunch(p->exec, s));
  } else {
    const int st = md::enqueue(p, s);
    if (st != MD_OK) return st;
  }
  MD_HIP_TRY(hipMemcpyAsync(d_gmi, p->d_gmi, sizeof(double) * p->nprob, hipMemcpyDeviceToDevice, s));
  return MD_OK;
}

int sweep_run_stats(const void* plan, int64_t* n_fallback, int* overflowed, void* stream) {
  md::set_error("");
  const md::SweepPlan* p = static_cast<const md::SweepPlan*>(plan);
  if (!p) return md::fail(MD_EINVAL, "plan is NULL");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  if (dev != p->device) return md::fail(MD_EINVAL, "the plan lives on another device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int h[3] = {0, 0, 0};
  MD_HIP_TRY(hipMemcpyAsync(h, p->d_counters, sizeof(h), hipMemcpyDeviceToHost, s));
  MD_HIP_TRY(hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = h[1];
  if (overflowed) *overflowed = h[2] != 0 ? 1 : 0;
  return MD_OK;
}

int sweep_plan_destroy(void* plan) {
  md::set_error("");
  md::SweepPlan* p = static_cast<md::SweepPlan*>(plan);
  if (!p) return MD_OK;
  MD_HIP_TRY(hipDeviceSynchronize());
  md::free_plan(p);
  return MD_OK;
}

}  // extern "C"
