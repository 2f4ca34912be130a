// Exact and max-log bit-wise LLRs: dispatch, the careful kernel and the score scales.
//
// Fast path (M >= 32, llr_fast.hpp).  A block of wavefronts stages the constellation
// fragments (prep.hip) in LDS; every wavefront takes one or two blocks of 32 received
// symbols.  Per tile of 32 labels it forms the 32x32 score block
// t = -c ||y - x||^2 + bias (base-2 exponent) with one v_mfma_f32_32x32x16_f16 per 16
// K slots of the split-FP16 contraction, then:
//   exact:   e = 2^t (v_exp_f32).  Because the shift -c ||y||^2 is part of the score,
//            t <= bias up to rounding and no running maximum is needed.  Lane l owns
//            labels 32 tau + 16 (l/32) + r, r = 0..15, of symbol l % 32; it keeps
//            E[r] += e (per-position sums over all tiles: label bits 0..3), per-tile
//            sums for the low tile-index bits, and group sums routed by the remaining
//            label bits.  Label bit 4 is the lane half.
//   max-log: the same with max in place of exp/add.
// The label-0/label-1 subset sums of bit b follow from those partial sums, and
// L = ln2 (log2 S0 - log2 S1).
//
// Exact path in three stages.  (1) The fast kernel appends to a first list every
// symbol with a subset sum outside [2^-96, 2^126] (its far subset lost FP32 range:
// the subset's best point lies more than 196 base-2 units below the bias) or with score
// operands outside the FP16 split range.  (2) The wide-range pass evaluates those
// symbols in two exponent windows 190 units apart and takes each subset sum from the
// window that kept it in range.  (3) What is left goes to the careful kernel: one
// wavefront per symbol, difference-form FP64 distances, per-subset maxima and
// log-sum-exp, robust for any finite input.  Max-log has only stages 1 and 3.
#include <cmath>
#include <cstdlib>

#include "common.hpp"
#include "llr_kernels.hpp"

namespace md {

namespace {

constexpr int kMaxM = 16;     // log2 of the largest M
constexpr int kMaxD = 30;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ careful kernel
// Four wavefronts per block, one symbol each.  The block stages the label-ordered points in
// LDS chunks of 512 that all four symbols read.  In a chunk, lane l takes the points
// j = c0 + l + 64 t (t = 0..7), so label bits 0..5 are the lane, bits 6..8 are t and the
// higher bits are the chunk index: each point is added to one position sum E[t] and to
// the chunk total, and the chunk totals are routed by the chunk-index bits (the same
// label-order geometry as the fast kernel, two FP64 adds per point instead of 2m).
// All arithmetic is FP64 (the inputs are FP32, so squared distances are exact to double
// rounding).
//   exact:   pass 1 finds the global maximum g of q = -||y - x||^2 / (2 sigma2); pass 2
//            accumulates e = exp(q - g).  A subset sum of at least 1e-290 has its
//            largest term in the normal FP64 range, and the terms lost to underflow
//            (below e^-745 of g) lie below e^-66 of that term, so its log-sum-exp is
//            g + ln(sum).  A smaller sum means the subset lies more than ~667 nats below
//            g: it is summed again against its own maximum (in practice never).
//   max-log: pass 1 alone, with max in place of the sums.
// Used for the symbols the fast passes hand over (M >= 32).
constexpr int kCarefulWaves = 4;
constexpr int kChunkPts = 512;                 // 512 rows of at most 31 floats: <= 62 KiB of LDS
constexpr int kChunkBits = 9;
constexpr int kMaxHigh = kMaxM - kChunkBits;   // label bits routed by chunk index
constexpr double kTinySum = 1e-290;

__device__ __forceinline__ double point_q(const double (&yv)[kMaxD], const float* __restrict__ x, int D, double cnat) {
  double d2 = 0.0;
#pragma unroll
  for (int d = 0; d < kMaxD; ++d) {
    if (d < D) {
      const double df = yv[d] - static_cast<double>(x[d]);
      d2 = fma(df, df, d2);
    }
  }
  return -cnat * d2;
}

// Log-sum-exp of subset (label bit b = bv) of received symbol yn straight from memory,
// against the subset's own maximum (the rare far-subset path; kept out of line).
__device__ __noinline__ double subset_lse(const float* __restrict__ yn, const float* __restrict__ xl, int M, int D,
                                          int b, int bv, double cnat, int lane) {
  double yv[kMaxD];
#pragma unroll
  for (int d = 0; d < kMaxD; ++d) yv[d] = d < D ? static_cast<double>(yn[d]) : 0.0;
  double mk = -INFINITY;
  for (int j = lane; j < M; j += 64)
    if (((j >> b) & 1) == bv) mk = fmax(mk, point_q(yv, xl + static_cast<int64_t>(j) * D, D, cnat));
  mk = wave_max(mk);
  double a = 0.0;
  for (int j = lane; j < M; j += 64)
    if (((j >> b) & 1) == bv) a += exp(point_q(yv, xl + static_cast<int64_t>(j) * D, D, cnat) - mk);
  return mk + log(wave_sum(a));
}

template <bool MAXLOG>
__device__ __forceinline__ double comb(double a, double b) {
  return MAXLOG ? fmax(a, b) : a + b;
}
template <bool MAXLOG>
__device__ __forceinline__ double wave_comb(double v) {
  return MAXLOG ? wave_max(v) : wave_sum(v);
}

template <bool MAXLOG>
__global__ void __launch_bounds__(kCarefulWaves * 64) llr_careful_kernel(const float* __restrict__ xl, int M, int m,
                                                                         int D, const float* __restrict__ y, int64_t N,
                                                                         double cnat, float* __restrict__ llr,
                                                                         const int* __restrict__ flags,
                                                                         const unsigned* __restrict__ list,
                                                                         int count_slot) {
  extern __shared__ float pts[];                 // kChunkPts rows of Dp floats
  const int Dp = D | 1;                          // odd row stride: no LDS bank conflicts
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t count = list ? static_cast<int64_t>(flags[count_slot]) : N;
  const bool invalid = flags[0] != 0;
  const double ident = MAXLOG ? -INFINITY : 0.0;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCarefulWaves; base < count;
       base += static_cast<int64_t>(gridDim.x) * kCarefulWaves) {
    const int64_t item = base + wave;
    const bool live = item < count;              // every wave still joins the block's barriers
    const int64_t n = live ? (list ? static_cast<int64_t>(list[item]) : item) : 0;
    double yv[kMaxD];
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) yv[d] = (live && d < D) ? static_cast<double>(y[n * D + d]) : 0.0;
    double E[8], H0[kMaxHigh], H1[kMaxHigh];
#pragma unroll
    for (int t = 0; t < 8; ++t) E[t] = ident;
#pragma unroll
    for (int q = 0; q < kMaxHigh; ++q) {
      H0[q] = ident;
      H1[q] = ident;
    }
    double gmax = -INFINITY;
    for (int pass = 0; pass < (MAXLOG ? 1 : 2); ++pass) {
      const bool sums = !MAXLOG && pass == 1;
      for (int c0 = 0; c0 < M; c0 += kChunkPts) {
        const int cn = min(kChunkPts, M - c0);
        __syncthreads();
        const float* src = xl + static_cast<int64_t>(c0) * D;
        for (int pt = threadIdx.x; pt < cn; pt += kCarefulWaves * 64)
          for (int d = 0; d < D; ++d) pts[pt * Dp + d] = src[pt * D + d];
        __syncthreads();
        double ctot = ident;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int jj = lane + 64 * t;
          if (jj < cn) {
            const double q = point_q(yv, pts + jj * Dp, D, cnat);
            if (MAXLOG) {
              E[t] = fmax(E[t], q);
              ctot = fmax(ctot, q);
            } else if (!sums) {
              gmax = fmax(gmax, q);
            } else {
              const double e = exp(q - gmax);
              E[t] += e;
              ctot += e;
            }
          }
        }
        if (MAXLOG || sums) {
          const int chunk = c0 >> kChunkBits;
#pragma unroll
          for (int q = 0; q < kMaxHigh; ++q) {
            const bool bit = (chunk >> q) & 1;
            H1[q] = bit ? comb<MAXLOG>(H1[q], ctot) : H1[q];
            H0[q] = bit ? H0[q] : comb<MAXLOG>(H0[q], ctot);
          }
        }
      }
      if (!MAXLOG && pass == 0) gmax = wave_max(gmax);
    }
    if (!live) continue;
    if (invalid) {
      if (lane < m) llr[n * m + lane] = __builtin_nanf("");
      continue;
    }
    // label-0 / label-1 subset sums (or maxima) of label bit b
    double lane_tot = ident;
#pragma unroll
    for (int t = 0; t < 8; ++t) lane_tot = comb<MAXLOG>(lane_tot, E[t]);
    double S0[kMaxM], S1[kMaxM];
#pragma unroll
    for (int b = 0; b < kMaxM; ++b) {
      S0[b] = ident;
      S1[b] = ident;
      if (b >= m) continue;
      if (b < 6) {
        const bool bit = (lane >> b) & 1;
        S0[b] = wave_comb<MAXLOG>(bit ? ident : lane_tot);
        S1[b] = wave_comb<MAXLOG>(bit ? lane_tot : ident);
      } else if (b < kChunkBits) {
        double a0 = ident, a1 = ident;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if ((t >> (b - 6)) & 1) a1 = comb<MAXLOG>(a1, E[t]);
          else a0 = comb<MAXLOG>(a0, E[t]);
        }
        S0[b] = wave_comb<MAXLOG>(a0);
        S1[b] = wave_comb<MAXLOG>(a1);
      } else {
        S0[b] = wave_comb<MAXLOG>(H0[b - kChunkBits]);
        S1[b] = wave_comb<MAXLOG>(H1[b - kChunkBits]);
      }
    }
#pragma unroll
    for (int b = 0; b < kMaxM; ++b) {
      if (b >= m) continue;
      double l0, l1;
      if (MAXLOG) {
        l0 = S0[b];
        l1 = S1[b];
      } else {
        // wave-uniform: far subsets are summed again against their own maximum
        l0 = S0[b] >= kTinySum ? gmax + log(S0[b]) : subset_lse(y + n * D, xl, M, D, b, 0, cnat, lane);
        l1 = S1[b] >= kTinySum ? gmax + log(S1[b]) : subset_lse(y + n * D, xl, M, D, b, 1, cnat, lane);
      }
      const int k = m - 1 - b;                  // column k holds label bit m-1-k
      if (lane == k) llr[n * m + k] = static_cast<float>(l0 - l1);
    }
  }
}

// ------------------------------------------------------------------ small constellations
// M <= 16: one thread per symbol.  The M scores q_j = -||y - x_j||^2 / (2 sigma2) are
// formed in FP64 (difference form); per label subset the maximum is taken in FP64 and the
// sum of exp(q - max) <= 1 in FP32 (hardware exponential, every term relative to the
// subset's own maximum, so nothing underflows that matters); LSE = max + ln(sum).
constexpr int kSmallM = 16;

template <bool MAXLOG>
__global__ void __launch_bounds__(256) llr_small_kernel(const float* __restrict__ xl, int M, int m, int D,
                                                        const float* __restrict__ y, int64_t N, double cnat,
                                                        float* __restrict__ llr, const int* __restrict__ flags) {
  const bool invalid = flags[0] != 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t n = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
    if (invalid) {
      for (int k = 0; k < m; ++k) llr[n * m + k] = __builtin_nanf("");
      continue;
    }
    double q[kSmallM];
#pragma unroll
    for (int j = 0; j < kSmallM; ++j) {
      q[j] = -INFINITY;
      if (j < M) {
        double d2 = 0.0;
        for (int d = 0; d < D; ++d) {
          const double df = static_cast<double>(y[n * D + d]) - static_cast<double>(xl[j * D + d]);
          d2 = fma(df, df, d2);
        }
        q[j] = -cnat * d2;
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b >= m) continue;
      double mx[2] = {-INFINITY, -INFINITY};
#pragma unroll
      for (int j = 0; j < kSmallM; ++j)
        if (j < M) mx[(j >> b) & 1] = fmax(mx[(j >> b) & 1], q[j]);
      double lse[2];
      if (MAXLOG) {
        lse[0] = mx[0];
        lse[1] = mx[1];
      } else {
        float sum[2] = {0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < kSmallM; ++j)
          if (j < M) sum[(j >> b) & 1] += __expf(static_cast<float>(q[j] - mx[(j >> b) & 1]));
        lse[0] = mx[0] + log(static_cast<double>(sum[0]));
        lse[1] = mx[1] + log(static_cast<double>(sum[1]));
      }
      llr[n * m + (m - 1 - b)] = static_cast<float>(lse[0] - lse[1]);
    }
  }
}

template <bool MAXLOG>
int launch_small_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                   hipStream_t stream) {
  const int m = ilog2_pow2(M);
  int64_t grid = (N + 255) / 256;
  if (grid > 65536) grid = 65536;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(llr_small_kernel<MAXLOG>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, P.xl, M, m, D,
                     d_y, N, 1.0 / (2.0 * sigma2), d_llr, P.flags);
  MD_LAUNCH_CHECK("llr_small_kernel launch");
  return MD_OK;
}

// list == nullptr: every symbol; otherwise the list with its length in flags[count_slot].
template <bool MAXLOG>
int launch_careful_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                     const unsigned* list, int count_slot, hipStream_t stream) {
  const int m = ilog2_pow2(M);
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int64_t grid = list ? static_cast<int64_t>(ncu) * 2 : (N + kCarefulWaves - 1) / kCarefulWaves;
  if (grid > static_cast<int64_t>(ncu) * 16) grid = static_cast<int64_t>(ncu) * 16;
  if (grid < 1) grid = 1;
  const double cnat = 1.0 / (2.0 * sigma2);
  const size_t lds = sizeof(float) * static_cast<size_t>(kChunkPts) * (D | 1);
  hipLaunchKernelGGL(llr_careful_kernel<MAXLOG>, dim3(static_cast<unsigned>(grid)), dim3(kCarefulWaves * 64), lds,
                     stream, P.xl, M, m, D, d_y, N, cnat, d_llr, P.flags, list, count_slot);
  MD_LAUNCH_CHECK("llr_careful_kernel launch");
  return MD_OK;
}

}  // namespace

void score_scales(double sigma2, float* alpha, float* c_over_alpha) {
  const double c = 1.4426950408889634 / (2.0 * sigma2);
  int e = static_cast<int>(std::lround(std::log2(c) / 2.0));
  e = e < -14 ? -14 : (e > 14 ? 14 : e);           // a stays a normal FP16 power of two
  *alpha = std::ldexp(1.0f, e);
  *c_over_alpha = static_cast<float>(c / std::ldexp(1.0, e));
}

int launch_llr(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, bool maxlog,
               int prec, float* d_llr, hipStream_t stream) {
  if (M <= kSmallM) {
    return maxlog ? launch_small_t<true>(P, M, D, d_y, N, sigma2, d_llr, stream)
                  : launch_small_t<false>(P, M, D, d_y, N, sigma2, d_llr, stream);
  }
  if (maxlog) {
    // max-log never loses range; its list holds only operands outside the FP16 split range
    const int slot = timing_begin(stream);
    int st = (vec_exact_supported(M, D) && P.vx) ? launch_vec_exact(P, M, D, d_y, N, d_llr, stream, true)
                                                 : launch_fast_maxlog(P, M, D, d_y, N, sigma2, d_llr, stream);
    timing_end(stream, slot);
    if (st != MD_OK) return st;
    return launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, P.fb_list, 1, stream);
  }
  if (P.sc != 0) {
    // reduced-precision scores: symbols outside the fast pass's range go straight to the
    // FP64 kernel (their LLRs are then exact)
    const int slot = timing_begin(stream);
    int st = P.gmi_terms ? launch_fast_gmi(P, M, D, d_y, N, sigma2, d_llr, stream)
                         : launch_fast_lowp(P, M, D, d_y, N, sigma2, d_llr, stream);
    timing_end(stream, slot);
    if (st != MD_OK) return st;
    return launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, P.fb_list, 1, stream);
  }
  const int slot = timing_begin(stream);
  // M = 32 and 64 (D <= 8): one thread per symbol, for llr_exact and llr_exact_gmi alike,
  // so that both give the same LLRs
  const bool vec = prec != MD_PREC_BF16 && vec_exact_supported(M, D) && P.vx;
  int st = vec ? launch_vec_exact(P, M, D, d_y, N, d_llr, stream)
           : P.gmi_terms ? launch_fast_gmi(P, M, D, d_y, N, sigma2, d_llr, stream)
           : prec == MD_PREC_BF16 ? launch_fast_bf16(P, M, D, d_y, N, d_llr, stream)
                                  : launch_fast_exact(P, M, D, d_y, N, sigma2, d_llr, stream);
  timing_end(stream, slot);
  if (st != MD_OK) return st;
  st = launch_wide_exact(P, M, D, d_y, d_llr, stream);
  if (st != MD_OK) return st;
  st = launch_wide3_exact(P, M, D, d_y, d_llr, stream);
  if (st != MD_OK) return st;
  return launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, P.fb_list, 4, stream);
}

int launch_llr_careful_all(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, bool maxlog,
                           float* d_llr, hipStream_t stream) {
  return maxlog ? launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, nullptr, 0, stream)
                : launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, nullptr, 0, stream);
}

}  // namespace md
