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
// A symbol whose smaller subset sum falls below 2^-96 (its far subset lost FP32
// range), or whose score operands leave the FP16 split range, is appended to a
// fallback list and recomputed by the careful kernel: one wavefront per symbol,
// difference-form FP64 distances, per-subset maxima by wavefront reductions, then
// per-subset log-sum-exp -- the textbook evaluation, robust for any finite input.
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
// One wavefront per symbol, all arithmetic in FP64 (the inputs are FP32, so squared
// distances are exact to double rounding): per-subset maxima by wavefront
// reductions, then per-subset log-sum-exp.  Used for every symbol when M < 32 and for
// the rare symbols the fast kernel hands over.
template <bool MAXLOG>
__global__ void __launch_bounds__(256) llr_careful_kernel(const float* __restrict__ xl, int M, int m, int D,
                                                          const float* __restrict__ y, int64_t N, double cnat,
                                                          float* __restrict__ llr, const int* __restrict__ flags,
                                                          const unsigned* __restrict__ list, int use_list) {
  const int lane = threadIdx.x & 63;
  const int64_t wave_id = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  const int64_t count = use_list ? static_cast<int64_t>(flags[1]) : N;
  const bool invalid = flags[0] != 0;
  for (int64_t item = wave_id; item < count; item += nwaves) {
    const int64_t n = use_list ? static_cast<int64_t>(list[item]) : item;
    if (invalid) {
      if (lane < m) llr[n * m + lane] = __builtin_nanf("");
      continue;
    }
    double yv[kMaxD];
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) yv[d] = d < D ? static_cast<double>(y[n * D + d]) : 0.0;
    double mx0[kMaxM], mx1[kMaxM];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      mx0[k] = -INFINITY;
      mx1[k] = -INFINITY;
    }
    for (int j = lane; j < M; j += 64) {
      double d2 = 0.0;
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) {
        if (d < D) {
          const double df = yv[d] - static_cast<double>(xl[static_cast<int64_t>(j) * D + d]);
          d2 = fma(df, df, d2);
        }
      }
      const double q = -cnat * d2;
#pragma unroll
      for (int k = 0; k < kMaxM; ++k) {
        if (k < m) {
          const bool b = (j >> (m - 1 - k)) & 1;
          if (b) mx1[k] = fmax(mx1[k], q);
          else mx0[k] = fmax(mx0[k], q);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k < m) {
        mx0[k] = wave_max(mx0[k]);
        mx1[k] = wave_max(mx1[k]);
      }
    }
    if (MAXLOG) {
#pragma unroll
      for (int k = 0; k < kMaxM; ++k)
        if (k < m && lane == k) llr[n * m + k] = static_cast<float>(mx0[k] - mx1[k]);
      continue;
    }
    double s0[kMaxM], s1[kMaxM];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      s0[k] = 0.0;
      s1[k] = 0.0;
    }
    for (int j = lane; j < M; j += 64) {
      double d2 = 0.0;
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) {
        if (d < D) {
          const double df = yv[d] - static_cast<double>(xl[static_cast<int64_t>(j) * D + d]);
          d2 = fma(df, df, d2);
        }
      }
      const double q = -cnat * d2;
#pragma unroll
      for (int k = 0; k < kMaxM; ++k) {
        if (k < m) {
          const bool b = (j >> (m - 1 - k)) & 1;
          const double e = exp(q - (b ? mx1[k] : mx0[k]));
          if (b) s1[k] += e;
          else s0[k] += e;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k < m) {
        const double a0 = wave_sum(s0[k]);
        const double a1 = wave_sum(s1[k]);
        if (lane == k) llr[n * m + k] = static_cast<float>((mx0[k] + log(a0)) - (mx1[k] + log(a1)));
      }
    }
  }
}

template <bool MAXLOG>
int launch_careful_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                     bool use_list, hipStream_t stream) {
  const int m = ilog2_pow2(M);
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int64_t grid = use_list ? static_cast<int64_t>(ncu) * 8 : (N + 3) / 4;
  if (grid > static_cast<int64_t>(ncu) * 64) grid = static_cast<int64_t>(ncu) * 64;
  if (grid < 1) grid = 1;
  const double cnat = 1.0 / (2.0 * sigma2);
  hipLaunchKernelGGL(llr_careful_kernel<MAXLOG>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, P.xl, M,
                     m, D, d_y, N, cnat, d_llr, P.flags, P.fb_list, use_list ? 1 : 0);
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
               bool bf16, float* d_llr, hipStream_t stream) {
  if (M < 32) {
    return maxlog ? launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, false, stream)
                  : launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, false, stream);
  }
  const int st = maxlog ? launch_fast_maxlog(P, M, D, d_y, N, sigma2, d_llr, stream)
                 : bf16   ? launch_fast_bf16(P, M, D, d_y, N, d_llr, stream)
                          : launch_fast_exact(P, M, D, d_y, N, sigma2, d_llr, stream);
  if (st != MD_OK) return st;
  return maxlog ? launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, true, stream)
                : launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, true, stream);
}

int launch_llr_careful_all(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, bool maxlog,
                           float* d_llr, hipStream_t stream) {
  return maxlog ? launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, false, stream)
                : launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, false, stream);
}

}  // namespace md
