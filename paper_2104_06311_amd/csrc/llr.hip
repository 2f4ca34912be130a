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
// One wavefront per symbol, all arithmetic in FP64 (the inputs are FP32, so squared
// distances are exact to double rounding).  Pass 1: per-subset maxima (wavefront
// reductions) and the global maximum g.  Pass 2: one exponential per point,
// e = exp(q - g), added to the m subsets the point belongs to.  A subset whose maximum
// lies within kNearNat of g keeps every term that matters (a term lost to FP64
// underflow is below e^-745 of g, so below e^-145 of the subset's largest term), and
// its log-sum-exp is g + ln(sum); a subset further below g is summed again against its
// own maximum in a pass of its own (in practice never).  Used for every symbol when M < 32 and for the symbols the fast
// passes hand over.
constexpr double kNearNat = 600.0;

__device__ __forceinline__ double point_q(const double (&yv)[kMaxD], const float* __restrict__ xl, int j, int D,
                                          double cnat) {
  double d2 = 0.0;
#pragma unroll
  for (int d = 0; d < kMaxD; ++d) {
    if (d < D) {
      const double df = yv[d] - static_cast<double>(xl[static_cast<int64_t>(j) * D + d]);
      d2 = fma(df, df, d2);
    }
  }
  return -cnat * d2;
}

template <bool MAXLOG>
__global__ void __launch_bounds__(256) llr_careful_kernel(const float* __restrict__ xl, int M, int m, int D,
                                                          const float* __restrict__ y, int64_t N, double cnat,
                                                          float* __restrict__ llr, const int* __restrict__ flags,
                                                          const unsigned* __restrict__ list, int count_slot) {
  const int lane = threadIdx.x & 63;
  const int64_t wave_id = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  const int64_t count = list ? static_cast<int64_t>(flags[count_slot]) : N;
  const bool invalid = flags[0] != 0;
  for (int64_t item = wave_id; item < count; item += nwaves) {
    const int64_t n = list ? static_cast<int64_t>(list[item]) : item;
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
      const double q = point_q(yv, xl, j, D, cnat);
#pragma unroll
      for (int k = 0; k < kMaxM; ++k) {
        if (k < m) {
          const bool b = (j >> (m - 1 - k)) & 1;
          if (b) mx1[k] = fmax(mx1[k], q);
          else mx0[k] = fmax(mx0[k], q);
        }
      }
    }
    double gmax = -INFINITY;
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k < m) {
        mx0[k] = wave_max(mx0[k]);
        mx1[k] = wave_max(mx1[k]);
        gmax = fmax(gmax, fmax(mx0[k], mx1[k]));
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
      const double e = exp(point_q(yv, xl, j, D, cnat) - gmax);
#pragma unroll
      for (int k = 0; k < kMaxM; ++k) {
        if (k < m) {
          const bool b = (j >> (m - 1 - k)) & 1;
          s1[k] += b ? e : 0.0;
          s0[k] += b ? 0.0 : e;
        }
      }
    }
    double lse0[kMaxM], lse1[kMaxM];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k < m) {
        lse0[k] = gmax + log(wave_sum(s0[k]));
        lse1[k] = gmax + log(wave_sum(s1[k]));
      }
    }
    // subsets far below the global maximum: sum again against their own maximum
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k >= m) continue;
#pragma unroll
      for (int bv = 0; bv < 2; ++bv) {
        const double mk = bv ? mx1[k] : mx0[k];
        if (!(gmax - mk > kNearNat)) continue;     // wave-uniform
        double a = 0.0;
        for (int j = lane; j < M; j += 64)
          if (((j >> (m - 1 - k)) & 1) == bv) a += exp(point_q(yv, xl, j, D, cnat) - mk);
        const double l = mk + log(wave_sum(a));
        if (bv) lse1[k] = l;
        else lse0[k] = l;
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxM; ++k)
      if (k < m && lane == k) llr[n * m + k] = static_cast<float>(lse0[k] - lse1[k]);
  }
}

// list == nullptr: every symbol; otherwise the list with its length in flags[count_slot].
template <bool MAXLOG>
int launch_careful_t(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                     const unsigned* list, int count_slot, hipStream_t stream) {
  const int m = ilog2_pow2(M);
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int64_t grid = list ? static_cast<int64_t>(ncu) * 8 : (N + 3) / 4;
  if (grid > static_cast<int64_t>(ncu) * 64) grid = static_cast<int64_t>(ncu) * 64;
  if (grid < 1) grid = 1;
  const double cnat = 1.0 / (2.0 * sigma2);
  hipLaunchKernelGGL(llr_careful_kernel<MAXLOG>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, P.xl, M,
                     m, D, d_y, N, cnat, d_llr, P.flags, list, count_slot);
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
    return maxlog ? launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, nullptr, 0, stream)
                  : launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, nullptr, 0, stream);
  }
  if (maxlog) {
    // max-log never loses range; its list holds only operands outside the FP16 split range
    int st = launch_fast_maxlog(P, M, D, d_y, N, sigma2, d_llr, stream);
    if (st != MD_OK) return st;
    return launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, P.fb_list, 1, stream);
  }
  int st = bf16 ? launch_fast_bf16(P, M, D, d_y, N, d_llr, stream)
                : launch_fast_exact(P, M, D, d_y, N, sigma2, d_llr, stream);
  if (st != MD_OK) return st;
  st = launch_wide_exact(P, M, D, d_y, d_llr, stream);
  if (st != MD_OK) return st;
  return launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, P.fb_list2, 3, stream);
}

int launch_llr_careful_all(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, bool maxlog,
                           float* d_llr, hipStream_t stream) {
  return maxlog ? launch_careful_t<true>(P, M, D, d_y, N, sigma2, d_llr, nullptr, 0, stream)
                : launch_careful_t<false>(P, M, D, d_y, N, sigma2, d_llr, nullptr, 0, stream);
}

}  // namespace md
