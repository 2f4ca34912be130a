// Exact (and max-log) LLRs of small constellations (M = 32 or 64, D <= 8) with one thread
// per symbol.
//
// With 64 points per symbol the matrix-core kernel does two tiles per 32-symbol block, so
// its per-symbol prologue and epilogue (operand staging, subset combine) cost more than its
// tile work.  Here each thread takes a whole symbol: the score of point j (label order),
//   t_j = bias - c ||y - x_j||^2 = sum_d y_d (2c x_jd) + (-c ||x_j||^2) + (bias - c ||y||^2),
// from the two per-point terms prep writes (read at uniform addresses through the constant
// address space, so by scalar loads that the vector instructions take as operands), D + 1
// FP32 operations per point; e_j = 2^t_j with the fast kernel's fixed bias; the label-0
// and label-1 subset sums of every bit by one pass per bit over block sums; LLRs as
// ln 2 (log2 S0 - log2 S1).  A symbol whose sums leave the FP32 range joins the fast
// pass's fallback list, which the wide-range passes and the FP64 kernel then finish, as
// for the matrix-core kernel.  Rounding: t_j carries about 2^-23 of c (|x_j| + |y|)^2,
// the same order as the split-FP16 contraction's dropped low-by-low product.
#include "common.hpp"
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {
namespace {

constexpr int kVecThreads = 256;

// GMI: also the loss term T_n = sum_k log2((S0_k + S1_k) / S_sent,k) of every finished
// symbol (NaN for the symbols left to the later passes), as the fast kernel's fused
// epilogue writes it.
// MAXLOG: max-log LLRs instead, ln 2 (max_{bit 0} t_j - max_{bit 1} t_j), from the same
// per-point terms with maxima in place of the exponentials and sums (scores never leave
// the FP32 range, so no symbol goes to the fallback list).
template <int MB, int D, bool GMI, bool MAXLOG = false>
__global__ void __launch_bounds__(kVecThreads) llr_vec_kernel(const float* __restrict__ vx_g,
                                                              const float* __restrict__ y, int64_t N, float c,
                                                              float* __restrict__ llr, int* __restrict__ flags,
                                                              unsigned* __restrict__ fb_list,
                                                              const uint32_t* __restrict__ gmi_tx,
                                                              const uint32_t* __restrict__ gmi_labels,
                                                              float* __restrict__ gmi_terms) {
  constexpr int M = 1 << MB;
  constexpr int m = MB;
  typedef const __attribute__((address_space(4))) float ConstFloat;
  const bool invalid = flags[0] != 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kVecThreads;
  for (int64_t n = static_cast<int64_t>(blockIdx.x) * kVecThreads + threadIdx.x; n < N; n += stride) {
    // the table's address passes through an empty asm statement on every symbol, so that
    // the compiler loads the M (D + 1) terms inside the loop as they are used, instead of
    // hoisting them all into scalar registers that spill
    uint64_t vaddr = reinterpret_cast<uint64_t>(vx_g);
    asm volatile("" : "+s"(vaddr));
    ConstFloat* vx = reinterpret_cast<ConstFloat*>(vaddr);
    float yv[D];
    float ysq = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      yv[d] = y[n * D + d];
      ysq = fmaf(yv[d], yv[d], ysq);
    }
    // max-log takes differences of scores only: the terms common to all points (the bias
    // and -c ||y||^2) drop out, and leaving them out keeps the scores' magnitude small
    const float r = MAXLOG ? 0.0f : fmaf(-c, ysq, fastk::kExpBias);
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      float t = vx[j * (D + 1) + D] + r;
#pragma unroll
      for (int d = 0; d < D; ++d) t = fmaf(yv[d], vx[j * (D + 1) + d], t);
      v[j] = MAXLOG ? t : __builtin_amdgcn_exp2f(t);
    }
    // level b: v[k] is the sum over the 2^b consecutive labels of block k, so bit b of a
    // label is the parity of its block index
    float S0[MB], S1[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int cnt = M >> b;
      float a0 = v[0], a1 = v[1];
#pragma unroll
      for (int k = 2; k < cnt; k += 2) {
        a0 = MAXLOG ? fmaxf(a0, v[k]) : a0 + v[k];
        a1 = MAXLOG ? fmaxf(a1, v[k + 1]) : a1 + v[k + 1];
      }
      S0[b] = a0;
      S1[b] = a1;
#pragma unroll
      for (int k = 0; k < cnt / 2; ++k) v[k] = MAXLOG ? fmaxf(v[2 * k], v[2 * k + 1]) : v[2 * k] + v[2 * k + 1];
    }
    if constexpr (MAXLOG) {
#pragma unroll
      for (int k = 0; k < m; ++k) {
        const int b = m - 1 - k;
        llr[n * m + k] = invalid ? __builtin_nanf("") : fastk::kLn2 * (S0[b] - S1[b]);
      }
      continue;
    }
    if (invalid) {
#pragma unroll
      for (int k = 0; k < m; ++k) llr[n * m + k] = __builtin_nanf("");
      if constexpr (GMI) gmi_terms[n] = __builtin_nanf("");
    } else if (!fastk::sums_in_range<MB>(S0, S1)) {
      const int idx = atomicAdd(&flags[1], 1);
      fb_list[idx] = static_cast<unsigned>(n);
      if constexpr (GMI) gmi_terms[n] = __builtin_nanf("");   // taken from its final LLRs later
    } else {
      float l2s0[MB], l2s1[MB];
#pragma unroll
      for (int k = 0; k < m; ++k) {
        const int b = m - 1 - k;
        l2s0[b] = fastk::log2_normal(S0[b]);
        l2s1[b] = fastk::log2_normal(S1[b]);
        llr[n * m + k] = fastk::kLn2 * (l2s0[b] - l2s1[b]);
      }
      if constexpr (GMI) {
        const uint32_t u = gmi_tx[n];
        const uint32_t lab = u < static_cast<uint32_t>(M) ? gmi_labels[u] : 0xFFFFFFFFu;
        // S0 + S1 is the sum over all points for every bit: one logarithm serves all
        const float l2tot = fastk::log2_normal(S0[0] + S1[0]);
        float T = lab != 0xFFFFFFFFu ? 0.0f : __builtin_nanf("");
#pragma unroll
        for (int b = 0; b < MB; ++b) T += l2tot - (((lab >> b) & 1u) ? l2s1[b] : l2s0[b]);
        gmi_terms[n] = T;
      }
    }
  }
}

template <int MB, int D, bool GMI, bool MAXLOG = false>
int launch_vec_g(const Prepared& P, const float* d_y, int64_t N, float* d_llr, hipStream_t stream) {
  auto kern = llr_vec_kernel<MB, D, GMI, MAXLOG>;
  int dev = 0, ncu = 0, occ = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), kVecThreads, 0));
  if (occ < 1) occ = 1;
  int64_t grid = (N + kVecThreads - 1) / kVecThreads;
  const int64_t full = static_cast<int64_t>(ncu) * occ * 4;
  if (grid > full) grid = full;
  const float c = P.c_over_alpha * P.alpha;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(kVecThreads), 0, stream, P.vx, d_y, N, c, d_llr,
                     P.flags, P.fb_list, P.gmi_tx, P.gmi_labels, P.gmi_terms);
  MD_LAUNCH_CHECK("llr_vec_kernel launch");
  return MD_OK;
}

template <int MB, int D>
int launch_vec_t(const Prepared& P, const float* d_y, int64_t N, bool maxlog, float* d_llr, hipStream_t stream) {
  if (maxlog) return launch_vec_g<MB, D, false, true>(P, d_y, N, d_llr, stream);
  return P.gmi_terms ? launch_vec_g<MB, D, true>(P, d_y, N, d_llr, stream)
                     : launch_vec_g<MB, D, false>(P, d_y, N, d_llr, stream);
}

template <int MB>
int launch_vec_m(const Prepared& P, int D, const float* d_y, int64_t N, bool maxlog, float* d_llr,
                 hipStream_t stream) {
  switch (D) {
    case 1: return launch_vec_t<MB, 1>(P, d_y, N, maxlog, d_llr, stream);
    case 2: return launch_vec_t<MB, 2>(P, d_y, N, maxlog, d_llr, stream);
    case 3: return launch_vec_t<MB, 3>(P, d_y, N, maxlog, d_llr, stream);
    case 4: return launch_vec_t<MB, 4>(P, d_y, N, maxlog, d_llr, stream);
    case 5: return launch_vec_t<MB, 5>(P, d_y, N, maxlog, d_llr, stream);
    case 6: return launch_vec_t<MB, 6>(P, d_y, N, maxlog, d_llr, stream);
    case 7: return launch_vec_t<MB, 7>(P, d_y, N, maxlog, d_llr, stream);
    default: return launch_vec_t<MB, 8>(P, d_y, N, maxlog, d_llr, stream);
  }
}

}  // namespace

bool vec_exact_supported(int M, int D) { return (M == 32 || M == 64) && D >= 1 && D <= 8; }

int launch_vec_exact(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr,
                     hipStream_t stream, bool maxlog) {
  if (!vec_exact_supported(M, D) || !P.vx) return fail(MD_EUNSUPPORTED, "vector demapper: M 32 or 64 and D <= 8");
  return M == 32 ? launch_vec_m<5>(P, D, d_y, N, maxlog, d_llr, stream)
                 : launch_vec_m<6>(P, D, d_y, N, maxlog, d_llr, stream);
}

}  // namespace md
