// gmi_reduce: Monte-Carlo GMI of bit-metric decoding from LLRs and transmitted labels.
//   T_n = sum_k log2(1 + exp(-s_nk L_nk))  (FP32 per symbol; s = +1 for a sent 0 bit)
//   GMI = m - (1/N) sum_n T_n,  GMI_k = 1 - (1/N) sum_n t_nk,  SE = std(T_n) / sqrt(N)
// Each thread keeps Neumaier-compensated FP32 sums over a grid-stride range of symbols;
// blocks reduce those in FP64 in a fixed order, one block per column adds the block
// partials in FP64, and one thread forms the outputs.  The grid depends only on N, so
// results are deterministic.
#include <cmath>

#include "common.hpp"
#include "llr_kernels.hpp"

namespace md {
namespace {

constexpr int kMaxM = 16;
constexpr int kBlock = 256;
constexpr int kMaxBlocks = 4096;

struct Kahan {
  float s, c;
  __device__ void add(float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  __device__ double get() const { return static_cast<double>(s) + static_cast<double>(c); }
};

// log2(1 + e^x) = max(x, 0) log2(e) + log2(1 + u), u = 2^(-|x| log2 e) in (0, 1], with
// the hardware base-2 exponential and logarithm.  log2(1 + u) is evaluated as
// log2(w) u / (w - 1), w = fl(1 + u), which cancels the rounding of w (the classic
// accurate log1p construction), so small terms keep their relative accuracy.
__device__ __forceinline__ float softplus_bits(float x) {
  constexpr float kLog2e = 1.4426950408889634f;
  const float u = __builtin_amdgcn_exp2f(-fabsf(x) * kLog2e);
  const float w = 1.0f + u;
  const float dw = w - 1.0f;
  const float a = __builtin_amdgcn_logf(w) * (u * __builtin_amdgcn_rcpf(dw));   // NaN when w == 1: not selected
  const float l1p = dw != 0.0f ? a : u * kLog2e;
  return fmaxf(x, 0.0f) * kLog2e + l1p;
}

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// partials: per block, [sum T, sum T^2, sum t_0 .. sum t_{m-1}, count of non-finite T].  Templated on m so that a
// symbol's m LLRs are loaded together and the per-bit work has no branches, and on PER_BIT
// (the per-bit columns are left at zero when the caller does not want them).
template <int MB, bool PER_BIT>
__global__ void __launch_bounds__(kBlock) gmi_partial_kernel(const float* __restrict__ llr, int64_t N,
                                                             const uint32_t* __restrict__ tx,
                                                             const uint32_t* __restrict__ labels,
                                                             double* __restrict__ partials) {
  __shared__ double sh[kBlock];
  Kahan sT{0.f, 0.f}, sT2{0.f, 0.f};
  Kahan sb[MB];
#pragma unroll
  for (int k = 0; k < MB; ++k) sb[k] = Kahan{0.f, 0.f};
  int nonfinite = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t n = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; n < N; n += stride) {
    float L[MB];
#pragma unroll
    for (int k = 0; k < MB; ++k) L[k] = llr[n * MB + k];
    const uint32_t u = tx[n];
    const bool ok = u < (1u << MB);                      // an index outside the labels gives NaN
    const uint32_t lab = labels[ok ? u : 0u];
    float T = ok ? 0.0f : __builtin_nanf("");
#pragma unroll
    for (int k = 0; k < MB; ++k) {
      const float s = ((lab >> (MB - 1 - k)) & 1u) ? 1.0f : -1.0f;   // -s_nk
      const float t = softplus_bits(s * L[k]);
      if (PER_BIT) sb[k].add(t);
      T += t;
    }
    nonfinite += !isfinite(T);
    sT.add(T);
    sT2.add(T * T);
  }
  // column-major partials: column c of block b at partials[c * gridDim.x + b]
  const int64_t nb = gridDim.x;
  double v = block_sum(sT.get(), sh);
  if (threadIdx.x == 0) partials[0 * nb + blockIdx.x] = v;
  v = block_sum(sT2.get(), sh);
  if (threadIdx.x == 0) partials[1 * nb + blockIdx.x] = v;
#pragma unroll
  for (int k = 0; k < MB; ++k) {
    v = PER_BIT ? block_sum(sb[k].get(), sh) : 0.0;
    if (threadIdx.x == 0) partials[(2 + k) * nb + blockIdx.x] = v;
  }
  v = block_sum(static_cast<double>(nonfinite), sh);
  if (threadIdx.x == 0) partials[(2 + MB) * nb + blockIdx.x] = v;
}

// Block partials of the per-symbol loss terms T_n that the fused demapping pass wrote,
// three columns [sum T, sum T^2, count of non-finite T] (column c of block b at
// partials[c * nblocks + b]); a NaN term marks a symbol the fast pass left to the later
// passes (or a bad index), whose term is formed here from its final LLRs like
// gmi_partial_kernel does.
constexpr int kTermsMaxBlocks = 1024;

template <int MB>
__global__ void __launch_bounds__(kBlock) gmi_terms_partial_kernel(const float* __restrict__ terms,
                                                                   const float* __restrict__ llr, int64_t N,
                                                                   const uint32_t* __restrict__ tx,
                                                                   const uint32_t* __restrict__ labels,
                                                                   double* __restrict__ partials) {
  __shared__ double sh[kBlock];
  Kahan sT{0.f, 0.f}, sT2{0.f, 0.f};
  int nonfinite = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  // eight coalesced loads in flight per thread before any of them is used: the pass reads
  // 4 bytes per symbol, so it is bound by load latency, not by bandwidth, one at a time
  constexpr int U = 8;
  for (int64_t n0 = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; n0 < N; n0 += U * stride) {
    float Tu[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t n = n0 + j * stride;
      Tu[j] = n < N ? terms[n] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t n = n0 + j * stride;
      if (n >= N) break;
      float T = Tu[j];
      if (isnan(T)) {
        const uint32_t u = tx[n];
        const bool ok = u < (1u << MB);
        const uint32_t lab = labels[ok ? u : 0u];
        T = ok ? 0.0f : __builtin_nanf("");
#pragma unroll
        for (int k = 0; k < MB; ++k) {
          const float s = ((lab >> (MB - 1 - k)) & 1u) ? 1.0f : -1.0f;
          T += softplus_bits(s * llr[n * MB + k]);
        }
      }
      nonfinite += !isfinite(T);
      sT.add(T);
      sT2.add(T * T);
    }
  }
  const int64_t nb = gridDim.x;
  double v = block_sum(sT.get(), sh);
  if (threadIdx.x == 0) partials[0 * nb + blockIdx.x] = v;
  v = block_sum(sT2.get(), sh);
  if (threadIdx.x == 0) partials[1 * nb + blockIdx.x] = v;
  v = block_sum(static_cast<double>(nonfinite), sh);
  if (threadIdx.x == 0) partials[2 * nb + blockIdx.x] = v;
}

// One block: the three columns of gmi_terms_partial_kernel summed in a fixed order, then
// GMI = m - sum T / N, its standard error, and the count of non-finite terms.
__global__ void __launch_bounds__(kBlock) gmi_terms_tail_kernel(const double* __restrict__ partials, int nblocks,
                                                                int64_t N, int m, double* __restrict__ gmi,
                                                                double* __restrict__ se,
                                                                long long* __restrict__ status) {
  __shared__ double sh[kBlock];
  double tot[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) a += partials[static_cast<int64_t>(c) * nblocks + b];
    tot[c] = block_sum(a, sh);
  }
  if (threadIdx.x == 0) {
    const double Nd = static_cast<double>(N);
    status[0] = static_cast<long long>(tot[2]);
    const double mean = tot[0] / Nd;
    gmi[0] = static_cast<double>(m) - mean;
    if (se) {
      const double var = N > 1 ? (tot[1] - tot[0] * mean) / (Nd - 1.0) : 0.0;
      se[0] = var > 0.0 ? sqrt(var) / sqrt(Nd) : 0.0;
    }
  }
}

// One block per column: the block partials of column c summed in a fixed order.
__global__ void __launch_bounds__(kBlock) gmi_column_kernel(const double* __restrict__ partials, int nblocks,
                                                            double* __restrict__ totals) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) a += partials[static_cast<int64_t>(c) * nblocks + b];
  const double t = block_sum(a, sh);
  if (threadIdx.x == 0) totals[c] = t;
}

__global__ void gmi_output_kernel(const double* __restrict__ tot, int64_t N, int m, double* __restrict__ gmi,
                                  double* __restrict__ gmi_per_bit, double* __restrict__ se,
                                  long long* __restrict__ status) {
  const int k = threadIdx.x;
  const double Nd = static_cast<double>(N);
  if (gmi_per_bit && k < m) gmi_per_bit[k] = 1.0 - tot[2 + k] / Nd;
  if (k == 0) {
    status[0] = static_cast<long long>(tot[2 + m]);   // symbols with a non-finite loss term
    const double mean = tot[0] / Nd;
    gmi[0] = static_cast<double>(m) - mean;
    if (se) {
      const double var = N > 1 ? (tot[1] - tot[0] * mean) / (Nd - 1.0) : 0.0;
      se[0] = var > 0.0 ? sqrt(var) / sqrt(Nd) : 0.0;
    }
  }
}

// Hard decisions from LLR signs (bit 1 where L < 0) against the sent labels: bit-error
// counts per LLR column, integer sums per block (column-major partials: column k of block b
// at partials[k * nblocks + b]), then one block per column sums them in a fixed order and
// one thread adds the columns.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(kBlock) ber_partial_kernel(const float* __restrict__ llr, int64_t N, int m,
                                                             const uint32_t* __restrict__ tx,
                                                             const uint32_t* __restrict__ labels,
                                                             unsigned long long* __restrict__ partials) {
  __shared__ unsigned long long sh[kBlock / 64][kMaxM];
  uint32_t cnt[kMaxM];
#pragma unroll
  for (int k = 0; k < kMaxM; ++k) cnt[k] = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t n = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; n < N; n += stride) {
    const uint32_t u = tx[n];
    const uint32_t lab = u < (1u << m) ? labels[u] : 0u;
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k < m) {
        const uint32_t sent = (lab >> (m - 1 - k)) & 1u;
        const uint32_t dec = llr[n * m + k] < 0.0f ? 1u : 0u;
        cnt[k] += sent ^ dec;
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kMaxM; ++k) {
    if (k < m) {
      const unsigned long long v = wave_sum_u64(cnt[k]);
      if (lane == 0) sh[wave][k] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < m) {
    unsigned long long a = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) a += sh[w][threadIdx.x];
    partials[static_cast<int64_t>(threadIdx.x) * gridDim.x + blockIdx.x] = a;
  }
}

// One block per column k: the block partials of the column summed in a fixed order.
__global__ void __launch_bounds__(kBlock) ber_column_kernel(const unsigned long long* __restrict__ partials,
                                                            int nblocks, unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long sh[kBlock / 64];
  const int k = blockIdx.x;
  unsigned long long a = 0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) a += partials[static_cast<int64_t>(k) * nblocks + b];
  a = wave_sum_u64(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
    totals[k] = t;
  }
}

__global__ void ber_output_kernel(const unsigned long long* __restrict__ totals, int m,
                                  unsigned long long* __restrict__ bit_errors, unsigned long long* __restrict__ errors) {
  if (threadIdx.x != 0) return;
  unsigned long long t = 0;
  for (int k = 0; k < m; ++k) {
    if (bit_errors) bit_errors[k] = totals[k];
    t += totals[k];
  }
  errors[0] = t;
}

// Q-factor of a bit-error count: BER = errors / n_bits, Q = sqrt2 erfcinv(2 BER) (the
// Gaussian-tail relation BER = erfc(Q / sqrt2) / 2), reported as 20 log10 Q; NaN where no
// finite Q exists (BER = 0 or BER >= 1/2).
__global__ void q_factor_kernel(const unsigned long long* __restrict__ errors, int64_t n_bits, double* __restrict__ q) {
  if (threadIdx.x != 0) return;
  const double ber = static_cast<double>(errors[0]) / static_cast<double>(n_bits);
  q[0] = (ber > 0.0 && ber < 0.5) ? 20.0 * log10(1.4142135623730951 * erfcinv(2.0 * ber)) : __builtin_nan("");
}

int gmi_blocks(int64_t N) {
  int64_t b = (N + kBlock - 1) / kBlock;
  if (b > kMaxBlocks) b = kMaxBlocks;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

}  // namespace

size_t gmi_workspace_bytes(int64_t N, int m) {
  return carve_size(sizeof(double) * static_cast<size_t>(gmi_blocks(N)) * (m + 3)) +
         carve_size(sizeof(double) * (m + 3));
}

namespace {
int launch_gmi_tail(double* partials, int nb, int64_t N, int m, double* d_gmi, double* d_gmi_per_bit, double* d_se,
                    long long* status, hipStream_t stream) {
  double* totals = partials + carve_size(sizeof(double) * static_cast<size_t>(nb) * (m + 3)) / sizeof(double);
  hipLaunchKernelGGL(gmi_column_kernel, dim3(m + 3), dim3(kBlock), 0, stream, partials, nb, totals);
  MD_LAUNCH_CHECK("gmi_column_kernel launch");
  hipLaunchKernelGGL(gmi_output_kernel, dim3(1), dim3(64), 0, stream, totals, N, m, d_gmi, d_gmi_per_bit, d_se,
                     status);
  MD_LAUNCH_CHECK("gmi_output_kernel launch");
  return MD_OK;
}
}  // namespace

int launch_gmi_terms(const float* d_terms, const float* d_llr, int64_t N, int m, const uint32_t* d_tx,
                     const uint32_t* d_labels, double* d_gmi, double* d_se, char* ws, long long* status,
                     hipStream_t stream) {
  // about 16 terms per thread, at most kTermsMaxBlocks blocks (3 partials each: within the
  // gmi_workspace_bytes of the per-bit reduction)
  int64_t nb64 = (N + 16 * kBlock - 1) / (16 * kBlock);
  if (nb64 > kTermsMaxBlocks) nb64 = kTermsMaxBlocks;
  if (nb64 < 1) nb64 = 1;
  const int nb = static_cast<int>(nb64);
  double* partials = reinterpret_cast<double*>(ws);
  switch (m) {
#define MD_GMI_CASE(MB_)                                                                                    \
  case MB_:                                                                                               \
    hipLaunchKernelGGL((gmi_terms_partial_kernel<MB_>), dim3(nb), dim3(kBlock), 0, stream, d_terms, d_llr, N, \
                       d_tx, d_labels, partials);                                                         \
    break;
    MD_GMI_CASE(5) MD_GMI_CASE(6) MD_GMI_CASE(7) MD_GMI_CASE(8) MD_GMI_CASE(9) MD_GMI_CASE(10) MD_GMI_CASE(11)
    MD_GMI_CASE(12) MD_GMI_CASE(13) MD_GMI_CASE(14) MD_GMI_CASE(15)
    default: MD_GMI_CASE(16)
#undef MD_GMI_CASE
  }
  MD_LAUNCH_CHECK("gmi_terms_partial_kernel launch");
  hipLaunchKernelGGL(gmi_terms_tail_kernel, dim3(1), dim3(kBlock), 0, stream, partials, nb, N, m, d_gmi, d_se,
                     status);
  MD_LAUNCH_CHECK("gmi_terms_tail_kernel launch");
  return MD_OK;
}

int launch_gmi(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels, double* d_gmi,
               double* d_gmi_per_bit, double* d_se, char* ws, long long* status, hipStream_t stream) {
  const int nb = gmi_blocks(N);
  double* partials = reinterpret_cast<double*>(ws);
  switch (m) {
#define MD_GMI_CASE(MB_)                                                                                    \
  case MB_:                                                                                               \
    if (d_gmi_per_bit)                                                                                    \
      hipLaunchKernelGGL((gmi_partial_kernel<MB_, true>), dim3(nb), dim3(kBlock), 0, stream, d_llr, N, d_tx,  \
                         d_labels, partials);                                                             \
    else                                                                                                  \
      hipLaunchKernelGGL((gmi_partial_kernel<MB_, false>), dim3(nb), dim3(kBlock), 0, stream, d_llr, N, d_tx, \
                         d_labels, partials);                                                             \
    break;
    MD_GMI_CASE(1) MD_GMI_CASE(2) MD_GMI_CASE(3) MD_GMI_CASE(4) MD_GMI_CASE(5) MD_GMI_CASE(6) MD_GMI_CASE(7)
    MD_GMI_CASE(8) MD_GMI_CASE(9) MD_GMI_CASE(10) MD_GMI_CASE(11) MD_GMI_CASE(12) MD_GMI_CASE(13) MD_GMI_CASE(14)
    MD_GMI_CASE(15)
    default: MD_GMI_CASE(16)
#undef MD_GMI_CASE
  }
  MD_LAUNCH_CHECK("gmi_partial_kernel launch");
  return launch_gmi_tail(partials, nb, N, m, d_gmi, d_gmi_per_bit, d_se, status, stream);
}

size_t ber_workspace_bytes(int64_t N, int m) {
  return carve_size(sizeof(unsigned long long) * static_cast<size_t>(gmi_blocks(N)) * m) +
         carve_size(sizeof(unsigned long long) * m);
}

int launch_ber(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels,
               uint64_t* d_bit_errors, uint64_t* d_errors, char* ws, hipStream_t stream) {
  const int nb = gmi_blocks(N);
  auto* partials = reinterpret_cast<unsigned long long*>(ws);
  auto* totals = partials + carve_size(sizeof(unsigned long long) * static_cast<size_t>(nb) * m) /
                                sizeof(unsigned long long);
  hipLaunchKernelGGL(ber_partial_kernel, dim3(nb), dim3(kBlock), 0, stream, d_llr, N, m, d_tx, d_labels, partials);
  MD_LAUNCH_CHECK("ber_partial_kernel launch");
  hipLaunchKernelGGL(ber_column_kernel, dim3(m), dim3(kBlock), 0, stream, partials, nb, totals);
  MD_LAUNCH_CHECK("ber_column_kernel launch");
  hipLaunchKernelGGL(ber_output_kernel, dim3(1), dim3(64), 0, stream, totals, m,
                     reinterpret_cast<unsigned long long*>(d_bit_errors),
                     reinterpret_cast<unsigned long long*>(d_errors));
  MD_LAUNCH_CHECK("ber_output_kernel launch");
  return MD_OK;
}

int launch_q_factor(const uint64_t* d_errors, int64_t n_bits, double* d_q, hipStream_t stream) {
  hipLaunchKernelGGL(q_factor_kernel, dim3(1), dim3(64), 0, stream,
                     reinterpret_cast<const unsigned long long*>(d_errors), n_bits, d_q);
  MD_LAUNCH_CHECK("q_factor_kernel launch");
  return MD_OK;
}

}  // namespace md
