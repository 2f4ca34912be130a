// awgn_sample: counter-based AWGN channel (Philox4x32-10 + Box-Muller), bit-exact by
// definition.  Every floating-point step below is a correctly rounded IEEE operation
// written out explicitly (contraction is off for this file), so any launch geometry --
// and any independent implementation of the same definition -- gives identical bits.
#include "common.hpp"
#include "rng.hpp"

#pragma clang fp contract(off)

namespace md {
namespace {

// One thread per channel use.  A wavefront draws 64 consecutive channel uses into its LDS
// rows (lane l writes the D values of use n0 + l) and then stores the 64 D floats of the
// block as one contiguous run -- 16-byte stores when y is 16-byte aligned (n0 is a multiple
// of 64, so y + n0 D keeps that alignment) -- instead of D scattered 4-byte stores per lane.
template <bool VEC>
__global__ void __launch_bounds__(256) awgn_kernel(const float* __restrict__ X, int m, int D,
                                                   uint32_t k0, uint32_t k1, uint64_t offset,
                                                   int64_t N, double sigma,
                                                   uint32_t* __restrict__ tx, float* __restrict__ y) {
  extern __shared__ float stage[];
  const int lane = threadIdx.x & 63;
  float* ws = stage + (threadIdx.x >> 6) * 64 * D;
  const int64_t wave0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t n0 = wave0 * 64; n0 < N; n0 += nwaves * 64) {
    const int64_t n = n0 + lane;
    if (n < N) tx[n] = rng::channel_symbol(X, m, D, k0, k1, offset + static_cast<uint64_t>(n), sigma, ws + lane * D);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int cnt = static_cast<int>(min<int64_t>(64, N - n0)) * D;    // floats of this block
    float* yb = y + n0 * D;
    int done = 0;
    if constexpr (VEC) {
      const int c4 = cnt >> 2;
      for (int i = lane; i < c4; i += 64)
        reinterpret_cast<float4*>(yb)[i] = reinterpret_cast<const float4*>(ws)[i];
      done = c4 << 2;
    }
    for (int i = done + lane; i < cnt; i += 64) yb[i] = ws[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

}  // namespace

int launch_awgn(const float* d_X, int M, int D, uint64_t seed, uint64_t offset, int64_t N,
                double sigma, uint32_t* d_tx, float* d_y, hipStream_t stream) {
  const int m = ilog2_pow2(M);
  const int block = 256;
  int64_t blocks = (N + block - 1) / block;
  if (blocks > 65536) blocks = 65536;
  const size_t lds = static_cast<size_t>(block) * D * sizeof(float);   // D <= 30: at most 30 KiB
  const bool vec = (reinterpret_cast<uintptr_t>(d_y) & 15) == 0;
  auto kern = vec ? awgn_kernel<true> : awgn_kernel<false>;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(block), lds, stream, d_X, m, D,
                     static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), offset, N, sigma,
                     d_tx, d_y);
  MD_LAUNCH_CHECK("awgn_kernel launch");
  return MD_OK;
}

}  // namespace md
