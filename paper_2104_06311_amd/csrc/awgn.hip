// awgn_sample: counter-based AWGN channel (Philox4x32-10 + Box-Muller), bit-exact by
// definition.  Every floating-point step below is a correctly rounded IEEE operation
// written out explicitly (contraction is off for this file), so any launch geometry --
// and any independent implementation of the same definition -- gives identical bits.
#include "common.hpp"
#include "rng.hpp"

#pragma clang fp contract(off)

namespace md {
namespace {

using rng::Philox4;
using rng::philox10;
using rng::gen_normal_pair;

// One thread per channel use; the D outputs of a symbol are contiguous.
__global__ void __launch_bounds__(256) awgn_kernel(const float* __restrict__ X, int m, int D,
                                                   uint32_t k0, uint32_t k1, uint64_t offset,
                                                   int64_t N, double sigma,
                                                   uint32_t* __restrict__ tx, float* __restrict__ y) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t n = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; n < N; n += stride) {
    const uint64_t g = offset + static_cast<uint64_t>(n);
    const uint32_t glo = static_cast<uint32_t>(g), ghi = static_cast<uint32_t>(g >> 32);
    const Philox4 rt = philox10(glo, ghi, 0u, 1u, k0, k1);
    const uint32_t u = rt.w[0] >> (32 - m);
    tx[n] = u;
    const float* xu = X + static_cast<int64_t>(u) * D;
    float* yn = y + n * D;
    const int npairs = (D + 1) >> 1;
    for (int p = 0; p < npairs; ++p) {
      const Philox4 r = philox10(glo, ghi, static_cast<uint32_t>(p), 2u, k0, k1);
      float z0, z1;
      gen_normal_pair(r, &z0, &z1);
      const int d0 = 2 * p;
      yn[d0] = static_cast<float>(__builtin_fma(sigma, static_cast<double>(z0), static_cast<double>(xu[d0])));
      if (d0 + 1 < D)
        yn[d0 + 1] = static_cast<float>(__builtin_fma(sigma, static_cast<double>(z1), static_cast<double>(xu[d0 + 1])));
    }
  }
}

}  // namespace

int launch_awgn(const float* d_X, int M, int D, uint64_t seed, uint64_t offset, int64_t N,
                double sigma, uint32_t* d_tx, float* d_y, hipStream_t stream) {
  const int m = ilog2_pow2(M);
  const int block = 256;
  int64_t blocks = (N + block - 1) / block;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(awgn_kernel, dim3(static_cast<unsigned>(blocks)), dim3(block), 0, stream, d_X, m, D,
                     static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), offset, N, sigma,
                     d_tx, d_y);
  MD_LAUNCH_CHECK("awgn_kernel launch");
  return MD_OK;
}

}  // namespace md
