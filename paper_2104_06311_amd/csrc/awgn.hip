// awgn_sample: counter-based AWGN channel (Philox4x32-10 + Box-Muller), bit-exact by
// definition.  Every floating-point step below is an IEEE double operation written out
// explicitly (contraction is off for this file), so any launch geometry -- and any
// independent implementation of the same definition -- gives identical bits.
#include "common.hpp"

#pragma clang fp contract(off)

namespace md {
namespace {

struct Philox4 {
  uint32_t w[4];
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 2x 32x32->64
// multiply-xor S-box with Weyl-sequence key schedule.
__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

// ln(K 2^-53) for odd K < 2^53: f 2^b = K, atanh series of (f-1)/(f+1) in f^2, fdlibm ln2 split.
__device__ __forceinline__ double gen_log_u(uint64_t K) {
  const int b = 63 - __clzll(static_cast<long long>(K));
  double f = static_cast<double>(K);
  f = __builtin_ldexp(f, -b);
  double e = static_cast<double>(b - 53);
  if (f > 0x1.6a09e667f3bcdp+0) {
    f = f * 0.5;
    e = e + 1.0;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double w = s * s;
  double p = 1.0 / 19.0;
  p = __builtin_fma(p, w, 1.0 / 17.0);
  p = __builtin_fma(p, w, 1.0 / 15.0);
  p = __builtin_fma(p, w, 1.0 / 13.0);
  p = __builtin_fma(p, w, 1.0 / 11.0);
  p = __builtin_fma(p, w, 1.0 / 9.0);
  p = __builtin_fma(p, w, 1.0 / 7.0);
  p = __builtin_fma(p, w, 1.0 / 5.0);
  p = __builtin_fma(p, w, 1.0 / 3.0);
  p = __builtin_fma(p, w, 1.0);
  const double lnf = (2.0 * s) * p;
  return __builtin_fma(e, 0x1.62e42feep-1, __builtin_fma(e, 0x1.a39ef35793c76p-33, lnf));
}

// sin/cos of ((2T+1) 2^-51) * pi/2 for T < 2^49 by Taylor polynomials (degree 17 / 18).
__device__ __forceinline__ void gen_sincos_quarter(uint64_t T, double* s_out, double* c_out) {
  const double t = static_cast<double>(2 * T + 1) * 0x1p-51;
  const double phi = t * 0x1.921fb54442d18p+0;
  const double w = phi * phi;
  double S = 1.0 / 355687428096000.0;
  S = __builtin_fma(S, w, -1.0 / 1307674368000.0);
  S = __builtin_fma(S, w, 1.0 / 6227020800.0);
  S = __builtin_fma(S, w, -1.0 / 39916800.0);
  S = __builtin_fma(S, w, 1.0 / 362880.0);
  S = __builtin_fma(S, w, -1.0 / 5040.0);
  S = __builtin_fma(S, w, 1.0 / 120.0);
  S = __builtin_fma(S, w, -1.0 / 6.0);
  S = __builtin_fma(S, w, 1.0);
  double C = -1.0 / 6402373705728000.0;
  C = __builtin_fma(C, w, 1.0 / 20922789888000.0);
  C = __builtin_fma(C, w, -1.0 / 87178291200.0);
  C = __builtin_fma(C, w, 1.0 / 479001600.0);
  C = __builtin_fma(C, w, -1.0 / 3628800.0);
  C = __builtin_fma(C, w, 1.0 / 40320.0);
  C = __builtin_fma(C, w, -1.0 / 720.0);
  C = __builtin_fma(C, w, 1.0 / 24.0);
  C = __builtin_fma(C, w, -1.0 / 2.0);
  C = __builtin_fma(C, w, 1.0);
  *s_out = phi * S;
  *c_out = C;
}

__device__ __forceinline__ void gen_normal_pair(const Philox4& r, double* z0, double* z1) {
  const uint64_t J1 = (static_cast<uint64_t>(r.w[0] >> 6) << 26) | static_cast<uint64_t>(r.w[1] >> 6);
  const uint64_t J2 = (static_cast<uint64_t>(r.w[2] >> 6) << 26) | static_cast<uint64_t>(r.w[3] >> 6);
  const double R = __builtin_sqrt(-2.0 * gen_log_u(2 * J1 + 1));
  const uint32_t q = static_cast<uint32_t>(J2 >> 50);
  const uint64_t T = J2 & ((1ull << 50) - 1);
  const bool upper = T >= (1ull << 49);
  double sq, cq;
  gen_sincos_quarter(upper ? ((1ull << 50) - 1 - T) : T, &sq, &cq);
  const double c = upper ? sq : cq;
  const double s = upper ? cq : sq;
  double ct, st;
  switch (q) {
    case 0: ct = c; st = s; break;
    case 1: ct = -s; st = c; break;
    case 2: ct = -c; st = -s; break;
    default: ct = s; st = -c; break;
  }
  *z0 = R * ct;
  *z1 = R * st;
}

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
      double z0, z1;
      gen_normal_pair(r, &z0, &z1);
      const int d0 = 2 * p;
      yn[d0] = static_cast<float>(__builtin_fma(sigma, z0, static_cast<double>(xu[d0])));
      if (d0 + 1 < D) yn[d0 + 1] = static_cast<float>(__builtin_fma(sigma, z1, static_cast<double>(xu[d0 + 1])));
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
