// Device side of the counter-based AWGN channel (Philox4x32-10 + Box-Muller), shared by
// awgn_sample and the batched sweep.  The definition is written out in mdemap.h; every
// floating-point step is an IEEE double operation with contraction switched off, so the
// bits do not depend on where or how the generator runs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace md {
namespace rng {

struct Philox4 {
  uint32_t w[4];
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 2x 32x32->64
// multiply-xor S-box with Weyl-sequence key schedule.
__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product per multiplier (a single v_mad_u64_u32 each), not separate
    // low and high multiplies
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
    // three-input XORs in one instruction each (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
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
#pragma clang fp contract(off)
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
#pragma clang fp contract(off)
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
#pragma clang fp contract(off)
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


// Channel use n (global index g = offset + n): transmitted index and the D received values.
__device__ __forceinline__ uint32_t channel_symbol(const float* __restrict__ X, int m, int D, uint32_t k0,
                                                   uint32_t k1, uint64_t g, double sigma, float* yout) {
#pragma clang fp contract(off)
  const uint32_t glo = static_cast<uint32_t>(g), ghi = static_cast<uint32_t>(g >> 32);
  const Philox4 rt = philox10(glo, ghi, 0u, 1u, k0, k1);
  const uint32_t u = rt.w[0] >> (32 - m);
  const float* xu = X + static_cast<int64_t>(u) * D;
  const int npairs = (D + 1) >> 1;
  for (int p = 0; p < npairs; ++p) {
    const Philox4 r = philox10(glo, ghi, static_cast<uint32_t>(p), 2u, k0, k1);
    double z0, z1;
    gen_normal_pair(r, &z0, &z1);
    const int d0 = 2 * p;
    yout[d0] = static_cast<float>(__builtin_fma(sigma, z0, static_cast<double>(xu[d0])));
    if (d0 + 1 < D) yout[d0 + 1] = static_cast<float>(__builtin_fma(sigma, z1, static_cast<double>(xu[d0 + 1])));
  }
  return u;
}

}  // namespace rng
}  // namespace md
