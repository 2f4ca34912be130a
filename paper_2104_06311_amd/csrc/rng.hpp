// Device side of the counter-based AWGN channel (Philox4x32-10 + Box-Muller), shared by
// awgn_sample and the batched sweep.  The definition is written out in mdemap.h; every
// floating-point step is a correctly rounded IEEE operation (single precision for the
// normal pair, one double fma for the received value) with contraction switched off, so
// the bits do not depend on where or how the generator runs.
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

// One normal pair from the four words of (symbol g, pair p, domain 2), in IEEE single
// precision (correctly rounded +, -, *, /, sqrt and fma; no contraction):
//   radius: U = f 2^-e, f = 1 + (r0 >> 9) 2^-23, e = 1 + clz(r1) (33 when r1 = 0);
//     ln U = ln f - k ln 2 with f halved and k = e - 1 when f > sqrt2 (else k = e),
//     ln f = 2s P(s^2), s = (f - 1)/(f + 1), P = Horner of 1/(2i+1), i = 5..0;
//     R = sqrt(-2 ln U);
//   angle: quadrant q = r2 >> 30, T = (r2 >> 7) mod 2^23, t = (2T + 1) 2^-24 of the
//     quadrant; sin and cos by Taylor polynomials on [0, pi/4] (t folded at 1/2);
//   z0 = R cos, z1 = R sin after q quarter turns.
constexpr float kGenSqrt2 = 0x1.6a09e6p+0f;
constexpr float kGenLn2Hi = 0x1.62e300p-1f;     // 0.693145751953125: k * hi exact for k < 2^8
constexpr float kGenLn2Lo = 0x1.2fefa2p-17f;    // ln 2 - hi, rounded
constexpr float kGenPio2 = 0x1.921fb6p+0f;

__device__ __forceinline__ float gen_log_u(uint32_t r0, uint32_t r1) {
#pragma clang fp contract(off)
  const int e = r1 == 0u ? 33 : 1 + __clz(static_cast<int>(r1));
  float f = 1.0f + static_cast<float>(r0 >> 9) * 0x1p-23f;      // exact
  float k = static_cast<float>(e);
  if (f > kGenSqrt2) {
    f = f * 0.5f;
    k = k - 1.0f;
  }
  const float s = (f - 1.0f) / (f + 1.0f);
  const float w = s * s;
  float P = 1.0f / 11.0f;
  P = __builtin_fmaf(P, w, 1.0f / 9.0f);
  P = __builtin_fmaf(P, w, 1.0f / 7.0f);
  P = __builtin_fmaf(P, w, 1.0f / 5.0f);
  P = __builtin_fmaf(P, w, 1.0f / 3.0f);
  P = __builtin_fmaf(P, w, 1.0f);
  const float lnf = (2.0f * s) * P;
  return __builtin_fmaf(-k, kGenLn2Hi, __builtin_fmaf(-k, kGenLn2Lo, lnf));
}

// sin and cos of phi = t pi/2, t = (2T + 1) 2^-24 <= 1/2, by Taylor polynomials in
// w = phi^2 (sin to phi^11, cos to phi^12), Horner with fma.
__device__ __forceinline__ void gen_sincos_quarter(uint32_t T, float* s_out, float* c_out) {
#pragma clang fp contract(off)
  const float t = static_cast<float>(2u * T + 1u) * 0x1p-24f;     // exact
  const float phi = t * kGenPio2;
  const float w = phi * phi;
  float S = -1.0f / 39916800.0f;
  S = __builtin_fmaf(S, w, 1.0f / 362880.0f);
  S = __builtin_fmaf(S, w, -1.0f / 5040.0f);
  S = __builtin_fmaf(S, w, 1.0f / 120.0f);
  S = __builtin_fmaf(S, w, -1.0f / 6.0f);
  S = __builtin_fmaf(S, w, 1.0f);
  float C = 1.0f / 479001600.0f;
  C = __builtin_fmaf(C, w, -1.0f / 3628800.0f);
  C = __builtin_fmaf(C, w, 1.0f / 40320.0f);
  C = __builtin_fmaf(C, w, -1.0f / 720.0f);
  C = __builtin_fmaf(C, w, 1.0f / 24.0f);
  C = __builtin_fmaf(C, w, -1.0f / 2.0f);
  C = __builtin_fmaf(C, w, 1.0f);
  *s_out = phi * S;
  *c_out = C;
}

__device__ __forceinline__ void gen_normal_pair(const Philox4& r, float* z0, float* z1) {
#pragma clang fp contract(off)
  const float R = __builtin_sqrtf(-2.0f * gen_log_u(r.w[0], r.w[1]));
  const uint32_t q = r.w[2] >> 30;
  const uint32_t T = (r.w[2] >> 7) & 0x7FFFFFu;
  const bool upper = T >= (1u << 22);
  float sq, cq;
  gen_sincos_quarter(upper ? ((1u << 23) - 1u - T) : T, &sq, &cq);
  const float c = upper ? sq : cq;
  const float s = upper ? cq : sq;
  float ct, st;
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
    float z0, z1;
    gen_normal_pair(r, &z0, &z1);
    const int d0 = 2 * p;
    yout[d0] = static_cast<float>(__builtin_fma(sigma, static_cast<double>(z0), static_cast<double>(xu[d0])));
    if (d0 + 1 < D)
      yout[d0 + 1] = static_cast<float>(__builtin_fma(sigma, static_cast<double>(z1), static_cast<double>(xu[d0 + 1])));
  }
  return u;
}

}  // namespace rng
}  // namespace md
