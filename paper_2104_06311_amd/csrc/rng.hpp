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

// One normal pair from two Philox words (a radius word and an angle word), in IEEE single
// precision (correctly rounded +, -, *, /, sqrt, fma and integer-to-float conversion; no
// contraction):
//   radius: v = float(a | 1) (round to nearest even), U = v 2^-32 in [2^-32, 1];
//     v = f 2^E with f in [1, 2) from its bits; k = E - 32, and f halved, k + 1 when
//     f > sqrt2; ln U = ln f + k ln 2 with ln f = 2s P(s^2), s = (f - 1)/(f + 1),
//     P = Horner of 1/(2i+1), i = 5..0; R = sqrt(-2 ln U);
//   angle: quadrant q = b >> 30, T = (b >> 7) mod 2^23, t = (2T + 1) 2^-24 of the
//     quadrant; sin and cos by Taylor polynomials on [0, pi/4] (t folded at 1/2);
//   z0 = R cos, z1 = R sin after q quarter turns.
constexpr float kGenSqrt2 = 0x1.6a09e6p+0f;
constexpr float kGenLn2Hi = 0x1.62e300p-1f;     // 0.693145751953125: k * hi exact for |k| < 2^8
constexpr float kGenLn2Lo = 0x1.2fefa2p-17f;    // ln 2 - hi, rounded
constexpr float kGenPio2 = 0x1.921fb6p+0f;

__device__ __forceinline__ float gen_log_u(uint32_t a) {
#pragma clang fp contract(off)
  const float v = static_cast<float>(a | 1u);                     // in [1, 2^32], rounded to nearest even
  const uint32_t bits = __float_as_uint(v);
  float f = __uint_as_float((bits & 0x007FFFFFu) | 0x3F800000u);   // mantissa in [1, 2)
  float k = static_cast<float>(static_cast<int>(bits >> 23) - 127 - 32);
  if (f > kGenSqrt2) {
    f = f * 0.5f;
    k = k + 1.0f;
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
  return __builtin_fmaf(k, kGenLn2Hi, __builtin_fmaf(k, kGenLn2Lo, lnf));
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

__device__ __forceinline__ void gen_normal_pair(uint32_t a, uint32_t b, float* z0, float* z1) {
#pragma clang fp contract(off)
  const float R = __builtin_sqrtf(-2.0f * gen_log_u(a));
  const uint32_t q = b >> 30;
  const uint32_t T = (b >> 7) & 0x7FFFFFu;
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

// Channel use g (counter words g_lo, g_hi): the Philox blocks (g_lo, g_hi, j, 1), j = 0, 1, ...
// give one stream of words w_{4j+i} = r_i.  Word w_0 gives the transmitted index
// u = w_0 >> (32 - m); pair p takes the radius word w_{2p+1} and the angle word w_{2p+2}
// and gives dimensions 2p and 2p + 1 (the last pair of an odd D uses only its first
// value).  Each received value is y_d = fl32(x_d + sigma z_d), one double fma.  So 8D
// takes three blocks and 2D one.
__device__ __forceinline__ uint32_t channel_symbol(const float* __restrict__ X, int m, int D, uint32_t k0,
                                                   uint32_t k1, uint64_t g, double sigma, float* yout) {
#pragma clang fp contract(off)
  const uint32_t glo = static_cast<uint32_t>(g), ghi = static_cast<uint32_t>(g >> 32);
  const int npairs = (D + 1) >> 1;
  uint32_t u = 0, radius = 0;
  const float* xu = X;
  int p = 0;
  for (uint32_t j = 0; p < npairs; ++j) {
    const Philox4 r = philox10(glo, ghi, j, 1u, k0, k1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if ((i & 1) != 0) {            // odd word: the radius word of the next pair
        radius = r.w[i];
        continue;
      }
      if (j == 0 && i == 0) {        // word 0: the transmitted index
        u = r.w[0] >> (32 - m);
        xu = X + static_cast<int64_t>(u) * D;
        continue;
      }
      if (p >= npairs) break;
      float z0, z1;
      gen_normal_pair(radius, r.w[i], &z0, &z1);
      const int d0 = 2 * p;
      yout[d0] = static_cast<float>(__builtin_fma(sigma, static_cast<double>(z0), static_cast<double>(xu[d0])));
      if (d0 + 1 < D)
        yout[d0 + 1] =
            static_cast<float>(__builtin_fma(sigma, static_cast<double>(z1), static_cast<double>(xu[d0 + 1])));
      ++p;
    }
  }
  return u;
}

// The same channel use for a compile-time D: every word index, block and output dimension
// is a constant, so the D values stay in registers without the selects that a run-time
// index into a register array costs.  Identical results to channel_symbol.
template <int D>
__device__ __forceinline__ uint32_t channel_symbol_d(const float* __restrict__ X, int m, uint32_t k0, uint32_t k1,
                                                     uint64_t g, double sigma, float (&yout)[8]) {
#pragma clang fp contract(off)
  constexpr int NP = (D + 1) / 2;          // normal pairs
  constexpr int NB = (1 + 2 * NP + 3) / 4;  // Philox blocks of the word stream
  const uint32_t glo = static_cast<uint32_t>(g), ghi = static_cast<uint32_t>(g >> 32);
  uint32_t w[4 * NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const Philox4 r = philox10(glo, ghi, static_cast<uint32_t>(j), 1u, k0, k1);
#pragma unroll
    for (int i = 0; i < 4; ++i) w[4 * j + i] = r.w[i];
  }
  const uint32_t u = w[0] >> (32 - m);
  const float* xu = X + static_cast<int64_t>(u) * D;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    float z0, z1;
    gen_normal_pair(w[2 * p + 1], w[2 * p + 2], &z0, &z1);
    yout[2 * p] = static_cast<float>(__builtin_fma(sigma, static_cast<double>(z0), static_cast<double>(xu[2 * p])));
    if (2 * p + 1 < D)
      yout[2 * p + 1] =
          static_cast<float>(__builtin_fma(sigma, static_cast<double>(z1), static_cast<double>(xu[2 * p + 1])));
  }
  return u;
}

}  // namespace rng
}  // namespace md
