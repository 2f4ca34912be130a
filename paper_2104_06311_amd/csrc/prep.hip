// Per-call constellation preparation: label-order permutation, label validation and
// the MFMA A-operand fragments of the score contraction.
//
// Score contraction.  For a symbol y and a point x the demappers need
//   t = -c ||y - x||^2 + bias,  c = log2(e) / (2 sigma2)   (exponent in base 2),
// written as u.w + p a + a r with
//   u = a x,  w = (2c/a) y,  p = -(c/a) ||x||^2,  r = (bias - c ||y||^2)/a
// and a power of two a that balances the magnitudes of both operands.  Every factor is
// split into an FP16 high part and an FP16 low part, and the MFMA's K dimension
// carries the partial products as separate slots (3D + 4 of them):
//   point (A) side:  [ u_hi (D), u_lo (D), u_hi (D), p_hi, p_lo, a, a, 0 ... ]
//   symbol (B) side: [ w_hi (D), w_hi (D), w_lo (D), a,    a,    r_hi, r_lo, 0 ... ]
// so that one FP32-accumulating v_mfma_f32_32x32x16_f16 per 16 slots forms
// u_hi w_hi + u_lo w_hi + u_hi w_lo (the dropped u_lo w_lo is ~2^-22 |u||w|).
//
// Fragment layout.  Points are grouped in tiles of 32 consecutive labels.  Inside a
// tile, MFMA row i (0..31) holds the point whose label offset is
//   p(i) = 16 * ((i / 4) % 2) + 4 * (i / 8) + i % 4,
// chosen so that in the 32x32 MFMA result lane l, register r holds label offset
// 16 * (l / 32) + r: every lane owns 16 consecutive labels of one symbol.
// frag[(tile * KS + ks) * 64 + lane] is the 8-half A operand of that lane: row lane % 32,
// slots 16 ks + 8 (lane / 32) .. +7.
//
// One-pass layouts (the reduced-precision variants of llr_exact): each factor is rounded
// once, to FP16 or to BF16, and the K dimension holds D + 4 slots
//   point (A) side:  [ u (D), p_hi, p_lo, a, a, 0 ... ]
//   symbol (B) side: [ w (D), a,    a,    r_hi, r_lo, 0 ... ]
// (the biases keep a hi/lo split in the same format), so one MFMA per tile serves
// D <= 12 at a score error of about 2^-10 (FP16) or 2^-8 (BF16) of sum_k |u_k w_k|.
#include <cmath>

#include "common.hpp"
#include "llr_kernels.hpp"

namespace md {
namespace {

constexpr int kMaxSlots = 96;   // 16 * frag_ksteps(30)

__global__ void prep_init_kernel(uint32_t* __restrict__ inv, int M, int* __restrict__ flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < M) inv[s] = 0xFFFFFFFFu;
  if (s < 8) flags[s] = 0;
}

__global__ void prep_scatter_kernel(const uint32_t* __restrict__ labels, int M, uint32_t* __restrict__ inv,
                                    int* __restrict__ flags) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const uint32_t l = labels[j];
  if (l >= static_cast<uint32_t>(M)) {
    flags[0] = 1;
    return;
  }
  inv[l] = static_cast<uint32_t>(j);
}

__device__ __forceinline__ void split_half(float v, _Float16* hi, _Float16* lo) {
  const _Float16 h = static_cast<_Float16>(v);
  *hi = h;
  *lo = static_cast<_Float16>(v - static_cast<float>(h));
}

// The BF16 bits of v (round to nearest even), carried in an FP16 slot of the row.
__device__ __forceinline__ _Float16 bf16_bits(float v) {
  return __builtin_bit_cast(_Float16, static_cast<__bf16>(v));
}
__device__ __forceinline__ void split_bf16(float v, _Float16* hi, _Float16* lo) {
  const __bf16 h = static_cast<__bf16>(v);
  *hi = __builtin_bit_cast(_Float16, h);
  *lo = bf16_bits(v - static_cast<float>(h));
}

// One thread per label slot s (padded to a multiple of 32).
__global__ void prep_build_kernel(const float* __restrict__ X, const uint32_t* __restrict__ labels,
                                  const uint32_t* __restrict__ inv, int M, int Mpad, int D, int KS, int sc,
                                  float alpha, float c_over_alpha, float* __restrict__ xl,
                                  uint4* __restrict__ frag, int* __restrict__ flags, float* __restrict__ vx) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Mpad) return;
  if (vx && s < M) {
    // the vector demapper's terms: 2c x (D floats) and -c ||x||^2, FP32 as it computes
    const uint32_t jv = inv[s];
    const bool okv = jv < static_cast<uint32_t>(M) && labels[jv] == static_cast<uint32_t>(s);
    const float c = c_over_alpha * alpha;
    float n32 = 0.0f;
    for (int d = 0; d < D; ++d) {
      const float v = okv ? X[static_cast<int64_t>(jv) * D + d] : 0.0f;
      vx[static_cast<int64_t>(s) * (D + 1) + d] = 2.0f * c * v;
      n32 = fmaf(v, v, n32);
    }
    vx[static_cast<int64_t>(s) * (D + 1) + D] = -c * n32;
  }
  _Float16 row[kMaxSlots];
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k) row[k] = static_cast<_Float16>(0.0f);
  if (s < M) {
    const uint32_t j = inv[s];
    const bool ok = j < static_cast<uint32_t>(M) && labels[j] == static_cast<uint32_t>(s);
    if (!ok) flags[0] = 1;
    double nrm = 0.0;
    bool range = false;
    for (int d = 0; d < D; ++d) {
      const float v = ok ? X[static_cast<int64_t>(j) * D + d] : 0.0f;
      xl[static_cast<int64_t>(s) * D + d] = v;
      nrm += static_cast<double>(v) * static_cast<double>(v);
      const float u = alpha * v;
      range |= !(fabsf(u) <= 30000.0f);
      if (sc == 0) {
        _Float16 hi, lo;
        split_half(u, &hi, &lo);
        row[d] = hi;
        row[D + d] = lo;
        row[2 * D + d] = hi;
      } else {
        row[d] = sc == 1 ? static_cast<_Float16>(u) : bf16_bits(u);
      }
    }
    const float p = -c_over_alpha * static_cast<float>(nrm);
    range |= !(fabsf(p) <= 30000.0f);
    _Float16 hi, lo;
    const int nb = sc == 0 ? 3 * D : D;       // first bias slot
    if (sc == 2) {
      split_bf16(p, &hi, &lo);
      row[nb + 2] = bf16_bits(alpha);
      row[nb + 3] = bf16_bits(alpha);
    } else {
      split_half(p, &hi, &lo);
      row[nb + 2] = static_cast<_Float16>(alpha);
      row[nb + 3] = static_cast<_Float16>(alpha);
    }
    row[nb] = hi;
    row[nb + 1] = lo;
    if (range) flags[2] = 1;          // outside the FP16 split range (or NaN)
  }
  // padded slots (s >= M, only when M < 32) keep an all-zero row; the kernels that use
  // the fragments require M >= 32, so these rows are never read.
  const int tile = s >> 5;
  const int p = s & 31;
  const int h = p >> 4, r = p & 15;
  const int i = 8 * (r >> 2) + 4 * h + (r & 3);
  for (int ks = 0; ks < KS; ++ks) {
    for (int g = 0; g < 2; ++g) {
      uint4 v;
      __builtin_memcpy(&v, &row[16 * ks + 8 * g], 16);
      frag[(static_cast<int64_t>(tile) * KS + ks) * 64 + i + 32 * g] = v;
    }
  }
}

}  // namespace

int frag_ksteps(int D) { return (3 * D + 4 + 15) / 16; }
int frag_ksteps_single(int D) { return (D + 4 + 15) / 16; }

size_t prep_bytes(int M, int D, int64_t N) {
  const int Mpad = ((M + 31) / 32) * 32;
  const int KS = frag_ksteps(D);
  size_t b = 0;
  b += carve_size(sizeof(float) * static_cast<size_t>(M) * D);                 // xl
  b += carve_size(sizeof(uint4) * static_cast<size_t>(Mpad / 32) * KS * 64);      // frag
  b += carve_size(sizeof(uint32_t) * M);                                       // inv
  b += carve_size(sizeof(int) * 8);                                            // flags
  b += 2 * carve_size(sizeof(unsigned) * static_cast<size_t>(N > 0 ? N : 1)); // fallback lists
  if (vec_exact_supported(M, D)) b += carve_size(sizeof(float) * static_cast<size_t>(M) * (D + 1));   // vx
  return b;
}

int prepare(const float* d_X, const uint32_t* d_labels, int M, int D, int64_t N, float alpha,
            float c_over_alpha, char* ws, hipStream_t stream, Prepared* out, int* flags_given, int sc) {
  const int Mpad = ((M + 31) / 32) * 32;
  const int KS = sc == 0 ? frag_ksteps(D) : frag_ksteps_single(D);
  Carver cv{ws, 0};
  float* xl = cv.take<float>(static_cast<size_t>(M) * D);
  uint4* frag = cv.take<uint4>(static_cast<size_t>(Mpad / 32) * KS * 64);
  uint32_t* inv = cv.take<uint32_t>(M);
  int* flags_carved = cv.take<int>(8);
  int* flags = flags_given ? flags_given : flags_carved;
  unsigned* fb = cv.take<unsigned>(static_cast<size_t>(N > 0 ? N : 1));
  unsigned* fb2 = cv.take<unsigned>(static_cast<size_t>(N > 0 ? N : 1));
  float* vx = (sc == 0 && vec_exact_supported(M, D)) ? cv.take<float>(static_cast<size_t>(M) * (D + 1)) : nullptr;
  const int bs = 256;
  hipLaunchKernelGGL(prep_init_kernel, dim3((M + bs - 1) / bs), dim3(bs), 0, stream, inv, M, flags);
  MD_LAUNCH_CHECK("prep_init_kernel launch");
  hipLaunchKernelGGL(prep_scatter_kernel, dim3((M + bs - 1) / bs), dim3(bs), 0, stream, d_labels, M, inv, flags);
  MD_LAUNCH_CHECK("prep_scatter_kernel launch");
  hipLaunchKernelGGL(prep_build_kernel, dim3((Mpad + bs - 1) / bs), dim3(bs), 0, stream, d_X, d_labels, inv, M,
                     Mpad, D, KS, sc, alpha, c_over_alpha, xl, frag, flags, vx);
  MD_LAUNCH_CHECK("prep_build_kernel launch");
  out->xl = xl;
  out->frag = frag;
  out->flags = flags;
  out->fb_list = fb;
  out->fb_list2 = fb2;
  out->vx = vx;
  out->ks = KS;
  out->sc = sc;
  out->alpha = alpha;
  out->c_over_alpha = c_over_alpha;
  return MD_OK;
}

}  // namespace md
