// Learned demapper: a D -> H -> H -> m GELU network trained on (y, exact LLR) pairs by
// the library's own BF16 MFMA kernels, and its inference.
//
//   f(y) = W3 g(W2 g(W1 y + b1) + b2) + b3,  g(a) = a Phi(a)  (GELU; Phi is the standard
//   normal distribution function).
//   loss = mean over the batch of sum_k p_k softplus(-f_k) + (1 - p_k) softplus(f_k),
//   p_k = sigmoid(L_exact_k), so that dloss/df = (sigmoid(f) - p) / B.
//
// Parameters live on the device as one FP32 vector (W1, b1, W2, b2, W3, b3, row-major
// [out][in]) with FP32 Adam moments.  Every product is a BF16 MFMA with FP32
// accumulation: operands are rounded to BF16 when they are staged into LDS.
//
// Training: a tiled GEMM (64x64 block tile, v_mfma_f32_32x32x16_bf16) with fused
// epilogues (bias + GELU storing pre- and post-activation; multiplication by GELU'),
// a loss kernel that also forms dloss/df, column sums for the bias gradients, and
// an elementwise Adam kernel.  Inference (llr_learned) for H <= 256 and D <= 15: one fused
// kernel holds all weights in LDS as BF16 MFMA fragments; each wavefront pushes 32 symbols
// through the three layers, and the hidden units of each layer are ordered so that the
// MFMA result registers of one layer are directly the B operand of the next.  For H up to
// 512 (or D up to 30) the same fragments are used, but the layer-2 weights are streamed
// through LDS one output block at a time; other shapes use the training GEMMs.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "llr_kernels.hpp"

namespace md {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

// GELU, g(a) = a Phi(a).  The upper tail Q(u) = erfc(u / sqrt 2) / 2 at u = |a| comes from
// Abramowitz & Stegun 7.1.26 (Hastings' approximation; its error in erf is below 1.5e-7):
//   erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-x^2),  t = 1 / (1 + p x),  x >= 0,
// so Phi(a) = 1 - Q(|a|) for a >= 0 and Q(|a|) below, with an absolute error under 1e-7.
// The derivative g'(a) = Phi(a) + a phi(a) reuses the same e^(-a^2/2).  The coefficients
// below are A&S's halved (Q = erfc / 2) and p / sqrt 2 (x = |a| / sqrt 2).
constexpr float kAsP = static_cast<float>(0.3275911 / 1.4142135623730951);
constexpr float kAs1 = 0.5f * 0.254829592f;
constexpr float kAs2 = 0.5f * -0.284496736f;
constexpr float kAs3 = 0.5f * 1.421413741f;
constexpr float kAs4 = 0.5f * -1.453152027f;
constexpr float kAs5 = 0.5f * 1.061405429f;
constexpr float kHalfLog2e = -0.72134752044448170f;   // -log2(e) / 2
constexpr float kInvSqrt2Pi = 0.39894228040143268f;  // 1 / sqrt(2 pi)

// Phi(a) and e^(-a^2/2); Phi is exactly 0 or 1 once the exponential underflows.
__device__ __forceinline__ float normal_cdf(float a, float* ex) {
  const float t = __builtin_amdgcn_rcpf(fmaf(kAsP, fabsf(a), 1.0f));
  const float e = __builtin_amdgcn_exp2f(kHalfLog2e * (a * a));
  const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, kAs5, kAs4), kAs3), kAs2), kAs1);
  const float q = poly * e;
  *ex = e;
  return a >= 0.0f ? 1.0f - q : q;
}
__device__ __forceinline__ float gelu(float a) {
  float e;
  return a * normal_cdf(a, &e);
}
__device__ __forceinline__ float gelu_grad(float a) {
  float e;
  const float p = normal_cdf(a, &e);
  return fmaf(a * kInvSqrt2Pi, e, p);
}
__device__ __forceinline__ float softplusf(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }
__device__ __forceinline__ float sigmoidf_acc(float t) {
  return t >= 0.0f ? 1.0f / (1.0f + expf(-t)) : expf(t) / (1.0f + expf(t));
}

// ------------------------------------------------------------------ generic GEMM
// C[i][j] = sum_k A(i,k) B(k,j), A(i,k) = A[i*sar + k*sac], B(k,j) = B[k*sbr + j*sbc]
// (FP32 in memory, BF16 in the MFMA), C row-major with leading dimension ldc.
enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

template <int EPI>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(const float* __restrict__ A, int64_t sar, int64_t sac,
                                                        const float* __restrict__ B, int64_t sbr, int64_t sbc,
                                                        int M, int N, int K, float* __restrict__ C, int64_t ldc,
                                                        const float* __restrict__ bias, float* __restrict__ C2,
                                                        const float* __restrict__ Z, float ascale, float bscale,
                                                        float cscale) {
  // K is staged 64 at a time (four 16-deep products per wavefront per barrier pair); the
  // next stage is read from global memory into registers while the current one is
  // multiplied.  Rows of the LDS tiles are padded to 144 bytes (9 x 16), so the 16-byte
  // fragment reads of 32 consecutive rows hit distinct banks.
  constexpr int KT = 64;
  __shared__ __attribute__((aligned(16))) __bf16 As[64][KT + 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[64][KT + 8];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // split K: slice z of gridDim.z covers [kb, ke) and writes its own partial product
  const int kper = ((K + 15) / 16 + gridDim.z - 1) / gridDim.z * 16;
  const int kb = blockIdx.z * kper;
  const int ke = min(K, kb + kper);
  C += static_cast<int64_t>(blockIdx.z) * M * ldc;
  // staging map of element e of this thread: consecutive threads take consecutive k when
  // the operand's k stride is 1, consecutive rows otherwise (coalesced either way)
  const bool a_kfast = sac == 1, b_kfast = sbr == 1;
  auto coord = [&](bool kfast, int e, int* r, int* kk) {
    const int idx = tid + 256 * e;
    *r = kfast ? idx >> 6 : idx & 63;
    *kk = kfast ? idx & 63 : idx >> 6;
  };
  float ra[16], rb[16];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      int r, kk;
      coord(a_kfast, e, &r, &kk);
      const int gi = i0 + r, gka = k0 + kk;
      ra[e] = (gi < M && gka < ke) ? A[gi * sar + gka * sac] : 0.0f;
      coord(b_kfast, e, &r, &kk);
      const int gj = j0 + r, gkb = k0 + kk;
      rb[e] = (gj < N && gkb < ke) ? B[gkb * sbr + gj * sbc] : 0.0f;
    }
  };
  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  if (kb < ke) load_stage(kb);
  for (int k0 = kb; k0 < ke; k0 += KT) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      int r, kk;
      coord(a_kfast, e, &r, &kk);
      As[r][kk] = static_cast<__bf16>(ra[e] * ascale);
      coord(b_kfast, e, &r, &kk);
      Bs[r][kk] = static_cast<__bf16>(rb[e] * bscale);
    }
    __syncthreads();
    if (k0 + KT < ke) load_stage(k0 + KT);
#pragma unroll
    for (int sst = 0; sst < KT / 16; ++sst) {
      if (k0 + 16 * sst < ke) {
        bf16x8 a, b;
        __builtin_memcpy(&a, &As[wi + (lane & 31)][16 * sst + 8 * h], 16);
        __builtin_memcpy(&b, &Bs[wj + (lane & 31)][16 * sst + 8 * h], 16);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int j = j0 + wj + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = i0 + wi + 8 * (r >> 2) + 4 * h + (r & 3);
    if (i < M && j < N) {
      float v = acc[r];
      const int64_t o = static_cast<int64_t>(i) * ldc + j;
      if (EPI == EPI_STORE) {
        if (bias) v += bias[j];
        C[o] = v * cscale;
      } else if (EPI == EPI_BIAS_GELU) {
        v += bias[j];
        C[o] = v;
        C2[o] = gelu(v);
      } else {
        C[o] = v * gelu_grad(Z[o]);
      }
    }
  }
}

// ascale / bscale multiply the A / B values as they are staged, cscale the stored result
// (EPI_STORE): the network's fixed input and output scales.
template <int EPI>
int gemm(const float* A, int64_t sar, int64_t sac, const float* B, int64_t sbr, int64_t sbc, int M, int N, int K,
         float* C, int64_t ldc, const float* bias, float* C2, const float* Z, hipStream_t s, float ascale = 1.0f,
         float bscale = 1.0f, float cscale = 1.0f) {
  dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
  hipLaunchKernelGGL(gemm_bf16_kernel<EPI>, grid, dim3(256), 0, s, A, sar, sac, B, sbr, sbc, M, N, K, C, ldc, bias,
                     C2, Z, ascale, bscale, cscale);
  MD_LAUNCH_CHECK("gemm_bf16_kernel launch");
  return MD_OK;
}

// Sums the `slices` partial products of a split-K GEMM in a fixed order.
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const float* __restrict__ part, int slices, int64_t n,
                                                            float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.0f;
  for (int z = 0; z < slices; ++z) acc += part[z * n + i];
  out[i] = acc;
}

constexpr int kSplitK = 16;

// Weight-gradient products (small M x N, K = batch): K split over kSplitK slices so
// that the grid covers the chip, partials in `part` (kSplitK * M * N floats).
int gemm_splitk(const float* A, int64_t sar, int64_t sac, const float* B, int64_t sbr, int64_t sbc, int M, int N,
                int K, float* C, float* part, hipStream_t s, float bscale = 1.0f) {
  dim3 grid((N + 63) / 64, (M + 63) / 64, kSplitK);
  hipLaunchKernelGGL(gemm_bf16_kernel<EPI_STORE>, grid, dim3(256), 0, s, A, sar, sac, B, sbr, sbc, M, N, K, part,
                     static_cast<int64_t>(N), nullptr, nullptr, nullptr, 1.0f, bscale, 1.0f);
  MD_LAUNCH_CHECK("gemm_bf16_kernel (split K) launch");
  const int64_t n = static_cast<int64_t>(M) * N;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, part,
                     kSplitK, n, C);
  MD_LAUNCH_CHECK("splitk_reduce_kernel launch");
  return MD_OK;
}

// ------------------------------------------------------------------ loss, bias grads, Adam
// One thread per sample: loss terms of z = oscale f and dloss/df = oscale (sigmoid(z) - sigmoid(L)) / B.
// partials[block] = sum of the block's per-sample losses (FP64, fixed order).
__global__ void __launch_bounds__(256) loss_grad_kernel(const float* __restrict__ f, const float* __restrict__ tgt,
                                                        int64_t B, int m, float oscale, float* __restrict__ df,
                                                        double* __restrict__ partials) {
  __shared__ double sh[256];
  double acc = 0.0;
  const int64_t b = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (b < B) {
    const float invB = 1.0f / static_cast<float>(B);
    for (int k = 0; k < m; ++k) {
      const float z = oscale * f[b * m + k];       // the network output is oscale times the last layer
      const float p = sigmoidf_acc(tgt[b * m + k]);
      acc += static_cast<double>(p * softplusf(-z) + (1.0f - p) * softplusf(z));
      df[b * m + k] = (sigmoidf_acc(z) - p) * (oscale * invB);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void loss_final_kernel(const double* __restrict__ partials, int nb, int64_t B, double* __restrict__ loss) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) a += partials[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = sh[0] / static_cast<double>(B);
}

// Column sums out[j] = sum_b G[b][j] in two deterministic stages: block (x, slice) sums the
// rows of one slice for 64 columns (4 row lanes of compensated sums, combined in a fixed
// order), then one thread per column adds the slice partials in order.
constexpr int kColSlices = 32;

__global__ void __launch_bounds__(256) colsum_partial_kernel(const float* __restrict__ G, int64_t B, int n,
                                                             float* __restrict__ partial) {
  __shared__ float sh[4][64];
  const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  const int64_t per = (B + kColSlices - 1) / kColSlices;
  const int64_t b0 = static_cast<int64_t>(blockIdx.y) * per;
  const int64_t b1 = min(B, b0 + per);
  float s = 0.0f, comp = 0.0f;
  if (j < n) {
    for (int64_t b = b0 + r; b < b1; b += 4) {
      const float x = G[b * n + j];
      const float t = s + x;
      comp += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
      s = t;
    }
  }
  sh[r][c] = s + comp;
  __syncthreads();
  if (r == 0 && j < n)
    partial[static_cast<int64_t>(blockIdx.y) * n + j] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
}

__global__ void __launch_bounds__(256) colsum_final_kernel(const float* __restrict__ partial, int n,
                                                           float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float s = 0.0f, comp = 0.0f;
  for (int q = 0; q < kColSlices; ++q) {
    const float x = partial[static_cast<int64_t>(q) * n + j];
    const float t = s + x;
    comp += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  out[j] = s + comp;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; w -= lr m^ / (sqrt(v^) + eps)
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, int64_t P, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Gathers the rows idx[b] of y (D columns) and t (m columns) into contiguous batches.
__global__ void gather_kernel(const float* __restrict__ y, const float* __restrict__ t, int D, int m, int64_t N,
                              uint64_t seed, uint64_t step, int64_t B, float* __restrict__ yb,
                              float* __restrict__ tb) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;
  // index = floor(u * N / 2^32) from a 64-bit mix of (seed, step, b): uniform up to N / 2^32
  uint64_t x = seed ^ (step * 0x9E3779B97F4A7C15ull) ^ (static_cast<uint64_t>(b) * 0xD1B54A32D192ED03ull);
  x ^= x >> 31;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 29;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 32;
  const int64_t idx = static_cast<int64_t>(((x & 0xFFFFFFFFull) * static_cast<uint64_t>(N)) >> 32);
  for (int d = 0; d < D; ++d) yb[b * D + d] = y[idx * D + d];
  for (int k = 0; k < m; ++k) tb[b * m + k] = t[idx * m + k];
}

// ------------------------------------------------------------------ fused inference
// LDS image (BF16 fragments, built by pack_infer_kernel from the FP32 master weights):
//   f1[rb][s][lane]        layer 1, hidden rows 32 rb + lane % 32, K slots 16 s + 8 (lane/32)
//                          .. +7 of [y (D), 1 (bias), 0 ...], s < ks1 = ceil((D + 1) / 16)
//   f2[ob][rb][q][lane]    layer 2: output rows 32 ob + lane % 32, input units of K step
//                          (rb, q) in the order of the layer-1 result registers
//   f3[rb][q][lane]        layer 3, output rows lane % 32 (rows >= m are zero)
//   b2[H], b3[32]          FP32 biases
// The K slot kk = 8 h + v of step (rb, q) is hidden unit 32 rb + 8 (2q + v/4) + 4h + v%4,
// exactly the unit that lane half h holds in register 8q + v of block rb.
__device__ __forceinline__ int unit_of_slot(int rb, int q, int kk) {
  const int hh = kk >> 3, v = kk & 7;
  return 32 * rb + 8 * (2 * q + (v >> 2)) + 4 * hh + (v & 3);
}

__device__ __forceinline__ floatx16 zero16() {
  floatx16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.0f;
  return z;
}
// One 32x32x16 BF16 product; the A fragment is read from LDS.
__device__ __forceinline__ floatx16 mfma_bf16(const uint4& a_lds, const bf16x8& b, const floatx16& c) {
  bf16x8 a;
  __builtin_memcpy(&a, &a_lds, 16);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

struct InferLayout {
  int H, nrb, ks1;                      // hidden width, H / 32, layer-1 K steps of 16 slots
  size_t f1, f2, f3, b2, b3, bytes;     // byte offsets
};

inline InferLayout infer_layout(int H, int D) {
  InferLayout L;
  L.H = H;
  L.nrb = H / 32;
  L.ks1 = (D + 1 + 15) / 16;
  size_t o = 0;
  L.f1 = o;
  o += static_cast<size_t>(L.nrb) * L.ks1 * 64 * 16;
  L.f2 = o;
  o += static_cast<size_t>(L.nrb) * L.nrb * 2 * 64 * 16;
  L.f3 = o;
  o += static_cast<size_t>(L.nrb) * 2 * 64 * 16;
  L.b2 = o;
  o += static_cast<size_t>(H) * 4;
  L.b3 = o;
  o += 32 * 4;
  L.bytes = o;
  return L;
}

__global__ void pack_infer_kernel(const float* __restrict__ w, int D, int H, int m, InferLayout L,
                                  char* __restrict__ img) {
  const int nrb = L.nrb;
  const float* W1 = w;
  const float* b1 = W1 + static_cast<int64_t>(H) * D;
  const float* W2 = b1 + H;
  const float* b2 = W2 + static_cast<int64_t>(H) * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + static_cast<int64_t>(m) * H;
  const int64_t n1 = static_cast<int64_t>(nrb) * L.ks1 * 64;
  const int64_t n2 = static_cast<int64_t>(nrb) * nrb * 2 * 64;
  const int64_t n3 = static_cast<int64_t>(nrb) * 2 * 64;
  const int64_t total = n1 + n2 + n3 + H + 32;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (t < n1) {
      const int rb = static_cast<int>(t / (64 * L.ks1)), st = static_cast<int>((t / 64) % L.ks1);
      const int lane = static_cast<int>(t % 64);
      const int row = 32 * rb + (lane & 31), hh = lane >> 5;
      __bf16 v8[8];
      for (int v = 0; v < 8; ++v) {
        const int k = 16 * st + 8 * hh + v;
        const float x = k < D ? W1[static_cast<int64_t>(row) * D + k] : (k == D ? b1[row] : 0.0f);
        v8[v] = static_cast<__bf16>(x);
      }
      __builtin_memcpy(img + L.f1 + t * 16, v8, 16);
    } else if (t < n1 + n2) {
      const int64_t u = t - n1;
      const int lane = static_cast<int>(u % 64);
      const int q = static_cast<int>((u / 64) % 2);
      const int rb = static_cast<int>((u / 128) % nrb);
      const int ob = static_cast<int>(u / (128 * nrb));
      const int row = 32 * ob + (lane & 31), hh = lane >> 5;
      __bf16 v8[8];
      for (int v = 0; v < 8; ++v)
        v8[v] = static_cast<__bf16>(W2[static_cast<int64_t>(row) * H + unit_of_slot(rb, q, 8 * hh + v)]);
      __builtin_memcpy(img + L.f2 + u * 16, v8, 16);
    } else if (t < n1 + n2 + n3) {
      const int64_t u = t - n1 - n2;
      const int lane = static_cast<int>(u % 64);
      const int q = static_cast<int>((u / 64) % 2);
      const int rb = static_cast<int>(u / 128);
      const int row = lane & 31, hh = lane >> 5;
      __bf16 v8[8];
      for (int v = 0; v < 8; ++v)
        v8[v] = static_cast<__bf16>(row < m ? W3[static_cast<int64_t>(row) * H + unit_of_slot(rb, q, 8 * hh + v)]
                                            : 0.0f);
      __builtin_memcpy(img + L.f3 + u * 16, v8, 16);
    } else if (t < n1 + n2 + n3 + H) {
      const int64_t i = t - n1 - n2 - n3;
      reinterpret_cast<float*>(img + L.b2)[i] = b2[i];
    } else {
      const int64_t i = t - n1 - n2 - n3 - H;
      reinterpret_cast<float*>(img + L.b3)[i] = i < m ? b3[i] : 0.0f;
    }
  }
}

template <int NRB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2))) mlp_infer_kernel(const char* __restrict__ img, InferLayout L, int D, int m,
                                                        const float* __restrict__ y, int64_t N, float in_scale,
                                                        float out_scale, float* __restrict__ llr) {
  extern __shared__ uint4 smem[];
  char* lds = reinterpret_cast<char*>(smem);
  for (size_t i = threadIdx.x; i < L.bytes / 16; i += blockDim.x)
    smem[i] = reinterpret_cast<const uint4*>(img)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int h = lane >> 5;
  const uint4* f1 = reinterpret_cast<const uint4*>(lds + L.f1);
  const uint4* f2 = reinterpret_cast<const uint4*>(lds + L.f2);
  const uint4* f3 = reinterpret_cast<const uint4*>(lds + L.f3);
  const float* b2 = reinterpret_cast<const float*>(lds + L.b2);
  const float* b3 = reinterpret_cast<const float*>(lds + L.b3);
  const int64_t ntile = (N + 31) / 32;
  for (int64_t tile = static_cast<int64_t>(blockIdx.x) * nw + wave; tile < ntile;
       tile += static_cast<int64_t>(gridDim.x) * nw) {
    const int64_t n = tile * 32 + (lane & 31);
    const bool live = n < N;
    // layer-1 B operand: [y (D), 1, 0 ...], lane half h holds K slots 8h .. 8h+7
    bf16x8 yb;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int k = 8 * h + v;
      const float x = (k < D) ? (live ? y[n * D + k] * in_scale : 0.0f) : (k == D ? 1.0f : 0.0f);
      yb[v] = static_cast<__bf16>(x);
    }
    // Layer 1 and the first block of layer 2.  The product of hidden block rb + 1 is issued
    // before the activations of block rb are formed, and each block's activations enter the
    // first layer-2 accumulation right away, so that matrix products and activations overlap.
    bf16x8 act[NRB][2];
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = b2[8 * (r >> 2) + 4 * h + (r & 3)];
    floatx16 h1 = mfma_bf16(f1[lane], yb, zero16());
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      floatx16 h1n;
      if (rb + 1 < NRB) h1n = mfma_bf16(f1[(rb + 1) * 64 + lane], yb, zero16());
#pragma unroll
      for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int v = 0; v < 8; ++v) act[rb][q][v] = static_cast<__bf16>(gelu(h1[8 * q + v]));
        acc = mfma_bf16(f2[(rb * 2 + q) * 64 + lane], act[rb][q], acc);
      }
      if (rb + 1 < NRB) h1 = h1n;
      __builtin_amdgcn_sched_barrier(0);   // keeps one hidden block in flight (no spills)
    }
    // Layer 2 block ob is accumulated while the activations of block ob - 1 are formed and
    // pushed through layer 3.
    floatx16 out;
#pragma unroll
    for (int r = 0; r < 16; ++r) out[r] = b3[8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll 1
    for (int ob = 1; ob < NRB; ++ob) {
      floatx16 nxt;
#pragma unroll
      for (int r = 0; r < 16; ++r) nxt[r] = b2[32 * ob + 8 * (r >> 2) + 4 * h + (r & 3)];
      // all A fragments of this block are requested before the first product, so that LDS
      // latency is paid once per block rather than once per product
      const uint4* f2o = f2 + ob * NRB * 2 * 64 + lane;
      uint4 fa[NRB][2];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int q = 0; q < 2; ++q) fa[rb][q] = f2o[(rb * 2 + q) * 64];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int q = 0; q < 2; ++q) nxt = mfma_bf16(fa[rb][q], act[rb][q], nxt);
      const uint4* f3o = f3 + (ob - 1) * 2 * 64 + lane;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bf16x8 act2;
#pragma unroll
        for (int v = 0; v < 8; ++v) act2[v] = static_cast<__bf16>(gelu(acc[8 * q + v]));
        out = mfma_bf16(f3o[q * 64], act2, out);
      }
      acc = nxt;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bf16x8 act2;
#pragma unroll
      for (int v = 0; v < 8; ++v) act2[v] = static_cast<__bf16>(gelu(acc[8 * q + v]));
      out = mfma_bf16(f3[((NRB - 1) * 2 + q) * 64 + lane], act2, out);
    }
    if (live) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = 8 * (r >> 2) + 4 * h + (r & 3);
        if (k < m) llr[n * m + k] = out[r] * out_scale;
      }
    }
  }
}

// Inference for wider networks (H up to 512, D up to 31), whose layer-2 weights do not fit
// in LDS.  A block of 8 wavefronts (256 symbols) keeps layer 1, layer 3 and the biases in
// LDS and streams the layer-2 fragments one output block (32 rows, 2 H / 32 fragments) at a
// time through two LDS buffers: while block ob is multiplied out of one buffer, block ob + 1
// is loaded into the other, with one barrier per block.  The sequence of blocks continues
// across symbol tiles (block 0 of the next tile follows block NRB - 1), so buffer j mod 2
// always holds the j-th block of the block's stream.  Layer-1 activations of the
// wavefront's 32 symbols stay in registers (H / 4 per lane).
template <int NRB>
__device__ __forceinline__ void stream_request(const uint4* __restrict__ g2, int ob, uint4 (&pre)[(NRB * 128 + 511) / 512]) {
  constexpr int kChunk = NRB * 2 * 64;
#pragma unroll
  for (int i = 0; i < (kChunk + 511) / 512; ++i) {
    const int idx = min(static_cast<int>(threadIdx.x) + 512 * i, kChunk - 1);   // in range; stored only if < kChunk
    pre[i] = g2[static_cast<int64_t>(ob) * kChunk + idx];
  }
}
template <int NRB>
__device__ __forceinline__ void stream_store(uint4* __restrict__ dst, const uint4 (&pre)[(NRB * 128 + 511) / 512]) {
  constexpr int kChunk = NRB * 2 * 64;
#pragma unroll
  for (int i = 0; i < (kChunk + 511) / 512; ++i) {
    const int idx = static_cast<int>(threadIdx.x) + 512 * i;
    if (idx < kChunk) dst[idx] = pre[i];
  }
}

template <int NRB, int KS1>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
mlp_infer_stream_kernel(const char* __restrict__ img, InferLayout L, int D, int m, const float* __restrict__ y,
                        int64_t N, float in_scale, float out_scale, float* __restrict__ llr) {
  constexpr int kChunk = NRB * 2 * 64;              // uint4 per layer-2 output block
  constexpr int kPre = (kChunk + 511) / 512;
  extern __shared__ uint4 smem[];
  const int s1 = NRB * KS1 * 64;                    // layer-1 fragments (uint4)
  const int s3 = static_cast<int>((L.bytes - L.f3) / 16);   // layer-3 fragments and biases
  uint4* lf1 = smem;
  uint4* lf3 = smem + s1;
  uint4* lch = smem + s1 + s3;                      // two buffers of kChunk
  const uint4* g1 = reinterpret_cast<const uint4*>(img + L.f1);
  const uint4* g2 = reinterpret_cast<const uint4*>(img + L.f2);
  const uint4* g3 = reinterpret_cast<const uint4*>(img + L.f3);
  for (int i = threadIdx.x; i < s1; i += 512) lf1[i] = g1[i];
  for (int i = threadIdx.x; i < s3; i += 512) lf3[i] = g3[i];
  {
    uint4 pre[kPre];
    stream_request<NRB>(g2, 0, pre);
    stream_store<NRB>(lch, pre);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const float* b2 = reinterpret_cast<const float*>(lf3 + NRB * 2 * 64);
  const float* b3 = b2 + 32 * NRB;
  const int64_t nbt = (N + 255) / 256;
  int buf = 0;
  for (int64_t bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
    const int64_t n = bt * 256 + wave * 32 + (lane & 31);
    const bool live = n < N;
    bf16x8 yb[KS1];
#pragma unroll
    for (int st = 0; st < KS1; ++st)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int k = 16 * st + 8 * h + v;
        const float x = (k < D) ? (live ? y[n * D + k] * in_scale : 0.0f) : (k == D ? 1.0f : 0.0f);
        yb[st][v] = static_cast<__bf16>(x);
      }
    bf16x8 act[NRB][2];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      floatx16 h1 = zero16();
#pragma unroll
      for (int st = 0; st < KS1; ++st) h1 = mfma_bf16(lf1[(rb * KS1 + st) * 64 + lane], yb[st], h1);
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 8; ++v) act[rb][q][v] = static_cast<__bf16>(gelu(h1[8 * q + v]));
      __builtin_amdgcn_sched_barrier(0);
    }
    floatx16 out, acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) out[r] = b3[8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll 1
    for (int ob = 0; ob < NRB; ++ob) {
      // the next block of the stream: block ob + 1 of this tile, or block 0 of the next
      uint4 pre[kPre];
      stream_request<NRB>(g2, ob + 1 < NRB ? ob + 1 : 0, pre);
      floatx16 nxt;
#pragma unroll
      for (int r = 0; r < 16; ++r) nxt[r] = b2[32 * ob + 8 * (r >> 2) + 4 * h + (r & 3)];
      const uint4* cb = lch + buf * kChunk + lane;
#pragma unroll
      for (int g = 0; g < NRB; g += 4) {
        // four hidden blocks (eight fragments) requested together
        uint4 fa[4][2];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (g + rb < NRB) fa[rb][q] = cb[((g + rb) * 2 + q) * 64];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (g + rb < NRB) nxt = mfma_bf16(fa[rb][q], act[g + rb][q], nxt);
      }
      if (ob > 0) {
        const uint4* f3o = lf3 + (ob - 1) * 2 * 64 + lane;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          bf16x8 act2;
#pragma unroll
          for (int v = 0; v < 8; ++v) act2[v] = static_cast<__bf16>(gelu(acc[8 * q + v]));
          out = mfma_bf16(f3o[q * 64], act2, out);
        }
      }
      acc = nxt;
      stream_store<NRB>(lch + (buf ^ 1) * kChunk, pre);
      __syncthreads();
      buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bf16x8 act2;
#pragma unroll
      for (int v = 0; v < 8; ++v) act2[v] = static_cast<__bf16>(gelu(acc[8 * q + v]));
      out = mfma_bf16(lf3[((NRB - 1) * 2 + q) * 64 + lane], act2, out);
    }
    if (live) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = 8 * (r >> 2) + 4 * h + (r & 3);
        if (k < m) llr[n * m + k] = out[r] * out_scale;
      }
    }
  }
}

// ------------------------------------------------------------------ initialisation
// Philox4x32-10 on the host for the initial weights (uniform in +-1/sqrt(fan_in)).
void philox_host(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = 0xD2511F53ull * c0, p1 = 0xCD9E8D57ull * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = static_cast<uint32_t>(p1);
    c2 = n2;
    c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

}  // namespace

// ------------------------------------------------------------------ handle
struct Mlp {
  int D = 0, H = 0, m = 0;
  int64_t P = 0;
  int device = 0;
  int64_t step = 0;
  uint64_t seed = 0;
  float* w = nullptr;     // FP32 parameters
  float* g = nullptr;     // gradients
  float* m1 = nullptr;    // Adam first moment
  float* m2 = nullptr;    // Adam second moment
  char* img = nullptr;    // inference image
  int64_t img_version = -1;
  int64_t version = 0;    // bumped whenever w changes
  float* scratch = nullptr;
  size_t scratch_cap = 0;
  float in_scale = 1.0f;  // fixed input scale: the first layer sees in_scale * y
  float out_scale = 1.0f; // fixed output scale: f = out_scale * (last layer)
};

namespace {

int64_t param_count(int D, int H, int m) {
  return static_cast<int64_t>(H) * D + H + static_cast<int64_t>(H) * H + H + static_cast<int64_t>(m) * H + m;
}

int check_handle(const Mlp* p) {
  if (!p) return fail(MD_EINVAL, "MLP handle is NULL");
  return MD_OK;
}

int ensure_scratch(Mlp* p, size_t floats) {
  if (p->scratch_cap >= floats) return MD_OK;
  if (p->scratch) {
    MD_HIP_TRY(hipDeviceSynchronize());
    MD_HIP_TRY(md::dev_free(p->scratch));
    p->scratch = nullptr;
    p->scratch_cap = 0;
  }
  void* q = nullptr;
  if (md::dev_malloc(&q, floats * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MD_ENOMEM, "MLP scratch allocation failed");
  }
  p->scratch = static_cast<float*>(q);
  p->scratch_cap = floats;
  return MD_OK;
}

void init_params(int D, int H, int m, uint64_t seed, std::vector<float>* out) {
  out->resize(static_cast<size_t>(param_count(D, H, m)));
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  int64_t idx = 0;
  auto fill = [&](int64_t count, int fan_in) {
    const float bound = 1.0f / std::sqrt(static_cast<float>(fan_in));
    for (int64_t i = 0; i < count; ++i, ++idx) {
      uint32_t r[4];
      philox_host(static_cast<uint32_t>(idx), static_cast<uint32_t>(idx >> 32), 0u, 3u, k0, k1, r);
      const float u = (static_cast<float>(r[0] >> 8) + 0.5f) * (1.0f / 16777216.0f);   // (0, 1)
      (*out)[static_cast<size_t>(idx)] = (2.0f * u - 1.0f) * bound;
    }
  };
  fill(static_cast<int64_t>(H) * D, D);
  fill(H, D);
  fill(static_cast<int64_t>(H) * H, H);
  fill(H, H);
  fill(static_cast<int64_t>(m) * H, H);
  fill(m, H);
}

int colsum(const float* G, int64_t B, int n, float* partial, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((n + 63) / 64, kColSlices), dim3(256), 0, s, G, B, n, partial);
  MD_LAUNCH_CHECK("colsum_partial_kernel launch");
  hipLaunchKernelGGL(colsum_final_kernel, dim3((n + 255) / 256), dim3(256), 0, s, partial, n, out);
  MD_LAUNCH_CHECK("colsum_final_kernel launch");
  return MD_OK;
}

// forward (saving activations) + loss + backward into p->g.  Scratch layout for a batch B:
// Z1, A1, Z2, A2 (B x H each), F, dF (B x m), dZ2, dZ1 (B x H), loss partials.
int forward_backward(Mlp* p, const float* d_y, const float* d_t, int64_t B, double* d_loss, hipStream_t s) {
  const int D = p->D, H = p->H, m = p->m;
  const size_t BH = static_cast<size_t>(B) * H, Bm = static_cast<size_t>(B) * m;
  const int nb = static_cast<int>((B + 255) / 256);
  const size_t colpart = static_cast<size_t>(kColSlices) * (H > m ? H : m);
  const size_t kpart = static_cast<size_t>(kSplitK) * H * (H > D ? (H > m ? H : m) : D);
  int st = ensure_scratch(p, 6 * BH + 2 * Bm + 2 * static_cast<size_t>(nb) + 64 + colpart + kpart);
  if (st != MD_OK) return st;
  float* Z1 = p->scratch;
  float* A1 = Z1 + BH;
  float* Z2 = A1 + BH;
  float* A2 = Z2 + BH;
  float* F = A2 + BH;
  float* dF = F + Bm;
  float* dZ2 = dF + Bm;
  float* dZ1 = dZ2 + BH;
  double* part = reinterpret_cast<double*>(dZ1 + BH);     // 6 BH + 2 Bm floats: 8-byte aligned
  float* cpart = reinterpret_cast<float*>(part + nb + 32);
  float* kpartb = cpart + colpart;
  const float* W1 = p->w;
  const float* b1 = W1 + static_cast<int64_t>(H) * D;
  const float* W2 = b1 + H;
  const float* b2 = W2 + static_cast<int64_t>(H) * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + static_cast<int64_t>(m) * H;
  float* gW1 = p->g;
  float* gb1 = gW1 + static_cast<int64_t>(H) * D;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + static_cast<int64_t>(H) * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + static_cast<int64_t>(m) * H;
  const int Bi = static_cast<int>(B);
  // forward: Z1 = Y W1^T + b1, A1 = g(Z1); Z2 = A1 W2^T + b2, A2 = g(Z2); F = A2 W3^T + b3
  if ((st = gemm<EPI_BIAS_GELU>(d_y, D, 1, W1, 1, D, Bi, H, D, Z1, H, b1, A1, nullptr, s, p->in_scale))) return st;
  if ((st = gemm<EPI_BIAS_GELU>(A1, H, 1, W2, 1, H, Bi, H, H, Z2, H, b2, A2, nullptr, s))) return st;
  if ((st = gemm<EPI_STORE>(A2, H, 1, W3, 1, H, Bi, m, H, F, m, b3, nullptr, nullptr, s))) return st;
  hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(256), 0, s, F, d_t, B, m, p->out_scale, dF, part);
  MD_LAUNCH_CHECK("loss_grad_kernel launch");
  if (d_loss) {
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, part, nb, B, d_loss);
    MD_LAUNCH_CHECK("loss_final_kernel launch");
  }
  // backward
  // gW3 = dF^T A2 (m x H); gb3 = colsum dF
  if ((st = gemm_splitk(dF, 1, m, A2, H, 1, m, H, Bi, gW3, kpartb, s))) return st;
  if ((st = colsum(dF, B, m, cpart, gb3, s))) return st;
  // dZ2 = (dF W3) * g'(Z2)   (B x H)
  if ((st = gemm<EPI_GELU_GRAD>(dF, m, 1, W3, H, 1, Bi, H, m, dZ2, H, nullptr, nullptr, Z2, s))) return st;
  // gW2 = dZ2^T A1 (H x H); gb2 = colsum dZ2
  if ((st = gemm_splitk(dZ2, 1, H, A1, H, 1, H, H, Bi, gW2, kpartb, s))) return st;
  if ((st = colsum(dZ2, B, H, cpart, gb2, s))) return st;
  // dZ1 = (dZ2 W2) * g'(Z1)
  if ((st = gemm<EPI_GELU_GRAD>(dZ2, H, 1, W2, H, 1, Bi, H, H, dZ1, H, nullptr, nullptr, Z1, s))) return st;
  // gW1 = dZ1^T Y (H x D); gb1 = colsum dZ1
  if ((st = gemm_splitk(dZ1, 1, H, d_y, D, 1, H, D, Bi, gW1, kpartb, s, p->in_scale))) return st;
  if ((st = colsum(dZ1, B, H, cpart, gb1, s))) return st;
  return MD_OK;
}

int adam(Mlp* p, float lr, hipStream_t s) {
  p->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(p->step)));
  const float c2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(p->step)));
  hipLaunchKernelGGL(adam_kernel, dim3(static_cast<unsigned>((p->P + 255) / 256)), dim3(256), 0, s, p->w, p->g,
                     p->m1, p->m2, p->P, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
  MD_LAUNCH_CHECK("adam_kernel launch");
  p->version += 1;
  return MD_OK;
}

// Generic-GEMM inference (any H): the forward pass of training without the loss.
int infer_gemm(Mlp* p, const float* d_y, int64_t N, float* d_llr, hipStream_t s) {
  const int D = p->D, H = p->H, m = p->m;
  const int64_t chunk = 1 << 16;
  int st = ensure_scratch(p, static_cast<size_t>(4 * chunk * H));
  if (st != MD_OK) return st;
  const float* W1 = p->w;
  const float* b1 = W1 + static_cast<int64_t>(H) * D;
  const float* W2 = b1 + H;
  const float* b2 = W2 + static_cast<int64_t>(H) * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + static_cast<int64_t>(m) * H;
  float* Z = p->scratch;
  float* A1 = Z + chunk * H;
  float* A2 = A1 + chunk * H;
  for (int64_t n0 = 0; n0 < N; n0 += chunk) {
    const int nb = static_cast<int>(N - n0 < chunk ? N - n0 : chunk);
    if ((st = gemm<EPI_BIAS_GELU>(d_y + n0 * D, D, 1, W1, 1, D, nb, H, D, Z, H, b1, A1, nullptr, s, p->in_scale)))
      return st;
    if ((st = gemm<EPI_BIAS_GELU>(A1, H, 1, W2, 1, H, nb, H, H, Z, H, b2, A2, nullptr, s))) return st;
    if ((st = gemm<EPI_STORE>(A2, H, 1, W3, 1, H, nb, m, H, d_llr + n0 * m, m, b3, nullptr, nullptr, s, 1.0f, 1.0f,
                              p->out_scale)))
      return st;
  }
  return MD_OK;
}

template <int NRB>
int infer_fused_t(Mlp* p, const float* d_y, int64_t N, float* d_llr, hipStream_t s) {
  const InferLayout L = infer_layout(p->H, p->D);
  auto kern = mlp_infer_kernel<NRB>;
  {
    const int st_attr = set_lds_limit(reinterpret_cast<const void*>(kern), 160 * 1024);
    if (st_attr != MD_OK) return st_attr;
  }
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int block = 512;
  int64_t grid = ncu;
  const int64_t tiles = (N + 31) / 32;
  if (grid > (tiles + 7) / 8) grid = (tiles + 7) / 8;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(block), L.bytes, s, p->img, L, p->D, p->m, d_y, N,
                     p->in_scale, p->out_scale, d_llr);
  MD_LAUNCH_CHECK("mlp_infer_kernel launch");
  return MD_OK;
}

// LDS of the streaming kernel: layer 1, layer 3 + biases, two layer-2 output blocks.
size_t stream_lds_bytes(const InferLayout& L) {
  return static_cast<size_t>(L.nrb) * L.ks1 * 1024 + (L.bytes - L.f3) + 2 * static_cast<size_t>(L.nrb) * 2 * 1024;
}

template <int NRB, int KS1>
int infer_stream_t(Mlp* p, const float* d_y, int64_t N, float* d_llr, hipStream_t s) {
  const InferLayout L = infer_layout(p->H, p->D);
  auto kern = mlp_infer_stream_kernel<NRB, KS1>;
  {
    const int st_attr = set_lds_limit(reinterpret_cast<const void*>(kern), 160 * 1024);
    if (st_attr != MD_OK) return st_attr;
  }
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int64_t grid = ncu;
  const int64_t btiles = (N + 255) / 256;
  if (grid > btiles) grid = btiles;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(512), stream_lds_bytes(L), s, p->img, L, p->D,
                     p->m, d_y, N, p->in_scale, p->out_scale, d_llr);
  MD_LAUNCH_CHECK("mlp_infer_stream_kernel launch");
  return MD_OK;
}

#define MD_STREAM_CASE(NRB_, KS1_) \
  case NRB_: return infer_stream_t<NRB_, KS1_>(p, d_y, N, d_llr, s);

int infer(Mlp* p, const float* d_y, int64_t N, float* d_llr, hipStream_t s) {
  const InferLayout L = infer_layout(p->H, p->D);
  const bool shape_ok = p->H % 32 == 0 && p->m <= 32;
  const bool fused = shape_ok && p->H <= 256 && L.ks1 == 1 && L.bytes <= 160 * 1024;
  const bool stream = shape_ok && !fused && p->H <= 512 && L.ks1 <= 2 && stream_lds_bytes(L) <= 160 * 1024;
  if (!fused && !stream) return infer_gemm(p, d_y, N, d_llr, s);
  if (!p->img) {
    void* q = nullptr;
    if (md::dev_malloc(&q, L.bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MD_ENOMEM, "MLP inference image allocation failed");
    }
    p->img = static_cast<char*>(q);
  }
  if (p->img_version != p->version) {
    hipLaunchKernelGGL(pack_infer_kernel, dim3(256), dim3(256), 0, s, p->w, p->D, p->H, p->m, L, p->img);
    MD_LAUNCH_CHECK("pack_infer_kernel launch");
    p->img_version = p->version;
  }
  if (fused) {
    switch (L.nrb) {
      case 1: return infer_fused_t<1>(p, d_y, N, d_llr, s);
      case 2: return infer_fused_t<2>(p, d_y, N, d_llr, s);
      case 3: return infer_fused_t<3>(p, d_y, N, d_llr, s);
      case 4: return infer_fused_t<4>(p, d_y, N, d_llr, s);
      case 5: return infer_fused_t<5>(p, d_y, N, d_llr, s);
      case 6: return infer_fused_t<6>(p, d_y, N, d_llr, s);
      case 7: return infer_fused_t<7>(p, d_y, N, d_llr, s);
      default: return infer_fused_t<8>(p, d_y, N, d_llr, s);
    }
  }
  if (L.ks1 == 1) {
    switch (L.nrb) {
      MD_STREAM_CASE(9, 1) MD_STREAM_CASE(10, 1) MD_STREAM_CASE(11, 1) MD_STREAM_CASE(12, 1)
      MD_STREAM_CASE(13, 1) MD_STREAM_CASE(14, 1) MD_STREAM_CASE(15, 1) MD_STREAM_CASE(16, 1)
      default: break;
    }
  } else {
    switch (L.nrb) {
      MD_STREAM_CASE(1, 2) MD_STREAM_CASE(2, 2) MD_STREAM_CASE(3, 2) MD_STREAM_CASE(4, 2)
      MD_STREAM_CASE(5, 2) MD_STREAM_CASE(6, 2) MD_STREAM_CASE(7, 2) MD_STREAM_CASE(8, 2)
      MD_STREAM_CASE(9, 2) MD_STREAM_CASE(10, 2) MD_STREAM_CASE(11, 2) MD_STREAM_CASE(12, 2)
      MD_STREAM_CASE(13, 2) MD_STREAM_CASE(14, 2) MD_STREAM_CASE(15, 2) MD_STREAM_CASE(16, 2)
      default: break;
    }
  }
  return fail(MD_EINVAL, "no inference kernel for this network shape");
}
#undef MD_STREAM_CASE

uint32_t crc32(const void* data, size_t n, uint32_t crc = 0) {
  crc = ~crc;
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    crc ^= b[i];
    for (int k = 0; k < 8; ++k) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
  }
  return ~crc;
}

struct CkptHeader {
  char magic[8];          // "MDMLP\0\0\2"
  int32_t D, H, m, pad;
  int64_t P, step;
  uint64_t seed;
  uint32_t crc, pad2;
  float in_scale, out_scale;
};

}  // namespace
}  // namespace md

extern "C" {

int mlp_create(int D, int hidden, int m, uint64_t seed, void** out) {
  md::set_error("");
  if (!out) return md::fail(MD_EINVAL, "out is NULL");
  *out = nullptr;
  if (D < 1 || D > 30) return md::fail(MD_EDIM, "D outside [1, 30]");
  if (hidden < 1 || hidden > 4096) return md::fail(MD_EINVAL, "hidden outside [1, 4096]");
  if (m < 1 || m > 16) return md::fail(MD_EINVAL, "m outside [1, 16]");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  md::Mlp* p = new md::Mlp();
  p->D = D;
  p->H = hidden;
  p->m = m;
  p->P = md::param_count(D, hidden, m);
  p->device = dev;
  p->seed = seed;
  void* q = nullptr;
  if (md::dev_malloc(&q, sizeof(float) * 4 * static_cast<size_t>(p->P)) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return md::fail(MD_ENOMEM, "MLP parameter allocation failed");
  }
  p->w = static_cast<float*>(q);
  p->g = p->w + p->P;
  p->m1 = p->g + p->P;
  p->m2 = p->m1 + p->P;
  std::vector<float> init;
  md::init_params(D, hidden, m, seed, &init);
  std::vector<float> zeros(static_cast<size_t>(3 * p->P), 0.0f);
  if (hipMemcpy(p->w, init.data(), sizeof(float) * p->P, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->g, zeros.data(), sizeof(float) * 3 * p->P, hipMemcpyHostToDevice) != hipSuccess) {
    hipError_t e = hipGetLastError();
    (void)md::dev_free(p->w);
    delete p;
    return md::hip_fail(e, "MLP parameter upload");
  }
  *out = p;
  return MD_OK;
}

int mlp_destroy(void* mlp) {
  md::set_error("");
  md::Mlp* p = static_cast<md::Mlp*>(mlp);
  if (!p) return MD_OK;
  MD_HIP_TRY(hipDeviceSynchronize());
  if (p->w) MD_HIP_TRY(md::dev_free(p->w));
  if (p->img) MD_HIP_TRY(md::dev_free(p->img));
  if (p->scratch) MD_HIP_TRY(md::dev_free(p->scratch));
  delete p;
  return MD_OK;
}

int64_t mlp_num_params(const void* mlp) {
  const md::Mlp* p = static_cast<const md::Mlp*>(mlp);
  return p ? p->P : -1;
}

int mlp_get(const void* mlp, int which, float* h_out) {
  md::set_error("");
  const md::Mlp* p = static_cast<const md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (!h_out || which < 0 || which > 3) return md::fail(MD_EINVAL, "bad buffer or selector");
  MD_HIP_TRY(hipDeviceSynchronize());
  MD_HIP_TRY(hipMemcpy(h_out, p->w + which * p->P, sizeof(float) * p->P, hipMemcpyDeviceToHost));
  return MD_OK;
}

int mlp_set(void* mlp, int which, const float* h_in) {
  md::set_error("");
  md::Mlp* p = static_cast<md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (!h_in || which < 0 || which > 3) return md::fail(MD_EINVAL, "bad buffer or selector");
  MD_HIP_TRY(hipDeviceSynchronize());
  MD_HIP_TRY(hipMemcpy(p->w + which * p->P, h_in, sizeof(float) * p->P, hipMemcpyHostToDevice));
  if (which == 0) p->version += 1;
  return MD_OK;
}

int mlp_grad(void* mlp, const float* d_y, const float* d_target, int64_t B, double* d_loss, void* stream) {
  md::set_error("");
  md::Mlp* p = static_cast<md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (B < 1 || B > (1 << 24)) return md::fail(MD_EINVAL, "batch size outside [1, 2^24]");
  if (!d_y || !d_target) return md::fail(MD_EINVAL, "y or target is NULL");
  return md::forward_backward(p, d_y, d_target, B, d_loss, reinterpret_cast<hipStream_t>(stream));
}

int mlp_adam_step(void* mlp, float lr, void* stream) {
  md::set_error("");
  md::Mlp* p = static_cast<md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (!(lr >= 0.0f)) return md::fail(MD_EINVAL, "learning rate must be >= 0");
  return md::adam(p, lr, reinterpret_cast<hipStream_t>(stream));
}

int mlp_train_step(void* mlp, const float* d_y, const float* d_target, int64_t B, float lr, double* d_loss,
                   void* stream) {
  int st = mlp_grad(mlp, d_y, d_target, B, d_loss, stream);
  if (st != MD_OK) return st;
  return mlp_adam_step(mlp, lr, stream);
}

int mlp_fit(void* mlp, const float* d_y, const float* d_target, int64_t N, int64_t steps, int64_t B, float lr_max,
            float lr_min, uint64_t shuffle_seed, double* d_loss_trace, void* stream) {
  md::set_error("");
  md::Mlp* p = static_cast<md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (N < 1 || N >= (int64_t(1) << 32) || steps < 0 || B < 1 || B > (1 << 20))
    return md::fail(MD_EINVAL, "bad N, steps or batch size");
  if (!d_y || !d_target) return md::fail(MD_EINVAL, "y or target is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* q = nullptr;
  // the batch buffers are private to this call (freed after the stream drains)
  if (md::dev_malloc(&q, sizeof(float) * static_cast<size_t>(B) * (p->D + p->m)) != hipSuccess) {
    (void)hipGetLastError();
    return md::fail(MD_ENOMEM, "batch allocation failed");
  }
  float* yb = static_cast<float*>(q);
  float* tb = yb + B * p->D;
  const int64_t start = p->step;
  for (int64_t i = 0; i < steps && st == MD_OK; ++i) {
    const double frac = steps > 1 ? static_cast<double>(i) / static_cast<double>(steps - 1) : 0.0;
    const float lr = static_cast<float>(lr_min + 0.5 * (lr_max - lr_min) * (1.0 + std::cos(M_PI * frac)));
    hipLaunchKernelGGL(md::gather_kernel, dim3(static_cast<unsigned>((B + 255) / 256)), dim3(256), 0, s, d_y,
                       d_target, p->D, p->m, N, shuffle_seed, static_cast<uint64_t>(start + i), B, yb, tb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      st = md::hip_fail(e, "gather_kernel launch");
      break;
    }
    st = md::forward_backward(p, yb, tb, B, d_loss_trace ? d_loss_trace + i : nullptr, s);
    if (st == MD_OK) st = md::adam(p, lr, s);
  }
  hipError_t e1 = hipStreamSynchronize(s);
  hipError_t e2 = md::dev_free(yb);
  if (st != MD_OK) return st;
  if (e1 != hipSuccess) return md::hip_fail(e1, "hipStreamSynchronize");
  if (e2 != hipSuccess) return md::hip_fail(e2, "hipFree");
  return MD_OK;
}

int llr_learned(const void* mlp, const float* d_y, int64_t N, float* d_llr, void* stream) {
  md::set_error("");
  md::Mlp* p = const_cast<md::Mlp*>(static_cast<const md::Mlp*>(mlp));
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (N < 0) return md::fail(MD_EINVAL, "N is negative");
  if (N == 0) return MD_OK;
  if (!d_y || !d_llr) return md::fail(MD_EINVAL, "y or llr is NULL");
  return md::infer(p, d_y, N, d_llr, reinterpret_cast<hipStream_t>(stream));
}

int mlp_save(const void* mlp, const char* path) {
  md::set_error("");
  const md::Mlp* p = static_cast<const md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (!path) return md::fail(MD_EINVAL, "path is NULL");
  std::vector<float> buf(static_cast<size_t>(3 * p->P));
  MD_HIP_TRY(hipDeviceSynchronize());
  MD_HIP_TRY(hipMemcpy(buf.data(), p->w, sizeof(float) * p->P, hipMemcpyDeviceToHost));
  MD_HIP_TRY(hipMemcpy(buf.data() + p->P, p->m1, sizeof(float) * 2 * p->P, hipMemcpyDeviceToHost));
  md::CkptHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, "MDMLP\0\0\2", 8);
  hd.D = p->D;
  hd.H = p->H;
  hd.m = p->m;
  hd.P = p->P;
  hd.step = p->step;
  hd.seed = p->seed;
  hd.in_scale = p->in_scale;
  hd.out_scale = p->out_scale;
  hd.crc = md::crc32(&hd.in_scale, 2 * sizeof(float), md::crc32(buf.data(), buf.size() * sizeof(float)));
  FILE* f = std::fopen(path, "wb");
  if (!f) return md::fail(MD_EINVAL, std::string("cannot open ") + path);
  const bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 &&
                  std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  std::fclose(f);
  return ok ? MD_OK : md::fail(MD_EINVAL, "short write");
}

int mlp_load(const char* path, void** out) {
  md::set_error("");
  if (!path || !out) return md::fail(MD_EINVAL, "path or out is NULL");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return md::fail(MD_EINVAL, std::string("cannot open ") + path);
  md::CkptHeader hd;
  if (std::fread(&hd, sizeof(hd), 1, f) != 1 || std::memcmp(hd.magic, "MDMLP\0\0\2", 8) != 0 ||
      !(hd.in_scale > 0.0f && hd.in_scale < INFINITY && hd.out_scale > 0.0f && hd.out_scale < INFINITY) ||
      hd.P != md::param_count(hd.D, hd.H, hd.m)) {
    std::fclose(f);
    return md::fail(MD_EINVAL, "not an MLP checkpoint of this version");
  }
  std::vector<float> buf(static_cast<size_t>(3 * hd.P));
  const bool ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok || md::crc32(&hd.in_scale, 2 * sizeof(float), md::crc32(buf.data(), buf.size() * sizeof(float))) != hd.crc)
    return md::fail(MD_EINVAL, "checkpoint is truncated or corrupt (CRC mismatch)");
  void* h = nullptr;
  int st = mlp_create(hd.D, hd.H, hd.m, hd.seed, &h);
  if (st != MD_OK) return st;
  md::Mlp* p = static_cast<md::Mlp*>(h);
  MD_HIP_TRY(hipMemcpy(p->w, buf.data(), sizeof(float) * p->P, hipMemcpyHostToDevice));
  MD_HIP_TRY(hipMemcpy(p->m1, buf.data() + p->P, sizeof(float) * 2 * p->P, hipMemcpyHostToDevice));
  p->step = hd.step;
  p->in_scale = hd.in_scale;
  p->out_scale = hd.out_scale;
  p->version += 1;
  *out = p;
  return MD_OK;
}

int mlp_set_scales(void* mlp, float in_scale, float out_scale) {
  md::set_error("");
  md::Mlp* p = static_cast<md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (!(in_scale > 0.0f && in_scale < INFINITY && out_scale > 0.0f && out_scale < INFINITY))
    return md::fail(MD_EINVAL, "scales must be finite and > 0");
  p->in_scale = in_scale;
  p->out_scale = out_scale;
  return MD_OK;
}

int mlp_get_scales(const void* mlp, float* in_scale, float* out_scale) {
  md::set_error("");
  const md::Mlp* p = static_cast<const md::Mlp*>(mlp);
  int st = md::check_handle(p);
  if (st != MD_OK) return st;
  if (in_scale) *in_scale = p->in_scale;
  if (out_scale) *out_scale = p->out_scale;
  return MD_OK;
}

int mlp_info(const void* mlp, int* D, int* hidden, int* m, int64_t* step) {
  const md::Mlp* p = static_cast<const md::Mlp*>(mlp);
  if (!p) return md::fail(MD_EINVAL, "MLP handle is NULL");
  if (D) *D = p->D;
  if (hidden) *hidden = p->H;
  if (m) *m = p->m;
  if (step) *step = p->step;
  return MD_OK;
}

}  // extern "C"
