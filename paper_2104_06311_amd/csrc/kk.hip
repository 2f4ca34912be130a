// kk_frontend: the Kramers-Kronig front end of the paper's receiver (section "Experimental
// setup", DSP-chain paragraph): square root and logarithm of the detected samples, the
// phase by a Hilbert transform computed with 1024-point overlap-save FFTs, the field
// rebuilt from amplitude and phase, the carrier removed and the result downshifted to DC.
//
// One workgroup per 512 output samples: it reads the 1024 samples around them (zero
// outside the stream), takes l = 0.5 ln x, runs a 1024-point FFT in LDS, applies the
// analytic-signal mask, transforms back, and keeps the middle 512 phases.  The FFT is a
// radix-4 decimation-in-time over base-4 digit-reversed loads, in place: five stages of
// one butterfly per thread on disjoint quadruples, one barrier per stage.  The inverse is
// conj(FFT(conj X)) / 1024.
#include "common.hpp"

namespace md {
namespace {

constexpr int kKkN = 1024;
constexpr int kKkHop = 512;
constexpr int kKkPad = 256;
constexpr int kKkThreads = 256;

// reversal of the five base-4 digits of a 10-bit index: the bit reversal with each bit
// pair swapped back
__device__ __forceinline__ int digrev4(int i) {
  const int r = static_cast<int>(__brev(static_cast<unsigned>(i)) >> 22);
  return ((r & 0x155) << 1) | ((r & 0x2AA) >> 1);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-4 DIT over a[] holding its input in digit-reversed order; stage s
// combines four transforms of length L/4 into length L = 4^s with twiddles W_L^{k pos}.
__device__ __forceinline__ void fft1024(float2* a, const float2* tw) {
  for (int st = 1; st <= 5; ++st) {
    const int lq = 2 * (st - 1);               // log2 of a quarter of L
    const int q = 1 << lq;
    const int step = kKkN >> (2 * st);         // twiddle index step: 1024 / L
    const int g = threadIdx.x >> lq;
    const int p = threadIdx.x & (q - 1);
    const int i0 = (g << (2 * st)) + p;
    const int i1 = i0 + q, i2 = i1 + q, i3 = i2 + q;
    const float2 a0 = a[i0];
    const float2 a1 = cmul(a[i1], tw[p * step]);
    const float2 a2 = cmul(a[i2], tw[2 * p * step]);
    const float2 a3 = cmul(a[i3], tw[3 * p * step]);
    const float2 t0 = make_float2(a0.x + a2.x, a0.y + a2.y);
    const float2 t1 = make_float2(a0.x - a2.x, a0.y - a2.y);
    const float2 t2 = make_float2(a1.x + a3.x, a1.y + a3.y);
    const float2 t3 = make_float2(a1.x - a3.x, a1.y - a3.y);
    a[i0] = make_float2(t0.x + t2.x, t0.y + t2.y);
    a[i2] = make_float2(t0.x - t2.x, t0.y - t2.y);
    a[i1] = make_float2(t1.x + t3.y, t1.y - t3.x);   // t1 - i t3
    a[i3] = make_float2(t1.x - t3.y, t1.y + t3.x);   // t1 + i t3
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kKkThreads) kk_kernel(const float* __restrict__ x, int64_t T, float A, double nu,
                                                        float2* __restrict__ out) {
  __shared__ float2 a[kKkN];
  __shared__ float2 b[kKkN];
  __shared__ float2 tw[3 * kKkN / 4];
  __shared__ float lmid[kKkHop];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int64_t start = blk * kKkHop - kKkPad;
  for (int j = tid; j < 3 * kKkN / 4; j += kKkThreads) {
    double s, c;
    sincospi(static_cast<double>(j) / 512.0, &s, &c);   // exp(-2 pi i j / 1024)
    tw[j] = make_float2(static_cast<float>(c), static_cast<float>(-s));
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = tid + q * kKkThreads;
    const int64_t t = start + i;
    const float l = (t >= 0 && t < T) ? 0.5f * logf(fmaxf(x[t], 0x1p-126f)) : 0.0f;   // floor: see kk_frontend
    a[digrev4(i)] = make_float2(l, 0.0f);
    if (i >= kKkPad && i < kKkPad + kKkHop) lmid[i - kKkPad] = l;
  }
  __syncthreads();
  fft1024(a, tw);
  // analytic mask (1, 2 .. 2, 1, 0 .. 0), conjugated into digit-reversed order
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = tid + q * kKkThreads;
    const float m = (i == 0 || i == kKkN / 2) ? 1.0f : (i < kKkN / 2 ? 2.0f : 0.0f);
    const float2 v = a[i];
    b[digrev4(i)] = make_float2(m * v.x, -(m * v.y));
  }
  __syncthreads();
  fft1024(b, tw);
  // middle 512 samples: phase = Im(conj(B) / 1024) = -Im(B) / 1024
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = kKkPad + tid + q * kKkThreads;
    const float phi = -b[i].y * (1.0f / kKkN);
    const float amp = expf(lmid[i - kKkPad]);
    float sp, cp;
    sincosf(phi, &sp, &cp);
    const float er = amp * cp - A;
    const float ei = amp * sp;
    const int64_t t = start + i;
    const double ph = nu * static_cast<double>(t);
    const double frac = ph - floor(ph);
    double rs, rc;
    sincospi(2.0 * frac, &rs, &rc);                    // exp(-2 pi i frac) = (rc, -rs)
    const float2 rot = make_float2(static_cast<float>(rc), static_cast<float>(-rs));
    out[t] = cmul(make_float2(er, ei), rot);
  }
}

}  // namespace
}  // namespace md

extern "C" {

int kk_frontend(const float* d_x, int64_t T, float A, double nu, float* d_out, void* stream) {
  using namespace md;
  if (T < 0 || T % kKkHop != 0) return fail(MD_EINVAL, "kk_frontend: T must be a non-negative multiple of 512");
  if (!std::isfinite(A) || A < 0.0f) return fail(MD_EINVAL, "kk_frontend: A must be finite and >= 0");
  if (!std::isfinite(nu)) return fail(MD_EINVAL, "kk_frontend: nu must be finite");
  if (T == 0) return MD_OK;
  if (d_x == nullptr || d_out == nullptr) return fail(MD_EINVAL, "kk_frontend: d_x and d_out are required");
  const int64_t blocks = T / kKkHop;
  if (blocks > 0x7fffffff) return fail(MD_EINVAL, "kk_frontend: T too large");
  hipLaunchKernelGGL(kk_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kKkThreads), 0,
                     static_cast<hipStream_t>(stream), d_x, T, A, nu, reinterpret_cast<float2*>(d_out));
  MD_LAUNCH_CHECK("kk_kernel launch");
  return MD_OK;
}

}  // extern "C"
