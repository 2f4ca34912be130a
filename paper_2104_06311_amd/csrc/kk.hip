// kk_frontend: the Kramers-Kronig front end of the paper's receiver (section "Experimental
// setup", DSP-chain paragraph): square root and logarithm of the detected samples, the
// phase by a Hilbert transform computed with 1024-point overlap-save FFTs, the field
// rebuilt from amplitude and phase, the carrier removed and the result downshifted to DC.
//
// One workgroup per 1024 output samples, i.e. two 512-sample blocks a and b of the
// overlap-save scheme.  Both blocks' log-amplitudes are real, so they share one complex
// FFT pair: z = l_a + i l_b (each the 1024 samples around its block, zero outside the
// stream), Z = FFT(z), then w = IFFT(-i sgn(k) Z) (sgn 0 at k = 0 and k = 512).  The
// multiplier -i sgn(k) maps the spectrum of a real signal to that of its Hilbert
// transform (the analytic mask 1 + sgn(k) applied to l gives l + i H(l)), and it is
// linear, so w = H(l_a) + i H(l_b): the real part holds block a's phases, the imaginary
// part block b's.  The FFT is a radix-4 decimation-in-time over base-4 digit-reversed
// loads, in place in LDS: five stages of one butterfly per thread on disjoint
// quadruples, one barrier per stage; the inverse is conj(FFT(conj W)) / 1024.  The
// twiddle factors are computed once per device (FP64, rounded to FP32) into a device
// table that every workgroup copies to LDS.  Logarithm, exponential, sine and cosine use
// the hardware instructions (base 2, and revolutions for sine and cosine); the
// downshift phase frac(nu t) is formed in FP64 from one product per workgroup.
#include <mutex>

#include "common.hpp"

namespace md {
namespace {

constexpr int kKkN = 1024;
constexpr int kKkHop = 512;
constexpr int kKkPad = 256;
constexpr int kKkThreads = 256;
constexpr int kKkSpan = kKkN + kKkHop;     // samples a workgroup reads: 1536
constexpr int kKkTw = 3 * kKkN / 4;

__device__ float2 g_kk_tw[kKkTw];          // exp(-2 pi i j / 1024), j < 768, one table per device

__global__ void kk_twiddle_kernel() {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kKkTw) return;
  double s, c;
  sincospi(static_cast<double>(j) / 512.0, &s, &c);
  g_kk_tw[j] = make_float2(static_cast<float>(c), static_cast<float>(-s));
}

std::mutex g_tw_mu;
bool g_tw_done[64] = {};

// Fills this device's twiddle table once, on a private stream that the call waits for
// (so the caller's stream, even one being captured, is not involved).
int ensure_twiddles() {
  int dev = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MD_ENODEV, "kk_frontend: device index above 63");
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if (g_tw_done[dev]) return MD_OK;
  hipStream_t ts = nullptr;
  MD_HIP_TRY(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking));
  hipLaunchKernelGGL(kk_twiddle_kernel, dim3((kKkTw + 255) / 256), dim3(256), 0, ts);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(ts);
  (void)hipStreamDestroy(ts);
  if (e != hipSuccess) return hip_fail(e, "kk_twiddle_kernel");
  g_tw_done[dev] = true;
  return MD_OK;
}

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

constexpr float kHalfLn2 = 0.34657359027997265471f;     // ln(2) / 2
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kInv2Pi = 0.15915494309189533577f;

__global__ void __launch_bounds__(kKkThreads) kk_kernel(const float* __restrict__ x, int64_t T, float A, double nu,
                                                        float2* __restrict__ out) {
  __shared__ float2 a[kKkN];
  __shared__ float2 tw[kKkTw];
  __shared__ float l[kKkSpan];
  const int tid = threadIdx.x;
  const int64_t start = static_cast<int64_t>(blockIdx.x) * (2 * kKkHop) - kKkPad;   // first sample of block a's window
  const bool has_b = start + kKkPad + kKkHop < T;                                    // block b lies inside the stream
  for (int j = tid; j < kKkTw; j += kKkThreads) tw[j] = g_kk_tw[j];
  // l = 0.5 ln x over the workgroup's 1536 samples (block a's window, then the 512 more of b's)
#pragma unroll
  for (int q = 0; q < kKkSpan / kKkThreads; ++q) {
    const int i = tid + q * kKkThreads;
    const int64_t t = start + i;
    // floor: see kk_frontend
    l[i] = (t >= 0 && t < T) ? kHalfLn2 * __builtin_amdgcn_logf(fmaxf(x[t], 0x1p-126f)) : 0.0f;
  }
  __syncthreads();
  // z = l_a + i l_b in digit-reversed order (block b's window starts 512 samples later)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = tid + q * kKkThreads;
    a[digrev4(i)] = make_float2(l[i], has_b ? l[i + kKkHop] : 0.0f);
  }
  __syncthreads();
  fft1024(a, tw);
  // W = -i sgn(k) Z, stored as conj(W) in digit-reversed order for the inverse; the
  // butterfly partners read in place, so go through registers and a barrier
  float2 v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = tid + q * kKkThreads;
    const float2 z = a[k];
    // -i z = (z.y, -z.x); conj of that = (z.y, z.x); for sgn = -1 the negatives
    const float sg = (k == 0 || k == kKkN / 2) ? 0.0f : (k < kKkN / 2 ? 1.0f : -1.0f);
    v[q] = make_float2(sg * z.y, sg * z.x);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) a[digrev4(tid + q * kKkThreads)] = v[q];
  __syncthreads();
  fft1024(a, tw);
  // w = conj(a) / 1024: H(l_a) = a.x / 1024, H(l_b) = -a.y / 1024; the middle 512 of each
  const double fb = nu * static_cast<double>(start) - floor(nu * static_cast<double>(start));
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = tid + (q & 1) * kKkThreads;       // 0 .. 511 within the block's kept part
    const int blkb = q >> 1;
    if (blkb && !has_b) continue;
    const int i = kKkPad + r;                         // index in the block's window
    const float2 w = a[i];
    const float phi = (blkb ? -w.y : w.x) * (1.0f / kKkN);
    const float amp = __builtin_amdgcn_exp2f(kLog2e * l[i + blkb * kKkHop]);
    const float rev = phi * kInv2Pi;                  // the hardware sine and cosine take revolutions
    const float er = amp * __builtin_amdgcn_cosf(rev) - A;
    const float ei = amp * __builtin_amdgcn_sinf(rev);
    const int off = i + blkb * kKkHop;                // offset of the sample from start
    double ph = fb + nu * static_cast<double>(off);
    ph -= floor(ph);                                  // frac(nu t), t = start + off
    const float f = static_cast<float>(ph);
    const float2 rot = make_float2(__builtin_amdgcn_cosf(f), -__builtin_amdgcn_sinf(f));
    out[start + off] = cmul(make_float2(er, ei), rot);
  }
}

}  // namespace
}  // namespace md

extern "C" {

int kk_frontend(const float* d_x, int64_t T, float A, double nu, float* d_out, void* stream) {
  using namespace md;
  set_error("");
  if (T < 0 || T % kKkHop != 0) return fail(MD_EINVAL, "kk_frontend: T must be a non-negative multiple of 512");
  if (!std::isfinite(A) || A < 0.0f) return fail(MD_EINVAL, "kk_frontend: A must be finite and >= 0");
  if (!std::isfinite(nu)) return fail(MD_EINVAL, "kk_frontend: nu must be finite");
  if (T == 0) return MD_OK;
  if (d_x == nullptr || d_out == nullptr) return fail(MD_EINVAL, "kk_frontend: d_x and d_out are required");
  const int64_t blocks = (T / kKkHop + 1) / 2;
  if (blocks > 0x7fffffff) return fail(MD_EINVAL, "kk_frontend: T too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = ensure_twiddles();
  if (st != MD_OK) return st;
  hipLaunchKernelGGL(kk_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kKkThreads), 0, s, d_x, T, A, nu,
                     reinterpret_cast<float2*>(d_out));
  MD_LAUNCH_CHECK("kk_kernel launch");
  return MD_OK;
}

}  // extern "C"
