// kk_frontend: the Kramers-Kronig front end of the paper's receiver (section "Experimental
// setup", DSP-chain paragraph): square root and logarithm of the detected samples, the
// phase by a Hilbert transform computed with 1024-point overlap-save FFTs, the field
// rebuilt from amplitude and phase, the carrier removed and the result downshifted to DC.
//
// One wavefront per 1024 output samples, i.e. two 512-sample blocks a and b of the
// overlap-save scheme.  Both blocks' log-amplitudes are real, so they share one complex
// FFT pair: z = l_a + i l_b (each the 1024 samples around its block, zero outside the
// stream), Z = FFT(z), then w = IFFT(-i sgn(k) Z) (sgn 0 at k = 0 and k = 512).  The
// multiplier -i sgn(k) maps the spectrum of a real signal to that of its Hilbert
// transform (the analytic mask 1 + sgn(k) applied to l gives l + i H(l)), and it is
// linear, so w = H(l_a) + i H(l_b): the real part holds block a's phases, the imaginary
// part block b's.  The inverse is conj(FFT(conj W)) / 1024.
//
// The 1024-point FFT lives in the wavefront's registers: lane j holds the 16 points
// n = j + 64 m (m = 0..15), in and out.  With N = 64 x 16 and k = k1 + 16 k2:
//   A   16-point DFTs over m in every lane, times the twiddle W_1024^(j k1);
//   B1  for each (k1, jb) -- one lane each -- a 16-point DFT over ja of the values at
//       j = jb + 4 ja, times W_64^(jb k2a)  (k2 = k2a + 16 k2b);
//   B2  4-point DFTs over jb, placed so that lane k mod 64 holds X[k] in register k div 64.
// The two re-distributions go through LDS inside the wavefront (no workgroup barrier);
// the 16-point DFTs are two radix-4 stages in registers.  Twiddles come from a 1024-entry
// table computed once per device (FP64, rounded to FP32).  Logarithm, exponential, sine
// and cosine use the hardware instructions (base 2, and revolutions for sine and
// cosine); the downshift phase frac(nu t) is formed in FP64 from one product per
// wavefront.
#include <mutex>

#include "common.hpp"

namespace md {
namespace {

constexpr int kKkN = 1024;
constexpr int kKkHop = 512;
constexpr int kKkPad = 256;
constexpr int kKkLds = 16 * 68;            // float2 slots of the exchange buffer (rows of 64 + 4 pad)

__device__ float2 g_kk_tw[kKkN];           // W_1024^e = exp(-2 pi i e / 1024), one table per device

__global__ void kk_twiddle_kernel() {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kKkN) return;
  double s, c;
  sincospi(static_cast<double>(e) / 512.0, &s, &c);
  g_kk_tw[e] = make_float2(static_cast<float>(c), static_cast<float>(-s));
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
  hipLaunchKernelGGL(kk_twiddle_kernel, dim3(kKkN / 256), dim3(256), 0, ts);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(ts);
  (void)hipStreamDestroy(ts);
  if (e != hipSuccess) return hip_fail(e, "kk_twiddle_kernel");
  g_tw_done[dev] = true;
  return MD_OK;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // -i a

// 4-point DFT in place: X_k = sum_m a_m (-i)^(m k).
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 16-point DFT in place, input a[m], output A[k] at a[k]: m = m1 + 4 m2, k = k2 + 4 k1,
// A[k2 + 4 k1] = sum_m1 W16^(m1 k2) W4^(m1 k1) sum_m2 a[m1 + 4 m2] W4^(m2 k2).
__device__ __forceinline__ void dft16(float2 (&a)[16]) {
  constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, r2 = 0.70710678118654752440f;
  // W16^e = (cos, -sin)(2 pi e / 16), e = m1 k2 in {1, 2, 3, 2, 4, 6, 3, 6, 9}
  const float2 w[10] = {make_float2(1.0f, 0.0f), make_float2(c1, -s1), make_float2(r2, -r2), make_float2(s1, -c1),
                        make_float2(0.0f, -1.0f), make_float2(-s1, -c1), make_float2(-r2, -r2),
                        make_float2(-c1, -s1), make_float2(-1.0f, 0.0f), make_float2(-c1, s1)};
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) dft4(a[m1], a[m1 + 4], a[m1 + 8], a[m1 + 12]);   // now a[m1 + 4 k2]
#pragma unroll
  for (int m1 = 1; m1 < 4; ++m1)
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) a[m1 + 4 * k2] = cmul(a[m1 + 4 * k2], w[m1 * k2]);
  float2 b[16];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 x0 = a[0 + 4 * k2], x1 = a[1 + 4 * k2], x2 = a[2 + 4 * k2], x3 = a[3 + 4 * k2];
    dft4(x0, x1, x2, x3);                 // over m1: x_k1
    b[k2 + 0] = x0;
    b[k2 + 4] = x1;
    b[k2 + 8] = x2;
    b[k2 + 12] = x3;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = b[k];
}

// Orders the wavefront's LDS accesses around an exchange (one wavefront per workgroup).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Forward 1024-point DFT of the wavefront's points: lane j holds n = j + 64 m in v[m] on
// entry and X[k] for k = j + 64 m in v[m] on return.
__device__ __forceinline__ void fft1024(float2 (&v)[16], float2* sh, const float2* __restrict__ tw, int lane) {
  // A: DFT over m, twiddle W_1024^(j k1); Y[j][k1] to sh[k1][j]
  dft16(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[(lane * k1) & (kKkN - 1)]);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) sh[k1 * 68 + lane] = v[k1];
  wave_lds_sync();
  // B1: lane = k1 + 16 jb takes j = jb + 4 ja, ja = 0..15
  const int k1 = lane & 15, jb = lane >> 4;
#pragma unroll
  for (int ja = 0; ja < 16; ++ja) v[ja] = sh[k1 * 68 + jb + 4 * ja];
  wave_lds_sync();
  dft16(v);                                               // v[k2a]
#pragma unroll
  for (int k2a = 1; k2a < 16; ++k2a) v[k2a] = cmul(v[k2a], tw[(16 * jb * k2a) & (kKkN - 1)]);
  // to sh[k1][k2a][jb]: row k1 holds 64 values at k2a * 4 + jb
#pragma unroll
  for (int k2a = 0; k2a < 16; ++k2a) sh[k1 * 68 + 4 * k2a + jb] = v[k2a];
  wave_lds_sync();
  // B2: lane = k1 + 16 q takes k2a = q + 4 t (t = 0..3), 4-point DFTs over jb; output
  // k = k1 + 16 k2a + 256 k2b = lane + 64 (t + 4 k2b)
  const int q = jb;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float2 x0 = sh[k1 * 68 + 4 * (q + 4 * t) + 0], x1 = sh[k1 * 68 + 4 * (q + 4 * t) + 1];
    float2 x2 = sh[k1 * 68 + 4 * (q + 4 * t) + 2], x3 = sh[k1 * 68 + 4 * (q + 4 * t) + 3];
    dft4(x0, x1, x2, x3);                                 // over jb: x_k2b
    v[t + 0] = x0;
    v[t + 4] = x1;
    v[t + 8] = x2;
    v[t + 12] = x3;
  }
  wave_lds_sync();
}

constexpr float kHalfLn2 = 0.34657359027997265471f;     // ln(2) / 2
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kInv2Pi = 0.15915494309189533577f;

__global__ void __launch_bounds__(64) kk_kernel(const float* __restrict__ x, int64_t T, float A, double nu,
                                                float2* __restrict__ out) {
  __shared__ float2 sh[kKkLds];
  const int lane = threadIdx.x;
  const int64_t start = static_cast<int64_t>(blockIdx.x) * (2 * kKkHop) - kKkPad;   // block a's window
  const bool has_b = start + kKkPad + kKkHop < T;                                    // block b in the stream
  // l = 0.5 ln x at window offsets i = lane + 64 m, m = 0..23 (block a's window, then the
  // 512 more samples of block b's); the floor: see kk_frontend
  float l[24];
#pragma unroll
  for (int m = 0; m < 24; ++m) {
    const int64_t t = start + lane + 64 * m;
    l[m] = (t >= 0 && t < T) ? kHalfLn2 * __builtin_amdgcn_logf(fmaxf(x[t], 0x1p-126f)) : 0.0f;
  }
  // z[n] = l_a[n] + i l_b[n], l_b[n] = l[n + 512]; n = lane + 64 m
  float2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = make_float2(l[m], has_b ? l[m + 8] : 0.0f);
  fft1024(v, sh, g_kk_tw, lane);
  // conj(W), W = -i sgn(k) Z: -i z = (z.y, -z.x), conj = (z.y, z.x), sign by k = lane + 64 m
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = lane + 64 * m;
    const float sg = (k == 0 || k == kKkN / 2) ? 0.0f : (m < 8 ? 1.0f : -1.0f);
    v[m] = make_float2(sg * v[m].y, sg * v[m].x);
  }
  fft1024(v, sh, g_kk_tw, lane);
  // w = conj(v) / 1024: H(l_a)[n] = v.x / 1024, H(l_b)[n] = -v.y / 1024; keep n in [256, 768)
  const double fb = nu * static_cast<double>(start) - floor(nu * static_cast<double>(start));
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    if (blk == 1 && !has_b) break;
#pragma unroll
    for (int m = 4; m < 12; ++m) {
      const int n = lane + 64 * m;
      const float phi = (blk ? -v[m].y : v[m].x) * (1.0f / kKkN);
      const float amp = __builtin_amdgcn_exp2f(kLog2e * l[m + 8 * blk]);
      const float rev = phi * kInv2Pi;                  // the hardware sine and cosine take revolutions
      const float er = amp * __builtin_amdgcn_cosf(rev) - A;
      const float ei = amp * __builtin_amdgcn_sinf(rev);
      const int off = n + blk * kKkHop;                 // offset of the sample from start
      double ph = fb + nu * static_cast<double>(off);
      ph -= floor(ph);                                  // frac(nu t), t = start + off
      const float f = static_cast<float>(ph);
      const float2 rot = make_float2(__builtin_amdgcn_cosf(f), -__builtin_amdgcn_sinf(f));
      out[start + off] = cmul(make_float2(er, ei), rot);
    }
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
  hipLaunchKernelGGL(kk_kernel, dim3(static_cast<unsigned>(blocks)), dim3(64), 0, s, d_x, T, A, nu,
                     reinterpret_cast<float2*>(d_out));
  MD_LAUNCH_CHECK("kk_kernel launch");
  return MD_OK;
}

}  // extern "C"
