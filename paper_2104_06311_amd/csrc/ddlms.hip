// ddlms_equalize: four-tap widely-linear decision-directed LMS equaliser, the step that
// feeds the demapper in the paper's receiver (section "Experimental setup": a four-tap
// adaptive time-domain DD-LMS widely-linear equaliser after downsampling to 2 samples per
// symbol, whose sequential recursion the receiver hides by running many buffers at once).
//
// The recursion of one equaliser is sequential, so the parallelism is across independent
// instances (buffers, sub-blocks, channels): one thread per instance, samples stored
// time-major so that every step of all threads reads consecutive addresses.  The state is
// FP64 and every operation is written out with contraction off, in the order the header
// states, so the results do not depend on the launch geometry.
#include "common.hpp"

#pragma clang fp contract(off)

namespace md {
namespace {

constexpr int kEqThreads = 256;
constexpr int kEqMaxPoints = 1024;

struct Taps {
  double v[16];   // h re/im for j = 0..3, then g re/im for j = 0..3
};

// h_in, g_in: NULL (every instance starts from t0) or B x 8 doubles, each instance's own
// starting taps; they may be the same arrays as h_out, g_out (each thread reads its
// instance's taps before it writes them).
__global__ void __launch_bounds__(kEqThreads) ddlms_kernel(const float2* __restrict__ x, int64_t B, int64_t N,
                                                          const float2* __restrict__ C, int M, Taps t0, double mu,
                                                          uint32_t* __restrict__ dec, float2* __restrict__ z,
                                                          const double* h_in, const double* g_in, double* h_out,
                                                          double* g_out) {
  __shared__ float2 pts[kEqMaxPoints];
  for (int i = threadIdx.x; i < M; i += blockDim.x) pts[i] = C[i];
  __syncthreads();
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;   // after the only barrier

  double hr[4], hi[4], gr[4], gi[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hr[j] = h_in ? h_in[8 * b + 2 * j] : t0.v[2 * j];
    hi[j] = h_in ? h_in[8 * b + 2 * j + 1] : t0.v[2 * j + 1];
    gr[j] = g_in ? g_in[8 * b + 2 * j] : t0.v[8 + 2 * j];
    gi[j] = g_in ? g_in[8 * b + 2 * j + 1] : t0.v[8 + 2 * j + 1];
  }
  // window w_j = u_{2n+j}; samples 2n and 2n+1 carry over from the previous symbol
  double wr[4] = {0.0, 0.0, 0.0, 0.0}, wi[4] = {0.0, 0.0, 0.0, 0.0};
  float2 p2 = make_float2(0.0f, 0.0f), p3 = make_float2(0.0f, 0.0f);
  if (N > 0) {
    const float2 s0 = x[b], s1 = x[B + b];
    wr[0] = static_cast<double>(s0.x);
    wi[0] = static_cast<double>(s0.y);
    wr[1] = static_cast<double>(s1.x);
    wi[1] = static_cast<double>(s1.y);
    p2 = x[2 * B + b];
    p3 = x[3 * B + b];
  }
  for (int64_t n = 0; n < N; ++n) {
    wr[2] = static_cast<double>(p2.x);
    wi[2] = static_cast<double>(p2.y);
    wr[3] = static_cast<double>(p3.x);
    wi[3] = static_cast<double>(p3.y);
    if (n + 1 < N) {   // the next symbol's new samples 2n+4, 2n+5 (at most 2N+1)
      p2 = x[(2 * n + 4) * B + b];
      p3 = x[(2 * n + 5) * B + b];
    }
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zr = zr + (hr[j] * wr[j] - hi[j] * wi[j]);
      zr = zr + (gr[j] * wr[j] + gi[j] * wi[j]);
      zi = zi + (hr[j] * wi[j] + hi[j] * wr[j]);
      zi = zi + (gi[j] * wr[j] - gr[j] * wi[j]);
    }
    double best = INFINITY;
    int arg = 0;
    for (int i = 0; i < M; ++i) {
      const float2 c = pts[i];
      const double dr = zr - static_cast<double>(c.x);
      const double di = zi - static_cast<double>(c.y);
      const double d2 = dr * dr + di * di;
      if (d2 < best) {
        best = d2;
        arg = i;
      }
    }
    const float2 c = pts[arg];
    const double er = static_cast<double>(c.x) - zr;
    const double ei = static_cast<double>(c.y) - zi;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hr[j] = hr[j] + mu * (er * wr[j] + ei * wi[j]);
      hi[j] = hi[j] + mu * (ei * wr[j] - er * wi[j]);
      gr[j] = gr[j] + mu * (er * wr[j] - ei * wi[j]);
      gi[j] = gi[j] + mu * (er * wi[j] + ei * wr[j]);
    }
    dec[n * B + b] = static_cast<uint32_t>(arg);
    if (z) z[n * B + b] = make_float2(static_cast<float>(zr), static_cast<float>(zi));
    wr[0] = wr[2];
    wi[0] = wi[2];
    wr[1] = wr[3];
    wi[1] = wi[3];
  }
  if (h_out) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      h_out[8 * b + 2 * j] = hr[j];
      h_out[8 * b + 2 * j + 1] = hi[j];
    }
  }
  if (g_out) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      g_out[8 * b + 2 * j] = gr[j];
      g_out[8 * b + 2 * j + 1] = gi[j];
    }
  }
}

bool finite_taps(const double* t) {
  for (int i = 0; i < 8; ++i)
    if (!std::isfinite(t[i])) return false;
  return true;
}

}  // namespace

int launch_ddlms(const float* d_x, int64_t B, int64_t N, const float* d_C, int M, const double* t0_h,
                 const double* t0_g, const double* d_h_in, const double* d_g_in, double mu, uint32_t* d_dec,
                 float* d_z, double* d_h, double* d_g, hipStream_t stream) {
  if (B == 0) return MD_OK;
  Taps t0;
  for (int i = 0; i < 8; ++i) {
    t0.v[i] = t0_h ? t0_h[i] : 0.0;
    t0.v[8 + i] = t0_g ? t0_g[i] : 0.0;
  }
  const int64_t blocks = (B + kEqThreads - 1) / kEqThreads;
  if (blocks > 0x7fffffff) return fail(MD_EINVAL, "ddlms: B too large");
  hipLaunchKernelGGL(ddlms_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kEqThreads), 0, stream,
                     reinterpret_cast<const float2*>(d_x), B, N, reinterpret_cast<const float2*>(d_C), M, t0, mu,
                     d_dec, reinterpret_cast<float2*>(d_z), d_h_in, d_g_in, d_h, d_g);
  MD_LAUNCH_CHECK("ddlms_kernel launch");
  return MD_OK;
}

}  // namespace md

extern "C" {

int ddlms_equalize(const float* d_x, int64_t B, int64_t N, const float* d_C, int M, const double* h_h0,
                   const double* h_g0, double mu, uint32_t* d_dec, float* d_z, double* d_h, double* d_g,
                   void* stream) {
  using namespace md;
  if (B < 0 || N < 0) return fail(MD_EINVAL, "ddlms_equalize: B and N must be >= 0");
  if (M < 1 || M > kEqMaxPoints) return fail(MD_EINVAL, "ddlms_equalize: M must be in [1, 1024]");
  if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(MD_EINVAL, "ddlms_equalize: mu must be finite and >= 0");
  if (h_h0 == nullptr || h_g0 == nullptr) return fail(MD_EINVAL, "ddlms_equalize: starting taps are required");
  if (!finite_taps(h_h0) || !finite_taps(h_g0)) return fail(MD_EINVAL, "ddlms_equalize: starting taps must be finite");
  if (d_x == nullptr || d_C == nullptr) return fail(MD_EINVAL, "ddlms_equalize: d_x and d_C are required");
  if (N > 0 && d_dec == nullptr) return fail(MD_EINVAL, "ddlms_equalize: d_dec is required");
  if (N > (int64_t(1) << 40) / (B > 0 ? B : 1)) return fail(MD_EINVAL, "ddlms_equalize: (2N + 2) B too large");
  return launch_ddlms(d_x, B, N, d_C, M, h_h0, h_g0, nullptr, nullptr, mu, d_dec, d_z, d_h, d_g,
                      static_cast<hipStream_t>(stream));
}

int ddlms_equalize_chain(const float* d_x, int64_t B, int64_t N, const float* d_C, int M, double mu,
                         uint32_t* d_dec, float* d_z, double* d_h, double* d_g, void* stream) {
  using namespace md;
  if (B < 0 || N < 0) return fail(MD_EINVAL, "ddlms_equalize_chain: B and N must be >= 0");
  if (M < 1 || M > kEqMaxPoints) return fail(MD_EINVAL, "ddlms_equalize_chain: M must be in [1, 1024]");
  if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(MD_EINVAL, "ddlms_equalize_chain: mu must be finite and >= 0");
  if (d_x == nullptr || d_C == nullptr) return fail(MD_EINVAL, "ddlms_equalize_chain: d_x and d_C are required");
  if (d_h == nullptr || d_g == nullptr) return fail(MD_EINVAL, "ddlms_equalize_chain: d_h and d_g are required");
  if (N > 0 && d_dec == nullptr) return fail(MD_EINVAL, "ddlms_equalize_chain: d_dec is required");
  if (N > (int64_t(1) << 40) / (B > 0 ? B : 1)) return fail(MD_EINVAL, "ddlms_equalize_chain: (2N + 2) B too large");
  return launch_ddlms(d_x, B, N, d_C, M, nullptr, nullptr, d_h, d_g, mu, d_dec, d_z, d_h, d_g,
                      static_cast<hipStream_t>(stream));
}

}  // extern "C"
