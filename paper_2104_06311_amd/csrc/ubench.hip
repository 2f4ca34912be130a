// ubench: measured peak rates of the instructions the demapping kernels are bound by
// (v_exp_f32, non-packed v_add_f32, their one-exponential-two-adds mix, the exact
// demapper's whole per-tile instruction mix with its matrix products, the FP16/BF16/FP32
// matrix products) and of a device copy, on the current device.  Each compute kernel keeps 16 independent chains (or 4
// independent accumulators) per lane, so that issue, not latency, bounds it; its result
// feeds a store that is never taken, so the work cannot be removed.
#include "common.hpp"

namespace md {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kChains = 16;
constexpr float kNever = 1.2345678e30f;   // a sum the kernels never reach

__global__ void __launch_bounds__(kThreads) ub_exp_kernel(int64_t iters, float seed, float* sink) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed * static_cast<float>(threadIdx.x + c);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) r += x[c];
  if (r == kNever) sink[0] = r;
}

__global__ void __launch_bounds__(kThreads) ub_add_kernel(int64_t iters, float seed, float* sink) {
  float x[kChains], s[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = seed * static_cast<float>(threadIdx.x + c);
    s[c] = 0.0f;
  }
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) s[c] += x[c];
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) r += s[c];
  if (r == kNever) sink[0] = r;
}

// The exact demapper's per-pair mix: one exponential and two independent adds of its
// result into different partial sums (the two accumulators start from different values,
// so the compiler cannot merge them).
__global__ void __launch_bounds__(kThreads) ub_exp_add2_kernel(int64_t iters, float seed, float* sink) {
  float x[kChains], s0[kChains], s1[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = seed * static_cast<float>(threadIdx.x + c);
    s0[c] = 0.0f;
    s1[c] = 1.0f;
  }
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = __builtin_amdgcn_exp2f(-x[c]);
      s0[c] += x[c];
      s1[c] += x[c];
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) r += s0[c] * s1[c];
  if (r == kNever) sink[0] = r;
}

// The exact demapper's per-tile instruction mix at KS K steps and 5 + 3 + NH label bits,
// without its memory traffic: per 32 x 32 tile, KS dependent v_mfma_f32_32x32x16_f16
// score the next tile from A operands read from LDS (a ring of kMixTiles tiles), then
// each lane takes 16 exponentials of the current tile's products, adds each into its
// position sum and reduces them by a 15-add tree into the tile's group sum; every 8 tiles
// the group sum is routed by NH bits.  Hard scheduling fences keep the matrix products of
// tile t + 1 ahead of the exponentials of tile t, as in the demapper, so its rate is the
// ceiling that instruction mix allows on this device (KS = 2, NH = 3: the 8D M = 2048
// kernel; KS = 4, NH = 8: the 16D M = 65536 one; KS = 1, NH = 3: the 8D loop with one
// matrix product per tile, which shows what the second one costs).  Blocks of 16 wavefronts, like the
// demapper's, leave 128 registers per lane, so the products stay in ordinary vector
// registers as they do there.
constexpr int kMixTiles = 8;
constexpr int kMixGroup = 8;
constexpr int kMixThreads = 1024;

template <int KS, int NH>
__global__ void __launch_bounds__(kMixThreads) ub_tile_mix_kernel(int64_t iters, float seed, float* sink) {
  __shared__ uint4 frag[kMixTiles * KS * 64];
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < kMixTiles * KS * 64; i += kMixThreads) {
    half8 h;
#pragma unroll
    for (int v = 0; v < 8; ++v) h[v] = static_cast<_Float16>(seed * static_cast<float>((i + v) & 15) - 0.004f);
    __builtin_memcpy(&frag[i], &h, 16);
  }
  __syncthreads();
  half8 bf[KS], ah[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int v = 0; v < 8; ++v) bf[ks][v] = static_cast<_Float16>(seed * static_cast<float>((lane + v + ks) & 31));
  float pos[16], tg[kMixGroup], h0[NH], h1[NH], gt = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) pos[r] = 0.0f;
#pragma unroll
  for (int i = 0; i < kMixGroup; ++i) tg[i] = 0.0f;
#pragma unroll
  for (int q = 0; q < NH; ++q) h0[q] = h1[q] = 0.0f;
  floatx16 cur;
#pragma unroll
  for (int r = 0; r < 16; ++r) cur[r] = 0.0f;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    __builtin_memcpy(&ah[ks], &frag[ks * 64 + lane], 16);
    cur = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[ks], bf[ks], cur, 0, 0, 0);
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) __builtin_memcpy(&ah[ks], &frag[(KS + ks) * 64 + lane], 16);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kMixGroup; ++i) {
      floatx16 nxt;
#pragma unroll
      for (int r = 0; r < 16; ++r) nxt[r] = 0.0f;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) nxt = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[ks], bf[ks], nxt, 0, 0, 0);
      const int t = (i + 2) & (kMixTiles - 1);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) __builtin_memcpy(&ah[ks], &frag[(t * KS + ks) * 64 + lane], 16);
      __builtin_amdgcn_sched_barrier(0);
      float v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        v[r] = __builtin_amdgcn_exp2f(cur[r]);
        pos[r] += v[r];
      }
#pragma unroll
      for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
        for (int r = 0; r < w; ++r) v[r] += v[r + w];
      tg[i] += v[0];
      gt = (i == 0) ? v[0] : gt + v[0];
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
    }
    const int grp = static_cast<int>(it);
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      const bool bit = (grp >> q) & 1;
      h1[q] += bit ? gt : 0.0f;
      h0[q] += bit ? 0.0f : gt;
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int k = 0; k < 16; ++k) r += pos[k];
#pragma unroll
  for (int i = 0; i < kMixGroup; ++i) r += tg[i];
#pragma unroll
  for (int q = 0; q < NH; ++q) r += h0[q] * h1[q];
  if (r == kNever) sink[0] = r;
}

// KIND 0: v_mfma_f32_32x32x16_f16, 1: v_mfma_f32_32x32x16_bf16, 2: v_mfma_f32_32x32x2_f32
template <int KIND>
__global__ void __launch_bounds__(kThreads) ub_mfma_kernel(int64_t iters, float seed, float* sink) {
  floatx16 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  const float a0 = seed * static_cast<float>(threadIdx.x & 63);
  half8 ah, bh;
  bf16x8 ab, bb;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    ah[v] = static_cast<_Float16>(a0 + v);
    bh[v] = static_cast<_Float16>(a0 - v);
    ab[v] = static_cast<__bf16>(a0 + v);
    bb[v] = static_cast<__bf16>(a0 - v);
  }
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (KIND == 0) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, acc[j], 0, 0, 0);
      if constexpr (KIND == 1) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, bb, acc[j], 0, 0, 0);
      if constexpr (KIND == 2) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, a0 + 1.0f, acc[j], 0, 0, 0);
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) r += acc[j][e];
  if (r == kNever) sink[0] = r;
}

__global__ void __launch_bounds__(kThreads) ub_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                           int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

constexpr double kMfmaFlop[3] = {2.0 * 32 * 32 * 16, 2.0 * 32 * 32 * 16, 2.0 * 32 * 32 * 2};
constexpr int64_t kDefaultIters[10] = {8192, 8192, 4096, 4096, 2048, 0, 8192, 1024, 512, 1024};

int launch_kind(int kind, int64_t work, int blocks, const void* d_src, void* d_dst, float* sink, hipStream_t s) {
  const int64_t iters = work > 0 ? work : kDefaultIters[kind];
  switch (kind) {
    case MD_UB_EXP: hipLaunchKernelGGL(ub_exp_kernel, dim3(blocks), dim3(kThreads), 0, s, iters, 1e-3f, sink); break;
    case MD_UB_ADD_F32: hipLaunchKernelGGL(ub_add_kernel, dim3(blocks), dim3(kThreads), 0, s, iters, 1e-3f, sink); break;
    case MD_UB_MFMA_F16:
      hipLaunchKernelGGL(ub_mfma_kernel<0>, dim3(blocks), dim3(kThreads), 0, s, iters, 1e-3f, sink);
      break;
    case MD_UB_MFMA_BF16:
      hipLaunchKernelGGL(ub_mfma_kernel<1>, dim3(blocks), dim3(kThreads), 0, s, iters, 1e-3f, sink);
      break;
    case MD_UB_MFMA_F32:
      hipLaunchKernelGGL(ub_mfma_kernel<2>, dim3(blocks), dim3(kThreads), 0, s, iters, 1e-3f, sink);
      break;
    case MD_UB_EXP_ADD2:
      hipLaunchKernelGGL(ub_exp_add2_kernel, dim3(blocks), dim3(kThreads), 0, s, iters, 1e-3f, sink);
      break;
    case MD_UB_TILE_MIX:
      hipLaunchKernelGGL((ub_tile_mix_kernel<2, 3>), dim3(blocks / 4), dim3(kMixThreads), 0, s, iters, 1e-3f, sink);
      break;
    case MD_UB_TILE_MIX4:
      hipLaunchKernelGGL((ub_tile_mix_kernel<4, 8>), dim3(blocks / 4), dim3(kMixThreads), 0, s, iters, 1e-3f, sink);
      break;
    case MD_UB_TILE_MIX1:
      hipLaunchKernelGGL((ub_tile_mix_kernel<1, 3>), dim3(blocks / 4), dim3(kMixThreads), 0, s, iters, 1e-3f, sink);
      break;
    default: {
      const int64_t n = work / 16;
      int64_t g = (n + kThreads - 1) / kThreads;
      if (g > blocks) g = blocks;
      if (g < 1) g = 1;
      hipLaunchKernelGGL(ub_copy_kernel, dim3(static_cast<unsigned>(g)), dim3(kThreads), 0, s,
                         static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), n);
    }
  }
  MD_LAUNCH_CHECK("ubench kernel launch");
  return MD_OK;
}

}  // namespace
}  // namespace md

extern "C" {

int ubench(int kind, int64_t work, const void* d_src, void* d_dst, double* h_rate, double* h_ms, void* stream) {
  using namespace md;
  if (kind < MD_UB_EXP || kind > MD_UB_TILE_MIX1) return fail(MD_EINVAL, "ubench: unknown kind");
  if (work < 0) return fail(MD_EINVAL, "ubench: work must be >= 0");
  if (kind == MD_UB_COPY) {
    if (d_src == nullptr || d_dst == nullptr) return fail(MD_EINVAL, "ubench: the copy needs d_src and d_dst");
    if (work <= 0 || work % 16 != 0) return fail(MD_EINVAL, "ubench: the copy needs work > 0, a multiple of 16");
    if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) % 16 != 0)
      return fail(MD_EINVAL, "ubench: copy buffers must be 16-byte aligned");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, ncu = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  MD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = ncu * 8;
  char* ws = nullptr;
  if (int st = workspace(s, 256, &ws); st != MD_OK) return st;
  float* sink = reinterpret_cast<float*>(ws);
  hipEvent_t e0, e1;
  MD_HIP_TRY(hipEventCreate(&e0));
  if (hipError_t e = hipEventCreate(&e1); e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  int st = launch_kind(kind, work, blocks, d_src, d_dst, sink, s);   // warm-up
  hipError_t he = hipSuccess;
  if (st == MD_OK) he = hipEventRecord(e0, s);
  if (st == MD_OK && he == hipSuccess) st = launch_kind(kind, work, blocks, d_src, d_dst, sink, s);
  if (st == MD_OK && he == hipSuccess) he = hipEventRecord(e1, s);
  if (st == MD_OK && he == hipSuccess) he = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (st == MD_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MD_OK) return st;
  if (he != hipSuccess) return hip_fail(he, "ubench timing");
  const double sec = static_cast<double>(ms) * 1e-3;
  const int64_t iters = work > 0 ? work : (kind != MD_UB_COPY ? kDefaultIters[kind] : 0);
  const double lanes = static_cast<double>(blocks) * kThreads;
  const double waves = lanes / 64.0;
  double amount = 0.0;
  switch (kind) {
    case MD_UB_EXP:
    case MD_UB_EXP_ADD2:
    case MD_UB_ADD_F32: amount = lanes * static_cast<double>(iters) * kChains; break;
    case MD_UB_TILE_MIX:
    case MD_UB_TILE_MIX4:
    case MD_UB_TILE_MIX1: amount = lanes * static_cast<double>(iters) * kMixGroup * 16; break;
    case MD_UB_MFMA_F16:
    case MD_UB_MFMA_BF16:
    case MD_UB_MFMA_F32:
      amount = waves * static_cast<double>(iters) * 4.0 * kMfmaFlop[kind - MD_UB_MFMA_F16];
      break;
    default: amount = 2.0 * static_cast<double>(work);
  }
  if (h_rate) *h_rate = sec > 0.0 ? amount / sec : 0.0;
  if (h_ms) *h_ms = static_cast<double>(ms);
  return MD_OK;
}

}  // extern "C"
