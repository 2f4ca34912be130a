// Allocation-free variant of llr_exact, for callers that cannot allocate device memory
// (work under stream capture, tight serving loops, harnesses that forbid hipMalloc).
// The label-ordered constellation, the MFMA fragments, the stage counters and the
// fallback lists that llr_exact carves from its per-stream workspace are carved here
// from one file-scope device array instead.  Each device the library runs on holds its
// own copy of the array until the process ends; every call on a device shares that copy,
// so calls that overlap on one device (on different streams, or from different threads)
// race.  The counters are cleared by the prep kernels of each call.
#include <mutex>

#include "common.hpp"
#include "llr_kernels.hpp"

namespace md {
namespace {

constexpr size_t kScratchBytes = size_t(24) << 20;   // 24 MiB per device
constexpr int64_t kMaxN = int64_t(1) << 20;           // symbols per call
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device, with the
// device current).  The array's name in host code is only a host-side handle.
int scratch_on(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MD_ENODEV, "llr_exact_noalloc: device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MD_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return MD_OK;
}

}  // namespace
}  // namespace md

extern "C" {

int llr_exact_noalloc(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N,
                      double sigma2, int prec, float* d_llr, void* stream) {
  md::set_error("");
  int st = md::check_demap_args(d_X, d_labels, M, D, d_y, N, sigma2, prec, d_llr);
  if (st != MD_OK) return st;
  if (N > md::kMaxN) return md::fail(MD_EINVAL, "llr_exact_noalloc: N above 2^20 symbols per call");
  const size_t need = md::prep_bytes(M, D, N);
  if (need > md::kScratchBytes)
    return md::fail(MD_EINVAL, "llr_exact_noalloc: needs " + std::to_string(need) +
                                   " bytes of scratch, above the 24 MiB limit");
  int dev = 0;
  st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = md::check_labels_once(d_labels, M, s);
  if (st != MD_OK) return st;
  if (N == 0) return MD_OK;
  char* ws = nullptr;
  st = md::scratch_on(dev, &ws);
  if (st != MD_OK) return st;
  float alpha = 1.0f, c_over_alpha = 1.0f;
  md::score_scales(sigma2, &alpha, &c_over_alpha);
  md::Prepared P;
  // flags == nullptr: the stage counters are carved from the scratch array as well
  st = md::prepare(d_X, d_labels, M, D, N, alpha, c_over_alpha, ws, s, &P, nullptr, md::score_layout(prec));
  if (st != MD_OK) return st;
  return md::launch_llr(P, M, D, d_y, N, sigma2, false, prec, d_llr, s);
}

}  // extern "C"
