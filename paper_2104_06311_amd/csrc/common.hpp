// Internal definitions shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/mdemap.h"

namespace md {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define MD_HIP_TRY(expr)                                  \
  do {                                                    \
    hipError_t md_e_ = (expr);                            \
    if (md_e_ != hipSuccess) return md::hip_fail(md_e_, #expr); \
  } while (0)

// Checks that a launch was accepted (grid/block/LDS limits).
#define MD_LAUNCH_CHECK(name)                                          \
  do {                                                                 \
    hipError_t md_e_ = hipGetLastError();                              \
    if (md_e_ != hipSuccess) return md::hip_fail(md_e_, name);         \
  } while (0)

inline int ilog2_pow2(int M) {
  int m = 0;
  while ((1 << m) < M) ++m;
  return m;
}
inline bool is_pow2(int M) { return M >= 2 && (M & (M - 1)) == 0; }

// ---------------------------------------------------------------- workspace
// One growable device buffer per (device, stream); sub-buffers are carved from it
// with 256-byte alignment.
struct Carver {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};
inline size_t carve_size(size_t bytes) { return ((bytes + 255) & ~size_t(255)); }

// Returns a device buffer of at least `bytes` bytes private to (current device, stream).
int workspace(hipStream_t stream, size_t bytes, char** out);

// hipMalloc behind the library's allocation-failure injection (alloc_fault_inject): every
// device allocation the library makes goes through here.
hipError_t dev_malloc(void** p, size_t bytes);
// hipFree of memory from dev_malloc (keeps the library's count of live allocations).
hipError_t dev_free(void* p);

// Stage counters of the demapping calls on (current device, stream): a 16-byte device
// buffer that stays at one address until release_cache, plus what the last call was.
struct LastCall {
  bool valid = false;
  bool maxlog = false;
  int64_t N = 0;
};
int stream_flags(hipStream_t stream, int** out);
// The GMI status word inside a stream's counter buffer: the number of symbols whose
// loss term was not finite in the last gmi_reduce / llr_exact_gmi on that stream.
inline long long* gmi_status_word(int* flags) { return reinterpret_cast<long long*>(flags + 32); }
void record_last_call(hipStream_t stream, const LastCall& lc);
int last_call(hipStream_t stream, LastCall* lc, int** flags);

// Host-side label check cache: returns MD_OK if the labels at d_labels (M entries)
// form a permutation; checks on the host the first time (pointer, M) is seen.
int check_labels_once(const uint32_t* d_labels, int M, hipStream_t stream);

int current_device(int* dev);

// Raises the dynamic-LDS limit of kernel `kern` to `bytes` on the current device.  The
// attribute belongs to a (kernel, device) pair, so it is set once per pair.
int set_lds_limit(const void* kern, int bytes);

// Event timing of the demappers' fast kernel on one (current device, stream) pair, when
// switched on by kernel_timing(): timing_begin records the first event of a pair before
// the launch and returns its slot (or -1 when timing is off or the stream is capturing),
// timing_end records the second after it.
// The DD-LMS equaliser's launcher (ddlms.hip): every instance starts from the taps t0_h /
// t0_g (host, 8 doubles each) or, when d_h_in / d_g_in are given, from its own B x 8 device
// taps (which may be d_h / d_g themselves).
int launch_ddlms(const float* d_x, int64_t B, int64_t N, const float* d_C, int M, const double* t0_h,
                 const double* t0_g, const double* d_h_in, const double* d_g_in, double mu, uint32_t* d_dec,
                 float* d_z, double* d_h, double* d_g, hipStream_t stream);

int timing_begin(hipStream_t stream);
void timing_end(hipStream_t stream, int slot);

// ---------------------------------------------------------------- prepared constellation
// Device-side view of a prepared constellation (label order).
struct Prepared {
  const float* xl;          // M x D float32, row s = point with label s
  const uint4* frag;        // MFMA A-operand fragments (see prep.hip)
  int* flags;               // [0] labels invalid, [1] first fallback count, [2] constellation
                            // outside the FP16 split range, [3] second fallback count,
                            // [4] third fallback count (8 ints)
  unsigned* fb_list;        // symbols the fast pass could not finish (capacity N); after the
                            // second pass it is reused for the third list (careful kernel)
  unsigned* fb_list2;       // symbols left after the two-window pass (capacity N)
  int ks;                   // number of 16-slot K steps of the fragment
  int sc;                   // score contraction: 0 split FP16, 1 one FP16 pass, 2 one BF16 pass
  float alpha;              // power-of-two operand balance a
  float c_over_alpha;       // c / a, c = log2(e) / (2 sigma2)
  // fused GMI epilogue (llr_exact_gmi): transmitted indices, labels and the per-symbol loss
  // terms T_n the fast pass writes (NaN for symbols it leaves to later passes); all null
  // when the call only demaps
  const uint32_t* gmi_tx = nullptr;
  const uint32_t* gmi_labels = nullptr;
  float* gmi_terms = nullptr;
  // per-point score terms of the one-thread-per-symbol demapper (label order, D + 1 floats
  // per point: 2c x_j, then -c ||x_j||^2); null for the shapes it does not take
  const float* vx = nullptr;
};

// Builds the label-ordered copy, fragments and flags for one call.  `ws` must point
// at a workspace of at least prep_bytes(M, D, N) bytes.
size_t prep_bytes(int M, int D, int64_t N);   // an upper bound for every fragment layout
// `flags` (8 ints) may be given by the caller; otherwise they are carved from ws.
// sc selects the fragment layout of the score contraction (Prepared::sc).
int prepare(const float* d_X, const uint32_t* d_labels, int M, int D, int64_t N, float alpha,
            float c_over_alpha, char* ws, hipStream_t stream, Prepared* out, int* flags = nullptr, int sc = 0);

int frag_ksteps(int D);    // ceil((3 D + 4) / 16) steps of 16 K slots (split FP16 scores)
int frag_ksteps_single(int D);   // ceil((D + 4) / 16) steps (one-pass FP16 or BF16 scores)

}  // namespace md
