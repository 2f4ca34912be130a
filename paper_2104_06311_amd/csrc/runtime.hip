// Host runtime of the library: error strings, per-(device, stream) workspaces and the
// host-side label check cache.
#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "common.hpp"

namespace md {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();   // consume the error so that later checks do not report it again
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory) return MD_ENOMEM;
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return MD_ENODEV;
  return MD_EHIP;
}

int current_device(int* dev) {
  (void)hipGetLastError();   // a stale error of earlier, unrelated work must not be reported here
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(MD_ENODEV, "no GPU visible");
  MD_HIP_TRY(hipGetDevice(dev));
  return MD_OK;
}

namespace {
// allocation-failure injection (alloc_fault_inject): -1 off, k >= 0 the k-th next fails
std::atomic<int> g_fail_in{-1};
}  // namespace

namespace {
std::mutex g_live_mu;
std::unordered_map<void*, size_t> g_live;   // device allocations the library holds
}  // namespace

hipError_t dev_malloc(void** p, size_t bytes) {
  int k = g_fail_in.load();
  while (k >= 0) {
    if (g_fail_in.compare_exchange_weak(k, k - 1)) {
      if (k == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
      }
      break;
    }
  }
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live[*p] = bytes;
  }
  return e;
}

hipError_t dev_free(void* p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.erase(p);
  }
  return hipFree(p);
}

namespace {
struct WsEntry {
  char* ptr = nullptr;
  size_t cap = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, WsEntry> g_ws;

std::mutex g_lab_mu;
std::set<std::tuple<int, const uint32_t*, int>> g_lab_ok;

struct FlagsEntry {
  int* ptr = nullptr;
  LastCall last;
};
std::mutex g_fl_mu;
std::map<std::pair<int, hipStream_t>, FlagsEntry> g_fl;
}  // namespace

namespace {
struct TimingEntry {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;   // recorded, not yet read
  std::vector<hipEvent_t> pool;                           // created, free
};
std::mutex g_tm_mu;
std::map<std::pair<int, hipStream_t>, TimingEntry> g_tm;

hipEvent_t pool_event(TimingEntry& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void drop_events(TimingEntry& t) {
  for (auto& pr : t.pairs) {
    if (pr.first) (void)hipEventDestroy(pr.first);
    if (pr.second) (void)hipEventDestroy(pr.second);
  }
  for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
  t.pairs.clear();
  t.pool.clear();
}
}  // namespace

int timing_begin(hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  std::lock_guard<std::mutex> lk(g_tm_mu);
  auto it = g_tm.find({dev, stream});
  if (it == g_tm.end() || !it->second.on) return -1;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return -1;
  }
  TimingEntry& t = it->second;
  hipEvent_t a = pool_event(t), b = pool_event(t);
  if (!a || !b || hipEventRecord(a, stream) != hipSuccess) {
    (void)hipGetLastError();
    if (a) t.pool.push_back(a);
    if (b) t.pool.push_back(b);
    return -1;
  }
  t.pairs.emplace_back(a, b);
  return static_cast<int>(t.pairs.size()) - 1;
}

void timing_end(hipStream_t stream, int slot) {
  if (slot < 0) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> lk(g_tm_mu);
  auto it = g_tm.find({dev, stream});
  if (it == g_tm.end() || slot >= static_cast<int>(it->second.pairs.size())) return;
  if (hipEventRecord(it->second.pairs[static_cast<size_t>(slot)].second, stream) != hipSuccess) {
    (void)hipGetLastError();
    it->second.pairs[static_cast<size_t>(slot)].second = nullptr;
  }
}

namespace {
std::mutex g_attr_mu;
std::set<std::tuple<int, const void*, int>> g_attr_done;
}  // namespace

int set_lds_limit(const void* kern, int bytes) {
  int dev = 0;
  MD_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_attr_mu);
  if (g_attr_done.count({dev, kern, bytes})) return MD_OK;
  MD_HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  g_attr_done.insert({dev, kern, bytes});
  return MD_OK;
}

int stream_flags(hipStream_t stream, int** out) {
  int dev = 0;
  int st = current_device(&dev);
  if (st != MD_OK) return st;
  std::lock_guard<std::mutex> lk(g_fl_mu);
  FlagsEntry& f = g_fl[{dev, stream}];
  if (!f.ptr) {
    void* p = nullptr;
    hipError_t e = dev_malloc(&p, 256);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MD_ENOMEM, "allocation of the stage counters failed");
    }
    // the GMI status word (bytes 128..135) reads 0 until a GMI call writes it
    e = hipMemset(p, 0, 256);
    if (e != hipSuccess) {
      (void)dev_free(p);
      return hip_fail(e, "hipMemset(stage counters)");
    }
    f.ptr = static_cast<int*>(p);
  }
  *out = f.ptr;
  return MD_OK;
}

void record_last_call(hipStream_t stream, const LastCall& lc) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> lk(g_fl_mu);
  g_fl[{dev, stream}].last = lc;
}

int last_call(hipStream_t stream, LastCall* lc, int** flags) {
  int dev = 0;
  int st = current_device(&dev);
  if (st != MD_OK) return st;
  std::lock_guard<std::mutex> lk(g_fl_mu);
  auto it = g_fl.find({dev, stream});
  if (it == g_fl.end() || !it->second.ptr) {
    *lc = LastCall{};
    *flags = nullptr;
    return MD_OK;
  }
  *lc = it->second.last;
  *flags = it->second.ptr;
  return MD_OK;
}

int workspace(hipStream_t stream, size_t bytes, char** out) {
  int dev = 0;
  int st = current_device(&dev);
  if (st != MD_OK) return st;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  WsEntry& w = g_ws[{dev, stream}];
  if (w.cap < bytes) {
    size_t cap = bytes + bytes / 4 + (1 << 20);
    if (w.ptr) {
      // the old buffer may still be in use by work queued on this stream
      MD_HIP_TRY(hipStreamSynchronize(stream));
      MD_HIP_TRY(dev_free(w.ptr));
      w.ptr = nullptr;
      w.cap = 0;
    }
    void* p = nullptr;
    hipError_t e = dev_malloc(&p, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MD_ENOMEM, "workspace allocation of " + std::to_string(cap) + " bytes failed");
    }
    w.ptr = static_cast<char*>(p);
    w.cap = cap;
  }
  *out = w.ptr;
  return MD_OK;
}

int check_labels_once(const uint32_t* d_labels, int M, hipStream_t stream) {
  int dev = 0;
  int st = current_device(&dev);
  if (st != MD_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_lab_mu);
    if (g_lab_ok.count({dev, d_labels, M})) return MD_OK;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  MD_HIP_TRY(hipStreamIsCapturing(stream, &cap));
  if (cap != hipStreamCaptureStatusNone) return MD_OK;   // the device-side check still applies
  std::vector<uint32_t> h(static_cast<size_t>(M));
  MD_HIP_TRY(hipMemcpyAsync(h.data(), d_labels, sizeof(uint32_t) * M, hipMemcpyDeviceToHost, stream));
  MD_HIP_TRY(hipStreamSynchronize(stream));
  std::vector<char> seen(static_cast<size_t>(M), 0);
  for (int j = 0; j < M; ++j) {
    if (h[j] >= static_cast<uint32_t>(M))
      return fail(MD_ELABEL, "label " + std::to_string(h[j]) + " of point " + std::to_string(j) +
                                 " is outside [0, M)");
    if (seen[h[j]]) return fail(MD_ELABEL, "label " + std::to_string(h[j]) + " is used twice");
    seen[h[j]] = 1;
  }
  std::lock_guard<std::mutex> lk(g_lab_mu);
  g_lab_ok.insert({dev, d_labels, M});
  return MD_OK;
}

// Frees the workspace and the stage counters of one (current device, stream) pair; the
// caller has synchronised the stream and is about to destroy it.
int release_stream_resources(hipStream_t stream) {
  int dev = 0;
  int st = current_device(&dev);
  if (st != MD_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({dev, stream});
    if (it != g_ws.end()) {
      if (it->second.ptr) MD_HIP_TRY(dev_free(it->second.ptr));
      g_ws.erase(it);
    }
  }
  std::lock_guard<std::mutex> lk(g_fl_mu);
  auto it = g_fl.find({dev, stream});
  if (it != g_fl.end()) {
    if (it->second.ptr) MD_HIP_TRY(dev_free(it->second.ptr));
    g_fl.erase(it);
  }
  return MD_OK;
}

int release_workspaces() {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (!g_ws.empty()) MD_HIP_TRY(hipDeviceSynchronize());
  for (auto& kv : g_ws) {
    if (kv.second.ptr) {
      int cur = 0;
      MD_HIP_TRY(hipGetDevice(&cur));
      MD_HIP_TRY(hipSetDevice(kv.first.first));
      hipError_t e = dev_free(kv.second.ptr);
      MD_HIP_TRY(hipSetDevice(cur));
      if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
    }
  }
  g_ws.clear();
  {
    std::lock_guard<std::mutex> lk2(g_lab_mu);
    g_lab_ok.clear();
  }
  std::lock_guard<std::mutex> lk3(g_fl_mu);
  for (auto& kv : g_fl) {
    if (kv.second.ptr) {
      int cur = 0;
      MD_HIP_TRY(hipGetDevice(&cur));
      MD_HIP_TRY(hipSetDevice(kv.first.first));
      hipError_t e = dev_free(kv.second.ptr);
      MD_HIP_TRY(hipSetDevice(cur));
      if (e != hipSuccess) return hip_fail(e, "hipFree(stage counters)");
    }
  }
  g_fl.clear();
  return MD_OK;
}

}  // namespace md

extern "C" {

int alloc_fault_inject(int k) {
  md::set_error("");
  md::g_fail_in.store(k < 0 ? -1 : k);
  return MD_OK;
}

int alloc_stats(int64_t* live_bytes, int64_t* live_allocs) {
  md::set_error("");
  if (!live_bytes || !live_allocs) return md::fail(MD_EINVAL, "output pointer is NULL");
  std::lock_guard<std::mutex> lk(md::g_live_mu);
  int64_t b = 0;
  for (const auto& kv : md::g_live) b += static_cast<int64_t>(kv.second);
  *live_bytes = b;
  *live_allocs = static_cast<int64_t>(md::g_live.size());
  return MD_OK;
}

int kernel_timing(int enable, void* stream) {
  md::set_error("");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(md::g_tm_mu);
  md::TimingEntry& t = md::g_tm[{dev, s}];
  if (!enable) {
    MD_HIP_TRY(hipStreamSynchronize(s));
    md::drop_events(t);
  }
  t.on = enable != 0;
  return MD_OK;
}

int kernel_timing_read(double* total_ms, int64_t* launches, void* stream) {
  md::set_error("");
  if (!total_ms || !launches) return md::fail(MD_EINVAL, "output pointer is NULL");
  *total_ms = 0.0;
  *launches = 0;
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(md::g_tm_mu);
  auto it = md::g_tm.find({dev, s});
  if (it == md::g_tm.end()) return MD_OK;
  md::TimingEntry& t = it->second;
  MD_HIP_TRY(hipStreamSynchronize(s));
  double sum = 0.0;
  int64_t n = 0;
  for (auto& pr : t.pairs) {
    float ms = 0.0f;
    if (pr.second && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      sum += ms;
      ++n;
    } else {
      (void)hipGetLastError();
    }
    t.pool.push_back(pr.first);
    if (pr.second) t.pool.push_back(pr.second);
  }
  t.pairs.clear();
  *total_ms = sum;
  *launches = n;
  return MD_OK;
}

int release_cache(void) {
  md::set_error("");
  return md::release_workspaces();
}

const char* last_error(void) { return md::g_last_error.c_str(); }

int mdemap_version(void) { return 100; }

}  // extern "C"
