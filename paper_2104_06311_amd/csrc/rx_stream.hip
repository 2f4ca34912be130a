// Streaming receiver (rx_* in mdemap.h): a host-resident symbol stream cut into buffers
// that go round-robin to several HIP streams ("lanes").  Per buffer a lane copies the
// symbols in, demaps them with the library's own entry points, reduces the statistics of
// the bins the buffer touches and copies the results out; an event at the end of each
// buffer lets the host retire it, fold its statistics in stream order and reuse the lane.
// With the equaliser stage a buffer's samples pass the DD-LMS equaliser first; its taps
// carry over from buffer to buffer, so each lane's equaliser waits for an event that the
// previous buffer's lane records after its own (a dependency chain through the lanes),
// while the copies and demapping of neighbouring buffers run beside it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace md {

int release_stream_resources(hipStream_t stream);

namespace {

// Hard decision from the LLR signs: label bit m-1-k is 1 where column k is negative (for
// max-log LLRs, the label of the nearest point).
__global__ void __launch_bounds__(256) rx_decide_kernel(const float* __restrict__ llr, int64_t N, int m,
                                                        uint32_t* __restrict__ dec) {
  const int64_t n = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (n >= N) return;
  uint32_t lab = 0;
  for (int k = 0; k < m; ++k) lab = (lab << 1) | (llr[n * m + k] < 0.0f ? 1u : 0u);
  dec[n] = lab;
}

constexpr int kMaxPieces = 2;   // a bin spans at least one buffer: a buffer touches <= 2 bins

struct PieceResult {
  double gmi[kMaxPieces];
  unsigned long long err[kMaxPieces];
};

struct Lane {
  hipStream_t s = nullptr;
  hipEvent_t beg = nullptr, end = nullptr;
  hipEvent_t eq = nullptr;           // after the buffer's equaliser (equaliser stage only)
  float* x = nullptr;                // the buffer's samples (equaliser stage only)
  float* y = nullptr;
  uint32_t* tx = nullptr;
  float* llr = nullptr;
  uint32_t* dec = nullptr;
  PieceResult* d_res = nullptr;      // device
  PieceResult* h_res = nullptr;      // pinned host
  bool busy = false;                 // a buffer is in flight
  int n_pieces = 0;
  int64_t piece_bin[kMaxPieces] = {0, 0};
  int64_t piece_n[kMaxPieces] = {0, 0};
};

}  // namespace

struct RxStream {
  int M = 0, D = 0, m = 0, mode = 0, S = 0, device = 0;
  int64_t B = 0, bin = 0;
  double sigma2 = 0.0;
  float* X = nullptr;
  uint32_t* labels = nullptr;
  std::vector<Lane> lanes;
  // equaliser stage: P channels, their taps (P x 8 doubles each, carried across buffers)
  int64_t P = 0;
  double mu = 0.0, h0[8] = {}, g0[8] = {};
  double* th = nullptr;
  double* tg = nullptr;
};

namespace {

int is_pinned(const void* p) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return a.type == hipMemoryTypeHost ? 1 : 0;
}

// Demap nb symbols of a lane (the mode's LLRs into lane.llr).
int lane_demap(RxStream* r, Lane& L, int64_t nb) {
  if (r->mode == MD_RX_EXACT)
    return llr_exact(r->X, r->labels, r->M, r->D, L.y, nb, r->sigma2, MD_PREC_FP32, L.llr, L.s);
  return llr_maxlog(r->X, r->labels, r->M, r->D, L.y, nb, r->sigma2, L.llr, L.s);
}

// Waits for the lane's buffer, folds its statistics and records its latency.
int retire(RxStream* r, Lane& L, std::vector<double>* sumT, std::vector<double>* cnt,
           std::vector<unsigned long long>* err, double* lat_sum, double* lat_max, int64_t* n_lat) {
  if (!L.busy) return MD_OK;
  MD_HIP_TRY(hipEventSynchronize(L.end));
  float ms = 0.0f;
  MD_HIP_TRY(hipEventElapsedTime(&ms, L.beg, L.end));
  *lat_sum += ms;
  *lat_max = std::max(*lat_max, static_cast<double>(ms));
  *n_lat += 1;
  for (int p = 0; p < L.n_pieces; ++p) {
    const int64_t b = L.piece_bin[p];
    if (b < 0 || (err && b >= static_cast<int64_t>(err->size()))) return fail(MD_EINVAL, "bin index out of range");
    const double n = static_cast<double>(L.piece_n[p]);
    if (sumT) (*sumT)[b] += (r->m - L.h_res->gmi[p]) * n;   // the piece's sum of GMI terms
    if (cnt) (*cnt)[b] += n;
    if (err) (*err)[b] += L.h_res->err[p];
  }
  L.busy = false;
  return MD_OK;
}

void free_lane(Lane& L) {
  if (L.s) {
    (void)hipStreamSynchronize(L.s);
    (void)release_stream_resources(L.s);
  }
  if (L.x) (void)md::dev_free(L.x);
  if (L.y) (void)md::dev_free(L.y);
  if (L.tx) (void)md::dev_free(L.tx);
  if (L.llr) (void)md::dev_free(L.llr);
  if (L.dec) (void)md::dev_free(L.dec);
  if (L.d_res) (void)md::dev_free(L.d_res);
  if (L.h_res) (void)hipHostFree(L.h_res);
  if (L.beg) (void)hipEventDestroy(L.beg);
  if (L.end) (void)hipEventDestroy(L.end);
  if (L.eq) (void)hipEventDestroy(L.eq);
  if (L.s) (void)hipStreamDestroy(L.s);
  L = Lane{};
}

void destroy(RxStream* r) {
  for (Lane& L : r->lanes) free_lane(L);
  if (r->th) (void)md::dev_free(r->th);
  if (r->tg) (void)md::dev_free(r->tg);
  if (r->X) (void)md::dev_free(r->X);
  if (r->labels) (void)md::dev_free(r->labels);
  (void)hipGetLastError();
  delete r;
}

template <class T>
int dev_alloc(T** p, size_t count) {
  void* q = nullptr;
  if (md::dev_malloc(&q, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MD_ENOMEM, "streaming receiver: device allocation failed");
  }
  *p = static_cast<T*>(q);
  return MD_OK;
}

}  // namespace
}  // namespace md

extern "C" {

int rx_create(const float* d_X, const uint32_t* d_labels, int M, int D, double sigma2, const md_rx_config* cfg,
              void** out) {
  md::set_error("");
  if (!out) return md::fail(MD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_X || !d_labels || !cfg) return md::fail(MD_EINVAL, "constellation, labels or config pointer is NULL");
  if (M < 2 || M > 65536 || !md::is_pow2(M))
    return md::fail(MD_ENOTPOW2, "M=" + std::to_string(M) + " is not a power of two in [2, 65536]");
  if (D < 1 || D > 30) return md::fail(MD_EDIM, "D=" + std::to_string(D) + " is outside [1, 30]");
  if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return md::fail(MD_EINVAL, "sigma2 must be finite and > 0");
  if (cfg->mode != MD_RX_HARD && cfg->mode != MD_RX_EXACT) return md::fail(MD_EINVAL, "unknown receiver mode");
  if (cfg->n_streams < 1 || cfg->n_streams > 8) return md::fail(MD_EINVAL, "n_streams must be in [1, 8]");
  if (cfg->buf_symbols < 1 || cfg->buf_symbols > (int64_t(1) << 24))
    return md::fail(MD_EINVAL, "buf_symbols must be in [1, 2^24]");
  if (cfg->bin_symbols < cfg->buf_symbols) return md::fail(MD_EINVAL, "bin_symbols must be >= buf_symbols");
  if (cfg->eq_instances < 0) return md::fail(MD_EINVAL, "eq_instances must be >= 0");
  if (cfg->eq_instances > 0) {
    if (D != 2) return md::fail(MD_EINVAL, "the equaliser stage needs a 2D (complex) constellation");
    if (M > 1024) return md::fail(MD_EINVAL, "the equaliser stage takes M <= 1024 reference points");
    if (cfg->buf_symbols % cfg->eq_instances != 0)
      return md::fail(MD_EINVAL, "buf_symbols must be a multiple of eq_instances");
    if (!(cfg->eq_mu >= 0.0) || !std::isfinite(cfg->eq_mu)) return md::fail(MD_EINVAL, "eq_mu must be finite and >= 0");
    for (int i = 0; i < 8; ++i)
      if (!std::isfinite(cfg->eq_h0[i]) || !std::isfinite(cfg->eq_g0[i]))
        return md::fail(MD_EINVAL, "the equaliser's starting taps must be finite");
  }
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  auto* r = new md::RxStream();
  r->M = M;
  r->D = D;
  r->m = md::ilog2_pow2(M);
  r->mode = cfg->mode;
  r->S = cfg->n_streams;
  r->B = cfg->buf_symbols;
  r->bin = cfg->bin_symbols;
  r->sigma2 = sigma2;
  r->device = dev;
  r->P = cfg->eq_instances;
  r->mu = cfg->eq_mu;
  for (int i = 0; i < 8; ++i) {
    r->h0[i] = cfg->eq_h0[i];
    r->g0[i] = cfg->eq_g0[i];
  }
  auto bail = [&](int status) {
    md::destroy(r);
    return status;
  };
  if ((st = md::dev_alloc(&r->X, static_cast<size_t>(M) * D)) != MD_OK) return bail(st);
  if ((st = md::dev_alloc(&r->labels, static_cast<size_t>(M))) != MD_OK) return bail(st);
  hipError_t e = hipMemcpy(r->X, d_X, sizeof(float) * M * D, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(r->labels, d_labels, sizeof(uint32_t) * M, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) return bail(md::hip_fail(e, "copy of the constellation"));
  const size_t B = static_cast<size_t>(r->B);
  if (r->P > 0) {
    if ((st = md::dev_alloc(&r->th, static_cast<size_t>(r->P) * 8)) != MD_OK) return bail(st);
    if ((st = md::dev_alloc(&r->tg, static_cast<size_t>(r->P) * 8)) != MD_OK) return bail(st);
  }
  r->lanes.resize(static_cast<size_t>(r->S));
  for (md::Lane& L : r->lanes) {
    e = hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&L.beg);
    if (e == hipSuccess) e = hipEventCreate(&L.end);
    if (e == hipSuccess && r->P > 0) e = hipEventCreateWithFlags(&L.eq, hipEventDisableTiming);
    if (e != hipSuccess) return bail(md::hip_fail(e, "stream or event creation"));
    if (r->P > 0) {
      // (2n + 2) rows of P complex samples
      const size_t rows = 2 * (B / static_cast<size_t>(r->P)) + 2;
      if ((st = md::dev_alloc(&L.x, rows * static_cast<size_t>(r->P) * 2)) != MD_OK) return bail(st);
    }
    if ((st = md::dev_alloc(&L.y, B * D)) != MD_OK) return bail(st);
    if ((st = md::dev_alloc(&L.tx, B)) != MD_OK) return bail(st);
    if ((st = md::dev_alloc(&L.llr, B * r->m)) != MD_OK) return bail(st);
    if ((st = md::dev_alloc(&L.dec, B)) != MD_OK) return bail(st);
    if ((st = md::dev_alloc(&L.d_res, 1)) != MD_OK) return bail(st);
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(md::PieceResult), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return bail(md::fail(MD_ENOMEM, "streaming receiver: pinned host allocation failed"));
    }
    L.h_res = static_cast<md::PieceResult*>(h);
    // one full buffer of zeros through every stage, so that every workspace of the lane's
    // stream is sized (and the labels are checked) before the first timed run
    e = hipMemsetAsync(L.y, 0, sizeof(float) * B * D, L.s);
    if (e == hipSuccess) e = hipMemsetAsync(L.tx, 0, sizeof(uint32_t) * B, L.s);
    if (e == hipSuccess && r->P > 0)
      e = hipMemsetAsync(L.x, 0, sizeof(float) * 2 * (2 * (B / r->P) + 2) * r->P, L.s);
    if (e != hipSuccess) return bail(md::hip_fail(e, "hipMemsetAsync"));
    if (r->P > 0 &&
        (st = md::launch_ddlms(L.x, r->P, r->B / r->P, r->X, M, r->h0, r->g0, nullptr, nullptr, r->mu, L.dec, L.y,
                               nullptr, nullptr, L.s)) != MD_OK)
      return bail(st);
    if ((st = md::lane_demap(r, L, r->B)) != MD_OK) return bail(st);
    if ((st = gmi_reduce(L.llr, r->B, r->m, L.tx, r->labels, &L.d_res->gmi[0], nullptr, nullptr, L.s)) != MD_OK)
      return bail(st);
    if ((st = ber_count(L.llr, r->B, r->m, L.tx, r->labels, nullptr,
                        reinterpret_cast<uint64_t*>(&L.d_res->err[0]), L.s)) != MD_OK)
      return bail(st);
    e = hipStreamSynchronize(L.s);
    if (e != hipSuccess) return bail(md::hip_fail(e, "hipStreamSynchronize"));
  }
  *out = r;
  return MD_OK;
}

int rx_run(void* rx, const float* h_y, const uint32_t* h_tx, int64_t N, int64_t total, void* h_out,
           uint64_t* h_bin_errors, double* h_bin_gmi, double* h_stats) {
  md::set_error("");
  auto* r = static_cast<md::RxStream*>(rx);
  if (!r) return md::fail(MD_EINVAL, "receiver handle is NULL");
  if (!h_y) return md::fail(MD_EINVAL, "h_y is NULL");
  if (N < 1) return md::fail(MD_EINVAL, "the host ring must hold N >= 1 symbols");
  if (total < 0) return md::fail(MD_EINVAL, "total is negative");
  if (total > N && N % r->B != 0)
    return md::fail(MD_EINVAL, "a ring that is read more than once must hold a multiple of buf_symbols symbols");
  if ((h_bin_errors || h_bin_gmi) && !h_tx) return md::fail(MD_EINVAL, "bin statistics need h_tx");
  if (r->P > 0 && (N % r->P != 0 || total % r->P != 0))
    return md::fail(MD_EINVAL, "with the equaliser stage N and total must be multiples of eq_instances");
  if (!md::is_pinned(h_y) || (h_tx && !md::is_pinned(h_tx)) || (h_out && !md::is_pinned(h_out)))
    return md::fail(MD_EINVAL, "host arrays must be pinned (hipHostMalloc or pin_memory)");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  if (dev != r->device) return md::fail(MD_EINVAL, "the receiver was created on another device");
  for (md::Lane& L : r->lanes) {   // buffers left in flight by a failed earlier run
    if (L.busy) MD_HIP_TRY(hipEventSynchronize(L.end));
    L.busy = false;
  }
  const int64_t n_bins = total > 0 ? (total + r->bin - 1) / r->bin : 0;
  std::vector<double> sumT(static_cast<size_t>(n_bins), 0.0), cnt(static_cast<size_t>(n_bins), 0.0);
  std::vector<unsigned long long> err(static_cast<size_t>(n_bins), 0ull);
  double lat_sum = 0.0, lat_max = 0.0;
  int64_t n_lat = 0;
  const int m = r->m, D = r->D;
  const bool stats = h_tx != nullptr;
  if (r->P > 0) {
    // every run starts the equaliser from the configured taps
    std::vector<double> th(static_cast<size_t>(r->P) * 8), tg(static_cast<size_t>(r->P) * 8);
    for (int64_t b = 0; b < r->P; ++b)
      for (int i = 0; i < 8; ++i) {
        th[static_cast<size_t>(b * 8 + i)] = r->h0[i];
        tg[static_cast<size_t>(b * 8 + i)] = r->g0[i];
      }
    MD_HIP_TRY(hipMemcpy(r->th, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice));
    MD_HIP_TRY(hipMemcpy(r->tg, tg.data(), sizeof(double) * tg.size(), hipMemcpyHostToDevice));
  }
  const md::Lane* prev = nullptr;   // the lane of the previous buffer (equaliser order)
  const auto t0 = std::chrono::steady_clock::now();
  int64_t k = 0;
  for (int64_t i0 = 0; i0 < total; i0 += r->B, ++k) {
    md::Lane& L = r->lanes[static_cast<size_t>(k % r->S)];
    if ((st = md::retire(r, L, &sumT, &cnt, &err, &lat_sum, &lat_max, &n_lat)) != MD_OK) return st;
    const int64_t nb = std::min(r->B, total - i0);
    const int64_t r0 = i0 % N;          // no buffer wraps: N % B == 0 whenever total > N
    MD_HIP_TRY(hipEventRecord(L.beg, L.s));
    if (r->P > 0) {
      // samples of channel rows [2 t0, 2 t0 + 2 nr + 2): the buffer's symbols and the two
      // samples it shares with the next buffer; the equaliser waits for the previous one
      const int64_t t0 = r0 / r->P, nr = nb / r->P;
      MD_HIP_TRY(hipMemcpyAsync(L.x, h_y + 2 * (2 * t0) * r->P, sizeof(float) * 2 * (2 * nr + 2) * r->P,
                                hipMemcpyHostToDevice, L.s));
      if (prev) MD_HIP_TRY(hipStreamWaitEvent(L.s, prev->eq, 0));
      if ((st = md::launch_ddlms(L.x, r->P, nr, r->X, r->M, nullptr, nullptr, r->th, r->tg, r->mu, L.dec, L.y, r->th,
                                 r->tg, L.s)) != MD_OK)
        return st;
      MD_HIP_TRY(hipEventRecord(L.eq, L.s));
      prev = &L;
    } else {
      MD_HIP_TRY(hipMemcpyAsync(L.y, h_y + r0 * D, sizeof(float) * nb * D, hipMemcpyHostToDevice, L.s));
    }
    if (stats) MD_HIP_TRY(hipMemcpyAsync(L.tx, h_tx + r0, sizeof(uint32_t) * nb, hipMemcpyHostToDevice, L.s));
    if ((st = md::lane_demap(r, L, nb)) != MD_OK) return st;
    L.n_pieces = 0;
    if (stats) {
      for (int64_t a = i0; a < i0 + nb;) {
        const int64_t b = std::min(i0 + nb, (a / r->bin + 1) * r->bin);
        const int p = L.n_pieces++;
        L.piece_bin[p] = a / r->bin;
        L.piece_n[p] = b - a;
        const int64_t off = a - i0;
        if ((st = gmi_reduce(L.llr + off * m, b - a, m, L.tx + off, r->labels, &L.d_res->gmi[p], nullptr, nullptr,
                             L.s)) != MD_OK)
          return st;
        if ((st = ber_count(L.llr + off * m, b - a, m, L.tx + off, r->labels, nullptr,
                            reinterpret_cast<uint64_t*>(&L.d_res->err[p]), L.s)) != MD_OK)
          return st;
        a = b;
      }
      MD_HIP_TRY(hipMemcpyAsync(L.h_res, L.d_res, sizeof(md::PieceResult), hipMemcpyDeviceToHost, L.s));
    }
    if (r->mode == MD_RX_HARD) {
      hipLaunchKernelGGL(md::rx_decide_kernel, dim3(static_cast<unsigned>((nb + 255) / 256)), dim3(256), 0, L.s,
                         L.llr, nb, m, L.dec);
      MD_LAUNCH_CHECK("rx_decide_kernel launch");
      if (h_out)
        MD_HIP_TRY(hipMemcpyAsync(static_cast<uint32_t*>(h_out) + r0, L.dec, sizeof(uint32_t) * nb,
                                  hipMemcpyDeviceToHost, L.s));
    } else if (h_out) {
      MD_HIP_TRY(hipMemcpyAsync(static_cast<float*>(h_out) + r0 * m, L.llr, sizeof(float) * nb * m,
                                hipMemcpyDeviceToHost, L.s));
    }
    MD_HIP_TRY(hipEventRecord(L.end, L.s));
    L.busy = true;
  }
  for (int64_t j = 0; j < r->S; ++j) {
    md::Lane& L = r->lanes[static_cast<size_t>((k + j) % r->S)];   // oldest first: stream order
    if ((st = md::retire(r, L, &sumT, &cnt, &err, &lat_sum, &lat_max, &n_lat)) != MD_OK) return st;
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int64_t b = 0; b < n_bins; ++b) {
    if (h_bin_errors) h_bin_errors[b] = err[static_cast<size_t>(b)];
    if (h_bin_gmi) h_bin_gmi[b] = m - sumT[static_cast<size_t>(b)] / cnt[static_cast<size_t>(b)];
  }
  if (h_stats) {
    h_stats[0] = wall;
    h_stats[1] = wall > 0.0 ? static_cast<double>(total) / wall : 0.0;
    h_stats[2] = n_lat ? lat_sum / static_cast<double>(n_lat) : 0.0;
    h_stats[3] = lat_max;
  }
  return MD_OK;
}

int rx_destroy(void* rx) {
  md::set_error("");
  if (!rx) return MD_OK;
  md::destroy(static_cast<md::RxStream*>(rx));
  return MD_OK;
}

}  // extern "C"
