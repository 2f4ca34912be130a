// C entry points: argument validation on the host, then prep + kernel launches on the
// caller's stream.  Nothing here computes on the host.
#include <climits>
#include <cmath>

#include "common.hpp"
#include "llr_kernels.hpp"

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int check_constellation(const void* d_X, int M, int D) {
  if (!d_X) return md::fail(MD_EINVAL, "constellation pointer is NULL");
  if (M < 2 || M > 65536 || !md::is_pow2(M))
    return md::fail(MD_ENOTPOW2, "M=" + std::to_string(M) + " is not a power of two in [2, 65536]");
  if (D < 1 || D > 30) return md::fail(MD_EDIM, "D=" + std::to_string(D) + " is outside [1, 30]");
  return MD_OK;
}

}  // namespace

namespace md {

int check_demap_args(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N,
                     double sigma2, int prec, const float* d_llr) {
  int st = check_constellation(d_X, M, D);
  if (st != MD_OK) return st;
  if (!d_labels) return fail(MD_EINVAL, "labels pointer is NULL");
  if (N < 0) return fail(MD_EINVAL, "N is negative");
  // the fallback lists hold 32-bit symbol indices behind a 32-bit counter
  if (N > INT32_MAX) return fail(MD_EINVAL, "N above 2^31 - 1 symbols in one call");
  if (N > 0 && (!d_y || !d_llr)) return fail(MD_EINVAL, "y or llr pointer is NULL");
  if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return fail(MD_EINVAL, "sigma2 must be finite and > 0");
  if (prec != MD_PREC_FP32 && prec != MD_PREC_FP16 && prec != MD_PREC_BF16 && prec != MD_PREC_BF16_SCORES)
    return fail(MD_EINVAL, "unknown precision");
  if ((prec == MD_PREC_FP16 || prec == MD_PREC_BF16_SCORES) && D > 12)
    return fail(MD_EUNSUPPORTED, "one-pass FP16 / BF16 scores take D <= 12");
  return MD_OK;
}

}  // namespace md

namespace {

int demap(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N, double sigma2,
          int prec, bool maxlog, float* d_llr, void* stream) {
  md::set_error("");
  int st = md::check_demap_args(d_X, d_labels, M, D, d_y, N, sigma2, prec, d_llr);
  if (st != MD_OK) return st;
  int dev = 0;
  st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = as_stream(stream);
  st = md::check_labels_once(d_labels, M, s);
  if (st != MD_OK) return st;
  if (N == 0) return MD_OK;
  char* ws = nullptr;
  st = md::workspace(s, md::prep_bytes(M, D, N), &ws);
  if (st != MD_OK) return st;
  md::Prepared P;
  float alpha = 1.0f, c_over_alpha = 1.0f;
  md::score_scales(sigma2, &alpha, &c_over_alpha);
  int* flags = nullptr;
  st = md::stream_flags(s, &flags);
  if (st != MD_OK) return st;
  st = md::prepare(d_X, d_labels, M, D, N, alpha, c_over_alpha, ws, s, &P, flags,
                   maxlog ? 0 : md::score_layout(prec));
  if (st != MD_OK) return st;
  md::LastCall lc;
  lc.valid = true;
  lc.maxlog = maxlog;
  lc.N = N;
  md::record_last_call(s, lc);
  return md::launch_llr(P, M, D, d_y, N, sigma2, maxlog, prec, d_llr, s);
}

}  // namespace

extern "C" {

int awgn_sample(const float* d_X, int M, int D, uint64_t seed, uint64_t offset, int64_t N, double sigma,
                uint32_t* d_tx, float* d_y, void* stream) {
  md::set_error("");
  int st = check_constellation(d_X, M, D);
  if (st != MD_OK) return st;
  if (N < 0) return md::fail(MD_EINVAL, "N is negative");
  if (N > 0 && (!d_tx || !d_y)) return md::fail(MD_EINVAL, "tx or y pointer is NULL");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return md::fail(MD_EINVAL, "sigma must be finite and >= 0");
  int dev = 0;
  st = md::current_device(&dev);
  if (st != MD_OK) return st;
  if (N == 0) return MD_OK;
  return md::launch_awgn(d_X, M, D, seed, offset, N, sigma, d_tx, d_y, as_stream(stream));
}

int llr_exact(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N, double sigma2,
              int prec, float* d_llr, void* stream) {
  return demap(d_X, d_labels, M, D, d_y, N, sigma2, prec, false, d_llr, stream);
}

int llr_maxlog(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N, double sigma2,
               float* d_llr, void* stream) {
  return demap(d_X, d_labels, M, D, d_y, N, sigma2, MD_PREC_FP32, true, d_llr, stream);
}

int llr_path_counts(void* stream, int64_t* n_wide, int64_t* n_careful) {
  md::set_error("");
  if (!n_wide || !n_careful) return md::fail(MD_EINVAL, "output pointer is NULL");
  *n_wide = 0;
  *n_careful = 0;
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = as_stream(stream);
  md::LastCall lc;
  int* flags = nullptr;
  st = md::last_call(s, &lc, &flags);
  if (st != MD_OK) return st;
  if (!lc.valid || !flags) return MD_OK;
  int h[5] = {0, 0, 0, 0, 0};
  MD_HIP_TRY(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s));
  MD_HIP_TRY(hipStreamSynchronize(s));
  if (lc.maxlog) {
    *n_careful = h[1];
  } else {
    *n_wide = h[1];
    *n_careful = h[4];
  }
  return MD_OK;
}

int gmi_reduce(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels, double* d_gmi,
               double* d_gmi_per_bit, double* d_se, void* stream) {
  md::set_error("");
  if (N <= 0) return md::fail(MD_EINVAL, "GMI needs N > 0 symbols");
  if (m < 1 || m > 16) return md::fail(MD_EINVAL, "m=" + std::to_string(m) + " is outside [1, 16]");
  if (!d_llr || !d_tx || !d_labels || !d_gmi) return md::fail(MD_EINVAL, "llr, tx, labels or gmi pointer is NULL");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = as_stream(stream);
  char* ws = nullptr;
  // calls on one stream run in order, so the partials may reuse the demappers' workspace
  st = md::workspace(s, md::gmi_workspace_bytes(N, m), &ws);
  if (st != MD_OK) return st;
  int* flags = nullptr;
  st = md::stream_flags(s, &flags);
  if (st != MD_OK) return st;
  return md::launch_gmi(d_llr, N, m, d_tx, d_labels, d_gmi, d_gmi_per_bit, d_se, ws, md::gmi_status_word(flags), s);
}

int gmi_status(void* stream, int64_t* n_nonfinite) {
  md::set_error("");
  if (!n_nonfinite) return md::fail(MD_EINVAL, "output pointer is NULL");
  *n_nonfinite = 0;
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = as_stream(stream);
  int* flags = nullptr;
  st = md::stream_flags(s, &flags);
  if (st != MD_OK) return st;
  long long h = 0;
  MD_HIP_TRY(hipMemcpyAsync(&h, md::gmi_status_word(flags), sizeof(h), hipMemcpyDeviceToHost, s));
  MD_HIP_TRY(hipStreamSynchronize(s));
  *n_nonfinite = h;
  if (h > 0)
    return md::fail(MD_ENONFINITE, std::to_string(h) + " symbols had a non-finite GMI term (non-finite LLR or a "
                                                         "transmitted index outside the labels)");
  return MD_OK;
}

int llr_exact_gmi(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N,
                  double sigma2, int prec, const uint32_t* d_tx, float* d_llr, double* d_gmi, double* d_se,
                  void* stream) {
  md::set_error("");
  int st = md::check_demap_args(d_X, d_labels, M, D, d_y, N, sigma2, prec, d_llr);
  if (st != MD_OK) return st;
  if (N <= 0) return md::fail(MD_EINVAL, "GMI needs N > 0 symbols");
  if (!d_tx || !d_gmi) return md::fail(MD_EINVAL, "tx or gmi pointer is NULL");
  const int m = md::ilog2_pow2(M);
  const int sc = md::score_layout(prec);
  const int ks = sc == 0 ? md::frag_ksteps(D) : md::frag_ksteps_single(D);
  if (M <= 16 || prec == MD_PREC_BF16 || !md::fused_gmi_supported(sc, ks)) {
    // no fused epilogue on these paths: the two calls in sequence
    st = demap(d_X, d_labels, M, D, d_y, N, sigma2, prec, false, d_llr, stream);
    if (st != MD_OK) return st;
    return gmi_reduce(d_llr, N, m, d_tx, d_labels, d_gmi, nullptr, d_se, stream);
  }
  int dev = 0;
  st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = as_stream(stream);
  st = md::check_labels_once(d_labels, M, s);
  if (st != MD_OK) return st;
  const size_t pb = md::prep_bytes(M, D, N);
  const size_t tb = md::carve_size(sizeof(float) * static_cast<size_t>(N));
  char* ws = nullptr;
  st = md::workspace(s, pb + tb + md::gmi_workspace_bytes(N, m), &ws);
  if (st != MD_OK) return st;
  int* flags = nullptr;
  st = md::stream_flags(s, &flags);
  if (st != MD_OK) return st;
  md::Prepared P;
  float alpha = 1.0f, c_over_alpha = 1.0f;
  md::score_scales(sigma2, &alpha, &c_over_alpha);
  st = md::prepare(d_X, d_labels, M, D, N, alpha, c_over_alpha, ws, s, &P, flags, md::score_layout(prec));
  if (st != MD_OK) return st;
  P.gmi_tx = d_tx;
  P.gmi_labels = d_labels;
  P.gmi_terms = reinterpret_cast<float*>(ws + pb);
  md::LastCall lc;
  lc.valid = true;
  lc.maxlog = false;
  lc.N = N;
  md::record_last_call(s, lc);
  st = md::launch_llr(P, M, D, d_y, N, sigma2, false, prec, d_llr, s);
  if (st != MD_OK) return st;
  return md::launch_gmi_terms(P.gmi_terms, d_llr, N, m, d_tx, d_labels, d_gmi, d_se, ws + pb + tb,
                              md::gmi_status_word(flags), s);
}

int ber_count(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels,
              uint64_t* d_bit_errors, uint64_t* d_errors, void* stream) {
  md::set_error("");
  if (N <= 0) return md::fail(MD_EINVAL, "bit-error counting needs N > 0 symbols");
  if (m < 1 || m > 16) return md::fail(MD_EINVAL, "m=" + std::to_string(m) + " is outside [1, 16]");
  if (!d_llr || !d_tx || !d_labels || !d_errors)
    return md::fail(MD_EINVAL, "llr, tx, labels or errors pointer is NULL");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  hipStream_t s = as_stream(stream);
  char* ws = nullptr;
  st = md::workspace(s, md::ber_workspace_bytes(N, m), &ws);
  if (st != MD_OK) return st;
  return md::launch_ber(d_llr, N, m, d_tx, d_labels, d_bit_errors, d_errors, ws, s);
}

int q_factor_db(const uint64_t* d_errors, int64_t n_bits, double* d_q_db, void* stream) {
  md::set_error("");
  if (n_bits <= 0) return md::fail(MD_EINVAL, "n_bits must be > 0");
  if (!d_errors || !d_q_db) return md::fail(MD_EINVAL, "errors or q pointer is NULL");
  int dev = 0;
  int st = md::current_device(&dev);
  if (st != MD_OK) return st;
  return md::launch_q_factor(d_errors, n_bits, d_q_db, as_stream(stream));
}

}  // extern "C"
