// Launchers implemented by the kernel translation units.
#pragma once

#include "common.hpp"

namespace md {

int launch_awgn(const float* d_X, int M, int D, uint64_t seed, uint64_t offset, int64_t N, double sigma,
                uint32_t* d_tx, float* d_y, hipStream_t stream);

// Power-of-two scale a that balances the two operands of the split-FP16 score
// contraction, and c / a with c = log2(e) / (2 sigma2).
void score_scales(double sigma2, float* alpha, float* c_over_alpha);

// Fast MFMA path (M >= 32) followed by the careful kernel on the fallback list, or the
// careful kernel on every symbol (M < 32).
int launch_llr(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, bool maxlog,
               int prec, float* d_llr, hipStream_t stream);
int launch_fast_exact(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                      hipStream_t stream);
int launch_fast_maxlog(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2,
                       float* d_llr, hipStream_t stream);
int launch_fast_bf16(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr,
                     hipStream_t stream);
// One-pass FP16 or BF16 scores (P.sc 1 or 2, one K step), exact LLRs.
int launch_fast_lowp(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                     hipStream_t stream);
// Exact LLRs with the fused GMI epilogue (P.gmi_terms set), for the shapes
// fused_gmi_supported(P.sc, P.ks) accepts.
int launch_fast_gmi(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                    hipStream_t stream);
bool fused_gmi_supported(int sc, int ks);
// Exact LLRs with one thread per symbol (FP32 scores from per-point terms in LDS), for
// M = 32 or 64 and D <= 8, where the matrix-core kernel's per-symbol work outweighs its
// two tiles; out-of-range symbols join the first fallback list like the fast pass's (the
// max-log form, from the same scores, never does).
bool vec_exact_supported(int M, int D);
int launch_vec_exact(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr,
                     hipStream_t stream, bool maxlog = false);
// Fragment layout (Prepared::sc) that llr_exact's precision `prec` needs.
inline int score_layout(int prec) {
  return prec == MD_PREC_FP16 ? 1 : (prec == MD_PREC_BF16_SCORES ? 2 : 0);
}
// Wide-range second pass over the first fallback list and third pass over the second
// (exact LLRs; two and three exponent windows).
int launch_wide_exact(const Prepared& P, int M, int D, const float* d_y, float* d_llr, hipStream_t stream);
int launch_wide3_exact(const Prepared& P, int M, int D, const float* d_y, float* d_llr, hipStream_t stream);
int launch_llr_careful_all(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2,
                           bool maxlog, float* d_llr, hipStream_t stream);

size_t gmi_workspace_bytes(int64_t N, int m);
// `status` (device) receives the number of symbols whose loss term was not finite.
int launch_gmi(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels, double* d_gmi,
               double* d_gmi_per_bit, double* d_se, char* ws, long long* status, hipStream_t stream);
// GMI from the loss terms of the fused demapping pass (NaN terms: formed from the LLRs).
int launch_gmi_terms(const float* d_terms, const float* d_llr, int64_t N, int m, const uint32_t* d_tx,
                     const uint32_t* d_labels, double* d_gmi, double* d_se, char* ws, long long* status,
                     hipStream_t stream);

size_t ber_workspace_bytes(int64_t N, int m);
int launch_ber(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels,
               uint64_t* d_bit_errors, uint64_t* d_errors, char* ws, hipStream_t stream);

// Host-side checks shared by the demapping entry points (the MD_* status, last_error set).
int check_demap_args(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N,
                     double sigma2, int prec, const float* d_llr);

int launch_q_factor(const uint64_t* d_errors, int64_t n_bits, double* d_q, hipStream_t stream);

}  // namespace md
