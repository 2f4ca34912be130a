// Instantiation of the fast exact demapping kernel with one-pass FP16 or BF16 scores
// (the reduced-precision variants of llr_exact).
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

int launch_fast_lowp(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                     hipStream_t stream) {
  return P.sc == 2 ? fastk::launch_fast_lowp<2>(P, M, D, d_y, N, sigma2, d_llr, stream)
                   : fastk::launch_fast_lowp<1>(P, M, D, d_y, N, sigma2, d_llr, stream);
}

}  // namespace md
