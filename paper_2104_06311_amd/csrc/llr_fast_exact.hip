// Instantiation of the fast demapping kernel for the exact (log-sum-exp) LLRs.
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

int launch_fast_exact(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                      hipStream_t stream) {
  return fastk::launch_fast<false>(P, M, D, d_y, N, sigma2, d_llr, stream);
}

}  // namespace md
