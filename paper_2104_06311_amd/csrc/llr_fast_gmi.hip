// Instantiation of the fast exact demapping kernel with the fused GMI epilogue
// (llr_exact_gmi).
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

int launch_fast_gmi(const Prepared& P, int M, int D, const float* d_y, int64_t N, double sigma2, float* d_llr,
                    hipStream_t stream) {
  return fastk::launch_fast_gmi<>(P, M, D, d_y, N, sigma2, d_llr, stream);
}

bool fused_gmi_supported(int sc, int ks) { return fastk::fused_gmi_supported(sc, ks); }

}  // namespace md
