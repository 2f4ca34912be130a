// Instantiation of the BF16 subset-sum variant of the exact demapping kernel.
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

int launch_fast_bf16(const Prepared& P, int M, int D, const float* d_y, int64_t N, float* d_llr,
                     hipStream_t stream) {
  return fastk::launch_bf16<>(P, M, D, d_y, N, d_llr, stream);
}

}  // namespace md
