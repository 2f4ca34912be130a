// Instantiation of the wide-range second pass of the exact demapper.
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

int launch_wide_exact(const Prepared& P, int M, int D, const float* d_y, float* d_llr, hipStream_t stream) {
  return fastk::launch_wide(P, M, D, d_y, d_llr, stream);
}

}  // namespace md
