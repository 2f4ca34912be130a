// Instantiation of the wide-range third pass of the exact demapper (three windows).
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

// list 2 (flags[3], fb_list2) -> list 3 (flags[4], fb_list: list 1 is no longer needed)
int launch_wide3_exact(const Prepared& P, int M, int D, const float* d_y, float* d_llr, hipStream_t stream) {
  return fastk::launch_wide<3>(P, M, D, d_y, d_llr, 3, 4, P.fb_list2, P.fb_list, stream);
}

}  // namespace md
