// Instantiation of the wide-range second pass of the exact demapper (two windows); the
// third pass is in llr_wide3.hip, a translation unit of its own so that the two compile in
// parallel.
#include "llr_fast.hpp"
#include "llr_kernels.hpp"

namespace md {

// list 1 (flags[1], fb_list) -> list 2 (flags[3], fb_list2), two windows
int launch_wide_exact(const Prepared& P, int M, int D, const float* d_y, float* d_llr, hipStream_t stream) {
  return fastk::launch_wide<2>(P, M, D, d_y, d_llr, 1, 3, P.fb_list, P.fb_list2, stream);
}

}  // namespace md
