// Instantiates the tail-estimate segment kernel at three workgroups per CU
// (solve_dev.h, k_segment_w3) for 16 and 64 rows per wavefront, FP32 and
// FP64 terms.
#include "solve_dev.h"

namespace prlib {

const void* seg_kernel_tail_w3(int rpw, bool fp64) {
  if (fp64) {
    if (rpw == 64) return (const void*)k_segment_w3<double, 64>;
    if (rpw == 16) return (const void*)k_segment_w3<double, 16>;
    return nullptr;
  }
  if (rpw == 64) return (const void*)k_segment_w3<float, 64>;
  if (rpw == 16) return (const void*)k_segment_w3<float, 16>;
  return nullptr;
}

}  // namespace prlib
