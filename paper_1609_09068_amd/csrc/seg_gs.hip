// Instantiates the segment kernel with block Gauss-Seidel sweeps in
// workgroup SCCs (solve_dev.h, k_segment_gs) for every rows-per-wavefront
// shape, FP32 and FP64 terms.
#include "solve_dev.h"

namespace prlib {

const void* seg_kernel_gs(int rpw, bool fp64) {
  if (fp64) {
    switch (rpw) {
      case 64: return (const void*)k_segment_gs<double, 64>;
      case 16: return (const void*)k_segment_gs<double, 16>;
      case 4: return (const void*)k_segment_gs<double, 4>;
      default: return (const void*)k_segment_gs<double, 1>;
    }
  }
  switch (rpw) {
    case 64: return (const void*)k_segment_gs<float, 64>;
    case 16: return (const void*)k_segment_gs<float, 16>;
    case 4: return (const void*)k_segment_gs<float, 4>;
    default: return (const void*)k_segment_gs<float, 1>;
  }
}

}  // namespace prlib
