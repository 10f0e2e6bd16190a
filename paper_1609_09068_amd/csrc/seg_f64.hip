// Instantiates the persistent segment kernel (solve_dev.h) with double series
// terms: one translation unit per variant family so the
// library's sources compile in parallel.
#include "solve_dev.h"

namespace prlib {

const void* seg_kernel_f64(int rpw, bool warm) {
  if (warm) {
    switch (rpw) {
      case 64: return (const void*)k_segment<double, 64, true, false>;
      case 16: return (const void*)k_segment<double, 16, true, false>;
      case 4: return (const void*)k_segment<double, 4, true, false>;
      default: return (const void*)k_segment<double, 1, true, false>;
    }
  }
  switch (rpw) {
    case 64: return (const void*)k_segment<double, 64, false, false>;
    case 16: return (const void*)k_segment<double, 16, false, false>;
    case 4: return (const void*)k_segment<double, 4, false, false>;
    default: return (const void*)k_segment<double, 1, false, false>;
  }
}

}  // namespace prlib
