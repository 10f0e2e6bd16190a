// Instantiates the persistent segment kernel (solve_dev.h) with float series
// terms and the tail-estimate stop: one translation unit per variant family so the
// library's sources compile in parallel.
#include "solve_dev.h"

namespace prlib {

const void* seg_kernel_f32_tail(int rpw, bool warm) {
  if (warm) {
    switch (rpw) {
      case 64: return (const void*)k_segment<float, 64, true, true>;
      case 16: return (const void*)k_segment<float, 16, true, true>;
      case 4: return (const void*)k_segment<float, 4, true, true>;
      default: return (const void*)k_segment<float, 1, true, true>;
    }
  }
  switch (rpw) {
    case 64: return (const void*)k_segment<float, 64, false, true>;
    case 16: return (const void*)k_segment<float, 16, false, true>;
    case 4: return (const void*)k_segment<float, 4, false, true>;
    default: return (const void*)k_segment<float, 1, false, true>;
  }
}

}  // namespace prlib
