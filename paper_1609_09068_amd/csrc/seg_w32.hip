// Instantiates the persistent segment kernel (solve_dev.h) for weighted
// graphs with float series terms (plain start, with and without the tail
// estimate): one translation unit per variant family so the library's
// sources compile in parallel.
#include "solve_dev.h"

namespace prlib {

const void* seg_kernel_w32(int rpw, bool tail) {
  if (tail) {
    switch (rpw) {
      case 64: return (const void*)k_segment<float, 64, false, true, true>;
      case 16: return (const void*)k_segment<float, 16, false, true, true>;
      case 4: return (const void*)k_segment<float, 4, false, true, true>;
      default: return (const void*)k_segment<float, 1, false, true, true>;
    }
  }
  switch (rpw) {
    case 64: return (const void*)k_segment<float, 64, false, false, true>;
    case 16: return (const void*)k_segment<float, 16, false, false, true>;
    case 4: return (const void*)k_segment<float, 4, false, false, true>;
    default: return (const void*)k_segment<float, 1, false, false, true>;
  }
}

}  // namespace prlib
