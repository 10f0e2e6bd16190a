// Instantiates the persistent segment kernel (solve_dev.h) for weighted
// graphs with double series terms (plain start, with and without the tail
// estimate): one translation unit per variant family so the library's
// sources compile in parallel.
#include "solve_dev.h"

namespace prlib {

const void* seg_kernel_w64(int rpw, bool tail) {
  if (tail) {
    switch (rpw) {
      case 64: return (const void*)k_segment<double, 64, false, true, true>;
      case 16: return (const void*)k_segment<double, 16, false, true, true>;
      case 4: return (const void*)k_segment<double, 4, false, true, true>;
      default: return (const void*)k_segment<double, 1, false, true, true>;
    }
  }
  switch (rpw) {
    case 64: return (const void*)k_segment<double, 64, false, false, true>;
    case 16: return (const void*)k_segment<double, 16, false, false, true>;
    case 4: return (const void*)k_segment<double, 4, false, false, true>;
    default: return (const void*)k_segment<double, 1, false, false, true>;
  }
}

}  // namespace prlib
