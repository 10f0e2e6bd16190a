// Learned warm start (per-vertex MLP): placeholder until the kernels land.
#include "internal.h"

namespace prlib {
void mlp_destroy(void* h) { (void)h; }
}  // namespace prlib
