// Device scan / sort helpers used by the plan build.
#pragma once

#include <vector>

#include "internal.h"

namespace prlib {

// Device allocations released when the object goes out of scope.  Users
// synchronise the stream before that happens.
struct DevScratch {
  std::vector<void*> ptrs;
  int32_t get(size_t bytes, void** p);
  ~DevScratch();
};

__host__ __device__ inline bool idx_last_block(unsigned b, unsigned nb) { return b + 1 == nb; }

// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total (uint32).
int32_t scan_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// key; the sorted pairs end up in keys / vals.
int32_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s);

int bit_length(uint64_t x);

}  // namespace prlib
