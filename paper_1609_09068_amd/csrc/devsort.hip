// Device building blocks for the plan build: exclusive scan and a stable
// LSD radix sort of (uint32 key, uint32 value) pairs.  Wave64 throughout.
#include "devsort.h"

namespace prlib {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;                 // elements per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kSortRounds = 16;               // rounds of 256 elements per sort tile
constexpr int kSortTile = kBlock * kSortRounds;

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive block scan of one value per thread; returns the prefix, writes total
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total, uint32_t* lds4) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v, lane);
  if (lane == 63) lds4[wave] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    uint32_t s = lds4[w];
    if (w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(const uint32_t* in, int64_t n, uint32_t* sums) {
  __shared__ uint32_t lds4[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < n) s += in[idx];
  }
  uint32_t tot;
  block_excl_scan(s, &tot, lds4);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t* in, int64_t n, const uint32_t* offs,
                                                       uint32_t* out) {
  __shared__ uint32_t lds4[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    v[i] = idx < n ? in[idx] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot, lds4) + (offs ? offs[blockIdx.x] : 0u);
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (idx_last_block(blockIdx.x, gridDim.x) && threadIdx.x == kBlock - 1) out[n] = run;
}

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t* keys, int64_t n, int shift, int nblocks,
                                                    uint32_t* hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t idx = base + r * kBlock + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t* keys, const uint32_t* vals, int64_t n,
                                                       int shift, int nblocks, const uint32_t* offs,
                                                       uint32_t* keys_out, uint32_t* vals_out) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  run[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t idx = base + r * kBlock + threadIdx.x;
    const bool valid = idx < n;
    const uint32_t k = valid ? keys[idx] : 0u;
    const uint32_t v = valid ? vals[idx] : 0u;
    const uint32_t d = (k >> shift) & 255u;
    unsigned long long mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bm = __ballot(valid && bit);
      mask &= bit ? bm : ~bm;
    }
    const uint32_t rank = __popcll(mask & lt);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(mask);
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
      const uint32_t pos = run[d] + pre + rank;
      keys_out[pos] = k;
      vals_out[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < 4; ++w) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

int32_t DevScratch::get(size_t bytes, void** p) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
  if (e != hipSuccess) {
    set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP;
  }
  ptrs.push_back(q);
  *p = q;
  return PR_OK;
}

DevScratch::~DevScratch() {
  for (void* q : ptrs) (void)hipFree(q);
}

int32_t scan_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  // out[0..n]: exclusive prefix sums, out[n] = total
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (n == 0) {
    PR_HIP_CHECK(hipMemsetAsync(out, 0, sizeof(uint32_t), s));
    return PR_OK;
  }
  if (nb == 1) {
    k_scan_apply<<<1, kBlock, 0, s>>>(in, n, nullptr, out);
    PR_HIP_CHECK(hipGetLastError());
    return PR_OK;
  }
  DevScratch scr;
  uint32_t *sums, *offs;
  int32_t rc;
  if ((rc = scr.get(sizeof(uint32_t) * nb, (void**)&sums))) return rc;
  if ((rc = scr.get(sizeof(uint32_t) * (nb + 1), (void**)&offs))) return rc;
  k_scan_sums<<<(unsigned)nb, kBlock, 0, s>>>(in, n, sums);
  PR_HIP_CHECK(hipGetLastError());
  if ((rc = scan_u32(sums, offs, nb, s))) return rc;
  k_scan_apply<<<(unsigned)nb, kBlock, 0, s>>>(in, n, offs, out);
  PR_HIP_CHECK(hipGetLastError());
  PR_HIP_CHECK(hipStreamSynchronize(s));  // scratch is freed on return
  return PR_OK;
}

int32_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
  if (n <= 1 || bits <= 0) return PR_OK;
  const int passes = (bits + 7) / 8;
  const int64_t nb64 = (n + kSortTile - 1) / kSortTile;
  if (nb64 * 256 > (int64_t)INT32_MAX) {
    set_error("radix sort of %lld elements is too large", (long long)n);
    return PR_EINVAL;
  }
  const int nb = (int)nb64;
  DevScratch scr;
  uint32_t *k2, *v2, *hist, *offs;
  int32_t rc;
  if ((rc = scr.get(sizeof(uint32_t) * n, (void**)&k2))) return rc;
  if ((rc = scr.get(sizeof(uint32_t) * n, (void**)&v2))) return rc;
  if ((rc = scr.get(sizeof(uint32_t) * 256 * (size_t)nb, (void**)&hist))) return rc;
  if ((rc = scr.get(sizeof(uint32_t) * (256 * (size_t)nb + 1), (void**)&offs))) return rc;
  uint32_t *ki = keys, *vi = vals, *ko = k2, *vo = v2;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    k_rs_hist<<<nb, kBlock, 0, s>>>(ki, n, shift, nb, hist);
    PR_HIP_CHECK(hipGetLastError());
    if ((rc = scan_u32(hist, offs, 256 * (int64_t)nb, s))) return rc;
    k_rs_scatter<<<nb, kBlock, 0, s>>>(ki, vi, n, shift, nb, offs, ko, vo);
    PR_HIP_CHECK(hipGetLastError());
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (ki != keys) {
    PR_HIP_CHECK(hipMemcpyAsync(keys, ki, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    PR_HIP_CHECK(hipMemcpyAsync(vals, vi, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
  }
  PR_HIP_CHECK(hipStreamSynchronize(s));
  return PR_OK;
}

int bit_length(uint64_t x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

}  // namespace prlib
