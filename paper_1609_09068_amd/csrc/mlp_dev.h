// Device side of the starting-guess network: 4 -> 64 -> 64 -> 1 with GELU
// after both hidden layers, BF16 operands on the matrix cores, FP32
// accumulation.
//
// The network runs transposed, 16 rows (vertices) at a time, on
// v_mfma_f32_16x16x16_bf16 (wave64).  For that instruction, with D = A B + C:
//   A (16 x 16, M x K): lane l holds A[l % 16][4 (l / 16) + j], j = 0..3
//   B (16 x 16, K x N): lane l holds B[4 (l / 16) + j][l % 16]
//   D (16 x 16, M x N): lane l holds D[4 (l / 16) + j][l % 16]
// With activations stored transposed (hidden unit x row), a layer's output
// in D layout is exactly the B operand of the next layer, so the forward
// pass needs no data exchange between lanes.  Weights are packed once into
// per-lane A fragments (MlpPacked).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace prlib {

constexpr int kMlpIn = 4;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
// offsets of the flat FP32 parameter vector (row-major matrices)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHidden * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden;
static_assert(kOffB3 + 1 == kMlpParams && kMlpParams == 4545, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// BF16 weight fragments, one 8-byte entry per lane and tile
struct MlpPacked {
  bf16x4 w1[4][64];       // layer 1, hidden tile t: W1[16t + l][0..3] on lanes 0..15, zero elsewhere
  bf16x4 w2[4][4][64];    // layer 2, [out tile u][in tile t]: W2[16u + l%16][16t + 4(l/16) + j]
  bf16x4 w2t[4][4][64];   // transposed, [in tile t][out tile u]: W2[16u + 4(l/16) + j][16t + l%16]
  bf16x4 w3[4][64];       // layer 3, [in tile u]: W3[16u + 4(l/16) + j] on lanes with l%16 == 0
  float b1[kMlpHidden], b2[kMlpHidden], b3;
};

// round to nearest even (finite inputs)
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__device__ inline bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}
__device__ inline bf16x4 pack4(f32x4 v) { return pack4(v[0], v[1], v[2], v[3]); }

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// GELU with the exact normal CDF, and its derivative
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Forward pass of one block of 16 rows.  xb: the B operand of the features
// (lanes 0..15 hold the four features of row l, other lanes zero).  Returns
// the output of row l % 16 on lanes 0..15 (other lanes: unspecified).
__device__ __attribute__((always_inline)) inline float mlp_forward16(const MlpPacked& w, bf16x4 xb) {
  const int lane = threadIdx.x & 63;
  const int hb = 4 * (lane >> 4);  // first hidden unit of this lane within a tile
  bf16x4 h1[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    z = mfma16(w.w1[t][lane], xb, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) z[j] = gelu(z[j] + w.b1[16 * t + hb + j]);
    h1[t] = pack4(z);
  }
  bf16x4 h2[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) z = mfma16(w.w2[u][t][lane], h1[t], z);
#pragma unroll
    for (int j = 0; j < 4; ++j) z[j] = gelu(z[j] + w.b2[16 * u + hb + j]);
    h2[u] = pack4(z);
  }
  f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < 4; ++u) y = mfma16(w.w3[u][lane], h2[u], y);
  return y[0] + w.b3;
}

// Forward pass for up to 64 rows held one per lane (features f0..f3 of the
// lane's row; inactive lanes pass anything).  Returns the lane's output.
// The weights are read from memory (L1/L2) for each block rather than held
// in registers, so a kernel that embeds this keeps its register budget.
__device__ __attribute__((always_inline)) inline float mlp_forward64(const MlpPacked& w, float f0, float f1, float f2, float f3) {
  const int lane = threadIdx.x & 63;
  float out = 0.f;
#pragma unroll 1
  for (int b = 0; b < 4; ++b) {
    uint64_t wa = (uint64_t)(uintptr_t)&w;
    asm volatile("" : "+v"(wa));  // not loop-invariant: the loads stay inside the loop
    const MlpPacked* wb = (const MlpPacked*)(uintptr_t)wa;
    const int srcl = 16 * b + (lane & 15);
    const float a0 = __shfl(f0, srcl, 64), a1 = __shfl(f1, srcl, 64);
    const float a2 = __shfl(f2, srcl, 64), a3 = __shfl(f3, srcl, 64);
    const bf16x4 xb = lane < 16 ? pack4(a0, a1, a2, a3) : pack4(0.f, 0.f, 0.f, 0.f);
    const float y = mlp_forward16(*wb, xb);
    // row 16b + i came out on lane i
    const float yb = __shfl(y, lane & 15, 64);
    if ((lane >> 4) == b) out = yb;
  }
  return out;
}

}  // namespace prlib
