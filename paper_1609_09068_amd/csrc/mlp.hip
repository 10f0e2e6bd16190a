// The starting-guess network: object, packing, inference, gradient, Adam,
// file format, and the per-vertex features of a solved plan.
//
// Training minimises the mean squared error between the network's output
// and a per-vertex target over a batch; the gradient is accumulated per
// wavefront on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 sums),
// written as one partial vector per wavefront and reduced in wavefront order,
// so a step is bitwise reproducible for a given batch.  Adam (Kingma and Ba,
// 2015: bias-corrected moment estimates) updates FP32 master weights, from
// which the BF16 fragments are repacked.
#include <mutex>
#include <cmath>
#include <cstdio>
#include <new>

#include "internal.h"

namespace prlib {

namespace {

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void k_mlp_pack(const float* __restrict__ p, MlpPacked* __restrict__ out) {
  const int l = threadIdx.x & 63, q = threadIdx.x >> 6;  // four groups of 64 lanes
  const int col = l & 15, hb = 4 * (l >> 4);
  const float* W1 = p + kOffW1;
  const float* W2 = p + kOffW2;
  const float* W3 = p + kOffW3;
  {
    const int t = q;
    out->w1[t][l] = l < 16 ? pack4(W1[(16 * t + l) * 4 + 0], W1[(16 * t + l) * 4 + 1], W1[(16 * t + l) * 4 + 2],
                                   W1[(16 * t + l) * 4 + 3])
                           : pack4(0.f, 0.f, 0.f, 0.f);
    out->w3[t][l] = col == 0 ? pack4(W3[16 * t + hb], W3[16 * t + hb + 1], W3[16 * t + hb + 2], W3[16 * t + hb + 3])
                             : pack4(0.f, 0.f, 0.f, 0.f);
  }
  for (int a = 0; a < 4; ++a) {
    const int u = q, t = a;
    out->w2[u][t][l] = pack4(W2[(16 * u + col) * 64 + 16 * t + hb], W2[(16 * u + col) * 64 + 16 * t + hb + 1],
                             W2[(16 * u + col) * 64 + 16 * t + hb + 2], W2[(16 * u + col) * 64 + 16 * t + hb + 3]);
    const int tt = q, uu = a;
    out->w2t[tt][uu][l] =
        pack4(W2[(16 * uu + hb) * 64 + 16 * tt + col], W2[(16 * uu + hb + 1) * 64 + 16 * tt + col],
              W2[(16 * uu + hb + 2) * 64 + 16 * tt + col], W2[(16 * uu + hb + 3) * 64 + 16 * tt + col]);
  }
  if (threadIdx.x < kMlpHidden) {
    out->b1[threadIdx.x] = p[kOffB1 + threadIdx.x];
    out->b2[threadIdx.x] = p[kOffB2 + threadIdx.x];
  }
  if (threadIdx.x == 0) out->b3 = p[kOffB3];
}

__global__ __launch_bounds__(kT) void k_mlp_predict(const MlpPacked* __restrict__ w, const float* __restrict__ X,
                                                     float* __restrict__ y, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t nchunk = (n + 63) / 64;
  for (int64_t ch = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6); ch < nchunk;
       ch += (int64_t)gridDim.x * (kT / 64)) {
    const int64_t r = ch * 64 + lane;
    const bool ok = r < n;
    const float f0 = ok ? X[4 * r] : 0.f, f1 = ok ? X[4 * r + 1] : 0.f;
    const float f2 = ok ? X[4 * r + 2] : 0.f, f3 = ok ? X[4 * r + 3] : 0.f;
    const float out = mlp_forward64(*w, f0, f1, f2, f3);
    if (ok) y[r] = out;
  }
}

// The A operand of a 16 x 16 tile held in D layout (lane l has
// D[4(l/16) + j][l % 16]): lane l gets D[l % 16][4(l/16) + j].  Goes through
// a per-wavefront LDS tile (row stride 17).
__device__ inline bf16x4 a_from_d(f32x4 d, float* tile) {
  const int lane = threadIdx.x & 63, col = lane & 15, hb = 4 * (lane >> 4);
#pragma unroll
  for (int j = 0; j < 4; ++j) tile[(hb + j) * 17 + col] = d[j];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const bf16x4 r = pack4(tile[col * 17 + hb], tile[col * 17 + hb + 1], tile[col * 17 + hb + 2], tile[col * 17 + hb + 3]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return r;
}

// sum over the 16 lanes of a row group (lanes with equal l / 16)
__device__ inline float sum16(float v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}

// Gradient of  dscale/2 * sum_rows (y - t)^2  (dscale = 2 / batch gives the
// mean squared error) for the rows of this launch; one partial vector per
// wavefront.
__global__ __launch_bounds__(kT) void k_mlp_grad(const MlpPacked* __restrict__ wp, const float* __restrict__ master,
                                                  const float* __restrict__ X, const float* __restrict__ T,
                                                  int64_t n, float dscale, float* __restrict__ gpart,
                                                  double* __restrict__ lpart) {
  __shared__ float s_tile[kT / 64][16 * 17];
  __shared__ float s_x[kT / 64][16 * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, hb = 4 * (lane >> 4);
  const MlpPacked& w = *wp;
  float* tile = s_tile[wave];
  float* sx = s_x[wave];
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gw2[4][4], gw1[4], pb1[4], pb2[4], pw3[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gw1[a] = pb1[a] = pb2[a] = pw3[a] = zero;
#pragma unroll
    for (int b = 0; b < 4; ++b) gw2[a][b] = zero;
  }
  float w3v[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) w3v[u][j] = master[kOffW3 + 16 * u + hb + j];
  float pb3 = 0.f;
  double ls = 0.0;
  const int64_t nblk = (n + 15) / 16;
  const int64_t gw = (int64_t)blockIdx.x * (kT / 64) + wave, nw = (int64_t)gridDim.x * (kT / 64);
  for (int64_t b = gw; b < nblk; b += nw) {
    const int64_t r = b * 16 + col;
    const bool valid = r < n;
    const float x0 = valid ? X[4 * r] : 0.f, x1 = valid ? X[4 * r + 1] : 0.f;
    const float x2 = valid ? X[4 * r + 2] : 0.f, x3 = valid ? X[4 * r + 3] : 0.f;
    const float tv = valid ? T[r] : 0.f;
    if (lane < 16) {
      sx[col * 4 + 0] = x0;
      sx[col * 4 + 1] = x1;
      sx[col * 4 + 2] = x2;
      sx[col * 4 + 3] = x3;
    }
    const bf16x4 xb = lane < 16 ? pack4(x0, x1, x2, x3) : pack4(0.f, 0.f, 0.f, 0.f);
    // forward, keeping pre-activations and activations
    f32x4 z1[4], g1[4], z2[4], g2[4];
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 z = mfma16(w.w1[t][lane], xb, zero);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        z1[t][j] = z[j] + w.b1[16 * t + hb + j];
        g1[t][j] = gelu(z1[t][j]);
      }
      h1[t] = pack4(g1[t]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      f32x4 z = zero;
#pragma unroll
      for (int t = 0; t < 4; ++t) z = mfma16(w.w2[u][t][lane], h1[t], z);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        z2[u][j] = z[j] + w.b2[16 * u + hb + j];
        g2[u][j] = gelu(z2[u][j]);
      }
      h2[u] = pack4(g2[u]);
    }
    f32x4 yv = zero;
#pragma unroll
    for (int u = 0; u < 4; ++u) yv = mfma16(w.w3[u][lane], h2[u], yv);
    const float y = yv[0] + w.b3;
    // output error (lanes 0..15 hold rows 0..15 of the block)
    const float d = (lane < 16 && valid) ? (y - tv) : 0.f;
    ls += (double)d * (double)d;
    const float dy = d * dscale;
    pb3 += dy;
    const float dyn = __shfl(dy, col, 64);  // dy of the row of this lane's column
    // layer 3 and the error at layer 2's pre-activation
    f32x4 dz2[4];
    bf16x4 dz2b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        pw3[u][j] += dyn * g2[u][j];
        dz2[u][j] = w3v[u][j] * dyn * gelu_grad(z2[u][j]);
        pb2[u][j] += dz2[u][j];
      }
      dz2b[u] = pack4(dz2[u]);
    }
    // error at layer 1's pre-activation: W2^T dZ2, then GELU'
    f32x4 dz1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = zero;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = mfma16(w.w2t[t][u][lane], dz2b[u], acc);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        dz1[t][j] = acc[j] * gelu_grad(z1[t][j]);
        pb1[t][j] += dz1[t][j];
      }
    }
    // dW2 += dZ2 H1^T over the block's rows
    bf16x4 ah1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ah1[t] = a_from_d(g1[t], tile);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bf16x4 adz = a_from_d(dz2[u], tile);
#pragma unroll
      for (int t = 0; t < 4; ++t) gw2[u][t] = mfma16(adz, ah1[t], gw2[u][t]);
    }
    // dW1 += dZ1 X over the block's rows (features padded to 16 columns)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bf16x4 bx = col < 4 ? pack4(sx[(hb + 0) * 4 + col], sx[(hb + 1) * 4 + col], sx[(hb + 2) * 4 + col],
                                      sx[(hb + 3) * 4 + col])
                              : pack4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 4; ++t) gw1[t] = mfma16(a_from_d(dz1[t], tile), bx, gw1[t]);
  }
  // this wavefront's partial gradient
  float* g = gpart + gw * (int64_t)kMlpParams;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (col < 4) g[kOffW1 + (16 * t + hb + j) * 4 + col] = gw1[t][j];
      const float sb1 = sum16(pb1[t][j]);
      const float sb2 = sum16(pb2[t][j]);
      const float sw3 = sum16(pw3[t][j]);
      if (col == 0) {
        g[kOffB1 + 16 * t + hb + j] = sb1;
        g[kOffB2 + 16 * t + hb + j] = sb2;
        g[kOffW3 + 16 * t + hb + j] = sw3;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) g[kOffW2 + (16 * u + hb + j) * 64 + 16 * t + col] = gw2[u][t][j];
  // b3 and the loss: lanes 0..15 hold the rows
  float s3 = lane < 16 ? pb3 : 0.f;
  s3 = sum16(s3);
  double l2 = lane < 16 ? ls : 0.0;
  for (int o = 1; o < 16; o <<= 1) l2 += __shfl_xor(l2, o, 64);
  if (lane == 0) {
    g[kOffB3] = s3;
    lpart[gw] = l2;
  }
}

// sum of the per-wavefront partials in wavefront order
__global__ __launch_bounds__(kT) void k_mlp_reduce(const float* __restrict__ gpart, int64_t P,
                                                    const double* __restrict__ lpart, float* __restrict__ grad,
                                                    double* __restrict__ loss) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < kMlpParams) {
    float s = 0.f;
    for (int64_t q = 0; q < P; ++q) s += gpart[q * kMlpParams + i];
    grad[i] = s;
  }
  if (i == 0) {
    double s = 0.0;
    for (int64_t q = 0; q < P; ++q) s += lpart[q];
    *loss = s;
  }
}

__global__ __launch_bounds__(kT) void k_mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g, float lr, float b1, float b2, float eps,
                                                  float bc1, float bc2) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= kMlpParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---- features of a solved plan (caller's vertex order)
__global__ __launch_bounds__(kT) void k_features(const int32_t* __restrict__ scc_ranks, int64_t n_scc,
                                                  const int32_t* __restrict__ comp_vbeg,
                                                  const uint32_t* __restrict__ bnd_ptr,
                                                  const uint32_t* __restrict__ int_ptr,
                                                  const int32_t* __restrict__ int_src,
                                                  const double* __restrict__ inv64, const int32_t* __restrict__ perm,
                                                  const double* __restrict__ wprime, const double* __restrict__ W,
                                                  double c, float* __restrict__ F, float* __restrict__ S,
                                                  uint8_t* __restrict__ mask) {
  __shared__ double red[kT / 64];
  for (int64_t q = blockIdx.x; q < n_scc; q += gridDim.x) {
    const int r = scc_ranks[q];
    const int vb = comp_vbeg[r], ve = comp_vbeg[r + 1];
    double part = 0.0;
    for (int v = vb + threadIdx.x; v < ve; v += kT) part += wprime[v];
    // fixed-order block sum
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    const double s = ((red[0] + red[1]) + (red[2] + red[3])) / (double)(ve - vb);
    __syncthreads();
    for (int v = vb + threadIdx.x; v < ve; v += kT) {
      double p1 = 0.0;
      for (uint32_t e = int_ptr[v]; e < int_ptr[v + 1]; ++e) {
        const int u = int_src[e];
        p1 += wprime[u] * inv64[u];
      }
      const double r1 = wprime[v] + c * p1;
      const double indeg = (double)((bnd_ptr[v + 1] - bnd_ptr[v]) + (int_ptr[v + 1] - int_ptr[v]));
      const double outdeg = rint(1.0 / inv64[v]);
      const int o = perm[v];
      const double sd = s > 0.0 ? s : 1.0;
      F[4 * (int64_t)o + 0] = (float)log1p(indeg);
      F[4 * (int64_t)o + 1] = (float)log1p(outdeg);
      F[4 * (int64_t)o + 2] = (float)log1p((wprime[v] - W[o]) / sd);
      F[4 * (int64_t)o + 3] = (float)log1p(r1 / sd);
      S[o] = (float)s;
      mask[o] = 1;
    }
  }
}

int32_t mlp_alloc(Mlp& m) {
  PR_HIP_CHECK(hipGetDevice(&m.device));
  PR_HIP_CHECK(hipMalloc(&m.master, sizeof(float) * kMlpParams));
  PR_HIP_CHECK(hipMalloc(&m.mom1, sizeof(float) * kMlpParams));
  PR_HIP_CHECK(hipMalloc(&m.mom2, sizeof(float) * kMlpParams));
  PR_HIP_CHECK(hipMalloc(&m.grad, sizeof(float) * kMlpParams));
  PR_HIP_CHECK(hipMalloc(&m.loss, sizeof(double)));
  PR_HIP_CHECK(hipMalloc(&m.packed, sizeof(MlpPacked)));
  PR_HIP_CHECK(hipMemset(m.mom1, 0, sizeof(float) * kMlpParams));
  PR_HIP_CHECK(hipMemset(m.mom2, 0, sizeof(float) * kMlpParams));
  return PR_OK;
}

int32_t mlp_upload(Mlp& m, const float* host) {
  PR_HIP_CHECK(hipMemcpy(m.master, host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
  k_mlp_pack<<<1, kT>>>(m.master, m.packed);
  PR_HIP_CHECK(hipGetLastError());
  PR_HIP_CHECK(hipDeviceSynchronize());
  return PR_OK;
}

// workgroups of the gradient kernel for n rows (at most 256, so at most
// 1024 wavefront partials whatever the batch)
int64_t grad_groups(int64_t n) {
  const int64_t nblk = (n + 15) / 16;
  return std::max<int64_t>(1, std::min<int64_t>(256, (nblk + 3) / 4));
}

// gradient of the batch into m.grad / m.loss on stream s, the per-wavefront
// partials in gpart / lpart (every partial the reduction reads is written)
int32_t launch_grad(Mlp& m, int64_t n, const float* X, const float* T, float* gpart, double* lpart,
                    hipStream_t s) {
  const int64_t G = grad_groups(n);
  const int64_t P = G * (kT / 64);
  k_mlp_grad<<<(unsigned)G, kT, 0, s>>>(m.packed, m.master, X, T, n, (float)(2.0 / (double)n), gpart, lpart);
  k_mlp_reduce<<<(kMlpParams + kT - 1) / kT, kT, 0, s>>>(gpart, P, lpart, m.grad, m.loss);
  PR_HIP_CHECK(hipGetLastError());
  return PR_OK;
}

// gradient of the batch into m.grad / m.loss on stream s
int32_t mlp_grad(Mlp& m, int64_t n, const float* X, const float* T, hipStream_t s) {
  const int64_t P = grad_groups(n) * (kT / 64);
  if (P > m.gpart_cap) {
    if (m.gpart) (void)hipFree(m.gpart);
    if (m.lpart) (void)hipFree(m.lpart);
    m.gpart = nullptr;
    m.lpart = nullptr;
    PR_HIP_CHECK(hipMalloc(&m.gpart, sizeof(float) * kMlpParams * P));
    PR_HIP_CHECK(hipMalloc(&m.lpart, sizeof(double) * P));
    m.gpart_cap = P;
  }
  return launch_grad(m, n, X, T, m.gpart, m.lpart, s);
}

// ------------------------------------------- gradient without allocation
// pr_mlp_grad_noalloc keeps the per-wavefront partials in this file-scope
// array instead of a buffer the network allocates on first use: room for
// kScratchParts partial gradients (the most the gradient kernel writes for
// any batch) and their loss partials, 17.8 MiB that every device the library
// runs on holds until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address): it
// uses the address hipGetSymbolAddress gave for the current device.
constexpr int64_t kScratchParts = 1024;
constexpr size_t kScratchGradBytes = sizeof(float) * (size_t)kMlpParams * kScratchParts;
constexpr size_t kScratchBytes = kScratchGradBytes + sizeof(double) * kScratchParts;
static_assert(kScratchGradBytes % 256 == 0, "loss partials start on a 256-byte boundary");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// the array's address on the current device, looked up once per device
int32_t scratch_address(void** out) {
  int dev = 0;
  PR_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d: the static gradient scratch supports devices 0..%d", dev, kMaxDevices - 1);
    return PR_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    PR_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the gradient scratch on device %d", dev);
      return PR_EHIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PR_OK;
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

Mlp* as_mlp(pr_mlp_t* h) { return reinterpret_cast<Mlp*>(h); }

int32_t check_mlp(const pr_mlp_t* h) {
  if (!registry_has(h, KIND_MLP)) {
    set_error("not a live pr_mlp handle");
    return PR_EHANDLE;
  }
  int dev = 0;
  PR_HIP_CHECK(hipGetDevice(&dev));
  if (dev != reinterpret_cast<const Mlp*>(h)->device) {
    set_error("network lives on device %d but device %d is current", reinterpret_cast<const Mlp*>(h)->device, dev);
    return PR_EINVAL;
  }
  return PR_OK;
}

constexpr char kMagic[8] = {'P', 'R', 'M', 'L', 'P', '0', '0', '1'};

}  // namespace

Mlp::~Mlp() {
  void* ps[] = {master, mom1, mom2, grad, loss, packed, gpart, lpart};
  for (void* p : ps)
    if (p) (void)hipFree(p);
}

void mlp_destroy(void* h) { delete reinterpret_cast<Mlp*>(h); }

}  // namespace prlib

using namespace prlib;

extern "C" {

int32_t pr_mlp_create(uint64_t seed, pr_mlp_t** out) {
  if (!out) {
    set_error("out is NULL");
    return PR_EINVAL;
  }
  Mlp* m = new (std::nothrow) Mlp();
  if (!m) {
    set_error("out of host memory");
    return PR_ENOMEM;
  }
  int32_t rc = mlp_alloc(*m);
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a counter-based stream
  std::vector<float> h(kMlpParams);
  uint64_t st = seed;
  for (int i = 0; i < kMlpParams; ++i) {
    const int fan = (i < kOffB1 || (i >= kOffB1 && i < kOffW2)) ? kMlpIn : kMlpHidden;
    const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
    h[i] = (float)((2.0 * u - 1.0) / std::sqrt((double)fan));
  }
  if (!rc) rc = mlp_upload(*m, h.data());
  if (rc) {
    delete m;
    return rc;
  }
  registry_add(m, KIND_MLP);
  *out = reinterpret_cast<pr_mlp_t*>(m);
  return PR_OK;
}

int32_t pr_mlp_set_params(pr_mlp_t* h, const float* host_params) {
  PR_TRY(check_mlp(h));
  if (!host_params) {
    set_error("host_params is NULL");
    return PR_EINVAL;
  }
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(host_params[i])) {
      set_error("parameter %d is not finite", i);
      return PR_EINVAL;
    }
  Mlp* m = as_mlp(h);
  PR_TRY(mlp_upload(*m, host_params));
  PR_HIP_CHECK(hipMemset(m->mom1, 0, sizeof(float) * kMlpParams));
  PR_HIP_CHECK(hipMemset(m->mom2, 0, sizeof(float) * kMlpParams));
  m->step = 0;
  return PR_OK;
}

int32_t pr_mlp_get_params(const pr_mlp_t* h, float* host_out) {
  PR_TRY(check_mlp(h));
  if (!host_out) {
    set_error("host_out is NULL");
    return PR_EINVAL;
  }
  PR_HIP_CHECK(hipMemcpy(host_out, reinterpret_cast<const Mlp*>(h)->master, sizeof(float) * kMlpParams,
                         hipMemcpyDeviceToHost));
  return PR_OK;
}

int32_t pr_mlp_predict(const pr_mlp_t* h, int64_t n, const float* X_dev, float* y_dev, void* hip_stream) {
  PR_TRY(check_mlp(h));
  if (n < 0 || (n > 0 && (!X_dev || !y_dev))) {
    set_error("bad arguments (n = %lld)", (long long)n);
    return PR_EINVAL;
  }
  if (n == 0) return PR_OK;
  const int64_t chunks = (n + 63) / 64;
  const unsigned G = (unsigned)std::min<int64_t>(4096, (chunks + 3) / 4);
  k_mlp_predict<<<G, kT, 0, (hipStream_t)hip_stream>>>(reinterpret_cast<const Mlp*>(h)->packed, X_dev, y_dev, n);
  PR_HIP_CHECK(hipGetLastError());
  PR_HIP_CHECK(hipStreamSynchronize((hipStream_t)hip_stream));
  return PR_OK;
}

int32_t pr_mlp_grad(pr_mlp_t* h, int64_t n, const float* X_dev, const float* t_dev, float* grad_host,
                    double* loss, void* hip_stream) {
  PR_TRY(check_mlp(h));
  if (n <= 0 || !X_dev || !t_dev) {
    set_error("bad arguments (n = %lld)", (long long)n);
    return PR_EINVAL;
  }
  Mlp* m = as_mlp(h);
  const hipStream_t s = (hipStream_t)hip_stream;
  PR_TRY(mlp_grad(*m, n, X_dev, t_dev, s));
  double l = 0.0;
  PR_HIP_CHECK(hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grad_host)
    PR_HIP_CHECK(hipMemcpyAsync(grad_host, m->grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  if (loss) *loss = l / (double)n;
  return PR_OK;
}

int32_t pr_mlp_grad_noalloc(pr_mlp_t* h, int64_t n, const float* X_dev, const float* t_dev, float* grad_host,
                            double* loss, void* hip_stream) {
  PR_TRY(check_mlp(h));
  if (n <= 0 || !X_dev || !t_dev) {
    set_error("bad arguments (n = %lld)", (long long)n);
    return PR_EINVAL;
  }
  const int64_t P = grad_groups(n) * (kT / 64);
  if (P > kScratchParts) {
    set_error("%lld gradient partials needed; the static scratch holds %lld", (long long)P,
              (long long)kScratchParts);
    return PR_EINVAL;
  }
  void* base = nullptr;
  PR_TRY(scratch_address(&base));
  Mlp* m = as_mlp(h);
  const hipStream_t s = (hipStream_t)hip_stream;
  float* gpart = reinterpret_cast<float*>(base);
  double* lpart = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(base) + kScratchGradBytes);
  PR_TRY(launch_grad(*m, n, X_dev, t_dev, gpart, lpart, s));
  double l = 0.0;
  PR_HIP_CHECK(hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grad_host)
    PR_HIP_CHECK(hipMemcpyAsync(grad_host, m->grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  if (loss) *loss = l / (double)n;
  return PR_OK;
}

int32_t pr_mlp_train_step(pr_mlp_t* h, int64_t n, const float* X_dev, const float* t_dev, float lr, double* loss,
                          void* hip_stream) {
  PR_TRY(check_mlp(h));
  if (n <= 0 || !X_dev || !t_dev || !(lr > 0.f) || !std::isfinite(lr)) {
    set_error("bad arguments (n = %lld, lr = %g)", (long long)n, (double)lr);
    return PR_EINVAL;
  }
  Mlp* m = as_mlp(h);
  const hipStream_t s = (hipStream_t)hip_stream;
  PR_TRY(mlp_grad(*m, n, X_dev, t_dev, s));
  m->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 - std::pow(b1, (double)m->step));
  const float bc2 = (float)(1.0 - std::pow(b2, (double)m->step));
  k_mlp_adam<<<(kMlpParams + kT - 1) / kT, kT, 0, s>>>(m->master, m->mom1, m->mom2, m->grad, lr, (float)b1,
                                                        (float)b2, 1e-8f, bc1, bc2);
  k_mlp_pack<<<1, kT, 0, s>>>(m->master, m->packed);
  PR_HIP_CHECK(hipGetLastError());
  double l = 0.0;
  PR_HIP_CHECK(hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  if (loss) *loss = l / (double)n;
  return PR_OK;
}

int32_t pr_mlp_save(const pr_mlp_t* h, const char* path) {
  PR_TRY(check_mlp(h));
  if (!path) {
    set_error("path is NULL");
    return PR_EINVAL;
  }
  const Mlp* m = reinterpret_cast<const Mlp*>(h);
  std::vector<float> buf(3 * (size_t)kMlpParams);
  PR_HIP_CHECK(hipMemcpy(buf.data(), m->master, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  PR_HIP_CHECK(hipMemcpy(buf.data() + kMlpParams, m->mom1, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  PR_HIP_CHECK(hipMemcpy(buf.data() + 2 * kMlpParams, m->mom2, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) {
    set_error("cannot open %s for writing", path);
    return PR_EINVAL;
  }
  const int32_t np = kMlpParams;
  const int64_t step = m->step;
  const bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 && fwrite(&step, 8, 1, f) == 1 &&
                  fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  if (fclose(f) != 0 || !ok) {
    set_error("writing %s failed", path);
    return PR_EINVAL;
  }
  return PR_OK;
}

int32_t pr_mlp_load(const char* path, pr_mlp_t** out) {
  if (!path || !out) {
    set_error("path / out is NULL");
    return PR_EINVAL;
  }
  FILE* f = fopen(path, "rb");
  if (!f) {
    set_error("cannot open %s", path);
    return PR_EINVAL;
  }
  char magic[8];
  int32_t np = 0;
  int64_t step = 0;
  std::vector<float> buf(3 * (size_t)kMlpParams);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(&np, 4, 1, f) == 1 &&
            np == kMlpParams && fread(&step, 8, 1, f) == 1 && step >= 0 &&
            fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  fclose(f);
  if (!ok) {
    set_error("%s is not a saved network (magic, size or length mismatch)", path);
    return PR_EINVAL;
  }
  for (float x : buf)
    if (!std::isfinite(x)) {
      set_error("%s holds a non-finite value", path);
      return PR_EINVAL;
    }
  Mlp* m = new (std::nothrow) Mlp();
  if (!m) {
    set_error("out of host memory");
    return PR_ENOMEM;
  }
  int32_t rc = mlp_alloc(*m);
  if (!rc) rc = mlp_upload(*m, buf.data());
  if (!rc) {
    hipError_t e1 = hipMemcpy(m->mom1, buf.data() + kMlpParams, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    hipError_t e2 =
        hipMemcpy(m->mom2, buf.data() + 2 * kMlpParams, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      set_error("hipMemcpy of the Adam moments failed");
      rc = PR_EHIP;
    }
  }
  if (rc) {
    delete m;
    return rc;
  }
  m->step = step;
  registry_add(m, KIND_MLP);
  *out = reinterpret_cast<pr_mlp_t*>(m);
  return PR_OK;
}

int32_t pr_warm_features(const pr_levels_t* lh, double c, const void* W_dev, float* F_dev, float* s_dev,
                         uint8_t* mask_dev, void* hip_stream) {
  if (!registry_has(lh, KIND_LEVELS)) {
    set_error("not a live pr_levels handle");
    return PR_EHANDLE;
  }
  const Levels& lv = *reinterpret_cast<const Levels*>(lh);
  if (!(c > 0.0 && c < 1.0)) {
    set_error("c = %g must lie in (0, 1)", c);
    return PR_EINVAL;
  }
  if (lv.n > 0 && (!W_dev || !F_dev || !s_dev || !mask_dev)) {
    set_error("a buffer is NULL");
    return PR_EINVAL;
  }
  if (lv.n == 0) return PR_OK;
  const hipStream_t s = (hipStream_t)hip_stream;
  std::vector<int32_t> ranks;
  for (int64_t r = 0; r < lv.n_comp; ++r)
    if (lv.h_comp_class[r] == 0) ranks.push_back((int32_t)r);
  PR_HIP_CHECK(hipMemsetAsync(F_dev, 0, sizeof(float) * 4 * lv.n, s));
  PR_HIP_CHECK(hipMemsetAsync(s_dev, 0, sizeof(float) * lv.n, s));
  PR_HIP_CHECK(hipMemsetAsync(mask_dev, 0, lv.n, s));
  if (!ranks.empty()) {
    int32_t* d_ranks = nullptr;
    PR_HIP_CHECK(hipMalloc(&d_ranks, sizeof(int32_t) * ranks.size()));
    hipError_t e = hipMemcpyAsync(d_ranks, ranks.data(), sizeof(int32_t) * ranks.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      const unsigned G = (unsigned)std::min<size_t>(ranks.size(), 4096);
      k_features<<<G, kT, 0, s>>>(d_ranks, (int64_t)ranks.size(), lv.comp_vbeg, lv.bnd_ptr, lv.int_ptr, lv.int_src,
                                  lv.inv_deg64, lv.perm, lv.wprime, (const double*)W_dev, c, F_dev, s_dev, mask_dev);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_ranks);
    if (e != hipSuccess) {
      set_error("features: %s", hipGetErrorString(e));
      return PR_EHIP;
    }
  }
  return PR_OK;
}

}  // extern "C"
