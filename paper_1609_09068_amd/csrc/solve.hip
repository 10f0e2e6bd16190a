// The PageRank step of Sec. 3.3 on the device: one persistent kernel that
// works through the plan's items in topological order.
//
// What one item computes (Sec. 3.3, loops ignored):
//  * ITEM_VERTS   up to 256 consecutive vertices that are one-vertex
//                 components or CAC vertices.  Every in-edge of such a vertex
//                 comes from an earlier position (a higher level, or earlier
//                 in the CAC's topological order), so
//                     R_v = W_v + sum_{u -> v} x_u,    x_u = c R_u / outdeg(u)
//                 computed once (eq. PR:levels plus the one-sweep CAC rule of
//                 Sec. 3.3.1).
//  * ITEM_SMALL   up to four SCCs, one wavefront each, with the series terms
//                 kept in LDS: W'_C from the rank flowing in (eq. PR:levels),
//                 then the power series P_0 = W'_C, P_{k+1} = c A_CC^T P_k,
//                 R_C = sum_k P_k (Sec. 3.3.2) until the stop rule holds.
//  * ITEM_TEAM    one member of a team of workgroups that runs the same
//                 series on one larger SCC; members share the vector through
//                 global memory and meet at a barrier once per term.
// Dependencies between items are data driven: x starts at -1 ("not ready")
// and every x_u is written exactly once, with an agent-scope store, after
// R_u is final; readers poll with agent-scope loads.  Items are handed out
// in plan order by an atomic counter, so every item an item waits for was
// handed out earlier to a workgroup that is running; teams are contiguous
// in the list and never larger than half the resident grid.
//
// Precision: series terms y_k = c P_k / outdeg and their row sums are FP32
// (PR_PREC_MIXED) or FP64; R, W', x, the norms and every sum across rows are
// FP64.  All reductions use a fixed order (butterflies, fixed trees, and
// fixed-point integer sums across workgroups), so a solve is bitwise
// reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "devsort.h"

namespace prlib {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSmallMax = 256;  // rows of a wavefront-resident SCC

enum : int { C_HEAD = 0, C_EDGE_ITERS = 1, C_ITERS_MAX = 2, C_ITERS_SUM = 3, C_N_ITERATED = 4,
             C_NOT_CONV = 5, C_ERROR = 6, C_BAD_W = 7, C_WS_ACC = 8, C_WS_REJ = 9, C_COUNT = 16 };

struct SolveParams {
  int32_t n;
  int32_t stop;
  int32_t plain;
  int32_t n_items;
  double c, eps, tol;
  int64_t max_iter;
  const double* W;
  double* Rout;
  const int32_t* perm;
  const uint32_t* bnd_ptr;
  const int32_t* bnd_src;
  const uint32_t* int_ptr;
  const int32_t* int_src;
  const float* inv32;
  const double* inv64;
  double* x;
  double* R;
  double* wprime;
  void* y0;
  void* y1;
  const Item* items;
  const TeamDesc* teams;
  TeamSync* tsync;
  double* tpartial;
  const int32_t* comp_vbeg;
  int32_t* iters;
  double* lastnorm;
  unsigned long long* counters;
  unsigned long long timeout;  // wall-clock ticks a wait may take before it is abandoned
};

// ------------------------------------------------------------------ helpers

__device__ inline double ld_x(const double* x, int u) {
  return __hip_atomic_load(const_cast<double*>(x) + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_x(double* x, int u, double v) {
  __hip_atomic_store(x + u, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long ld_u64(const unsigned long long* p) {
  return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a wait gives up when it exceeds the timeout or when any other wait of the
// grid already gave up (the solve then reports an internal error)
__device__ inline bool aborted(const SolveParams& p) {
  return __hip_atomic_load(&p.counters[C_ERROR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull;
}
__device__ inline bool timed_out(const SolveParams& p, unsigned long long t0) {
  if (aborted(p)) return true;
  if (wall_clock64() - t0 > p.timeout) {
    atomicOr(&p.counters[C_ERROR], 1ull);
    return true;
  }
  return false;
}

// butterfly sum: every lane ends with the same, bitwise identical value
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <int LPR, typename T>
__device__ inline T group_sum(T v) {
#pragma unroll
  for (int o = LPR / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double block_sum(double v, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return t;
}
__device__ inline double block_max(double v, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
  __syncthreads();
  return t;
}

// sum of x over the between-component in-edges of row v, waiting for
// sources that are not final yet; LPR lanes share the row
template <int LPR>
__device__ inline double gather_between(const SolveParams& p, int v, bool act, int sub) {
  double acc = 0.0;
  if (act) {
    const uint32_t lo = p.bnd_ptr[v], hi = p.bnd_ptr[v + 1];
    unsigned long long t0 = 0;
    bool first = true;
    while (true) {
      acc = 0.0;
      bool ok = true;
      for (uint32_t e = lo + sub; e < hi; e += LPR) {
        const double xv = ld_x(p.x, p.bnd_src[e]);
        ok &= (xv >= 0.0);
        acc += xv;
      }
      if (ok) break;
      if (first) {
        t0 = wall_clock64();
        first = false;
      } else if (timed_out(p, t0)) {
        acc = 0.0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  return group_sum<LPR>(acc);
}

// ------------------------------------------------------------------ items

// One-vertex components and CAC vertices (Sec. 3.3 first bullet, Sec. 3.3.1).
__device__ void run_verts(const SolveParams& p, int vbeg, int vend) {
  const int v = vbeg + (int)threadIdx.x;
  const bool act = v < vend;
  double acc = gather_between<1>(p, v, act, 0);
  if (act) {
    acc += p.W[p.perm[v]];
    p.wprime[v] = acc;
  }
  uint32_t e = act ? p.int_ptr[v] : 0u;
  const uint32_t hi = act ? p.int_ptr[v + 1] : 0u;
  bool done = !act;
  unsigned long long t0 = wall_clock64();
  while (true) {
    if (!done) {
      while (e < hi) {  // in-edges inside the CAC, in topological order
        const double xv = ld_x(p.x, p.int_src[e]);
        if (xv < 0.0) break;
        acc += xv;
        ++e;
      }
      if (e == hi) {
        st_x(p.x, v, p.c * acc * p.inv64[v]);
        p.Rout[p.perm[v]] = acc;
        done = true;
      }
    }
    if (__all(done)) break;
    if (timed_out(p, t0)) {
      if (!done) {
        p.Rout[p.perm[v]] = acc;
        st_x(p.x, v, 0.0);
      }
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

__device__ inline bool stop_now(const SolveParams& p, double norm, double mx, double thresh) {
  return p.stop == PR_STOP_CERT_L1 ? (norm <= thresh) : (mx < p.tol);
}

// An SCC with at most 256 vertices, iterated by one wavefront.
template <typename YT>
__device__ void run_small(const SolveParams& p, int rank, YT* ybuf) {
  const int lane = threadIdx.x & 63;
  const int vbeg = p.comp_vbeg[rank];
  const int nv = p.comp_vbeg[rank + 1] - vbeg;
  YT* ya = ybuf;
  YT* yb = ybuf + kSmallMax;
  double Rj[4];
  float inv[4];
  double part = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = lane + 64 * j;
    const bool act = i < nv;
    const int v = vbeg + i;
    const double wp = gather_between<1>(p, v, act, 0) + (act ? p.W[p.perm[v]] : 0.0);
    Rj[j] = wp;
    inv[j] = act ? p.inv32[v] : 0.0f;
    if (act) {
      if constexpr (sizeof(YT) == 8) ya[i] = (YT)(p.c * wp * p.inv64[v]);
      else ya[i] = (YT)(p.c * wp * (double)inv[j]);
      p.wprime[v] = wp;
      part += wp;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const double wsum = wave_sum(part);
  const double thresh = p.eps * (1.0 - p.c) * wsum;
  const YT cy = (YT)p.c;
  int64_t k = 0;
  double last = wsum;
  bool conv = true;
  if (!(p.stop == PR_STOP_CERT_L1 && wsum == 0.0)) {
    conv = false;
    while (k < p.max_iter) {
      ++k;
      part = 0.0;
      double pm = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = lane + 64 * j;
        if (i < nv) {
          const int v = vbeg + i;
          YT s = 0;
          for (uint32_t e = p.int_ptr[v]; e < p.int_ptr[v + 1]; ++e) s += ya[p.int_src[e] - vbeg];
          Rj[j] += (double)s;
          if constexpr (sizeof(YT) == 8) yb[i] = cy * s * p.inv64[v];
          else yb[i] = cy * s * inv[j];
          part += (double)s;
          pm = fmax(pm, (double)s);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      const double norm = wave_sum(part);
      const double mx = wave_max(pm);
      last = norm;
      YT* t = ya;
      ya = yb;
      yb = t;
      if (stop_now(p, norm, mx, thresh)) {
        conv = true;
        break;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = lane + 64 * j;
    if (i < nv) {
      const int v = vbeg + i;
      p.Rout[p.perm[v]] = Rj[j];
      st_x(p.x, v, p.c * Rj[j] * p.inv64[v]);
    }
  }
  if (lane == 0) {
    p.iters[rank] = (int32_t)k;
    p.lastnorm[rank] = last;
    const uint32_t ne = p.int_ptr[vbeg + nv] - p.int_ptr[vbeg];
    atomicAdd(&p.counters[C_EDGE_ITERS], (unsigned long long)k * ne);
    atomicMax(&p.counters[C_ITERS_MAX], (unsigned long long)k);
    atomicAdd(&p.counters[C_ITERS_SUM], (unsigned long long)k);
    atomicAdd(&p.counters[C_N_ITERATED], 1ull);
    if (!conv) atomicAdd(&p.counters[C_NOT_CONV], 1ull);
  }
}

struct TeamLds {
  double red[4];
  unsigned long long acc, mx;
  int flag;
};

// Barrier of generation `gen` among the T workgroups of a team; adds this
// member's fixed-point partial norm and max, returns the team totals.
__device__ void team_barrier(const SolveParams& p, TeamSync* ts, int member, int T, unsigned gen,
                             unsigned long long add, unsigned long long mx, TeamLds* L) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int slot = (int)(gen % 3u);
    if (add) atomicAdd(&ts->acc[slot], add);
    if (mx) atomicMax(&ts->mx[slot], mx);
    if (member == 0) {
      const int nxt = (int)((gen + 1u) % 3u);
      __hip_atomic_store(&ts->acc[nxt], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ts->mx[nxt], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    atomicAdd(&ts->count, 1ull);
    const unsigned long long target = (unsigned long long)gen * (unsigned long long)T;
    const unsigned long long t0 = wall_clock64();
    bool bad = false;
    while (ld_u64(&ts->count) < target) {
      if (timed_out(p, t0)) {
        bad = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
    L->acc = ld_u64(&ts->acc[slot]);
    L->mx = ld_u64(&ts->mx[slot]);
    L->flag = bad ? 1 : 0;
  }
  __syncthreads();
}

// One member of a team iterating SCC rows [vbeg, vend) (or the whole graph
// for method PLAIN).  LPR lanes share one row of the product.
template <typename YT, int LPR>
__device__ void run_team(const SolveParams& p, const TeamDesc& td, int member, TeamLds* L) {
  const int T = td.size;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % LPR, grp = lane / LPR;
  constexpr int RPW = 64 / LPR;
  const uint32_t* ptr = p.int_ptr;
  const int32_t* src = p.int_src;
  // nnz-balanced slice of the rows (edges plus one per row)
  const int vb = td.vbeg, ve = td.vend;
  const int64_t e0 = ptr[vb];
  const int64_t total = (int64_t)(ptr[ve] - ptr[vb]) + (ve - vb);
  auto find_row = [&](int64_t target) {
    int lo = vb, hi = ve;
    while (lo < hi) {
      int mid = lo + (hi - lo) / 2;
      if ((int64_t)(ptr[mid] - e0) + (mid - vb) < target) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  const int r0 = member == 0 ? vb : find_row(total * member / T);
  const int r1 = member == T - 1 ? ve : find_row(total * (member + 1) / T);
  YT* ya = (YT*)p.y0;
  YT* yb = (YT*)p.y1;
  const double c = p.c;
  // phase 0: weights raised by the rank flowing in (eq. PR:levels)
  double part = 0.0;
  for (int base = r0 + wave * RPW; base < r1; base += kWaves * RPW) {
    const int v = base + grp;
    const bool act = v < r1;
    double wp = p.plain ? 0.0 : gather_between<LPR>(p, v, act, sub);
    if (act && sub == 0) {
      wp += p.W[p.perm[v]];
      p.R[v] = wp;
      p.wprime[v] = wp;
      if constexpr (sizeof(YT) == 8) ya[v] = c * wp * p.inv64[v];
      else ya[v] = (YT)(c * wp * (double)p.inv32[v]);
      part += wp;
    }
  }
  double wsum;
  TeamSync* ts = p.tsync + td.sync;
  if (T == 1) {
    wsum = block_sum(part, L->red);
  } else {
    part = block_sum(part, L->red);
    if (threadIdx.x == 0) p.tpartial[td.poff + member] = part;
    team_barrier(p, ts, member, T, 1u, 0ull, 0ull, L);
    double s = 0.0;
    for (int j = threadIdx.x; j < T; j += kThreads)
      s += __hip_atomic_load(p.tpartial + td.poff + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wsum = block_sum(s, L->red);
  }
  const double thresh = p.eps * (1.0 - c) * wsum;
  const double scale = wsum > 0.0 ? 2305843009213693952.0 / wsum : 0.0;  // 2^61 / wsum
  const YT cy = (YT)c;
  int64_t k = 0;
  double last = wsum;
  bool conv = true;
  unsigned gen = 1;
  if (!(p.stop == PR_STOP_CERT_L1 && wsum == 0.0)) {
    conv = false;
    while (k < p.max_iter) {
      ++k;
      part = 0.0;
      double pm = 0.0;
      for (int base = r0 + wave * RPW; base < r1; base += kWaves * RPW) {
        const int v = base + grp;
        const bool act = v < r1;
        YT s = 0;
        if (act) {
          const uint32_t hi = ptr[v + 1];
          for (uint32_t e = ptr[v] + sub; e < hi; e += LPR) s += ya[src[e]];
        }
        s = group_sum<LPR>(s);
        if (act && sub == 0) {
          p.R[v] += (double)s;
          if constexpr (sizeof(YT) == 8) yb[v] = cy * s * p.inv64[v];
          else yb[v] = cy * s * p.inv32[v];
          part += (double)s;
          pm = fmax(pm, (double)s);
        }
      }
      double norm, mx;
      if (T == 1) {
        norm = block_sum(part, L->red);
        mx = block_max(pm, L->red);
      } else {
        part = block_sum(part, L->red);
        pm = block_max(pm, L->red);
        const unsigned long long fx = (unsigned long long)(part * scale);
        ++gen;
        team_barrier(p, ts, member, T, gen, fx, (unsigned long long)__double_as_longlong(pm), L);
        norm = scale > 0.0 ? (double)L->acc / scale : 0.0;
        mx = __longlong_as_double((long long)L->mx);
        if (L->flag) break;  // the grid gave up; results are reported as an error
      }
      last = norm;
      YT* t = ya;
      ya = yb;
      yb = t;
      if (stop_now(p, norm, mx, thresh)) {
        conv = true;
        break;
      }
    }
  }
  // results: R in the caller's order, x for the levels below
  for (int v = r0 + (int)threadIdx.x; v < r1; v += kThreads) {
    const double r = p.R[v];
    p.Rout[p.perm[v]] = r;
    if (!p.plain) st_x(p.x, v, c * r * p.inv64[v]);
  }
  if (member == 0 && threadIdx.x == 0) {
    if (td.rank >= 0) {
      p.iters[td.rank] = (int32_t)k;
      p.lastnorm[td.rank] = last;
    } else {
      p.lastnorm[0] = last;
    }
    const uint64_t ne = ptr[ve] - ptr[vb];
    atomicAdd(&p.counters[C_EDGE_ITERS], (unsigned long long)k * ne);
    atomicMax(&p.counters[C_ITERS_MAX], (unsigned long long)k);
    atomicAdd(&p.counters[C_ITERS_SUM], (unsigned long long)k);
    atomicAdd(&p.counters[C_N_ITERATED], 1ull);
    if (!conv) atomicAdd(&p.counters[C_NOT_CONV], 1ull);
  }
}

template <typename YT, int LPR>
__global__ __launch_bounds__(kThreads) void k_solve(SolveParams p) {
  __shared__ Item s_item;
  __shared__ TeamLds s_team;
  __shared__ YT s_y[kWaves][2 * kSmallMax];
  const int wave = threadIdx.x >> 6;
  while (true) {
    if (threadIdx.x == 0) {
      const unsigned i = atomicAdd((unsigned*)&p.counters[C_HEAD], 1u);
      s_item = (int)i < p.n_items ? p.items[i] : Item{-1, 0, 0, 0};
    }
    __syncthreads();
    const Item it = s_item;
    __syncthreads();
    if (it.kind < 0) break;
    if (it.kind == ITEM_VERTS) {
      run_verts(p, it.a, it.b);
    } else if (it.kind == ITEM_SMALL) {
      const int r = it.a + wave;
      if (r < it.b) run_small<YT>(p, r, s_y[wave]);
    } else {
      const TeamDesc td = p.teams[it.a];
      run_team<YT, LPR>(p, td, it.b, &s_team);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ setup kernels

__global__ void k_init(SolveParams p, int64_t K, int64_t n_sync, int64_t n_part) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < p.n; i += stride) {
    p.x[i] = -1.0;
    const double w = p.W[i];
    if (!(w >= 0.0) || !(w <= 1.7976931348623157e308)) atomicOr(&p.counters[C_BAD_W], 1ull);
  }
  for (int64_t i = tid; i < K; i += stride) {
    p.iters[i] = 0;
    p.lastnorm[i] = 0.0;
  }
  unsigned* ts = (unsigned*)p.tsync;
  const int64_t nts = n_sync * (int64_t)(sizeof(TeamSync) / sizeof(unsigned));
  for (int64_t i = tid; i < nts; i += stride) ts[i] = 0u;
  for (int64_t i = tid; i < n_part; i += stride) p.tpartial[i] = 0.0;
}

__global__ void k_zero_counters(unsigned long long* c) {
  if (threadIdx.x < C_COUNT) c[threadIdx.x] = 0ull;
}

// deterministic two-stage sums: ||R||_1 and sum of last series norms
constexpr int kRedBlocks = 256;
__global__ __launch_bounds__(kThreads) void k_reduce1(const double* a, int64_t na, const double* b, int64_t nb,
                                                      double* part) {
  __shared__ double lds[4];
  double sa = 0.0, sb = 0.0;
  const int64_t ca = (na + kRedBlocks - 1) / kRedBlocks, cb = (nb + kRedBlocks - 1) / kRedBlocks;
  for (int64_t i = blockIdx.x * ca + threadIdx.x; i < std::min<int64_t>(na, (blockIdx.x + 1) * ca); i += kThreads)
    sa += fabs(a[i]);
  for (int64_t i = blockIdx.x * cb + threadIdx.x; i < std::min<int64_t>(nb, (blockIdx.x + 1) * cb); i += kThreads)
    sb += b[i];
  sa = block_sum(sa, lds);
  sb = block_sum(sb, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa;
    part[2 * blockIdx.x + 1] = sb;
  }
}
__global__ __launch_bounds__(kThreads) void k_reduce2(const double* part, double* out) {
  __shared__ double lds[4];
  double sa = part[2 * threadIdx.x], sb = part[2 * threadIdx.x + 1];
  sa = block_sum(sa, lds);
  sb = block_sum(sb, lds);
  if (threadIdx.x == 0) {
    out[0] = sa;
    out[1] = sb;
  }
}

template <typename T>
int32_t dalloc(T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1));
  if (e != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP;
  }
  return PR_OK;
}

using KernelFn = void (*)(SolveParams);

KernelFn pick_kernel(int precision, int lpr) {
  if (precision == PR_PREC_FP64) {
    switch (lpr) {
      case 64: return k_solve<double, 64>;
      case 16: return k_solve<double, 16>;
      case 4: return k_solve<double, 4>;
      default: return k_solve<double, 1>;
    }
  }
  switch (lpr) {
    case 64: return k_solve<float, 64>;
    case 16: return k_solve<float, 16>;
    case 4: return k_solve<float, 4>;
    default: return k_solve<float, 1>;
  }
}

}  // namespace

#define PR_TRY(x)                 \
  do {                            \
    int32_t rc_ = (x);            \
    if (rc_ != PR_OK) return rc_; \
  } while (0)

// resident workgroups of the solve kernel for one rows-per-wave choice
static int32_t grid_for(int lpr, int* grid) {
  int dev, cus;
  PR_HIP_CHECK(hipGetDevice(&dev));
  PR_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int best = 1 << 30;
  for (int prec = 0; prec < 2; ++prec) {
    int occ = 0;
    PR_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)pick_kernel(prec, lpr), kThreads, 0));
    best = std::min(best, occ);
  }
  if (best < 1) {
    set_error("solve kernel cannot be resident (occupancy 0)");
    return PR_EHIP;
  }
  const int per_cu = std::min(best, 4);
  *grid = per_cu * cus;
  return PR_OK;
}

int32_t make_schedule(Levels& lv, hipStream_t s) {
  const int lpr = 64 / lv.opts.rows_per_wave;
  PR_TRY(grid_for(lpr, &lv.grid));
  const int G = lv.grid;
  const int team_cap = std::max(1, G / 2);
  const int64_t K = lv.n_comp;
  std::vector<Item> items;
  std::vector<TeamDesc> teams;
  int32_t poff = 0;
  int64_t max_team = 0;
  int64_t r = 0;
  while (r < K) {
    const int lev = lv.h_comp_level[r];
    int64_t e = r;
    while (e < K && lv.h_comp_level[e] == lev) ++e;
    // SCCs of the level: ranks [r, sc) in size order
    int64_t sc = r;
    while (sc < e && lv.h_comp_class[sc] == 0) ++sc;
    std::vector<int64_t> small;
    for (int64_t q = r; q < sc; ++q) {
      const int32_t nv = lv.h_comp_vbeg[q + 1] - lv.h_comp_vbeg[q];
      if (nv <= lv.opts.small_cutoff) {
        small.push_back(q);
        continue;
      }
      const int64_t ne = lv.h_comp_int_edges[q];
      int T = (int)std::min<int64_t>(team_cap, std::max<int64_t>(1, (ne + lv.opts.team_edges - 1) / lv.opts.team_edges));
      TeamDesc td{};
      td.rank = (int32_t)q;
      td.size = T;
      td.vbeg = lv.h_comp_vbeg[q];
      td.vend = lv.h_comp_vbeg[q + 1];
      td.poff = poff;
      td.sync = (int32_t)teams.size();
      poff += T;
      max_team = std::max<int64_t>(max_team, T);
      for (int j = 0; j < T; ++j) items.push_back(Item{ITEM_TEAM, (int32_t)teams.size(), j, T});
      teams.push_back(td);
    }
    for (size_t i = 0; i < small.size(); i += kWaves) {
      const int64_t a = small[i];
      const int64_t b = small[std::min(small.size() - 1, i + kWaves - 1)] + 1;
      items.push_back(Item{ITEM_SMALL, (int32_t)a, (int32_t)b, 0});
    }
    // CAC and one-vertex components of the level: one contiguous range
    if (sc < e) {
      const int32_t v0 = lv.h_comp_vbeg[sc], v1 = lv.h_comp_vbeg[e];
      for (int32_t v = v0; v < v1; v += kThreads)
        items.push_back(Item{ITEM_VERTS, v, std::min(v1, v + kThreads), 0});
    }
    r = e;
  }
  lv.n_items = (int64_t)items.size();
  lv.n_teams = (int64_t)teams.size();
  // whole-graph team for method PLAIN: every resident workgroup
  TeamDesc pt{};
  pt.rank = -1;
  pt.size = G;
  pt.vbeg = 0;
  pt.vend = (int32_t)lv.n;
  pt.poff = poff;
  pt.sync = (int32_t)teams.size();
  std::vector<Item> pitems;
  for (int j = 0; j < G; ++j) pitems.push_back(Item{ITEM_TEAM, 0, j, G});
  // device copies
  if (lv.items) (void)hipFree(lv.items);
  if (lv.teams) (void)hipFree(lv.teams);
  if (lv.plain_items) (void)hipFree(lv.plain_items);
  if (lv.plain_team) (void)hipFree(lv.plain_team);
  if (lv.tsync) (void)hipFree(lv.tsync);
  if (lv.tpartial) (void)hipFree(lv.tpartial);
  lv.items = nullptr;
  lv.teams = nullptr;
  lv.plain_items = nullptr;
  lv.plain_team = nullptr;
  lv.tsync = nullptr;
  lv.tpartial = nullptr;
  PR_TRY(dalloc(&lv.items, items.size()));
  PR_TRY(dalloc(&lv.teams, teams.size()));
  PR_TRY(dalloc(&lv.plain_items, pitems.size()));
  PR_TRY(dalloc(&lv.plain_team, 1));
  PR_TRY(dalloc(&lv.tsync, teams.size() + 1));
  PR_TRY(dalloc(&lv.tpartial, (size_t)poff + G));
  if (!items.empty())
    PR_HIP_CHECK(hipMemcpyAsync(lv.items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice, s));
  if (!teams.empty())
    PR_HIP_CHECK(hipMemcpyAsync(lv.teams, teams.data(), sizeof(TeamDesc) * teams.size(), hipMemcpyHostToDevice, s));
  PR_HIP_CHECK(hipMemcpyAsync(lv.plain_items, pitems.data(), sizeof(Item) * pitems.size(), hipMemcpyHostToDevice, s));
  PR_HIP_CHECK(hipMemcpyAsync(lv.plain_team, &pt, sizeof(TeamDesc), hipMemcpyHostToDevice, s));
  // per-solve buffers
  const int64_t n = lv.n;
  if (!lv.x) {
    PR_TRY(dalloc(&lv.x, n));
    PR_TRY(dalloc(&lv.R, n));
    PR_TRY(dalloc(&lv.wprime, n));
    PR_TRY(dalloc((double**)&lv.y0, n));
    PR_TRY(dalloc((double**)&lv.y1, n));
    PR_TRY(dalloc(&lv.iters, std::max<int64_t>(K, 1)));
    PR_TRY(dalloc(&lv.lastnorm, std::max<int64_t>(K, 1)));
    PR_TRY(dalloc(&lv.counters, C_COUNT));
    PR_TRY(dalloc(&lv.red, 2 * kRedBlocks + 8));
  }
  PR_HIP_CHECK(hipStreamSynchronize(s));
  pr_levels_info& I = lv.info;
  I.n_items = lv.n_items;
  I.n_teams = lv.n_teams;
  I.max_team = max_team;
  I.rows_per_wave = lv.opts.rows_per_wave;
  I.small_cutoff = lv.opts.small_cutoff;
  I.team_edges = lv.opts.team_edges;
  I.grid_wgs = G;
  // a new schedule invalidates a captured graph
  if (lv.graph_exec) (void)hipGraphExecDestroy(lv.graph_exec);
  if (lv.graph) (void)hipGraphDestroy(lv.graph);
  lv.graph_exec = nullptr;
  lv.graph = nullptr;
  lv.graph_key = 0;
  return PR_OK;
}

static uint64_t mix64(uint64_t h, uint64_t x) {
  h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

int32_t solve_levels(Levels& lv, double c, const double* W, double* R, const pr_solve_opts& o,
                     hipStream_t s, pr_solve_stats* st) {
  int dev;
  PR_HIP_CHECK(hipGetDevice(&dev));
  if (dev != lv.device) {
    set_error("plan lives on device %d but device %d is current", lv.device, dev);
    return PR_EINVAL;
  }
  pr_solve_stats local{};
  if (lv.n == 0) {
    if (st) *st = local;
    return PR_OK;
  }
  const bool plain = o.method == PR_METHOD_PLAIN;
  int clock_khz = 0;
  PR_HIP_CHECK(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
  SolveParams p{};
  p.n = (int32_t)lv.n;
  p.stop = o.stop;
  p.plain = plain ? 1 : 0;
  p.n_items = plain ? lv.grid : (int32_t)lv.n_items;
  p.c = c;
  p.eps = o.eps;
  p.tol = o.tol;
  p.max_iter = o.max_iter;
  p.W = W;
  p.Rout = R;
  p.perm = lv.perm;
  p.bnd_ptr = lv.bnd_ptr;
  p.bnd_src = lv.bnd_src;
  p.int_ptr = plain ? lv.full_ptr : lv.int_ptr;
  p.int_src = plain ? lv.full_src : lv.int_src;
  p.inv32 = lv.inv_deg32;
  p.inv64 = lv.inv_deg64;
  p.x = lv.x;
  p.R = lv.R;
  p.wprime = lv.wprime;
  p.y0 = lv.y0;
  p.y1 = lv.y1;
  p.items = plain ? lv.plain_items : lv.items;
  p.teams = plain ? lv.plain_team : lv.teams;
  p.tsync = lv.tsync;
  p.tpartial = lv.tpartial;
  p.comp_vbeg = lv.comp_vbeg;
  p.iters = lv.iters;
  p.lastnorm = lv.lastnorm;
  p.counters = lv.counters;
  p.timeout = (unsigned long long)clock_khz * 1000ull * 30ull;  // 30 s
  const int64_t K = std::max<int64_t>(lv.n_comp, 1);
  const int64_t n_sync = lv.n_teams + 1;
  const int64_t n_part = 0;
  const unsigned init_blocks = (unsigned)std::min<int64_t>(4096, (lv.n + kThreads - 1) / kThreads + 1);

  // the weights must be non-negative and finite (a negative x would read as
  // "not ready"); checked before the solve kernel runs
  k_zero_counters<<<1, 64, 0, s>>>(lv.counters);
  k_init<<<init_blocks, kThreads, 0, s>>>(p, K, n_sync, n_part);
  PR_HIP_CHECK(hipGetLastError());
  unsigned long long badw = 0;
  PR_HIP_CHECK(hipMemcpyAsync(&badw, lv.counters + C_BAD_W, sizeof(badw), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  if (badw) {
    set_error("W has a negative or non-finite entry");
    return PR_EINVAL;
  }
  const KernelFn fn = pick_kernel(o.precision, 64 / lv.opts.rows_per_wave);
  hipEvent_t ev0, ev1;
  PR_HIP_CHECK(hipEventCreate(&ev0));
  PR_HIP_CHECK(hipEventCreate(&ev1));
  auto launch_all = [&](bool graph_mode) -> int32_t {
    if (graph_mode) {
      k_zero_counters<<<1, 64, 0, s>>>(lv.counters);
      k_init<<<init_blocks, kThreads, 0, s>>>(p, K, n_sync, n_part);
    }
    void* args[] = {&p};
    if (graph_mode) {
      PR_HIP_CHECK(hipLaunchKernel((const void*)fn, dim3(lv.grid), dim3(kThreads), args, 0, s));
    } else {
      PR_HIP_CHECK(hipLaunchCooperativeKernel((const void*)fn, dim3(lv.grid), dim3(kThreads), args, 0, s));
    }
    k_reduce1<<<kRedBlocks, kThreads, 0, s>>>(R, lv.n, lv.lastnorm, plain ? 1 : lv.n_comp, lv.red + 8);
    k_reduce2<<<1, kThreads, 0, s>>>(lv.red + 8, lv.red);
    PR_HIP_CHECK(hipGetLastError());
    return PR_OK;
  };
  int32_t rc = PR_OK;
  if (o.use_graph) {
    uint64_t key = 1469598103934665603ull;
    key = mix64(key, (uint64_t)(uintptr_t)W);
    key = mix64(key, (uint64_t)(uintptr_t)R);
    key = mix64(key, (uint64_t)__builtin_bit_cast(uint64_t, c));
    key = mix64(key, (uint64_t)__builtin_bit_cast(uint64_t, o.eps));
    key = mix64(key, (uint64_t)__builtin_bit_cast(uint64_t, o.tol));
    key = mix64(key, (uint64_t)o.max_iter);
    key = mix64(key, (uint64_t)(o.stop * 16 + o.precision * 4 + o.method));
    key = mix64(key, (uint64_t)(uintptr_t)s);
    if (!lv.graph_exec || lv.graph_key != key) {
      if (lv.graph_exec) (void)hipGraphExecDestroy(lv.graph_exec);
      if (lv.graph) (void)hipGraphDestroy(lv.graph);
      lv.graph_exec = nullptr;
      lv.graph = nullptr;
      PR_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      rc = launch_all(true);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(s, &g);
      if (rc) return rc;
      if (ce != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ce));
        return PR_EHIP;
      }
      lv.graph = g;
      PR_HIP_CHECK(hipGraphInstantiate(&lv.graph_exec, g, nullptr, nullptr, 0));
      lv.graph_key = key;
    }
    PR_HIP_CHECK(hipEventRecord(ev0, s));
    PR_HIP_CHECK(hipGraphLaunch(lv.graph_exec, s));
    PR_HIP_CHECK(hipEventRecord(ev1, s));
  } else {
    PR_HIP_CHECK(hipEventRecord(ev0, s));
    rc = launch_all(false);
    if (rc) return rc;
    PR_HIP_CHECK(hipEventRecord(ev1, s));
  }
  unsigned long long cnt[C_COUNT];
  double red[2];
  PR_HIP_CHECK(hipMemcpyAsync(cnt, lv.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipMemcpyAsync(red, lv.red, sizeof(red), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  float ms = 0.f;
  PR_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (cnt[C_ERROR]) {
    set_error("internal: a dependency wait or team barrier timed out (flags %llu)", cnt[C_ERROR]);
    return PR_EHIP;
  }
  local.edge_iters = (int64_t)cnt[C_EDGE_ITERS] +
                     (plain ? 0 : (lv.info.m_between + lv.info.m_cac_internal));
  local.iters_max = (int64_t)cnt[C_ITERS_MAX];
  local.iters_sum = (int64_t)cnt[C_ITERS_SUM];
  local.n_iterated = (int64_t)cnt[C_N_ITERATED];
  local.n_not_converged = (int64_t)cnt[C_NOT_CONV];
  local.ws_accepted = (int64_t)cnt[C_WS_ACC];
  local.ws_rejected = (int64_t)cnt[C_WS_REJ];
  local.r_sum = red[0];
  local.cert_abs = c / (1.0 - c) * red[1];
  local.cert_rel = red[0] > 0.0 ? local.cert_abs / red[0] : 0.0;
  local.time_ms = ms;
  if (st) *st = local;
  return local.n_not_converged ? PR_NOT_CONVERGED : PR_OK;
}

}  // namespace prlib

extern "C" int32_t pr_levels_debug(const pr_levels_t* lh, int32_t what, void* host_out) {
  using namespace prlib;
  if (!registry_has(lh, KIND_LEVELS)) {
    set_error("not a live pr_levels handle");
    return PR_EHANDLE;
  }
  const Levels& lv = *reinterpret_cast<const Levels*>(lh);
  if (!host_out) {
    set_error("host_out is NULL");
    return PR_EINVAL;
  }
  const int64_t n = lv.n, K = lv.n_comp;
  if (what == 0) {
    std::vector<double> wp(n);
    std::vector<int32_t> perm(n);
    if (n) {
      PR_HIP_CHECK(hipMemcpy(wp.data(), lv.wprime, sizeof(double) * n, hipMemcpyDeviceToHost));
      PR_HIP_CHECK(hipMemcpy(perm.data(), lv.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    }
    double* out = (double*)host_out;
    for (int64_t i = 0; i < n; ++i) out[perm[i]] = wp[i];
    return PR_OK;
  }
  if (what == 1) {
    std::vector<int32_t> it(K);
    if (K) PR_HIP_CHECK(hipMemcpy(it.data(), lv.iters, sizeof(int32_t) * K, hipMemcpyDeviceToHost));
    int32_t* out = (int32_t*)host_out;
    for (int64_t r = 0; r < K; ++r) out[lv.h_comp_id_of_rank[r]] = it[r];
    return PR_OK;
  }
  if (what == 2) {
    if (n) PR_HIP_CHECK(hipMemcpy(host_out, lv.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    return PR_OK;
  }
  set_error("unknown debug array %d", what);
  return PR_EINVAL;
}
