// Device code of the solve (Sec. 4.3): parameters, helpers and every
// kernel template.  Included by solve.hip (host driver, gang kernels) and by
// the seg_*.hip files, which instantiate the persistent segment kernel
// variants in translation units of their own so they compile in parallel.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "devsort.h"

namespace prlib {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSmallMax = 256;  // rows of a wavefront-resident SCC
constexpr int kGsMaxBlocks = 8;  // most Gauss-Seidel row blocks per sweep
constexpr int kDirectMax = 24;  // largest SCC solved directly: 24 x 25 doubles fit a wavefront's tile
constexpr int kDirectMaxWG = 80;  // largest workgroup SCC solved directly: 80 x 81 doubles fit the segment LDS

// per-workgroup counters (LDS during a kernel, accumulated in global memory
// across the launches of a solve); the last ones are wall-clock ticks
enum : int { S_EDGE_ITERS = 0, S_VERT_ITERS = 1, S_ITERS_MAX = 2, S_ITERS_SUM = 3, S_N_ITERATED = 4,
             S_NOT_CONV = 5, S_WS_ACC = 6, S_WS_REJ = 7, S_T_VERTS = 8, S_T_SMALL = 9, S_T_MEDIUM = 10,
             S_T_GANG = 11, S_T_WAIT = 12, S_T_SEGMENT = 13, S_N_GANG = 14, S_T_MEDIUM_ITER = 15 };
// global counters: [0, kWgStats) reduced from the workgroup counters, then flags
enum : int { C_ERROR = 16, C_BAD_W = 17, C_COUNT = 32 };
// the reduction of the workgroup counters writes slots [0, kWgStats): the
// flags must lie beyond them
static_assert(C_ERROR >= kWgStats && C_BAD_W >= kWgStats && C_BAD_W < C_COUNT, "counter layout");

struct SolveParams {
  int32_t n;
  int32_t stop;
  int32_t plain;
  int32_t n_items;  // items of the segment being run
  int32_t direct_max;  // SCCs of a wavefront with at most this many vertices are solved directly
  int32_t tail;        // segment SCC series may stop on the certified geometric tail estimate
  int32_t signed_w;    // weights may be negative (the residual that a correction solve takes)
  int32_t gs_blocks;   // > 0: workgroup SCCs on the register path take block Gauss-Seidel sweeps
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
  // weighted graph (Def. 3.4 with a_uv = w_uv / s_u, s_u the total weight of
  // u's out-edges): the raw weight of every edge, parallel to bnd_src and
  // int_src (FP32 copy for FP32 terms), and inv32/inv64 hold 1/s_u; null
  // for a plain graph, where every weight is one and s_u the out-degree
  const double* bnd_w;
  const double* int_w64;
  const float* int_w32;
  double* x;
  double* R;
  double* wprime;
  // starting guess (null: start from W'_C): for SCCs of segment items
  // (mlp) and of gangs (gmlp)
  const MlpPacked* mlp;
  const MlpPacked* gmlp;
  double* wr0;   // [n] R_0 of the guess
  double* wx;    // [n] c R_0 / outdeg
  double* wres;  // [n] r_0 = W' + c A^T R_0 - R_0
  float4* wfeat; // [n] gang SCC rows: the four features of the guess
  // starting guess of gang SCCs: per-workgroup partial norms of the first
  // plain term, of r_0 and max |r_0| (slot layout of gpart), then per SCC
  // the decision (1 kept, 0 not, -1 none), ||r_0||_1 and max |r_0|
  double* gwp1;
  double* gwr0;
  double* gwm0;
  int32_t* gws;
  double* gwn;
  double* gwm;
  void* y0;
  void* y1;
  const Item* items;
  const uint32_t* vpath;
  const uint32_t* mslot_ptr;
  const uint4* mslot_src;
  const double* mslot_w64;  // weighted plan: eight edge weights per slot
  const float* mslot_w32;
  const int32_t* comp_vbeg;
  int32_t* iters;
  double* lastnorm;
  unsigned long long* counters;
  unsigned long long* wgstats;
  const GangDesc* gangs;
  const GangScc* gscc;
  const int32_t* gbounds;
  double* gpart;
  double* gpmx;
  double* gwsum;
  double* gpdiff;
  double* gnhist;
  int32_t* gdone;
  const GangHub* ghubs;
  const GangPiece* gpieces;
  const int32_t* gpiece_ptr;
  const int32_t* ghub_pieces;
  double* gpiece_part;
  int64_t n_gslots;
  unsigned* seg_head;          // item counter of the segment being run
  unsigned long long* trace;   // optional per-item timeline [n_items][4]
  int32_t item_base;           // index of this segment's first item in the plan
  unsigned long long timeout;  // wall-clock ticks a wait may take before it is abandoned
};

// ------------------------------------------------------------------ helpers

// x holds a quiet NaN until its vertex's rank is final: any other value, of
// either sign (a correction solve has signed weights), is a published value
__device__ inline bool x_ok(double v) { return v == v; }
constexpr double kXPending = __builtin_nan("");

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

// Waiting for a value another workgroup publishes: sleep 256, 512, 1024,
// then 2048 cycles between polls, so a wavefront that waits long costs the
// memory system little.
__device__ inline void backoff_sleep(int& n) {
  for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(4);
  if (n < 8) n <<= 1;
}

// Cross-lane reductions with DPP (quad_perm xor 1 / xor 2, row half mirror,
// row mirror) inside each 16-lane row, then the four row values read as
// scalars and combined in a fixed order.  Every butterfly step pairs a lane
// with its partner and both compute the same (commutative) sum, so every
// lane ends with the bitwise identical result.  All 64 lanes must be active.
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
template <int CTRL>
__device__ inline float dpp(float v) { return dpp_f<CTRL>(v); }
template <int CTRL>
__device__ inline double dpp(double v) { return dpp_d<CTRL>(v); }
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

__device__ inline double readlane_d(double v, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline float readlane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ inline double readlane(double v, int l) { return readlane_d(v, l); }
__device__ inline float readlane(float v, int l) { return readlane_f(v, l); }

template <typename T>
__device__ inline T row16_sum(T v) {
  v += dpp<kDppXor1>(v);
  v += dpp<kDppXor2>(v);
  v += dpp<kDppHalfMirror>(v);
  v += dpp<kDppMirror>(v);
  return v;
}
template <typename T>
__device__ inline T row16_max(T v) {
  v = fmax(v, dpp<kDppXor1>(v));
  v = fmax(v, dpp<kDppXor2>(v));
  v = fmax(v, dpp<kDppHalfMirror>(v));
  v = fmax(v, dpp<kDppMirror>(v));
  return v;
}
template <typename T>
__device__ inline T wave_sum(T v) {
  v = row16_sum(v);
  return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}
// two wavefront sums at once (independent chains, each in wave_sum's order)
template <typename T>
__device__ inline void wave_sum2(T a, T b, T& sa, T& sb) {
  a = row16_sum(a);
  b = row16_sum(b);
  sa = (readlane(a, 0) + readlane(a, 16)) + (readlane(a, 32) + readlane(a, 48));
  sb = (readlane(b, 0) + readlane(b, 16)) + (readlane(b, 32) + readlane(b, 48));
}
template <typename T>
__device__ inline T wave_max(T v) {
  v = row16_max(v);
  return fmax(fmax(readlane(v, 0), readlane(v, 16)), fmax(readlane(v, 32), readlane(v, 48)));
}
// sum over aligned groups of LPR lanes; every lane of a group gets the result
template <int LPR, typename T>
__device__ inline T group_sum(T v) {
  if constexpr (LPR >= 2) v += dpp<kDppXor1>(v);
  if constexpr (LPR >= 4) v += dpp<kDppXor2>(v);
  if constexpr (LPR >= 8) v += dpp<kDppHalfMirror>(v);
  if constexpr (LPR >= 16) v += dpp<kDppMirror>(v);
  if constexpr (LPR == 64) v = (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
  return v;
}

// sum and max over the workgroup with a single barrier; red holds 16
// doubles used by alternating parities
__device__ inline void block_sum_max(double v, double m, double* red, int parity, double* sum, double* mx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  m = wave_max(m);
  double* r = red + 8 * parity;
  if (lane == 0) {
    r[wave] = v;
    r[4 + wave] = m;
  }
  __syncthreads();
  *sum = (r[0] + r[1]) + (r[2] + r[3]);
  *mx = fmax(fmax(r[4], r[5]), fmax(r[6], r[7]));
}

// the same with a second sum (red holds 24 doubles)
__device__ inline void block_sum2_max(double v, double d, double m, double* red, int parity, double* sum,
                                      double* dsum, double* mx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  d = wave_sum(d);
  m = wave_max(m);
  double* r = red + 12 * parity;
  if (lane == 0) {
    r[wave] = v;
    r[4 + wave] = m;
    r[8 + wave] = d;
  }
  __syncthreads();
  *sum = (r[0] + r[1]) + (r[2] + r[3]);
  *mx = fmax(fmax(r[4], r[5]), fmax(r[6], r[7]));
  *dsum = (r[8] + r[9]) + (r[10] + r[11]);
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

// ---------------------------------------------------------------- gathers
// A vertex item hands a row with more than kLongLane CAC sources to the
// whole wavefront.
constexpr uint32_t kLongLane = 32;

// ------------------------------------------------------------ tiled gather
// A wavefront sums, for up to 64 consecutive rows [ra, ra+nr), the values
// val[src[e]] over each row's sources.  The tile's sources are streamed in
// chunks of kChunk edges: phase 1 has all 64 lanes load 8 source indices and
// 8 values each (independent, coalesced index loads) into LDS; phase 2 sums
// each row's part of the chunk from LDS, 64/RPW rows at a time with LPR
// lanes per row.  Row sums accumulate chunk by chunk in edge order, so the
// result does not depend on timing.  With WAIT_X the values are the x
// vector and a chunk is re-read until every source is final.  With WT every
// value is multiplied by its edge's weight wt[e] as it is staged.
constexpr int kChunk = 512;
constexpr uint32_t kBigPart = 16;  // per lane of a row: above this the whole wavefront sums the row's part

struct WaveTile {
  double buf[kChunk];
  double racc[64];
  uint32_t rlo[64], rhi[64];
  unsigned long long* wst;  // the workgroup's counters (time accounting)
  unsigned long long* rdy;  // latest end of a readiness wait in the current item (trace)
};

template <int RPW, typename VT, bool WAIT_X, bool WT = false>
__device__ __attribute__((always_inline)) VT wave_tile_gather(const SolveParams& p, const uint32_t* ptr, const int32_t* src, const VT* val,
                               int ra, int nr, WaveTile* t, const VT* wt = nullptr) {
  constexpr int LPR = 64 / RPW;
  const int lane = threadIdx.x & 63;
  VT* buf = reinterpret_cast<VT*>(t->buf);
  VT* racc = reinterpret_cast<VT*>(t->racc);
  const bool act = lane < nr;
  const uint32_t lo = act ? ptr[ra + lane] : 0u, hi = act ? ptr[ra + lane + 1] : 0u;
  const uint32_t E0 = __shfl(lo, 0, 64);
  const uint32_t E1 = __shfl(hi, nr - 1, 64);
  t->rlo[lane] = lo;
  t->rhi[lane] = hi;
  racc[lane] = (VT)0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (uint32_t cs = E0; cs < E1; cs += kChunk) {
    const uint32_t ce = cs + kChunk < E1 ? cs + kChunk : E1;
    int32_t idx[8];
    VT wv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t e = cs + lane + 64 * j;
      idx[j] = e < ce ? src[e] : -1;
      if constexpr (WT) wv[j] = e < ce ? wt[e] : (VT)0;
    }
    if constexpr (WAIT_X) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = idx[j] >= 0 ? ld_x(p.x, idx[j]) : 0.0;
      bool ok = true;
#pragma unroll
      for (int j = 0; j < 8; ++j) ok = ok && x_ok(v[j]);
      if (!__all(ok)) {
        // poll one missing source at a time (one address for the whole
        // wavefront), then re-read only the sources still missing
        const unsigned long long t0 = wall_clock64();
        int nap = 1;
        while (true) {
          int want = -1;
#pragma unroll
          for (int j = 7; j >= 0; --j)
            if (!x_ok(v[j])) want = idx[j];
          const unsigned long long m = __ballot(want >= 0);
          if (!m) break;
          const int a = __shfl(want, __ffsll(m) - 1, 64);
          bool late = false;
          unsigned polls = 0;
          while (!x_ok(ld_x(p.x, a))) {
            if ((++polls & 15u) == 0u && timed_out(p, t0)) {
              late = true;
              break;
            }
            backoff_sleep(nap);
          }
          if (late) break;
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (!x_ok(v[j])) v[j] = ld_x(p.x, idx[j]);
        }
        if (lane == 0) atomicAdd(&t->wst[S_T_WAIT], wall_clock64() - t0);
      }
      if (p.trace && lane == 0) atomicMax(t->rdy, wall_clock64());
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (WT) v[j] *= (double)wv[j];
        if (idx[j] >= 0) buf[lane + 64 * j] = (VT)v[j];
      }
    } else {
      VT v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = idx[j] >= 0 ? val[idx[j]] : (VT)0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (WT) v[j] *= wv[j];
        if (idx[j] >= 0) buf[lane + 64 * j] = v[j];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int b = 0; b < 64 / RPW; ++b) {
      const int row = b * RPW + lane / LPR;
      const int sub = lane % LPR;
      VT s = (VT)0;
      bool touch = false, big = false;
      uint32_t a = 0, z = 0;
      if (row < nr) {
        const uint32_t rl = t->rlo[row], rh = t->rhi[row];
        a = rl > cs ? rl : cs;
        z = rh < ce ? rh : ce;
        touch = a < z;
        // a row with many sources in this chunk is summed by the wavefront
        big = z > a + kBigPart * LPR;
        if (!big)
          for (uint32_t e = a + sub; e < z; e += LPR) s += buf[e - cs];
      }
      s = group_sum<LPR>(s);
      if (touch && !big && sub == 0) racc[row] += s;
      unsigned long long mb = __ballot(big && sub == 0);
      while (mb) {
        const int bl = __ffsll(mb) - 1;
        mb &= mb - 1;
        const uint32_t ba = __shfl(a, bl, 64), bz = __shfl(z, bl, 64);
        VT h = (VT)0;
        for (uint32_t e = ba + lane; e < bz; e += 64) h += buf[e - cs];
        h = wave_sum(h);
        if (lane == bl) racc[row] += h;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  return act ? racc[lane] : (VT)0;
}

// ------------------------------------------------------------------ items

// One-vertex components and CAC vertices (Sec. 4.3 first bullet, Sec. 4.3.1).
// R_v = W_v + (rank from higher levels) + sum over v's CAC in-edges u -> v of
// c R_u / outdeg(u).  The item's (up to 256) vertices are in topological order.
//  1. One thread per vertex: rank from higher levels (boundary rows, waited
//     for through the published x) plus W_v gives acc_v; v's CAC sources are
//     noted in edge order (up to four: an index in the item, or a vertex of
//     an earlier item).  A vertex with more CAC sources adds the ones of
//     earlier items here (waiting for them).
//  2. The plan covers the item by vertex-disjoint paths (k_item_paths).  One
//     lane walks each path in order with the x of the previous vertex in a
//     register: R_v = acc_v + the x of v's CAC sources in edge order, read
//     from LDS (sources in the item) or from the published x (earlier items)
//     once final (x still NaN means not yet; the lane then retries in the next
//     round).  A chain costs one multiply-add chain in one lane, and an item
//     starts walking while the items before it are still being walked.
// x_v = c R_v / outdeg(v) is published the moment R_v is final when a later
// item needs it (a CAC edge into a later item), else when the item ends.
// Every sum has a fixed order (the schedule depends only on the graph).
// With WT (a weighted graph) x_v = c R_v / s_v and every source's x is
// multiplied by its edge weight; the four listed sources keep their weights
// beside them in LDS.
constexpr int kWalkBatches = 2;
// Vertex items hold up to kVertMax positions, one per thread (kVertMaxW on
// a weighted plan).
constexpr int kVertMax = kThreads;
constexpr int kVertMaxW = kThreads;
// plan path order (vpath): local index in bits 0-9, bit 10 starts a path,
// bit 16 marks a vertex with a CAC edge into a later item
constexpr uint32_t kVIdx = 0x3ffu, kVStart = 0x400u, kVEarly = 0x10000u;
// byte offset of the listed sources' weights in a vertex item's LDS (after
// x, R, acc, c / outdeg, the source lists and the path tables)
constexpr size_t kVertWtOff =
    (4 * kThreads * sizeof(double) + kThreads * sizeof(uint4) + (3 * kThreads + 1 + kWaves) * sizeof(int32_t) + 31) &
    ~(size_t)31;
template <bool WT>
__device__ __attribute__((always_inline)) void run_verts(const SolveParams& p, int vbeg, int vend, WaveTile* tile,
                                                          double* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i = (int)threadIdx.x;
  const int v = vbeg + i;
  const int nvi = vend - vbeg;
  const bool act = v < vend;
  const int ra = vbeg + (int)(threadIdx.x & ~63u);
  const int nr = vend - ra < 64 ? vend - ra : 64;
  double* sX = lds;                 // by vertex: x when final, -1 before
  double* sR = lds + kThreads;      // by vertex: R
  double* sA = lds + 2 * kThreads;  // by path position: acc
  double* sC = lds + 3 * kThreads;  // by path position: c / outdeg
  uint4* sS = reinterpret_cast<uint4*>(lds + 4 * kThreads);  // by position: CAC sources (see kExt)
  uint32_t* sI = reinterpret_cast<uint32_t*>(sS + kThreads);  // by position: vertex | kind << 8 | count << 10
  int32_t* sQ = reinterpret_cast<int32_t*>(sI + kThreads);    // by vertex: path position | start << 16
  int32_t* sPB = sQ + kThreads;                               // path k: positions [sPB[k], sPB[k+1])
  int32_t* sWc = sPB + kThreads + 1;                          // path starts per wavefront
  // by position: the weights of the four listed sources (WT only)
  double* sWt = lds + kVertWtOff / sizeof(double);
  constexpr uint32_t kExt = 0x80000000u;  // source entry: vertex index of an earlier item (else local index)
  auto ld_lx = [&](int k) { return __hip_atomic_load(sX + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
  auto st_lx = [&](int k, double val) {
    __hip_atomic_store(sX + k, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  // path bounds: -1 until written after the barrier below; no barrier
  // follows those writes, so the walk reads its bounds with a wait on the mark
  auto ld_pb = [&](int k) { return __hip_atomic_load(sPB + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
  auto st_pb = [&](int k, int32_t val) {
    __hip_atomic_store(sPB + k, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  // path order: position i holds vertex pw & kVIdx; kVStart starts a path
  const uint32_t pw = act ? p.vpath[v] : 0u;
  const bool pstart = act && (pw & kVStart);
  const bool early = pw & kVEarly;  // v has a CAC edge into a later item
  if (act) sQ[pw & kVIdx] = i | (pstart ? 0x10000 : 0);
  sX[i] = kXPending;  // the LDS still holds the previous item's values
  sI[i] = 0u;    // bit 15 marks a position whose entries are written
  st_pb(i, -1);
  if (i == 0) st_pb(kThreads, -1);
  const unsigned long long sm = __ballot(pstart);
  if (lane == 0) sWc[wave] = (int32_t)__popcll(sm);
  __syncthreads();
  {
    int pid = (int)__popcll(sm & ((1ull << lane) - 1ull)), npath = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      if (w < wave) pid += sWc[w];
      npath += sWc[w];
    }
    if (pstart) st_pb(pid, i);
    if (i == 0) st_pb(npath, nvi);
  }
  // Everything that does not need other items' x is loaded before the
  // boundary gather waits for them: W, the CAC row and its source ids.
  // After the wait only the sums remain (one round trip for the x of
  // earlier items), so an item on the chain of dependencies starts its walk
  // soon after its last source is published.
  const int orig = act ? p.perm[v] : 0;
  const double wv = act ? p.W[orig] : 0.0;
  const double cinv = act ? p.c * p.inv64[v] : 0.0;
  const uint32_t lo = act ? p.int_ptr[v] : 0u;
  const uint32_t hi = act ? p.int_ptr[v + 1] : 0u;
  const bool lng = (hi - lo) > kLongLane;
  auto inside = [&](int u) { return u >= vbeg && u < vend; };
  auto wait_x = [&](int u) {
    double xv = ld_x(p.x, u);
    if (!x_ok(xv)) {
      const unsigned long long tw = wall_clock64();
      int nw = 1;
      unsigned polls = 0;
      while (!x_ok(xv = ld_x(p.x, u))) {
        if ((++polls & 15u) == 0u && timed_out(p, tw)) return 0.0;
        backoff_sleep(nw);
      }
    }
    return xv;
  };
  // edge weight of a CAC edge (one for a plain graph)
  auto ew = [&](uint32_t e) -> double {
    if constexpr (WT) return p.int_w64[e];
    else return 1.0;
  };
  // 1. note the CAC sources (four ids loaded at a time)
  uint32_t s0 = 0u, s1 = 0u, s2 = 0u, s3 = 0u, ns = 0u;
  double g0 = 1.0, g1 = 1.0, g2 = 1.0, g3 = 1.0;  // their weights (WT)
  if (act && !lng) {
    for (uint32_t e = lo; e < hi; e += 4) {
      int u[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = e + j < hi ? p.int_src[e + j] : -1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (u[j] >= 0) {
          const uint32_t w = inside(u[j]) ? (uint32_t)(u[j] - vbeg) : (kExt | (uint32_t)u[j]);
          const double g = (WT && ns < 4u) ? ew(e + j) : 1.0;
          if (ns == 0u) s0 = w, g0 = g;
          else if (ns == 1u) s1 = w, g1 = g;
          else if (ns == 2u) s2 = w, g2 = g;
          else if (ns == 3u) s3 = w, g3 = g;
          ++ns;
        }
      }
    }
  }
  // the rank from higher levels: W' = W + the boundary gather (eq. PR:levels)
  double acc = 0.0;
  if (nr > 0) acc = wave_tile_gather<64, double, true, WT>(p, p.bnd_ptr, p.bnd_src, p.x, ra, nr, tile, p.bnd_w);
  if (act) {
    acc += wv;
    p.wprime[v] = acc;
  }
  if (act && !lng) {
    if (ns <= 4u) {
      // sources of earlier items that are already published are added now
      // and dropped from the list.  The walk adds a vertex's sources of
      // earlier items before its sources in the item, each group in edge
      // order, so the sum is the same whether they are added here or there:
      // the result does not depend on timing.
      const uint32_t sl[4] = {s0, s1, s2, s3};
      const double gl[4] = {g0, g1, g2, g3};
      double xe[4];
      bool all = true;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bool ext = (uint32_t)m < ns && (sl[m] & kExt);
        xe[m] = ext ? ld_x(p.x, (int)(sl[m] & ~kExt)) : 0.0;
        all = all && (!ext || x_ok(xe[m]));
      }
      if (all) {
        uint32_t keep[4] = {0u, 0u, 0u, 0u};
        double gk[4] = {1.0, 1.0, 1.0, 1.0};
        uint32_t nk = 0u;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if ((uint32_t)m < ns && (sl[m] & kExt)) acc += WT ? xe[m] * gl[m] : xe[m];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if ((uint32_t)m < ns && !(sl[m] & kExt)) {
            if (nk == 0u) keep[0] = sl[m], gk[0] = gl[m];
            else if (nk == 1u) keep[1] = sl[m], gk[1] = gl[m];
            else if (nk == 2u) keep[2] = sl[m], gk[2] = gl[m];
            else keep[3] = sl[m], gk[3] = gl[m];
            ++nk;
          }
        }
        s0 = keep[0];
        s1 = keep[1];
        s2 = keep[2];
        s3 = keep[3];
        g0 = gk[0];
        g1 = gk[1];
        g2 = gk[2];
        g3 = gk[3];
        ns = nk;
      }
    }
    if (ns > 4u) {  // many sources: the ones of earlier items are added now, in edge order
      for (uint32_t e = lo; e < hi; e += 4) {
        int u[4];
        double xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          u[j] = e + j < hi ? p.int_src[e + j] : -1;
          xv[j] = (u[j] >= 0 && !inside(u[j])) ? ld_x(p.x, u[j]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (u[j] >= 0 && !inside(u[j])) {
            if (!x_ok(xv[j])) xv[j] = wait_x(u[j]);
            acc += WT ? xv[j] * ew(e + j) : xv[j];
          }
        }
      }
    }
  }
  // rows with many CAC sources: the wavefront waits for and sums the ones in
  // earlier items; the walk adds the ones in the item from the row itself
  unsigned long long lm = __ballot(act && lng);
  while (lm) {
    const int b = __ffsll(lm) - 1;
    lm &= lm - 1;
    const uint32_t blo = __shfl(lo, b, 64), bhi = __shfl(hi, b, 64);
    double part = 0.0;
    for (uint32_t e = blo + lane; e < bhi; e += 64) {
      const int u = p.int_src[e];
      if (!inside(u)) part += WT ? wait_x(u) * ew(e) : wait_x(u);
    }
    part = wave_sum(part);
    if (lane == b) acc += part;
  }
  if (act) {
    // hop kind: 0 no CAC source, 1 the path predecessor is the only one, 2 up
    // to four listed sources, 3 many (the walk reads the row)
    const int qw = sQ[i];
    const uint32_t kind =
        (lng || ns > 4u) ? 3u : ns == 0u ? 0u : (ns == 1u && !(s0 & kExt) && !(qw & 0x10000)) ? 1u : 2u;
    const int q = qw & 0xffff;
    sA[q] = acc;
    sC[q] = cinv;
    sS[q] = make_uint4(s0, s1, s2, s3);
    if constexpr (WT) {
      sWt[4 * q] = g0;
      sWt[4 * q + 1] = g1;
      sWt[4 * q + 2] = g2;
      sWt[4 * q + 3] = g3;
    }
    __hip_atomic_store(sI + q, (uint32_t)i | (kind << 8) | ((ns > 4u ? 7u : ns) << 10) | (early ? 0x2000u : 0u) | 0x8000u,
                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  if (p.trace && lane == 0) atomicMax(tile->rdy, wall_clock64());
  // 2. walk the paths; lanes retry in rounds until every path is done.  No
  // barrier: a lane walks as far as the positions whose entries are written
  // (sI bit 15), so a wavefront still waiting for rank from higher levels
  // holds back only the paths through its own vertices.
  int q = 0, qe = 0;
  {
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += sWc[w];
    if (i < tot) {
      // written by other wavefronts right after the barrier: almost never
      // still -1 here
      while ((q = ld_pb(i)) < 0) __builtin_amdgcn_s_sleep(1);
      while ((qe = ld_pb(i + 1)) < 0) __builtin_amdgcn_s_sleep(1);
    }
  }
  double xprev = 0.0;
  int prev = -1;
  unsigned rounds = 0;
  const unsigned long long t0 = wall_clock64();
  while (true) {
    const int qb = q;
    bool stop = q >= qe;
    // at most kWalkBatches batches per round: the lanes of a wavefront run in
    // lockstep, so a lane blocked on another path retries only when every
    // lane of its wavefront has ended the round
    int nb = 0;
    while (!stop && nb++ < kWalkBatches) {
      // the next eight positions in one LDS round trip; hops of kind 0 and 1
      // then run from registers
      double a8[8], c8[8], w8[8];
      uint32_t i8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int qq = q + j < qe ? q + j : qe - 1;
        i8[j] = __hip_atomic_load(sI + qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int qq = q + j < qe ? q + j : qe - 1;
        a8[j] = sA[qq];
        c8[j] = sC[qq];
        if constexpr (WT) w8[j] = sWt[4 * qq];  // kind 1: the weight of the one source
      }
      // eight written hops of kind 0 or 1 (kind bit 9 clear) inside the
      // path: a straight run with no per-hop branch on the kind
      const uint32_t all8 = ((i8[0] & i8[1]) & (i8[2] & i8[3])) & ((i8[4] & i8[5]) & (i8[6] & i8[7]));
      const uint32_t any8 = ((i8[0] | i8[1]) | (i8[2] | i8[3])) | ((i8[4] | i8[5]) | (i8[6] | i8[7]));
      if (q + 8 <= qe && (all8 & 0x8000u) && (any8 & 0x200u) == 0u) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int loc = (int)(i8[j] & 0xffu);
          const double r = (i8[j] & 0x100u) ? (WT ? a8[j] + w8[j] * xprev : a8[j] + xprev) : a8[j];
          const double xv = c8[j] * r;
          st_lx(loc, xv);
          sR[loc] = r;
          if (i8[j] & 0x2000u) st_x(p.x, vbeg + loc, xv);
          xprev = xv;
        }
        prev = (int)(i8[7] & 0xffu);
        q += 8;
        stop = q >= qe;
        continue;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (!stop) {
          const int loc = (int)(i8[j] & 0xffu);
          const uint32_t kind = (i8[j] >> 8) & 3u;
          double r = a8[j];
          bool ok = (i8[j] & 0x8000u) != 0u;
          if (!ok) {
          } else if (kind == 1u) {
            r += WT ? w8[j] * xprev : xprev;
          } else if (kind == 2u) {
            const uint32_t n = (i8[j] >> 10) & 7u;
            const uint4 s4 = sS[q];
            const uint32_t w4[4] = {s4.x, s4.y, s4.z, s4.w};
            double g4[4] = {1.0, 1.0, 1.0, 1.0};
            if constexpr (WT) {
#pragma unroll
              for (int m = 0; m < 4; ++m) g4[m] = sWt[4 * q + m];
            }
            double xs[4];
            double nl = 0.0;  // self-loops (a plan built with keep_loops), by weight
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const uint32_t w = w4[m];
              const bool self = (uint32_t)m < n && w == (uint32_t)loc;
              nl += self ? g4[m] : 0.0;
              xs[m] = ((uint32_t)m >= n || self) ? 0.0
                      : (w & kExt)              ? ld_x(p.x, (int)(w & ~kExt))
                      : (int)w == prev          ? xprev
                                                : ld_lx((int)w);
            }
            // sources of earlier items first, then the ones in the item
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              if ((uint32_t)m < n && (w4[m] & kExt)) {
                ok = ok && x_ok(xs[m]);
                r += WT ? xs[m] * g4[m] : xs[m];
              }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              if ((uint32_t)m < n && !(w4[m] & kExt)) {
                ok = ok && x_ok(xs[m]);
                r += WT ? xs[m] * g4[m] : xs[m];
              }
            }
            // the loop's share returns to the vertex: R = (W' + sources) / (1 - c a_vv)
            if (nl != 0.0) r /= 1.0 - nl * c8[j];
          } else if (kind == 3u) {
            const uint32_t l0 = p.int_ptr[vbeg + loc], l1 = p.int_ptr[vbeg + loc + 1];
            double nl = 0.0;
            for (uint32_t e = l0; e < l1 && ok; ++e) {
              const int u = p.int_src[e];
              if (!inside(u)) continue;
              if (u - vbeg == loc) {
                nl += ew(e);
                continue;
              }
              const double xv = u - vbeg == prev ? xprev : ld_lx(u - vbeg);
              if (!x_ok(xv)) ok = false;
              else r += WT ? xv * ew(e) : xv;
            }
            if (nl != 0.0) r /= 1.0 - nl * c8[j];
          }
          if (!ok) {
            stop = true;
          } else {
            const double xv = c8[j] * r;
            st_lx(loc, xv);
            sR[loc] = r;
            if (i8[j] & 0x2000u) st_x(p.x, vbeg + loc, xv);
            xprev = xv;
            prev = loc;
            ++q;
            if (q >= qe) stop = true;
          }
        }
      }
    }
    if (__all(q >= qe)) break;
    if (!__any(q != qb)) __builtin_amdgcn_s_sleep(1);
    // bounded: a malformed plan cannot hold the workgroup
    if ((++rounds & 255u) == 0u && timed_out(p, t0)) {
      for (; q < qe; ++q) {
        const int loc = (int)(sI[q] & 0xffu);
        sR[loc] = sA[q];
        st_lx(loc, 0.0);
        if (sI[q] & 0x2000u) st_x(p.x, vbeg + loc, 0.0);
      }
    }
  }
  // 3. publish the rest of the item's x in one coalesced store per
  // wavefront (single-lane stores, one per vertex of a path, would be issued
  // back to back to the same cache lines)
  __syncthreads();
  if (act) {
    if (!early) st_x(p.x, v, sX[i]);
    p.Rout[orig] = sR[i];
  }
}

__device__ inline bool stop_now(const SolveParams& p, double norm, double mx, double thresh) {
  return p.stop == PR_STOP_CERT_L1 ? (norm <= thresh) : (mx < p.tol);
}

// k: terms of the series; ws: -1 no starting guess, 0 guess rejected, 1
// kept (a guess costs two more passes over the component's edges)
__device__ inline void record_scc(const SolveParams& p, int rank, int64_t k, double last, bool conv, uint64_t ne,
                                  uint64_t nv, unsigned long long* wst, bool lds_stats, int ws = -1) {
  p.iters[rank] = (int32_t)k;
  p.lastnorm[rank] = last;
  const unsigned long long passes = (unsigned long long)k + (ws >= 0 ? 2ull : 0ull);
  if (lds_stats) {
    atomicAdd(&wst[S_EDGE_ITERS], passes * ne);
    atomicAdd(&wst[S_VERT_ITERS], passes * nv);
    atomicMax(&wst[S_ITERS_MAX], (unsigned long long)k);
    atomicAdd(&wst[S_ITERS_SUM], (unsigned long long)k);
    atomicAdd(&wst[S_N_ITERATED], 1ull);
    if (!conv) atomicAdd(&wst[S_NOT_CONV], 1ull);
    if (ws == 1) atomicAdd(&wst[S_WS_ACC], 1ull);
    if (ws == 0) atomicAdd(&wst[S_WS_REJ], 1ull);
  } else {
    wst[S_EDGE_ITERS] += passes * ne;
    wst[S_VERT_ITERS] += passes * nv;
    if ((unsigned long long)k > wst[S_ITERS_MAX]) wst[S_ITERS_MAX] = (unsigned long long)k;
    wst[S_ITERS_SUM] += (unsigned long long)k;
    wst[S_N_ITERATED] += 1ull;
    if (!conv) wst[S_NOT_CONV] += 1ull;
    if (ws == 1) wst[S_WS_ACC] += 1ull;
    if (ws == 0) wst[S_WS_REJ] += 1ull;
  }
}

// ---------------------------------------------------------- starting guess
// For the SCC on rows [vbeg, vbeg + nv), run by a group of G threads (one
// wavefront, G = 64, or the workgroup, G = kThreads) once its W' is final:
// the network's guess R_0 from the four features, the residual
// r_0 = W' + c A^T R_0 - R_0 in FP64 (into wr0 / wres), and the decision to
// keep it: ||r_0||_1 < ||c A^T W'||_1, the first term of the plain start.
// Every thread of the group returns the same decision, and with it
// ||r_0||_1 and max |r_0|.
struct WarmOut {
  bool keep;
  double n_r0, m_r0;
};

template <int G>
__device__ __attribute__((always_inline)) WarmOut warm_preamble(const SolveParams& p, int vbeg, int nv, double wsum, double* red) {
  const int tid = G == 64 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  auto gsum = [&](double v) { return G == 64 ? wave_sum(v) : block_sum(v, red); };
  auto gmax = [&](double v) { return G == 64 ? wave_max(v) : block_max(v, red); };
  auto gsync = [&]() {
    if constexpr (G == 64) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    else __syncthreads();
  };
  WarmOut o{false, 0.0, 0.0};
  gsync();  // every W' of the component is visible to the group
  const double s = wsum / (double)nv;
  if (!(s > 0.0)) return o;
  double np1 = 0.0;
  for (int base = 0; base < nv; base += G) {  // uniform trip count: the network needs whole wavefronts
    const int i = base + tid;
    const bool act = i < nv;
    const int v = vbeg + i;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
    double inv = 0.0;
    if (act) {
      const double wpv = p.wprime[v];
      inv = p.inv64[v];
      const uint32_t lo = p.int_ptr[v], hi = p.int_ptr[v + 1];
      double acc = 0.0;
      for (uint32_t e = lo; e < hi; ++e) {
        const int u = p.int_src[e];
        acc += p.wprime[u] * p.inv64[u];
      }
      const double p1 = p.c * acc;
      np1 += fabs(p1);
      const double indeg = (double)((p.bnd_ptr[v + 1] - p.bnd_ptr[v]) + (hi - lo));
      f0 = (float)log1p(indeg);
      f1 = (float)log1p(rint(1.0 / inv));
      f2 = (float)log1p((wpv - p.W[p.perm[v]]) / s);
      f3 = (float)log1p((wpv + p1) / s);
    }
    const float y = mlp_forward64(*p.mlp, f0, f1, f2, f3);
    if (act) {
      const double r0 = s * exp((double)y);
      p.wr0[v] = r0;
      p.wx[v] = p.c * r0 * inv;
    }
  }
  np1 = gsum(np1);
  gsync();
  double nr0 = 0.0, mr0 = 0.0;
  for (int i = tid; i < nv; i += G) {
    const int v = vbeg + i;
    double acc = 0.0;
    for (uint32_t e = p.int_ptr[v]; e < p.int_ptr[v + 1]; ++e) acc += p.wx[p.int_src[e]];
    const double r = p.wprime[v] + acc - p.wr0[v];
    p.wres[v] = r;
    nr0 += fabs(r);
    mr0 = fmax(mr0, fabs(r));
  }
  nr0 = gsum(nr0);
  mr0 = gmax(mr0);
  gsync();
  o.keep = nr0 < np1;  // false for a non-finite guess
  o.n_r0 = nr0;
  o.m_r0 = mr0;
  return o;
}

// the inside-component edge weights in the type of the series terms
template <typename YT>
__device__ inline const YT* term_w(const SolveParams& p) {
  if constexpr (sizeof(YT) == 8) return reinterpret_cast<const YT*>(p.int_w64);
  else return reinterpret_cast<const YT*>(p.int_w32);
}

// the slots' edge weights (eight per slot) in the type of the series terms
template <typename YT>
__device__ inline const YT* slot_w(const SolveParams& p) {
  if constexpr (sizeof(YT) == 8) return reinterpret_cast<const YT*>(p.mslot_w64);
  else return reinterpret_cast<const YT*>(p.mslot_w32);
}

// An SCC with at most 256 vertices, iterated by one wavefront.  After the
// weights are gathered, the component's internal rows are copied into LDS
// (one-byte local source ids, two-byte row offsets) when they fit, so every
// term touches only LDS and registers (R stays in registers, four rows per
// lane).  A weighted graph (WT) keeps a lane's first sixteen edge weights in
// registers on the one-row-per-lane path and reads the others from the plan.
template <typename YT, bool WARM, bool TAIL = false, bool WT = false>
__device__ __attribute__((always_inline)) void run_small(const SolveParams& p, int rank, YT* ybuf, unsigned long long* wst, WaveTile* tile) {
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
    double wp = 0.0;
    const int nr = nv - 64 * j < 64 ? nv - 64 * j : 64;
    if (nr > 0)
      wp = wave_tile_gather<64, double, true, WT>(p, p.bnd_ptr, p.bnd_src, p.x, vbeg + 64 * j, nr, tile, p.bnd_w);
    if (act) wp += p.W[p.perm[v]];
    Rj[j] = wp;
    inv[j] = act ? p.inv32[v] : 0.0f;
    if (act) {
      if constexpr (sizeof(YT) == 8) ya[i] = (YT)(p.c * wp * p.inv64[v]);
      else ya[i] = (YT)(p.c * wp * (double)inv[j]);
      p.wprime[v] = wp;
      part += fabs(wp);
    }
  }
  // stage the internal rows in LDS (the tile is free after the gathers)
  const uint32_t eb = p.int_ptr[vbeg];
  const uint32_t ne = p.int_ptr[vbeg + nv] - eb;
  const bool staged = ne <= (uint32_t)sizeof(tile->buf);
  const YT* ewt = nullptr;  // weights by staged edge index (WT)
  if constexpr (WT) ewt = term_w<YT>(p) + eb;
  uint8_t* lsrc = reinterpret_cast<uint8_t*>(tile->buf);
  uint16_t* lptr = reinterpret_cast<uint16_t*>(tile->racc);  // racc + rlo + rhi: 1 KB >= 2 * 257
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (staged) {
    for (uint32_t q = lane; q < ne; q += 64) lsrc[q] = (uint8_t)(p.int_src[eb + q] - vbeg);
    for (int q = lane; q <= nv; q += 64) lptr[q] = (uint16_t)(p.int_ptr[vbeg + q] - eb);
  }
  uint32_t rlo[4], rhi[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = lane + 64 * j;
    rlo[j] = i < nv ? p.int_ptr[vbeg + i] : 0u;
    rhi[j] = i < nv ? p.int_ptr[vbeg + i + 1] : 0u;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const double wsum = wave_sum(part);
  const double thresh = p.eps * (1.0 - p.c) * wsum;
  const YT cy = (YT)p.c;
  int64_t k = 0;
  double last = wsum;
  bool conv = true;
  bool skip = p.stop == PR_STOP_CERT_L1 && wsum == 0.0;
  int ws = -1;
  if (nv <= p.direct_max && nv <= kDirectMax && !skip) {
    // Direct solve (Sec. 4.3, small SCCs): Gauss-Jordan elimination of
    // [I - c A_CC^T | W'] in LDS, in FP64, without pivoting; every column of
    // I - c A_CC^T has diagonal 1 and off-diagonal sum at most c < 1, so the
    // pivots stay at least 1 - c.  The matrix takes the tile (its staged
    // rows are not needed on this path).
    double* M = reinterpret_cast<double*>(tile->buf);
    const int ld = nv + 1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int q = lane; q < nv * ld; q += 64) M[q] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const double wp = Rj[0];
    if (lane < nv) {
      M[lane * ld + lane] = 1.0;
      M[lane * ld + nv] = wp;
      for (uint32_t e = rlo[0]; e < rhi[0]; ++e) {
        const int u = p.int_src[e] - vbeg;
        if constexpr (WT) M[lane * ld + u] -= p.c * p.inv64[vbeg + u] * p.int_w64[e];
        else M[lane * ld + u] -= p.c * p.inv64[vbeg + u];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int kk = 0; kk < nv; ++kk) {
      const double inv_piv = 1.0 / M[kk * ld + kk];
      const int cols = nv - kk;  // columns kk+1 .. nv
      for (int q = lane; q < nv * cols; q += 64) {
        const int i = q / cols, j = kk + 1 + q % cols;
        if (i != kk) M[i * ld + j] -= (M[i * ld + kk] * inv_piv) * M[kk * ld + j];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    const double xr = lane < nv ? M[lane * ld + nv] / M[lane * ld + lane] : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < nv) M[lane * ld + nv] = xr;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // residual W' - (I - c A_CC^T) R in FP64: ||R - R*||_1 <= ||r||_1 / (1 - c)
    double rr = 0.0;
    if (lane < nv) {
      double acc = wp - xr;
      for (uint32_t e = rlo[0]; e < rhi[0]; ++e) {
        const int u = p.int_src[e] - vbeg;
        if constexpr (WT) acc += p.c * p.inv64[vbeg + u] * p.int_w64[e] * M[u * ld + nv];
        else acc += p.c * p.inv64[vbeg + u] * M[u * ld + nv];
      }
      rr = fabs(acc);
    }
    rr = wave_sum(rr);
    Rj[0] = xr;
    last = rr / p.c;  // the certificate adds c / (1 - c) * last
    skip = true;
  }
  double P0 = Rj[0];  // the lane's first term: W' (P_0), or r_0 after a kept guess
  if (WARM && !skip) {  // (the direct solve above has set skip)
    const WarmOut w = warm_preamble<64>(p, vbeg, nv, wsum, nullptr);
    ws = w.keep ? 1 : 0;
    if (w.keep) {  // start from R_0 + r_0 with the term r_0
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = lane + 64 * j;
        if (i < nv) {
          const int v = vbeg + i;
          const double r = p.wres[v];
          Rj[j] = p.wr0[v] + r;
          if (j == 0) P0 = r;
          if constexpr (sizeof(YT) == 8) ya[i] = (YT)(p.c * r * p.inv64[v]);
          else ya[i] = (YT)(p.c * r * (double)inv[j]);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      last = w.n_r0;
      if (stop_now(p, w.n_r0, w.m_r0, thresh)) skip = true;  // the guess already meets the rule
    }
  }
  if (staged && nv <= 64 && !skip) {
    // one row per lane; its first 16 sources packed in registers (entry 255
    // of the term buffers is a zero pad for lanes with fewer sources)
    conv = false;
    const bool act = lane < nv;
    const uint32_t lo = act ? lptr[lane] : 0u, hi = act ? lptr[lane + 1] : 0u;
    const uint32_t deg = hi - lo;
    uint32_t pk[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if ((uint32_t)q < deg) {
        const uint32_t sh = 8u * (q & 3);
        pk[q >> 2] = (pk[q >> 2] & ~(0xffu << sh)) | ((uint32_t)lsrc[lo + q] << sh);
      }
    }
    YT wr[16];  // the packed sources' edge weights (WT)
    if constexpr (WT) {
#pragma unroll
      for (int q = 0; q < 16; ++q) wr[q] = (uint32_t)q < deg ? ewt[lo + q] : (YT)0;
    }
    const int nq = (int)wave_max((double)(deg < 16u ? deg : 16u));  // wave-uniform
    const bool extra = wave_max((double)deg) > 16.0;
    if (lane == 0) {
      ya[kSmallMax - 1] = (YT)0;
      yb[kSmallMax - 1] = (YT)0;
    }
    const double inv64 = act ? p.inv64[vbeg + lane] : 0.0;
    const bool cert = p.stop == PR_STOP_CERT_L1;
    double R0 = Rj[0];
    // certified tail estimate: the previous term (r_0 after a kept guess) and the
    // norms of the last two terms
    const bool tail = TAIL && p.tail && cert;
    double svp = P0, nprev = last, nprev2 = -1.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    while (k < p.max_iter) {
      ++k;
      // the tail estimate's ratio is known before the term (its division
      // overlaps the gathers)
      const double rho = (tail && nprev2 > 0.0) ? nprev / nprev2 : -1.0;
      const bool rho_ok = rho > 0.0 && rho < 1.0;
      // all gathers issued before any is used (one LDS wait); unused slots
      // read the zero pad
      YT g[16];
      if (nq <= 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) g[q] = ya[(pk[q >> 2] >> (8u * (q & 3))) & 0xffu];
#pragma unroll
        for (int q = 8; q < 16; ++q) g[q] = (YT)0;
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) g[q] = ya[(pk[q >> 2] >> (8u * (q & 3))) & 0xffu];
      }
      if constexpr (WT) {
#pragma unroll
        for (int q = 0; q < 16; ++q) g[q] *= wr[q];
      }
      YT sv = (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) +
              (((g[8] + g[9]) + (g[10] + g[11])) + ((g[12] + g[13]) + (g[14] + g[15])));
      if (extra) {
        for (uint32_t e = lo + 16; e < hi; e += 8) {
          uint32_t ix[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) ix[j] = e + j < hi ? lsrc[e + j] : (uint32_t)(kSmallMax - 1);
          YT h[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) h[j] = ya[ix[j]];
          if constexpr (WT) {
#pragma unroll
            for (int j = 0; j < 8; ++j) h[j] *= e + j < hi ? ewt[e + j] : (YT)0;
          }
          sv += ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));
        }
      }
      if (act) {
        R0 += (double)sv;
        if constexpr (sizeof(YT) == 8) yb[lane] = cy * sv * inv64;
        else yb[lane] = cy * sv * inv[0];
      }
      const double sd = act ? fabs((double)sv) : 0.0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      YT* t = ya;
      ya = yb;
      yb = t;
      if (cert) {
        double norm, dsum = 0.0;  // both sums in one pass
        if (rho_ok) wave_sum2(sd, act ? fabs((double)sv - rho * svp) : 0.0, norm, dsum);
        else norm = wave_sum(sd);
        last = norm;
        if (norm <= thresh) {
          conv = true;
          break;
        }
        if (rho_ok && dsum <= thresh * (1.0 - rho)) {  // R' = R - P_k + rho/(1-rho) P_{k-1}
          R0 += rho / (1.0 - rho) * svp - (double)sv;
          last = dsum / (1.0 - rho) / p.c;
          conv = true;
          break;
        }
        if (tail) {
          nprev2 = nprev;
          nprev = norm;
          svp = (double)sv;
        }
      } else {
        const double mx = wave_max(sd);
        last = wave_sum(sd);
        if (mx < p.tol) {
          conv = true;
          break;
        }
      }
    }
    Rj[0] = R0;
  } else if (!skip) {
    conv = false;
    // tail estimate: a row's terms are read back from the term buffers
    const bool tail = TAIL && p.tail;
    double nprev = last, nprev2 = -1.0;
    auto scale = [&](int j, int i) -> double {  // the factor between P and the term buffer
      if constexpr (sizeof(YT) == 8) return (double)cy * p.inv64[vbeg + i];
      else return (double)cy * (double)inv[j];
    };
    while (k < p.max_iter) {
      ++k;
      part = 0.0;
      double pm = 0.0, dd = 0.0;
      const double rho = (tail && nprev2 > 0.0) ? nprev / nprev2 : -1.0;
      const bool rho_ok = rho > 0.0 && rho < 1.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = lane + 64 * j;
        if (i < nv) {
          YT s0 = 0, s1 = 0;
          if (staged) {
            const uint32_t lo = lptr[i], hi = lptr[i + 1];
            for (uint32_t e = lo; e < hi; e += 8) {
              YT h[8];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                if constexpr (WT) h[j] = e + j < hi ? ya[lsrc[e + j]] * ewt[e + j] : (YT)0;
                else h[j] = e + j < hi ? ya[lsrc[e + j]] : (YT)0;
              }
              s0 += (h[0] + h[1]) + (h[2] + h[3]);
              s1 += (h[4] + h[5]) + (h[6] + h[7]);
            }
          } else if constexpr (WT) {
            const YT* wt = term_w<YT>(p);
            uint32_t e = rlo[j];
            for (; e + 1 < rhi[j]; e += 2) {
              s0 += ya[p.int_src[e] - vbeg] * wt[e];
              s1 += ya[p.int_src[e + 1] - vbeg] * wt[e + 1];
            }
            if (e < rhi[j]) s0 += ya[p.int_src[e] - vbeg] * wt[e];
          } else {
            uint32_t e = rlo[j];
            for (; e + 1 < rhi[j]; e += 2) {
              s0 += ya[p.int_src[e] - vbeg];
              s1 += ya[p.int_src[e + 1] - vbeg];
            }
            if (e < rhi[j]) s0 += ya[p.int_src[e] - vbeg];
          }
          const YT s = s0 + s1;
          Rj[j] += (double)s;
          if (rho_ok) dd += fabs((double)s - rho * (double)ya[i] / scale(j, i));
          if constexpr (sizeof(YT) == 8) yb[i] = cy * s * p.inv64[vbeg + i];
          else yb[i] = cy * s * inv[j];
          part += fabs((double)s);
          pm = fmax(pm, fabs((double)s));
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      double norm, dsum = 0.0;
      if (rho_ok) wave_sum2(part, dd, norm, dsum);
      else norm = wave_sum(part);
      const double mx = wave_max(pm);
      last = norm;
      YT* t = ya;
      ya = yb;
      yb = t;
      if (stop_now(p, norm, mx, thresh)) {
        conv = true;
        break;
      }
      if (rho_ok && dsum <= thresh * (1.0 - rho)) {
        // R' = R - P_k + rho/(1-rho) P_{k-1}; ya: P_k, yb: P_{k-1}
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = lane + 64 * j;
          if (i < nv) Rj[j] += (rho / (1.0 - rho) * (double)yb[i] - (double)ya[i]) / scale(j, i);
        }
        last = dsum / (1.0 - rho) / p.c;
        conv = true;
        break;
      }
      nprev2 = nprev;
      nprev = norm;
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
  if (lane == 0) record_scc(p, rank, k, last, conv, ne, (uint64_t)nv, wst, true, ws);
}

// The direct solve of an SCC run by one workgroup (Sec. 4.3, small SCCs):
// Gauss-Jordan elimination of [I - c A_CC^T | W'] in FP64 without pivoting
// (every column of I - c A_CC^T has diagonal 1 and off-diagonal sum at most
// c < 1, so the pivots stay at least 1 - c), the matrix in the segment LDS.
// One row per thread builds it, a 16 x 16 grid of threads updates it, one
// barrier per step.  The arithmetic and its order are those of the
// wavefront's direct solve, so an SCC gets the same R on either path.  Kept
// apart from run_medium so that its registers do not add to the iteration's.
template <bool WT>
__device__ __attribute__((always_inline)) void run_direct_wg(const SolveParams& p, int rank, double* red, unsigned long long* wst,
                                                             WaveTile* tiles, unsigned char* raw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  const int vb = p.comp_vbeg[rank], ve = p.comp_vbeg[rank + 1];
  const int nv = ve - vb;
  const double c = p.c;
  // W' = W + the boundary mass (eq. PR:levels), 64 rows per wavefront
  for (int ra = vb + 64 * wave; ra < ve; ra += 64 * kWaves) {
    const int nr = ve - ra < 64 ? ve - ra : 64;
    double wp = wave_tile_gather<64, double, true, WT>(p, p.bnd_ptr, p.bnd_src, p.x, ra, nr, tiles + wave, p.bnd_w);
    if (lane < nr) p.wprime[ra + lane] = wp + p.W[p.perm[ra + lane]];
  }
  __syncthreads();  // the gathers are done with the tiles; W' is visible
  double* M = reinterpret_cast<double*>(raw);
  const int ld = nv + 1;
  for (int q = tid; q < nv * ld; q += kThreads) M[q] = 0.0;
  __syncthreads();
  const bool own = tid < nv;  // nv <= kDirectMaxWG < kThreads: one row per thread
  double wpv = 0.0;
  if (own) {
    const int v = vb + tid;
    double* row = M + (size_t)tid * ld;
    wpv = p.wprime[v];
    row[tid] = 1.0;
    row[nv] = wpv;
    for (uint32_t e = p.int_ptr[v]; e < p.int_ptr[v + 1]; ++e) {
      const int u = p.int_src[e] - vb;
      if constexpr (WT) row[u] -= c * p.inv64[vb + u] * p.int_w64[e];
      else row[u] -= c * p.inv64[vb + u];
    }
  }
  __syncthreads();
  const int ty = tid >> 4, tx = tid & 15;
  for (int kk = 0; kk < nv; ++kk) {
    const double inv_piv = 1.0 / M[kk * ld + kk];
    for (int i = ty; i < nv; i += 16) {
      if (i == kk) continue;
      const double f = M[i * ld + kk] * inv_piv;
      for (int j = kk + 1 + tx; j <= nv; j += 16) M[i * ld + j] -= f * M[kk * ld + j];
    }
    __syncthreads();
  }
  const double xr = own ? M[tid * ld + nv] / M[tid * ld + tid] : 0.0;
  __syncthreads();
  if (own) M[tid * ld + nv] = xr;
  __syncthreads();
  // residual W' - (I - c A_CC^T) R in FP64: ||R - R*||_1 <= ||r||_1 / (1 - c)
  double rr = 0.0;
  if (own) {
    const int v = vb + tid;
    double acc = wpv - xr;
    for (uint32_t e = p.int_ptr[v]; e < p.int_ptr[v + 1]; ++e) {
      const int u = p.int_src[e] - vb;
      if constexpr (WT) acc += c * p.inv64[vb + u] * p.int_w64[e] * M[u * ld + nv];
      else acc += c * p.inv64[vb + u] * M[u * ld + nv];
    }
    rr = fabs(acc);
    p.R[v] = xr;
    p.Rout[p.perm[v]] = xr;
    st_x(p.x, v, c * xr * p.inv64[v]);
  }
  rr = block_sum(rr, red);
  if (tid == 0) {
    const uint32_t ne = p.int_ptr[ve] - p.int_ptr[vb];
    record_scc(p, rank, 0, rr / c, true, ne, (uint64_t)nv, wst, false);  // the certificate adds rr / (1 - c)
  }
}

// One SCC iterated by one workgroup.  When the component fits, its rows
// (two-byte local sources), 1/outdeg, R and both term vectors live in LDS
// during the iteration; otherwise the vectors stay in global memory, touched
// only by this workgroup.  A weighted graph (WT) multiplies every slot entry
// by its edge weight: from LDS on the register path (the weights staged
// beside the slot sums), from the plan on the large-component path.
template <typename YT, int RPW, bool WARM, bool TAIL = false, bool WT = false, bool GS = false>
__device__ __attribute__((always_inline)) void run_medium(const SolveParams& p, int rank, double* red, unsigned long long* wst, WaveTile* tiles,
                           unsigned char* raw, size_t raw_bytes) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  WaveTile* tile = tiles + wave;
  const uint32_t* ptr = p.int_ptr;
  const int32_t* src = p.int_src;
  const int vb = p.comp_vbeg[rank], ve = p.comp_vbeg[rank + 1];
  const int nv = ve - vb;
  const uint32_t eb = ptr[vb];
  const uint32_t ne = ptr[ve] - eb;
  const int64_t total = (int64_t)ne + nv;
  auto find_row = [&](int64_t target) {
    int lo = vb, hi = ve;
    while (lo < hi) {
      int mid = lo + (hi - lo) / 2;
      if ((int64_t)(ptr[mid] - eb) + (mid - vb) < target) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  const int w0 = wave == 0 ? vb : find_row(total * wave / kWaves);
  const int w1 = wave == kWaves - 1 ? ve : find_row(total * (wave + 1) / kWaves);
  YT* ya = (YT*)p.y0;
  YT* yb = (YT*)p.y1;
  const double c = p.c;
  double part = 0.0;
  for (int ra = w0; ra < w1; ra += 64) {
    const int nr = w1 - ra < 64 ? w1 - ra : 64;
    double wp = wave_tile_gather<64, double, true, WT>(p, p.bnd_ptr, p.bnd_src, p.x, ra, nr, tile, p.bnd_w);
    if (lane < nr) {
      const int v = ra + lane;
      wp += p.W[p.perm[v]];
      p.R[v] = wp;
      p.wprime[v] = wp;
      if constexpr (sizeof(YT) == 8) ya[v] = c * wp * p.inv64[v];
      else ya[v] = (YT)(c * wp * (double)p.inv32[v]);
      part += fabs(wp);
    }
  }
  const double wsum = block_sum(part, red);  // also orders the phase-0 writes
  const double thresh = p.eps * (1.0 - c) * wsum;
  const YT cy = (YT)c;
  int64_t k = 0;
  double last = wsum;
  bool conv = true;
  bool skip = p.stop == PR_STOP_CERT_L1 && wsum == 0.0;
  int ws = -1;
  if (WARM && !skip) {
    const WarmOut w = warm_preamble<kThreads>(p, vb, nv, wsum, red);
    ws = w.keep ? 1 : 0;
    if (w.keep) {  // start from R_0 + r_0 with the term r_0
      for (int i = threadIdx.x; i < nv; i += kThreads) {
        const int v = vb + i;
        const double r = p.wres[v];
        p.R[v] = p.wr0[v] + r;
        if constexpr (sizeof(YT) == 8) ya[v] = c * r * p.inv64[v];
        else ya[v] = (YT)(c * r * (double)p.inv32[v]);
      }
      __syncthreads();
      last = w.n_r0;
      if (stop_now(p, w.n_r0, w.m_r0, thresh)) skip = true;  // the guess already meets the rule
    }
  }
  const unsigned long long t_it = wall_clock64();
  // Register-resident iteration when the component is small enough.  The
  // in-edges of each row are cut into slots of at most kSlot; slot s belongs
  // to thread s % 256 and row r to thread r % 256.  Each thread keeps its
  // slots' source ids, and its rows' R, 1/outdeg and slot ranges, in
  // registers; only the terms (y0, y1: nv values and a zero pad each) and the
  // slot sums live in LDS.  A term is (A) every thread sums its slots,
  // (B) every row adds its slot sums in slot order (a row with more than
  // kSlot slots: the whole wavefront), so the work of a term is spread evenly
  // over the workgroup whatever the in-degrees.
  constexpr uint32_t kSlot = 8;  // the plan's slot width (k_medium_slots)
  constexpr int kSPT = 4;         // slots per thread
  constexpr int kRPT = 4;         // rows per thread
  const uint32_t sb = p.mslot_ptr[vb];
  const uint32_t nslot = p.mslot_ptr[ve] - sb;
  const size_t need = (2 * ((size_t)nv + 1) + nslot) * sizeof(YT) + 64;
  const size_t need_w = WT ? 16 + (size_t)kSlot * nslot * sizeof(YT) : 0;  // the slots' weights (WT)
  // the Gauss-Seidel blocks' first slots follow the slot sums (GS)
  const size_t need_gs = GS ? sizeof(uint32_t) * (kGsMaxBlocks + 1) + 16 : 0;
  const bool staged =
      need + need_w + need_gs <= raw_bytes && nv <= kThreads * kRPT && nslot <= (uint32_t)(kThreads * kSPT);
  // (the plan cuts slots only for components of at most 65535 vertices: the
  // ids are 16-bit and the component size is the zero pad)
  // larger components: the same two phases with the slots read from the plan
  // every term (L2-resident) and R, 1/outdeg and the row slot ranges in LDS
  const size_t need_big = (3 * (size_t)nv + 2 + nslot) * sizeof(YT) + 8 * (size_t)nv + 4 * ((size_t)nv + 1) + 64;
  const bool staged_big = !staged && need_big <= raw_bytes && nv <= 65535;
  if (staged_big) {
    double* lR = reinterpret_cast<double*>(raw);
    YT* l0 = reinterpret_cast<YT*>(lR + nv);
    YT* l1 = l0 + nv + 1;
    YT* linv = l1 + nv + 1;
    YT* lpart = linv + nv;
    uint32_t* lfs = reinterpret_cast<uint32_t*>(lpart + nslot);
    for (int q = threadIdx.x; q < nv; q += kThreads) {
      lR[q] = p.R[vb + q];
      l0[q] = ya[vb + q];
      if constexpr (sizeof(YT) == 8) linv[q] = p.inv64[vb + q];
      else linv[q] = p.inv32[vb + q];
    }
    for (int q = threadIdx.x; q <= nv; q += kThreads) lfs[q] = p.mslot_ptr[vb + q] - sb;
    if (threadIdx.x == 0) {
      l0[nv] = (YT)0;
      l1[nv] = (YT)0;
    }
    __syncthreads();
    const uint4* gs = p.mslot_src + sb;
    const YT* gw = nullptr;  // the slots' weights (WT)
    if constexpr (WT) gw = slot_w<YT>(p) + (size_t)kSlot * sb;
    YT* la = l0;
    YT* lb = l1;
    // certified tail estimate as in the register path below
    const bool tail = TAIL && p.tail;
    double nprev = last, nprev2 = -1.0;
    if (!skip) {
      conv = false;
      while (k < p.max_iter) {
        ++k;
        const double rho = (tail && nprev2 > 0.0) ? nprev / nprev2 : -1.0;
        const bool rho_ok = rho > 0.0 && rho < 1.0;
        // (A) slot sums, four slots' ids in flight per thread
        for (uint32_t base = threadIdx.x; base < nslot; base += 4 * kThreads) {
          uint4 w[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t sl = base + kThreads * j;
            w[j] = sl < nslot ? gs[sl] : make_uint4(0u, 0u, 0u, 0u);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t sl = base + kThreads * j;
            if (sl < nslot) {
              const uint32_t wv[4] = {w[j].x, w[j].y, w[j].z, w[j].w};
              YT g[kSlot];
#pragma unroll
              for (uint32_t m = 0; m < kSlot; ++m) g[m] = la[(wv[m / 2] >> (16 * (m & 1))) & 0xffffu];
              if constexpr (WT) {
#pragma unroll
                for (uint32_t m = 0; m < kSlot; ++m) g[m] *= gw[kSlot * (size_t)sl + m];
              }
              lpart[sl] = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]));
            }
          }
        }
        __syncthreads();
        // (B) row sums
        double part = 0.0, pm = 0.0, dpart = 0.0;
        for (int rb = wave * 64; rb < nv; rb += kThreads) {
          const int r = rb + lane;
          const uint32_t f0 = r < nv ? lfs[r] : 0u, f1 = r < nv ? lfs[r + 1] : 0u;
          const bool wide = f1 - f0 > kSlot;
          YT sv = 0;
          if (r < nv && !wide) {
            YT h[kSlot];
#pragma unroll
            for (uint32_t m = 0; m < kSlot; ++m) h[m] = f0 + m < f1 ? lpart[f0 + m] : (YT)0;
            sv = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));
          }
          unsigned long long m = __ballot(r < nv && wide);
          while (m) {
            const int bl = __ffsll(m) - 1;
            m &= m - 1;
            const uint32_t blo = __shfl(f0, bl, 64), bhi = __shfl(f1, bl, 64);
            YT ws = 0;
            for (uint32_t e = blo + lane; e < bhi; e += 256) {
              YT g[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) g[q] = e + 64 * q < bhi ? lpart[e + 64 * q] : (YT)0;
              ws += (g[0] + g[1]) + (g[2] + g[3]);
            }
            ws = wave_sum(ws);
            if (lane == bl) sv = ws;
          }
          if (r < nv) {
            lR[r] += (double)sv;
            lb[r] = cy * sv * linv[r];
            part += fabs((double)sv);
            pm = fmax(pm, fabs((double)sv));
            if (rho_ok) dpart += fabs((double)sv - rho * (double)la[r] / ((double)cy * (double)linv[r]));
          }
        }
        double norm, mx, dsum = 0.0;
        // the barrier also publishes lb
        if (tail) block_sum2_max(part, dpart, pm, red, (int)(k & 1), &norm, &dsum, &mx);
        else block_sum_max(part, pm, red, (int)(k & 1), &norm, &mx);
        last = norm;
        YT* tt = la;
        la = lb;
        lb = tt;
        if (stop_now(p, norm, mx, thresh)) {
          conv = true;
          break;
        }
        if (rho_ok && dsum <= thresh * (1.0 - rho)) {  // lb: P_{k-1}, la: P_k; a thread's rows only
          for (int r = threadIdx.x; r < nv; r += kThreads) {
            const double sc = (double)cy * (double)linv[r];
            lR[r] += rho / (1.0 - rho) * ((double)lb[r] / sc) - (double)la[r] / sc;
          }
          last = dsum / (1.0 - rho) / p.c;
          conv = true;
          break;
        }
        nprev2 = nprev;
        nprev = norm;
      }
    }
    for (int q = threadIdx.x; q < nv; q += kThreads) {
      const double r = lR[q];
      p.Rout[p.perm[vb + q]] = r;
      st_x(p.x, vb + q, c * r * p.inv64[vb + q]);
    }
  } else if (staged) {
    YT* l0 = reinterpret_cast<YT*>(raw);
    YT* l1 = l0 + nv + 1;
    YT* lpart = l1 + nv + 1;
    // the slots' weights (WT), 16-byte aligned after the slot sums
    YT* lw = reinterpret_cast<YT*>(raw + ((reinterpret_cast<unsigned char*>(lpart + nslot) - raw + 15) & ~(size_t)15));
    if constexpr (WT) {
      const YT* gw = slot_w<YT>(p) + (size_t)kSlot * sb;
      for (uint32_t q = threadIdx.x; q < kSlot * nslot; q += kThreads) lw[q] = gw[q];
    }
    for (int q = threadIdx.x; q < nv; q += kThreads) l0[q] = ya[vb + q];
    if (threadIdx.x == 0) {
      l0[nv] = (YT)0;
      l1[nv] = (YT)0;
    }
    // this thread's slots (source ids, two per register; nv is the zero pad)
    // and rows
    uint32_t sid[kSPT][kSlot / 2];
#pragma unroll
    for (int j = 0; j < kSPT; ++j) {
      const uint32_t sl = threadIdx.x + kThreads * j;
      const uint4 w = sl < nslot ? p.mslot_src[sb + sl] : make_uint4(0u, 0u, 0u, 0u);
      sid[j][0] = w.x;
      sid[j][1] = w.y;
      sid[j][2] = w.z;
      sid[j][3] = w.w;
    }
    double Rr[kRPT];
    YT ir[kRPT];
    uint32_t fr[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int r = threadIdx.x + kThreads * j;
      Rr[j] = r < nv ? p.R[vb + r] : 0.0;
      if constexpr (sizeof(YT) == 8) ir[j] = r < nv ? p.inv64[vb + r] : 0.0;
      else ir[j] = r < nv ? p.inv32[vb + r] : 0.0f;
      fr[j] = r < nv ? ((p.mslot_ptr[vb + r] - sb) | ((p.mslot_ptr[vb + r + 1] - sb) << 16)) : 0u;
    }
    __syncthreads();
    YT* la = l0;
    YT* lb = l1;
    // certified tail estimate (from r_0 after a kept guess): the norms of the last two
    // terms; a row's terms are read back from the term buffers, which hold
    // c P_k / outdeg (a relative difference of one FP32 rounding)
    const bool tail = TAIL && p.tail;
    double nprev = last, nprev2 = -1.0;
    if constexpr (GS) {
      // Block Gauss-Seidel sweeps (the alternative to the series that Sec.
      // 4.3.2 names): the component's rows, in plan order, cut into
      // gs_blocks consecutive blocks; la holds c R / outdeg of the newest R
      // (R starts at W').  A block's rows take W' plus their slot sums,
      // formed from la once the earlier blocks of the sweep have written
      // theirs.  The component stops after the first sweep with
      // ||R_new - R_old||_1 <= eps (1 - c) ||W'||_1 (the paper's rule: max
      // |R_new - R_old| < tol); then ||R - R*||_1 <= c ||dR||_1 / (1 - c),
      // the bound the certificate adds for it.
      uint32_t* lqb = reinterpret_cast<uint32_t*>(lpart + nslot);  // the blocks' first slots
      const int B = p.gs_blocks < nv ? p.gs_blocks : nv;
      for (int b = threadIdx.x; b <= B; b += kThreads)
        lqb[b] = p.mslot_ptr[vb + (int)(((int64_t)nv * b) / B)] - sb;
      double wr[kRPT];  // W' of this thread's rows
#pragma unroll
      for (int j = 0; j < kRPT; ++j) wr[j] = Rr[j];
      __syncthreads();
      if (!skip) {
        conv = false;
        while (k < p.max_iter) {
          ++k;
          double dsum = 0.0, dmax = 0.0;
          for (int b = 0; b < B; ++b) {
            const int r0 = (int)(((int64_t)nv * b) / B), r1 = (int)(((int64_t)nv * (b + 1)) / B);
            const uint32_t q0 = lqb[b], q1 = lqb[b + 1];
            // (A) the block's slot sums
#pragma unroll
            for (int j = 0; j < kSPT; ++j) {
              const uint32_t sl = threadIdx.x + kThreads * j;
              if (sl >= q0 && sl < q1) {
                YT g[kSlot];
#pragma unroll
                for (uint32_t m = 0; m < kSlot; ++m) g[m] = la[(sid[j][m / 2] >> (16 * (m & 1))) & 0xffffu];
                lpart[sl] = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]));
              }
            }
            __syncthreads();
            // (B) the block's rows
#pragma unroll
            for (int j = 0; j < kRPT; ++j) {
              if (kThreads * j + wave * 64 < nv) {  // wave-uniform
                const int r = threadIdx.x + kThreads * j;
                const bool in = r >= r0 && r < r1;
                const uint32_t f0 = fr[j] & 0xffffu, f1 = fr[j] >> 16;
                const bool wide = f1 - f0 > kSlot;
                YT sv = 0;
                if (in && !wide) {
                  YT h[kSlot];
#pragma unroll
                  for (uint32_t m = 0; m < kSlot; ++m) h[m] = f0 + m < f1 ? lpart[f0 + m] : (YT)0;
                  sv = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));
                }
                unsigned long long m = __ballot(in && wide);
                while (m) {
                  const int bl = __ffsll(m) - 1;
                  m &= m - 1;
                  const uint32_t blo = __shfl(f0, bl, 64), bhi = __shfl(f1, bl, 64);
                  YT ws = 0;
                  for (uint32_t e = blo + lane; e < bhi; e += 256) {
                    YT g[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) g[q] = e + 64 * q < bhi ? lpart[e + 64 * q] : (YT)0;
                    ws += (g[0] + g[1]) + (g[2] + g[3]);
                  }
                  ws = wave_sum(ws);
                  if (lane == bl) sv = ws;
                }
                if (in) {
                  const double rn = wr[j] + (double)sv;
                  const double d = fabs(rn - Rr[j]);
                  Rr[j] = rn;
                  la[r] = (YT)(c * rn * (double)ir[j]);
                  dsum += d;
                  dmax = fmax(dmax, d);
                }
              }
            }
            __syncthreads();  // the block's new values before the next block's sums
          }
          double norm, mx;
          block_sum_max(dsum, dmax, red, (int)(k & 1), &norm, &mx);
          last = norm;
          if (stop_now(p, norm, mx, thresh)) {
            conv = true;
            break;
          }
        }
      }
    } else if (!skip) {
      conv = false;
      while (k < p.max_iter) {
        ++k;
        const double rho = (tail && nprev2 > 0.0) ? nprev / nprev2 : -1.0;
        const bool rho_ok = rho > 0.0 && rho < 1.0;
        // (A) slot sums
#pragma unroll
        for (int j = 0; j < kSPT; ++j) {
          const uint32_t sl = threadIdx.x + kThreads * j;
          if (sl < nslot) {
            YT g[kSlot];
#pragma unroll
            for (uint32_t m = 0; m < kSlot; ++m) g[m] = la[(sid[j][m / 2] >> (16 * (m & 1))) & 0xffffu];
            if constexpr (WT) {
#pragma unroll
              for (uint32_t m = 0; m < kSlot; ++m) g[m] *= lw[kSlot * sl + m];
            }
            lpart[sl] = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]));
          }
        }
        __syncthreads();
        // (B) row sums
        double part = 0.0, pm = 0.0, dpart = 0.0;
#pragma unroll
        for (int j = 0; j < kRPT; ++j) {
          if (kThreads * j + wave * 64 < nv) {  // wave-uniform
            const int r = threadIdx.x + kThreads * j;
            const uint32_t f0 = fr[j] & 0xffffu, f1 = fr[j] >> 16;
            const bool wide = f1 - f0 > kSlot;
            YT sv = 0;
            if (r < nv && !wide) {
              YT h[kSlot];
#pragma unroll
              for (uint32_t m = 0; m < kSlot; ++m) h[m] = f0 + m < f1 ? lpart[f0 + m] : (YT)0;
              sv = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));
            }
            unsigned long long m = __ballot(r < nv && wide);
            while (m) {
              const int b = __ffsll(m) - 1;
              m &= m - 1;
              const uint32_t blo = __shfl(f0, b, 64), bhi = __shfl(f1, b, 64);
              YT ws = 0;
              for (uint32_t e = blo + lane; e < bhi; e += 256) {
                YT g[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) g[q] = e + 64 * q < bhi ? lpart[e + 64 * q] : (YT)0;
                ws += (g[0] + g[1]) + (g[2] + g[3]);
              }
              ws = wave_sum(ws);
              if (lane == b) sv = ws;
            }
            if (r < nv) {
              Rr[j] += (double)sv;
              lb[r] = cy * sv * ir[j];
              part += fabs((double)sv);
              pm = fmax(pm, fabs((double)sv));
              if (rho_ok) dpart += fabs((double)sv - rho * (double)la[r] / ((double)cy * (double)ir[j]));
            }
          }
        }
        double norm, mx, dsum = 0.0;
        // the barrier also publishes lb
        if (tail) block_sum2_max(part, dpart, pm, red, (int)(k & 1), &norm, &dsum, &mx);
        else block_sum_max(part, pm, red, (int)(k & 1), &norm, &mx);
        last = norm;
        YT* tt = la;
        la = lb;
        lb = tt;
        if (stop_now(p, norm, mx, thresh)) {
          conv = true;
          break;
        }
        if (rho_ok && dsum <= thresh * (1.0 - rho)) {  // R' = R - P_k + rho/(1-rho) P_{k-1}
#pragma unroll
          for (int j = 0; j < kRPT; ++j) {
            const int r = threadIdx.x + kThreads * j;
            if (r < nv) {
              const double sc = (double)cy * (double)ir[j];
              Rr[j] += rho / (1.0 - rho) * ((double)lb[r] / sc) - (double)la[r] / sc;  // lb: P_{k-1}, la: P_k
            }
          }
          last = dsum / (1.0 - rho) / p.c;
          conv = true;
          break;
        }
        nprev2 = nprev;
        nprev = norm;
      }
    }
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int r = threadIdx.x + kThreads * j;
      if (r < nv) {
        p.Rout[p.perm[vb + r]] = Rr[j];
        st_x(p.x, vb + r, c * Rr[j] * p.inv64[vb + r]);
      }
    }
  } else {
    // certified tail estimate as in the register path above
    const bool tail = TAIL && p.tail;
    double nprev = last, nprev2 = -1.0;
    if (!skip) {
      conv = false;
      while (k < p.max_iter) {
        ++k;
        const double rho = (tail && nprev2 > 0.0) ? nprev / nprev2 : -1.0;
        const bool rho_ok = rho > 0.0 && rho < 1.0;
        part = 0.0;
        double pm = 0.0, dpart = 0.0;
        for (int ra = w0; ra < w1; ra += 64) {
          const int nr = w1 - ra < 64 ? w1 - ra : 64;
          const YT s = wave_tile_gather<RPW, YT, false, WT>(p, ptr, src, ya, ra, nr, tile, term_w<YT>(p));
          if (lane < nr) {
            const int v = ra + lane;
            YT iv;
            if constexpr (sizeof(YT) == 8) iv = p.inv64[v];
            else iv = p.inv32[v];
            p.R[v] += (double)s;
            if (rho_ok) dpart += fabs((double)s - rho * (double)ya[v] / ((double)cy * (double)iv));
            yb[v] = cy * s * iv;
            part += fabs((double)s);
            pm = fmax(pm, fabs((double)s));
          }
        }
        double norm, mx, dsum = 0.0;
        // the barrier also publishes yb
        if (tail) block_sum2_max(part, dpart, pm, red, (int)(k & 1), &norm, &dsum, &mx);
        else block_sum_max(part, pm, red, (int)(k & 1), &norm, &mx);
        last = norm;
        YT* tt = ya;
        ya = yb;
        yb = tt;
        if (stop_now(p, norm, mx, thresh)) {
          conv = true;
          break;
        }
        if (rho_ok && dsum <= thresh * (1.0 - rho)) {  // yb: P_{k-1}, ya: P_k; a lane's own rows
          for (int v = w0 + lane; v < w1; v += 64) {
            double iv;
            if constexpr (sizeof(YT) == 8) iv = p.inv64[v];
            else iv = (double)p.inv32[v];
            const double sc = (double)cy * iv;
            p.R[v] += rho / (1.0 - rho) * ((double)yb[v] / sc) - (double)ya[v] / sc;
          }
          last = dsum / (1.0 - rho) / p.c;
          conv = true;
          break;
        }
        nprev2 = nprev;
        nprev = norm;
      }
    }
    for (int v = w0 + lane; v < w1; v += 64) {
      const double r = p.R[v];
      p.Rout[p.perm[v]] = r;
      st_x(p.x, v, c * r * p.inv64[v]);
    }
  }
  if (threadIdx.x == 0) {
    wst[S_T_MEDIUM_ITER] += wall_clock64() - t_it;
    record_scc(p, rank, k, last, conv, ne, (uint64_t)nv, wst, false, ws);
  }
}

__device__ inline void flush_stats(const SolveParams& p, unsigned long long* s_stats) {
  __syncthreads();
  if (threadIdx.x < kWgStats) {
    unsigned long long* g = p.wgstats + (size_t)blockIdx.x * kWgStats + threadIdx.x;
    const unsigned long long v = s_stats[threadIdx.x];
    *g = threadIdx.x == S_ITERS_MAX ? (v > *g ? v : *g) : *g + v;
  }
}

// LDS of the segment kernel: four wavefront tiles followed by the small-SCC
// term vectors; a single-workgroup SCC may reuse all of it once its weights
// are gathered, and a vertex item keeps its local x values in the second part.
static_assert(kDirectMax * (kDirectMax + 1) * sizeof(double) <= 512 * sizeof(double) + 64 * (sizeof(double) + 8),
              "direct-solve matrix fits the tile");
constexpr size_t kSegLds = 52 * 1024;  // three workgroups per CU (the VGPR limit too)
static_assert(kDirectMaxWG * (kDirectMaxWG + 1) * sizeof(double) <= kSegLds && kDirectMaxWG < kThreads,
              "workgroup direct-solve matrix fits the segment LDS");
static_assert(kWaves * sizeof(WaveTile) + kWaves * 2 * kSmallMax * sizeof(double) <= kSegLds, "segment LDS");
static_assert(kWaves * sizeof(WaveTile) + 4 * kThreads * sizeof(double) + kThreads * sizeof(uint4) +
                      (3 * kThreads + 1 + kWaves) * sizeof(int32_t) <=
                  kSegLds,
              "vertex item LDS");
static_assert(kWaves * sizeof(WaveTile) + kVertWtOff + 4 * kThreads * sizeof(double) <= kSegLds,
              "vertex item LDS with edge weights");

// Persistent segment kernel.  Items are handed out in plan order by one
// atomic counter per segment (one atomic per item).  This cannot deadlock,
// whatever the number of resident workgroups: an item only waits for items
// handed out before it, and those are held by running workgroups; the
// lowest unfinished item has nothing left to wait for.
template <typename YT, int RPW, bool WARM, bool TAIL, bool WT, bool GS = false>
__device__ __attribute__((always_inline)) void segment_body(const SolveParams& p) {
  __shared__ double s_red[24];
  __shared__ __attribute__((aligned(16))) unsigned char s_raw[kSegLds];
  __shared__ unsigned long long s_stats[kWgStats];
  WaveTile* tiles = reinterpret_cast<WaveTile*>(s_raw);
  unsigned char* second = s_raw + kWaves * sizeof(WaveTile);
  __shared__ unsigned long long s_ready;
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x < kWgStats) s_stats[threadIdx.x] = 0ull;
  if ((threadIdx.x & 63) == 0) {
    tiles[wave].wst = s_stats;
    tiles[wave].rdy = &s_ready;
  }
  __syncthreads();
  const unsigned long long t_k = wall_clock64();
  __shared__ int s_next;
  while (true) {
    if (threadIdx.x == 0) s_next = (int)atomicAdd(p.seg_head, 1u);
    __syncthreads();
    const int i = s_next;
    if (i >= p.n_items) break;
    const Item it = p.items[i];
    const unsigned long long t_i = wall_clock64();
    if (p.trace && threadIdx.x == 0) {
      p.trace[4 * (size_t)(p.item_base + i)] = blockIdx.x | ((unsigned long long)it.kind << 32);
      p.trace[4 * (size_t)(p.item_base + i) + 1] = t_i;
      s_ready = t_i;
    }
    int slot;
    if (it.kind == ITEM_VERTS) {
      run_verts<WT>(p, it.a, it.b, &tiles[wave], reinterpret_cast<double*>(second));
      slot = S_T_VERTS;
    } else if (it.kind == ITEM_SMALL) {
      const int r = it.a + wave;
      YT* ybuf = reinterpret_cast<YT*>(second) + (size_t)wave * 2 * kSmallMax;
      if (r < it.b) run_small<YT, WARM, TAIL, WT>(p, r, ybuf, s_stats, &tiles[wave]);
      slot = S_T_SMALL;
    } else {
      const int nvm = p.comp_vbeg[it.a + 1] - p.comp_vbeg[it.a];
      if (nvm <= p.direct_max && nvm <= kDirectMaxWG) run_direct_wg<WT>(p, it.a, s_red, s_stats, tiles, s_raw);
      else run_medium<YT, RPW, WARM, TAIL, WT, GS>(p, it.a, s_red, s_stats, tiles, s_raw, kSegLds);
      slot = S_T_MEDIUM;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long t_e = wall_clock64();
      s_stats[slot] += t_e - t_i;
      if (p.trace) {
        p.trace[4 * (size_t)(p.item_base + i) + 2] = s_ready;
        p.trace[4 * (size_t)(p.item_base + i) + 3] = t_e;
      }
    }
    if ((threadIdx.x & 63) == 0) {  // a staged SCC may have overwritten them
      tiles[wave].wst = s_stats;
      tiles[wave].rdy = &s_ready;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) s_stats[S_T_SEGMENT] += wall_clock64() - t_k;
  flush_stats(p, s_stats);
}

// The segment kernel: the variants with the starting guess, the tail
// estimate, edge weights or fewer than 16 rows per wavefront need more
// registers and run two workgroups per CU; the others three.  k_segment_w3
// runs the tail-estimate variant at three workgroups per CU (168 registers,
// a few spills): faster where a segment is bound by throughput (many SCC
// items in flight), slower where it is bound by its chain of dependencies;
// the autotuner picks (pr_build_opts.seg_waves).
template <typename YT, int RPW, bool WARM, bool TAIL = false, bool WT = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WARM ? 1 : ((TAIL || WT || RPW < 16) ? 2 : 3)))) void k_segment(SolveParams p) {
  segment_body<YT, RPW, WARM, TAIL, WT>(p);
}
template <typename YT, int RPW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_segment_w3(SolveParams p) {
  segment_body<YT, RPW, false, true, false>(p);
}
// the segment kernel with block Gauss-Seidel sweeps in workgroup SCCs
// (gs_blocks > 0; no tail estimate, starting guess or edge weights)
template <typename YT, int RPW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_segment_gs(SolveParams p) {
  segment_body<YT, RPW, false, false, false, true>(p);
}

// ------------------------------------------------------------- gang phases
// Launch k = 0 raises the weights of the gang's rows (eq. PR:levels) and
// stores the first term; launch k >= 1 first decides, from the partial norms
// written by launch k-1, whether each SCC stopped after term k-1 (then its
// rows are finalised and it is skipped), and otherwise adds term k.  Every
// workgroup combines the same partials in the same order, so all reach the
// same decision.  No workgroup waits for another inside a launch.

struct GangCtx {
  int r0, r1;     // this workgroup's rows
  int s_lo, s_hi; // gang SCCs intersecting them
};

__device__ inline GangCtx gang_ctx(const SolveParams& p, const GangDesc& gd) {
  GangCtx g;
  g.r0 = p.gbounds[gd.boff + blockIdx.x];
  g.r1 = p.gbounds[gd.boff + blockIdx.x + 1];
  // first SCC with vend > r0
  int lo = gd.s0, hi = gd.s1;
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if (p.gscc[mid].vend <= g.r0) lo = mid + 1;
    else hi = mid;
  }
  g.s_lo = lo;
  int e = lo;
  while (e < gd.s1 && p.gscc[e].vbeg < g.r1) ++e;
  g.s_hi = e;
  return g;
}

// deterministic sum (and max) of an SCC's partials from launch `parity`;
// with `want_d`, also the sum of its tail-estimate partials (else 0)
__device__ inline void gang_total(const SolveParams& p, const GangScc& sc, int parity, double* red, double* tot,
                                  double* mx, bool want_d, double& dtot) {
  const int cnt = sc.nslot;
  const size_t off = (size_t)parity * p.n_gslots + sc.pbase;
  const double* pp = p.gpart + off;
  const double* pm = p.gpmx + off;
  double s = 0.0, m = 0.0, d = 0.0;
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    s += pp[j];
    m = fmax(m, pm[j]);
    if (want_d) d += p.gpdiff[off + j];
  }
  *tot = block_sum(s, red);
  *mx = block_max(m, red);
  dtot = want_d ? block_sum(d, red) : 0.0;
}

__device__ inline void gang_finalise(const SolveParams& p, const GangScc& sc, const GangCtx& g, int64_t iters,
                                     double last, bool conv, unsigned long long* wst) {
  const int a = sc.vbeg > g.r0 ? sc.vbeg : g.r0, z = sc.vend < g.r1 ? sc.vend : g.r1;
  for (int v = a + (int)threadIdx.x; v < z; v += kThreads) {
    const double r = p.R[v];
    p.Rout[p.perm[v]] = r;
    if (!p.plain) st_x(p.x, v, p.c * r * p.inv64[v]);
  }
  if (blockIdx.x == sc.wg_first && threadIdx.x == 0) {
    p.gdone[sc.gidx] = (int32_t)iters;
    if (sc.rank >= 0) {
      p.iters[sc.rank] = (int32_t)iters;
      p.lastnorm[sc.rank] = last;
    } else {
      p.lastnorm[0] = last;
    }
    const uint64_t ne = p.int_ptr[sc.vend] - p.int_ptr[sc.vbeg];
    const int ws = p.gmlp ? p.gws[sc.gidx] : -1;
    const unsigned long long passes = (unsigned long long)iters + (ws >= 0 ? 2ull : 0ull);
    wst[S_EDGE_ITERS] += passes * ne;
    wst[S_VERT_ITERS] += passes * (unsigned long long)(sc.vend - sc.vbeg);
    if (ws == 1) wst[S_WS_ACC] += 1ull;
    if (ws == 0) wst[S_WS_REJ] += 1ull;
    if ((unsigned long long)iters > wst[S_ITERS_MAX]) wst[S_ITERS_MAX] = (unsigned long long)iters;
    wst[S_ITERS_SUM] += (unsigned long long)iters;
    wst[S_N_ITERATED] += 1ull;
    if (!conv) wst[S_NOT_CONV] += 1ull;
  }
}

constexpr uint32_t kHubRow = 2048;   // rows with more in-edges are summed in pieces
constexpr uint32_t kHubPiece = 1024; // edges per piece

// first hub row >= r in the gang's (row-sorted) hub table
__device__ inline int first_hub(const SolveParams& p, const GangDesc& gd, int r) {
  int lo = gd.h0, hi = gd.h1;
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if (p.ghubs[mid].row < r) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename YT, int RPW, bool WT = false>
__global__ __launch_bounds__(kThreads) void k_gang(SolveParams p, int gang, int k, int final_launch) {
  __shared__ double s_red[4];
  __shared__ WaveTile s_tile[kWaves];
  __shared__ unsigned long long s_stats[kWgStats];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < kWgStats) s_stats[threadIdx.x] = 0ull;
  if (lane == 0) s_tile[wave].wst = s_stats;
  __syncthreads();
  const unsigned long long t_k = wall_clock64();
  const GangDesc gd = p.gangs[gang];
  const GangCtx g = gang_ctx(p, gd);
  const double c = p.c;
  YT* yr = (YT*)((k & 1) ? p.y0 : p.y1);  // term k-1
  YT* yw = (YT*)((k & 1) ? p.y1 : p.y0);  // term k
  const int par_w = k & 1, par_r = (k + 1) & 1;
  for (int si = g.s_lo; si < g.s_hi; ++si) {
    const GangScc sc = p.gscc[si];
    // skip SCCs finalised in an earlier launch; gdone holds the number of
    // terms, so the launch that detected the stop is gdone + 1 (the SCC is
    // finalised by every covering workgroup in that same launch)
    const int32_t done_terms = k > 0 ? p.gdone[si] : -1;
    if (done_terms >= 0 && done_terms + 1 < k) continue;
    const int a = sc.vbeg > g.r0 ? sc.vbeg : g.r0, z = sc.vend < g.r1 ? sc.vend : g.r1;
    // split this workgroup's rows of the SCC between its wavefronts by edges
    const uint32_t* ptr = p.int_ptr;
    const int64_t tot_w = (int64_t)(ptr[z] - ptr[a]) + (z - a);
    auto find_row = [&](int64_t target) {
      int lo = a, hi = z;
      while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if ((int64_t)(ptr[mid] - ptr[a]) + (mid - a) < target) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    const int w0 = wave == 0 ? a : find_row(tot_w * wave / kWaves);
    const int w1 = wave == kWaves - 1 ? z : find_row(tot_w * (wave + 1) / kWaves);
    double part = 0.0, pm = 0.0, dpart = 0.0, rho_k = -1.0;
    if (k == 0) {
      for (int ra = w0; ra < w1; ra += 64) {
        const int nr = w1 - ra < 64 ? w1 - ra : 64;
        double wp = p.plain ? 0.0
                            : wave_tile_gather<64, double, false, WT>(p, p.bnd_ptr, p.bnd_src, p.x, ra, nr,
                                                                      &s_tile[wave], p.bnd_w);
        if (lane < nr) {
          const int v = ra + lane;
          wp += p.W[p.perm[v]];
          p.R[v] = wp;
          p.wprime[v] = wp;
          if constexpr (sizeof(YT) == 8) yw[v] = c * wp * p.inv64[v];
          else yw[v] = (YT)(c * wp * (double)p.inv32[v]);
          part += fabs(wp);
        }
      }
    } else {
      double tot, mx, dtot = 0.0;
      gang_total(p, sc, par_r, s_red, &tot, &mx, p.tail != 0, dtot);
      double wsum;
      if (k == 1) {
        wsum = tot;
        if (blockIdx.x == sc.wg_first && threadIdx.x == 0) p.gwsum[si] = wsum;
      } else {
        wsum = p.gwsum[si];
      }
      const double thresh = p.eps * (1.0 - c) * wsum;
      bool stop;
      double last = k == 1 ? wsum : tot;
      if (k == 1) {
        stop = (p.stop == PR_STOP_CERT_L1 && wsum == 0.0);
        if (!stop && p.gmlp && p.gws[si] == 1) {  // kept guess: term 0 is r_0
          last = p.gwn[si];
          stop = stop_now(p, p.gwn[si], p.gwm[si], thresh);
        }
      } else {
        stop = stop_now(p, tot, mx, thresh);
      }
      // certified tail estimate: gnhist slot j % 3 holds ||P_{j-1}||_1 from
      // launch j (P_0 = r_0 after a kept guess); rho_t belongs to the
      // difference term k-1 carries, rho_k to the one this launch forms
      const YT cy = (YT)c;
      double rho_t = -1.0;
      if (p.tail) {
        double* hist = p.gnhist + 3 * (size_t)si;
        // launch 1: the first term's norm, r_0's for a kept starting guess
        if (blockIdx.x == sc.wg_first && threadIdx.x == 0) hist[k % 3] = last;
        if (k >= 2 && hist[(k - 1) % 3] > 0.0) rho_k = tot / hist[(k - 1) % 3];
        if (k >= 3 && hist[(k - 2) % 3] > 0.0) rho_t = hist[(k - 1) % 3] / hist[(k - 2) % 3];
        if (!stop && rho_t > 0.0 && rho_t < 1.0 && dtot <= thresh * (1.0 - rho_t)) {
          // R' = R - P_{k-1} + rho/(1-rho) P_{k-2}: the terms come back from
          // the term buffers (c P / outdeg), each row by the thread that
          // finalises it
          for (int v = a + (int)threadIdx.x; v < z; v += kThreads) {
            double iv;
            if constexpr (sizeof(YT) == 8) iv = p.inv64[v];
            else iv = (double)p.inv32[v];
            const double sc_v = (double)cy * iv;
            p.R[v] += rho_t / (1.0 - rho_t) * ((double)yw[v] / sc_v) - (double)yr[v] / sc_v;
          }
          last = dtot / (1.0 - rho_t) / c;
          stop = true;
        }
      }
      if (stop || final_launch) {
        gang_finalise(p, sc, g, k - 1, last, stop, s_stats);
        continue;
      }
      const bool rho_ok = rho_k > 0.0 && rho_k < 1.0;
      int hidx = first_hub(p, gd, w0);  // hub rows are summed in pieces below
      int ra = w0;
      while (ra < w1) {
        const int nexth = hidx < gd.h1 ? p.ghubs[hidx].row : 0x7fffffff;
        if (ra == nexth) {
          ++ra;
          ++hidx;
          continue;
        }
        int rb = ra + 64 < w1 ? ra + 64 : w1;
        if (nexth < rb) rb = nexth;
        const int nr = rb - ra;
        const YT sv = wave_tile_gather<RPW, YT, false, WT>(p, ptr, p.int_src, yr, ra, nr, &s_tile[wave], term_w<YT>(p));
        if (lane < nr) {
          const int v = ra + lane;
          YT iv;
          if constexpr (sizeof(YT) == 8) iv = p.inv64[v];
          else iv = p.inv32[v];
          p.R[v] += (double)sv;
          if (rho_ok) dpart += fabs((double)sv - rho_k * (double)yr[v] / ((double)cy * (double)iv));
          yw[v] = cy * sv * iv;
          part += fabs((double)sv);
          pm = fmax(pm, fabs((double)sv));
        }
        ra = rb;
      }
    }
    part = block_sum(part, s_red);
    pm = block_max(pm, s_red);
    if (p.tail) dpart = block_sum(dpart, s_red);
    if (threadIdx.x == 0) {
      const size_t slot = (size_t)par_w * p.n_gslots + sc.pbase + (blockIdx.x - sc.wg_first);
      p.gpart[slot] = part;
      p.gpmx[slot] = pm;
      if (p.tail) p.gpdiff[slot] = dpart;
    }
  }
  // pieces of hub rows assigned to this workgroup (terms k >= 1); a piece
  // of an SCC that has stopped is computed anyway and ignored by the combine
  if (k > 0 && !final_launch && gd.h1 > gd.h0) {
    const int pb = p.gpiece_ptr[gd.poff + blockIdx.x], pe = p.gpiece_ptr[gd.poff + blockIdx.x + 1];
    for (int q = pb + wave; q < pe; q += kWaves) {
      const GangPiece pc = p.gpieces[q];
      YT a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      uint32_t e = pc.ebeg + lane;
      if constexpr (WT) {
        const YT* wt = term_w<YT>(p);
        for (; e + 192 < pc.eend; e += 256) {
          const int32_t s0 = p.int_src[e], s1 = p.int_src[e + 64], s2 = p.int_src[e + 128], s3 = p.int_src[e + 192];
          a0 += yr[s0] * wt[e];
          a1 += yr[s1] * wt[e + 64];
          a2 += yr[s2] * wt[e + 128];
          a3 += yr[s3] * wt[e + 192];
        }
        for (; e < pc.eend; e += 64) a0 += yr[p.int_src[e]] * wt[e];
      } else {
        for (; e + 192 < pc.eend; e += 256) {
          const int32_t s0 = p.int_src[e], s1 = p.int_src[e + 64], s2 = p.int_src[e + 128], s3 = p.int_src[e + 192];
          a0 += yr[s0];
          a1 += yr[s1];
          a2 += yr[s2];
          a3 += yr[s3];
        }
        for (; e < pc.eend; e += 64) a0 += yr[p.int_src[e]];
      }
      const YT sum = wave_sum((a0 + a1) + (a2 + a3));
      if (lane == 0) p.gpiece_part[q] = (double)sum;
    }
  }
  if (threadIdx.x == 0) {
    s_stats[S_T_GANG] += wall_clock64() - t_k;
    s_stats[S_N_GANG] += 1;
  }
  flush_stats(p, s_stats);
}

// Combine the pieces of every hub row of a gang after launch k: one
// wavefront per hub sums its pieces in order and applies the row update
// (k = 0: the hub slots of the first launch are cleared).
template <typename YT>
__global__ __launch_bounds__(kThreads) void k_gang_hubs(SolveParams p, int gang, int k) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const GangDesc gd = p.gangs[gang];
  const int h = gd.h0 + blockIdx.x * kWaves + wave;
  if (h >= gd.h1 || lane != 0) return;
  const GangHub hb = p.ghubs[h];
  const size_t slot = (size_t)(k & 1) * p.n_gslots + hb.slot;
  if (k == 0) {
    p.gpart[slot] = 0.0;
    p.gpmx[slot] = 0.0;
    if (p.tail) p.gpdiff[slot] = 0.0;
    return;
  }
  if (p.gdone[hb.scc] >= 0) return;  // its SCC stopped in launch k
  YT s = 0;
  for (int q = hb.p0; q < hb.p1; ++q) s += (YT)p.gpiece_part[p.ghub_pieces[q]];
  YT* yw = (YT*)((k & 1) ? p.y1 : p.y0);
  const YT* yr = (const YT*)((k & 1) ? p.y0 : p.y1);
  const int v = hb.row;
  YT iv;
  if constexpr (sizeof(YT) == 8) iv = p.inv64[v];
  else iv = p.inv32[v];
  const YT cy = (YT)p.c;
  p.R[v] += (double)s;
  yw[v] = cy * s * iv;
  p.gpart[slot] = fabs((double)s);
  p.gpmx[slot] = fabs((double)s);
  if (p.tail) {  // the same rho_k as launch k (gnhist, see k_gang)
    const double* hist = p.gnhist + 3 * (size_t)hb.scc;
    const double rho = (k >= 2 && hist[(k - 1) % 3] > 0.0) ? hist[k % 3] / hist[(k - 1) % 3] : -1.0;
    p.gpdiff[slot] = (rho > 0.0 && rho < 1.0) ? fabs((double)s - rho * (double)yr[v] / ((double)cy * (double)iv)) : 0.0;
  }
}

// Starting guess for the SCCs of a gang (Sec. 4.3.2 series started from a
// predicted R_0, see warm_preamble): three launches between term 0 and
// term 1.  step 0: the first plain term p_1 = c A^T W' (from wx = c W' /
// outdeg), the features, the network and R_0 (wres = c R_0 / outdeg);
// step 1: r_0 = W' + c A^T R_0 - R_0 (into wx); step 2: every workgroup
// combines the partial norms in slot order and, if ||r_0||_1 < ||p_1||_1,
// replaces R by R_0 + r_0 and term 0 by r_0.
template <typename YT, int RPW>
__global__ __launch_bounds__(kThreads) void k_gang_warm(SolveParams p, int gang, int step) {
  __shared__ double s_red[4];
  __shared__ WaveTile s_tile[kWaves];
  __shared__ unsigned long long s_stats[kWgStats];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < kWgStats) s_stats[threadIdx.x] = 0ull;
  if (lane == 0) s_tile[wave].wst = s_stats;
  __syncthreads();
  const GangDesc gd = p.gangs[gang];
  const GangCtx g = gang_ctx(p, gd);
  const double c = p.c;
  for (int si = g.s_lo; si < g.s_hi; ++si) {
    const GangScc sc = p.gscc[si];
    const int a = sc.vbeg > g.r0 ? sc.vbeg : g.r0, z = sc.vend < g.r1 ? sc.vend : g.r1;
    const uint32_t* ptr = p.int_ptr;
    const int64_t tot_w = (int64_t)(ptr[z] - ptr[a]) + (z - a);
    auto find_row = [&](int64_t target) {
      int lo = a, hi = z;
      while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if ((int64_t)(ptr[mid] - ptr[a]) + (mid - a) < target) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    const int w0 = wave == 0 ? a : find_row(tot_w * wave / kWaves);
    const int w1 = wave == kWaves - 1 ? z : find_row(tot_w * (wave + 1) / kWaves);
    const size_t slot = (size_t)sc.pbase + (blockIdx.x - sc.wg_first);
    if (step == 0) {
      double tot, mx, dnone;
      gang_total(p, sc, 0, s_red, &tot, &mx, false, dnone);  // ||W'_C||_1 from term 0's partials
      const double sC = tot / (double)(sc.vend - sc.vbeg);
      double np1 = 0.0;
      for (int ra = w0; ra < w1; ra += 64) {
        const int nr = w1 - ra < 64 ? w1 - ra : 64;
        // the first plain term, gathered from term 0 (c W' / outdeg, written by
        // launch k = 0 in the precision of the terms); the features are FP32
        const double p1 = (double)wave_tile_gather<RPW, YT, false>(p, ptr, p.int_src, (const YT*)p.y0, ra, nr,
                                                                   &s_tile[wave]);
        const int v = ra + lane;
        const bool act = lane < nr && sC > 0.0;
        float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
        if (act) {
          const double wpv = p.wprime[v];
          np1 += fabs(p1);
          const uint32_t indeg = (p.bnd_ptr[v + 1] - p.bnd_ptr[v]) + (ptr[v + 1] - ptr[v]);
          f0 = log1pf((float)indeg);
          f1 = log1pf(rintf(1.0f / p.inv32[v]));
          f2 = log1pf((float)((wpv - p.W[p.perm[v]]) / sC));
          f3 = log1pf((float)((wpv + p1) / sC));
        }
        if (lane < nr) p.wfeat[v] = make_float4(f0, f1, f2, f3);
      }
      np1 = block_sum(np1, s_red);
      if (threadIdx.x == 0) p.gwp1[slot] = np1;
    } else if (step == 1) {
      double nr0 = 0.0, mr0 = 0.0;
      for (int ra = w0; ra < w1; ra += 64) {
        const int nr = w1 - ra < 64 ? w1 - ra : 64;
        const double acc = wave_tile_gather<RPW, double, false>(p, ptr, p.int_src, p.wres, ra, nr, &s_tile[wave]);
        if (lane < nr) {
          const int v = ra + lane;
          const double r = p.wprime[v] + acc - p.wr0[v];
          p.wx[v] = r;
          nr0 += fabs(r);
          mr0 = fmax(mr0, fabs(r));
        }
      }
      nr0 = block_sum(nr0, s_red);
      mr0 = block_max(mr0, s_red);
      if (threadIdx.x == 0) {
        p.gwr0[slot] = nr0;
        p.gwm0[slot] = mr0;
      }
    } else {
      double s1 = 0.0, s2 = 0.0, m2 = 0.0;
      for (int j = threadIdx.x; j < sc.nslot; j += kThreads) {
        s1 += p.gwp1[sc.pbase + j];
        s2 += p.gwr0[sc.pbase + j];
        m2 = fmax(m2, p.gwm0[sc.pbase + j]);
      }
      const double np1 = block_sum(s1, s_red), nr0 = block_sum(s2, s_red), mr0 = block_max(m2, s_red);
      const bool keep = nr0 < np1;  // false for a non-finite guess
      if (keep) {
        YT* y0 = (YT*)p.y0;
        for (int v = a + (int)threadIdx.x; v < z; v += kThreads) {
          const double r = p.wx[v];
          p.R[v] = p.wr0[v] + r;
          if constexpr (sizeof(YT) == 8) y0[v] = c * r * p.inv64[v];
          else y0[v] = (YT)(c * r * (double)p.inv32[v]);
        }
      }
      if (blockIdx.x == sc.wg_first && threadIdx.x == 0) {
        p.gws[si] = keep ? 1 : 0;
        p.gwn[si] = nr0;
        p.gwm[si] = mr0;
      }
    }
  }
}

// The network of the gang SCCs' starting guess, between steps 0 and 1 of
// k_gang_warm: R_0 = s_C exp(y) from the features step 0 stored, and
// c R_0 / outdeg for the residual.  A kernel of its own: without the gather
// and its tiles it keeps few registers, so many wavefronts share each SIMD
// while the network's matrix-core and GELU work runs.
__global__ __launch_bounds__(kThreads) void k_gang_warm_net(SolveParams p, int gang) {
  __shared__ double s_red[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const GangDesc gd = p.gangs[gang];
  const GangCtx g = gang_ctx(p, gd);
  for (int si = g.s_lo; si < g.s_hi; ++si) {
    const GangScc sc = p.gscc[si];
    const int a = sc.vbeg > g.r0 ? sc.vbeg : g.r0, z = sc.vend < g.r1 ? sc.vend : g.r1;
    double tot, mx, dnone;
    gang_total(p, sc, 0, s_red, &tot, &mx, false, dnone);  // ||W'_C||_1 from term 0's partials
    const double sC = tot / (double)(sc.vend - sc.vbeg);
    for (int ra = a + 64 * wave; ra < z; ra += kThreads) {  // wave-uniform trip count
      const int v = ra + lane;
      const bool act = v < z && sC > 0.0;
      const float4 f = act ? p.wfeat[v] : make_float4(0.f, 0.f, 0.f, 0.f);
      const float y = mlp_forward64(*p.gmlp, f.x, f.y, f.z, f.w);
      if (v < z) {
        const double r0 = act ? sC * exp((double)y) : 0.0;
        p.wr0[v] = r0;
        p.wres[v] = p.c * r0 * p.inv64[v];
      }
    }
  }
}

// ------------------------------------------------------------ setup kernels

__global__ void k_init(SolveParams p, int64_t K, int64_t n_gscc, int64_t n_stats, unsigned* seg_heads,
                       int64_t n_heads) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < p.n; i += stride) {
    p.x[i] = kXPending;
    const double w = p.W[i];
    // weights are non-negative and finite; a correction solve's weights (a
    // residual) only finite
    if (!((p.signed_w ? fabs(w) : w) >= 0.0) || !(fabs(w) <= 1.7976931348623157e308))
      atomicOr(&p.counters[C_BAD_W], 1ull);
  }
  for (int64_t i = tid; i < K; i += stride) {
    p.iters[i] = 0;
    p.lastnorm[i] = 0.0;
  }
  for (int64_t i = tid; i < n_gscc; i += stride) {
    p.gdone[i] = -1;
    p.gwsum[i] = 0.0;
  }
  for (int64_t i = tid; i < n_stats; i += stride) p.wgstats[i] = 0ull;
  for (int64_t i = tid; i < n_heads; i += stride) seg_heads[i] = 0u;
  if (p.gmlp) {
    for (int64_t i = tid; i < n_gscc; i += stride) {
      p.gws[i] = -1;
      p.gwn[i] = 0.0;
      p.gwm[i] = 0.0;
    }
    for (int64_t i = tid; i < p.n_gslots; i += stride) {
      p.gwp1[i] = 0.0;
      p.gwr0[i] = 0.0;
      p.gwm0[i] = 0.0;
    }
  }
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
__global__ __launch_bounds__(kThreads) void k_reduce2(const double* part, double* out,
                                                      const unsigned long long* wgstats, int G,
                                                      unsigned long long* counters) {
  __shared__ double lds[4];
  double sa = part[2 * threadIdx.x], sb = part[2 * threadIdx.x + 1];
  sa = block_sum(sa, lds);
  sb = block_sum(sb, lds);
  if (threadIdx.x == 0) {
    out[0] = sa;
    out[1] = sb;
  }
  // counter q = t % 16 over workgroups t/16, t/16 + 16, ...: independent
  // loads in flight; integer sums and maxima do not depend on the order
  __shared__ unsigned long long lacc[kThreads];
  const int q = threadIdx.x % kWgStats;
  unsigned long long acc = 0;
  for (int g = threadIdx.x / kWgStats; g < G; g += kThreads / kWgStats) {
    const unsigned long long v = wgstats[(size_t)g * kWgStats + q];
    acc = q == S_ITERS_MAX ? (v > acc ? v : acc) : acc + v;
  }
  lacc[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < kWgStats) {
    unsigned long long a = 0;
    for (int j = threadIdx.x; j < kThreads; j += kWgStats) {
      const unsigned long long v = lacc[j];
      a = threadIdx.x == S_ITERS_MAX ? (v > a ? v : a) : a + v;
    }
    counters[threadIdx.x] = a;
  }
}

// ------------------------------------------------------------ FP64 residual
// The certificate of a finished solve (Sec. 4.4).  With R the computed rank,
// r = W - (I - c A^T) R is formed in FP64 over every edge of the graph: the
// plan's between-component rows and inside-component rows together hold
// each edge once (kept self-loops included, in the inside rows).  Every
// column of c A^T sums to at most c, so ||R - R*||_1 <= ||r||_1 / (1 - c).
// Unlike the truncation bound of the series this covers the rounding of the
// FP32 terms too.
//   k_res_prep  R in plan order and xr = R / outdeg
//   k_residual  r per plan row, 64-row wavefront tiles; per-workgroup sums of
//               |r| and |R|; optionally r in the caller's order (the weights
//               of a correction solve)
//   k_res_sum   the workgroup sums added in a fixed order
constexpr int kResBlocks = 2048;
__global__ __launch_bounds__(kThreads) void k_res_prep(const double* Rout, const int32_t* perm, const double* inv64,
                                                       int64_t n, double* Rp, double* xr) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double r = Rout[perm[i]];
    Rp[i] = r;
    xr[i] = r * inv64[i];
  }
}
template <bool WT>
__global__ __launch_bounds__(kThreads) void k_residual(SolveParams p, const double* Rp, const double* xr, double* rw,
                                                       double* part) {
  __shared__ WaveTile s_tile[kWaves];
  __shared__ double lds[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double sr = 0.0, sR = 0.0;
  for (int64_t ra = ((int64_t)blockIdx.x * kWaves + wave) * 64; ra < p.n; ra += (int64_t)gridDim.x * kThreads) {
    const int nr = p.n - ra < 64 ? (int)(p.n - ra) : 64;
    const double sb =
        wave_tile_gather<64, double, false, WT>(p, p.bnd_ptr, p.bnd_src, xr, (int)ra, nr, &s_tile[wave], p.bnd_w);
    const double si =
        wave_tile_gather<64, double, false, WT>(p, p.int_ptr, p.int_src, xr, (int)ra, nr, &s_tile[wave], p.int_w64);
    if (lane < nr) {
      const int v = (int)ra + lane;
      const int o = p.perm[v];
      const double R = Rp[v];
      const double r = p.W[o] - R + p.c * (sb + si);
      if (rw) rw[o] = r;
      sr += fabs(r);
      sR += fabs(R);
    }
  }
  sr = block_sum(sr, lds);
  sR = block_sum(sR, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr;
    part[2 * blockIdx.x + 1] = sR;
  }
}
__global__ __launch_bounds__(kThreads) void k_res_sum(const double* part, int G, double* out) {
  __shared__ double lds[4];
  double a = 0.0, b = 0.0;
  for (int g = threadIdx.x; g < G; g += kThreads) {
    a += part[2 * g];
    b += part[2 * g + 1];
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}
// R += d (a refinement step)
__global__ __launch_bounds__(kThreads) void k_add(double* R, const double* d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    R[i] += d[i];
}

using SegFn = void (*)(SolveParams);

}  // namespace

// segment kernel variants by term type and stop rule, instantiated in the
// seg_*.hip files: the address of k_segment<YT, rpw, warm, tail> (cast to
// SegFn by the caller; rpw is rows per wavefront, warm selects the
// starting-guess variant), and of the weighted-graph variants (no guess)
const void* seg_kernel_f32(int rpw, bool warm);
const void* seg_kernel_f32_tail(int rpw, bool warm);
const void* seg_kernel_f64(int rpw, bool warm);
const void* seg_kernel_f64_tail(int rpw, bool warm);
const void* seg_kernel_w32(int rpw, bool tail);
const void* seg_kernel_w64(int rpw, bool tail);
// the tail-estimate variant at three workgroups per CU (rows per wavefront
// 16 or 64; null otherwise)
const void* seg_kernel_tail_w3(int rpw, bool fp64);
// the block Gauss-Seidel variant (gs_blocks > 0)
const void* seg_kernel_gs(int rpw, bool fp64);

}  // namespace prlib
