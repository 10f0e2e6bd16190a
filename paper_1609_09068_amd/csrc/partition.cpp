// Host SCC/CAC partition: the modified Tarjan depth-first search of Sec. 4.1.
//
// Per vertex the search keeps (Sec. 4.1): a discovery index, a lowlink, a
// level, a merge-find parent and depth (union by depth), and a state that
// says whether the vertex is still on the Tarjan stack or already placed in
// an SCC or a CAC.  The three steps per vertex are
//   Discover  index = lowlink = running counter, level = 1, push on stack;
//   Explore   every out-edge (v, w), self-loops skipped: an undiscovered w is
//             searched first; a placed w raises level(v) to level(w)+1, a w
//             still on the stack (same SCC) raises it to level(w) and lowers
//             lowlink(v) to lowlink(w);
//   Finish    when lowlink == index, pop v's SCC and give every member v's
//             level; a one-vertex SCC becomes a CAC and, as the head, merges
//             with every CAC on level(v)-1 it points to, unless it points to
//             an SCC of two or more vertices on that level (Theorem 3.1);
//             a merge lowers the head's level by one.
// The search is iterative (explicit frame stack), as in the paper's
// implementation (Sec. 5), so long paths cannot overflow the call stack.
// Levels are 1-based during the search and exported 0-based (Def. 3.3 and
// Fig. 1 put components without outgoing edges on level 0).
// Component ids: one pass over v = 0..n-1 numbering the merge-find roots in
// order of first appearance (Sec. 4.1, numbering pass).
#include <algorithm>
#include <cstring>
#include <new>

#include "internal.h"

namespace prlib {

int32_t validate_csr(int64_t n, const int64_t* row_ptr, const int32_t* col) {
  if (n < 0 || n > (int64_t)INT32_MAX - 1) {
    set_error("n = %lld outside [0, 2^31-2]", (long long)n);
    return PR_EINVAL;
  }
  if (!row_ptr) {
    set_error("row_ptr is NULL");
    return PR_EINVAL;
  }
  if (row_ptr[0] != 0) {
    set_error("row_ptr[0] = %lld, expected 0", (long long)row_ptr[0]);
    return PR_EINVAL;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (row_ptr[v + 1] < row_ptr[v]) {
      set_error("row_ptr decreases at row %lld", (long long)v);
      return PR_EINVAL;
    }
  }
  const int64_t m = row_ptr[n];
  if (m > 0 && !col) {
    set_error("col_idx is NULL with %lld edges", (long long)m);
    return PR_EINVAL;
  }
  for (int64_t e = 0; e < m; ++e) {
    if (col[e] < 0 || (int64_t)col[e] >= n) {
      set_error("col_idx[%lld] = %d outside [0, %lld)", (long long)e, col[e], (long long)n);
      return PR_EINVAL;
    }
  }
  return PR_OK;
}

uint64_t hash_csr(int64_t n, const int64_t* row_ptr, const int32_t* col) {
  // Fingerprint of the whole graph: every row pointer and every column index
  // enters it, so a plan is never built from a partition of another graph
  // with the same n and m (and autotune choices are keyed on the full CSR).
  // Four independent multiply-rotate lanes over 64-bit words keep it at
  // memory speed (about 0.1 s for 200M edges).
  constexpr uint64_t kP1 = 0x9E3779B97F4A7C15ull, kP2 = 0xC2B2AE3D27D4EB4Full;
  auto step = [](uint64_t h, uint64_t w) {
    h ^= w * kP1;
    h = (h << 31) | (h >> 33);
    return h * kP2;
  };
  const int64_t m = row_ptr[n];
  uint64_t h[4] = {0x243F6A8885A308D3ull ^ (uint64_t)n, 0x13198A2E03707344ull ^ (uint64_t)m,
                   0xA4093822299F31D0ull, 0x082EFA98EC4E6C89ull};
  int64_t v = 0;
  for (; v + 4 <= n + 1; v += 4)
    for (int j = 0; j < 4; ++j) h[j] = step(h[j], (uint64_t)row_ptr[v + j]);
  for (; v <= n; ++v) h[0] = step(h[0], (uint64_t)row_ptr[v]);
  int64_t e = 0;
  for (; e + 8 <= m; e += 8)
    for (int j = 0; j < 4; ++j)
      h[j] = step(h[j], (uint64_t)(uint32_t)col[e + 2 * j] | ((uint64_t)(uint32_t)col[e + 2 * j + 1] << 32));
  for (; e < m; ++e) h[1] = step(h[1], (uint64_t)(uint32_t)col[e] | ((uint64_t)e << 32));
  uint64_t r = (uint64_t)n * kP2;
  for (int j = 0; j < 4; ++j) r = step(r, h[j]);
  r ^= r >> 29;
  return r;
}

uint64_t hash_weights(int64_t m, const double* weight) {
  // fingerprint of the edge weights (their bit patterns), for the autotune
  // cache key of a weighted plan
  constexpr uint64_t kP1 = 0x9E3779B97F4A7C15ull, kP2 = 0xC2B2AE3D27D4EB4Full;
  uint64_t h = 0x452821E638D01377ull ^ (uint64_t)m;
  for (int64_t e = 0; e < m; ++e) {
    uint64_t w;
    std::memcpy(&w, weight + e, sizeof(w));
    h ^= w * kP1;
    h = ((h << 31) | (h >> 33)) * kP2;
  }
  return h ^ (h >> 29);
}

namespace {

enum : uint8_t { ST_NEW = 0, ST_STACK = 1, ST_SCC = 2, ST_CAC = 3 };

struct MergeFind {
  std::vector<int32_t> parent;
  std::vector<uint8_t> depth;
  explicit MergeFind(int64_t n) : parent(n), depth(n, 1) {
    for (int64_t i = 0; i < n; ++i) parent[i] = (int32_t)i;
  }
  int32_t find(int32_t v) {
    int32_t r = v;
    while (parent[r] != r) r = parent[r];
    while (parent[v] != r) {
      int32_t nx = parent[v];
      parent[v] = r;
      v = nx;
    }
    return r;
  }
  void merge(int32_t a, int32_t b) {
    int32_t ra = find(a), rb = find(b);
    if (ra == rb) return;
    if (depth[ra] < depth[rb]) std::swap(ra, rb);
    parent[rb] = ra;
    if (depth[ra] == depth[rb] && depth[ra] < 255) depth[ra]++;
  }
};

struct Frame {
  int32_t v;
  int64_t e;  // next out-edge to look at
};

}  // namespace

int32_t run_partition(int64_t n, const int64_t* row_ptr, const int32_t* col, Partition& out) {
  out.n = n;
  try {
    std::vector<int32_t> index(n, 0), low(n, 0), level(n, 0);
    std::vector<uint8_t> state(n, ST_NEW);
    std::vector<int32_t> tstack;
    std::vector<Frame> frames;
    MergeFind mf(n);
    out.emit_pos.assign(n, 0);
    tstack.reserve(1024);
    frames.reserve(1024);
    int32_t counter = 1;
    int32_t emitted = 0;

    auto settle = [&](int32_t v, int32_t w) {
      if (state[w] >= ST_SCC) {
        level[v] = std::max(level[v], level[w] + 1);
      } else {  // w on the stack: same SCC as v
        level[v] = std::max(level[v], level[w]);
        low[v] = std::min(low[v], low[w]);
      }
    };
    auto discover = [&](int32_t v) {
      index[v] = low[v] = counter++;
      level[v] = 1;
      state[v] = ST_STACK;
      tstack.push_back(v);
      frames.push_back(Frame{v, row_ptr[v]});
    };
    auto finish = [&](int32_t v) {
      if (low[v] != index[v]) return;
      int32_t size = 0;
      while (true) {
        int32_t w = tstack.back();
        tstack.pop_back();
        level[w] = level[v];
        state[w] = ST_SCC;
        mf.merge(w, v);
        out.emit_pos[w] = emitted++;
        ++size;
        if (w == v) break;
      }
      if (size != 1) return;
      state[v] = ST_CAC;
      // merge test: all out-edges, state kept across the whole loop
      const int32_t below = level[v] - 1;
      bool any = false, blocked = false;
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const int32_t w = col[e];
        if (w == v || level[w] != below) continue;
        if (state[w] == ST_SCC) {
          blocked = true;
          break;
        }
        if (state[w] == ST_CAC) any = true;
      }
      if (any && !blocked) {
        level[v] = below;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
          const int32_t w = col[e];
          if (w != v && state[w] == ST_CAC && level[w] == below) mf.merge(w, v);
        }
      }
    };

    for (int64_t r = 0; r < n; ++r) {
      if (state[r] != ST_NEW) continue;
      discover((int32_t)r);
      while (!frames.empty()) {
        Frame& f = frames.back();
        const int32_t v = f.v;
        if (f.e < row_ptr[v + 1]) {
          const int32_t w = col[f.e];
          if (w == v) {  // self-loop: ignored
            ++f.e;
            continue;
          }
          if (state[w] == ST_NEW) {
            discover(w);  // edge (v, w) is settled when w's frame closes
            continue;
          }
          ++f.e;
          settle(v, w);
          continue;
        }
        frames.pop_back();
        finish(v);
        if (!frames.empty()) {
          Frame& pf = frames.back();
          ++pf.e;
          settle(pf.v, v);
        }
      }
    }

    // numbering pass
    out.comp.assign(n, 0);
    std::vector<int32_t> id_of_root(n, -1);
    int32_t next = 0;
    for (int64_t v = 0; v < n; ++v) {
      const int32_t h = mf.find((int32_t)v);
      if (id_of_root[h] < 0) id_of_root[h] = next++;
      out.comp[v] = id_of_root[h];
    }
    out.n_comp = next;
    out.comp_level.assign(next, 0);
    out.comp_type.assign(next, 0);
    out.comp_size.assign(next, 0);
    int32_t maxlev = -1;
    for (int64_t v = 0; v < n; ++v) {
      const int32_t k = out.comp[v];
      out.comp_level[k] = level[v] - 1;
      out.comp_type[k] = state[v] == ST_SCC ? 1 : 0;
      out.comp_size[k]++;
      maxlev = std::max(maxlev, level[v] - 1);
    }
    out.n_levels = maxlev + 1;
  } catch (const std::bad_alloc&) {
    set_error("out of host memory in pr_partition (n = %lld)", (long long)n);
    return PR_ENOMEM;
  }
  return PR_OK;
}

}  // namespace prlib
