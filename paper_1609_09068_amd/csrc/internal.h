// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pr.h"
#include "mlp_dev.h"

namespace prlib {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

#define PR_HIP_CHECK(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      prlib::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                       __FILE__, __LINE__);                                         \
      return PR_EHIP;                                                               \
    }                                                                               \
  } while (0)

#define PR_TRY(x)                 \
  do {                            \
    int32_t rc_ = (x);            \
    if (rc_ != PR_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------- handles
enum HandleKind : uint32_t { KIND_PARTITION = 0x50415254u, KIND_LEVELS = 0x4c45564cu, KIND_MLP = 0x4d4c5050u };

void registry_add(void* h, HandleKind k);
bool registry_has(const void* h, HandleKind k);
bool registry_remove(void* h, HandleKind* k);

// --------------------------------------------------------------- partition
struct Partition {
  int64_t n = 0;
  int64_t n_comp = 0;
  int32_t n_levels = 0;
  std::vector<int32_t> comp;        // [n]
  std::vector<int32_t> comp_level;  // [K]
  std::vector<uint8_t> comp_type;   // [K]
  std::vector<int32_t> comp_size;   // [K]
  // position of each vertex in the order the depth-first search closed its
  // strongly connected component; reversed, it is a topological order of
  // the DAG of SCCs (used to lay out CAC vertices in dependency order)
  std::vector<int32_t> emit_pos;    // [n]
  uint64_t graph_hash = 0;
};

int32_t run_partition(int64_t n, const int64_t* row_ptr, const int32_t* col, Partition& out);
int32_t validate_csr(int64_t n, const int64_t* row_ptr, const int32_t* col);
uint64_t hash_csr(int64_t n, const int64_t* row_ptr, const int32_t* col);

// ---------------------------------------------------------------- the plan
// One work item of a persistent segment kernel.
struct Item {
  int32_t kind;  // ITEM_*
  int32_t a, b;  // ITEM_VERTS: positions [a, b); SMALL: ranks [a, b); MEDIUM: rank a
  int32_t c;     // ITEM_VERTS: longest chain of CAC edges inside the item (vertices)
};
enum : int32_t { ITEM_VERTS = 0, ITEM_SMALL = 1, ITEM_MEDIUM = 2 };

// A gang phase: the large SCCs of one level (or the whole graph for method
// PLAIN) iterated by every workgroup, one kernel launch per series term.
struct GangDesc {
  int32_t vbeg, vend;   // plan rows covered (the SCCs are contiguous)
  int32_t s0, s1;       // range in the GangScc table
  int32_t boff;         // offset of the grid+1 row bounds in the bounds table
  int32_t h0, h1;       // range in the GangHub table (sorted by row)
  int32_t poff;         // offset of the grid+1 per-workgroup piece pointers
};
struct GangScc {
  int32_t rank;         // component rank (-1: whole graph)
  int32_t vbeg, vend;
  int32_t wg_first, wg_last;  // workgroups whose rows intersect the SCC
  int32_t pbase;        // first partial-sum slot: one per covering workgroup, then one per hub row
  int32_t gidx;         // index of this entry in the table
  int32_t nslot;        // number of partial-sum slots
};
// A row whose in-degree exceeds the hub threshold is summed in pieces spread
// over the gang's workgroups, then combined by a separate small launch.
struct GangHub {
  int32_t row;
  int32_t scc;          // GangScc index
  int32_t p0, p1;       // its pieces [p0, p1) in the piece table
  int32_t slot;         // its partial-sum slot
  int32_t pad[3];
};
struct GangPiece {
  uint32_t ebeg, eend;  // edges of the hub row summed by this piece
  int32_t hub;          // GangHub index
  int32_t pad;
};

// Phase of a solve: a persistent segment over items [a, b) or gang a.
struct Phase {
  int32_t kind;  // 0 = segment, 1 = gang
  int32_t a, b;
};

constexpr int kWgStats = 16;  // per-workgroup counters accumulated over a solve

struct Levels {
  int64_t n = 0, m = 0, n_comp = 0;
  int32_t n_levels = 0;
  int device = 0;
  uint64_t graph_hash = 0;
  pr_build_opts opts{};
  pr_levels_info info{};
  // device arrays (plan order unless stated)
  int32_t* perm = nullptr;        // [n] plan position -> caller id
  int32_t* comp_vbeg = nullptr;   // [K+1] first plan position of each component (by rank)
  int32_t* comp_rank_of_id = nullptr;  // [K] caller component id -> rank
  int32_t* comp_id_of_rank = nullptr;  // [K]
  uint32_t* bnd_ptr = nullptr;    // [n+1] pull CSR of edges between components
  int32_t* bnd_src = nullptr;
  uint32_t* int_ptr = nullptr;    // [n+1] pull CSR of edges inside components
  int32_t* int_src = nullptr;
  uint32_t* full_ptr = nullptr;   // [n+1] whole-graph pull CSR (method PLAIN)
  int32_t* full_src = nullptr;
  float* inv_deg32 = nullptr;     // [n] 1/outdeg (0 for dangling); weighted: 1/s_u, s_u = total out-weight
  double* inv_deg64 = nullptr;    // [n]
  // weighted graph (Def. 3.4, a_uv = w_uv / s_u): the raw weight of every
  // edge, parallel to bnd_src, int_src and full_src (null when unweighted)
  bool weighted = false;
  uint64_t weight_hash = 0;
  double* bnd_w64 = nullptr;
  double* int_w64 = nullptr;
  float* int_w32 = nullptr;
  double* full_w64 = nullptr;
  float* full_w32 = nullptr;
  Item* items = nullptr;          // [n_items]
  uint32_t* vpath = nullptr;      // [n] vertex items: path order of the CAC sweep (see k_item_paths)
  uint32_t* mslot_ptr = nullptr;  // [n+1] first slot of each row (rows of workgroup SCCs own slots)
  uint4* mslot_src = nullptr;     // [slots] up to 8 source ids of a row, local to the SCC, two per word
  double* mslot_w64 = nullptr;    // [8 * slots] weighted plan: the slots' edge weights
  float* mslot_w32 = nullptr;
  int64_t n_mslots = 0;
  int64_t n_items = 0;
  int32_t grid = 0;               // workgroups of a segment kernel launch
  int32_t ggrid = 0;              // workgroups of a gang kernel launch
  int32_t sgrid = 0;              // max(grid, ggrid): per-workgroup counter rows
  unsigned* seg_heads = nullptr;  // [phases] item counters of the segments
  std::vector<Phase> phases;      // componentwise schedule
  GangDesc* gangs = nullptr;      // [n_gangs + 1]; the last one is the whole-graph gang
  GangScc* gsccs = nullptr;       // [n_gscc + 1]
  int32_t* gbounds = nullptr;     // [(n_gangs + 1) * (grid + 1)]
  int64_t n_gangs = 0, n_gscc = 0, n_gslots = 0;
  double* gpart = nullptr;        // [2 * n_gslots] partial 1-norms of the last two terms
  double* gpmx = nullptr;         // [2 * n_gslots] partial max-norms
  double* gwsum = nullptr;        // [n_gscc + 1] ||W'_C||_1 of each gang SCC
  double* gpdiff = nullptr;       // [2 * n_gslots] partial 1-norms of P_k - rho P_{k-1} (tail estimate)
  double* gnhist = nullptr;       // [3 * n_gscc] ||P_{k-1}||_1 of each gang SCC, written by launch k at k % 3
  GangHub* ghubs = nullptr;       // hub rows of all gangs
  GangPiece* gpieces = nullptr;   // hub pieces, grouped by workgroup within a gang
  int32_t* gpiece_ptr = nullptr;  // per gang: grid+1 offsets into gpieces
  int32_t* ghub_pieces = nullptr; // per hub: its piece positions in edge order
  double* gpiece_part = nullptr;  // [n_pieces] piece sums of the current term
  std::vector<int32_t> h_gang_nhub;  // hubs per gang (host)
  std::vector<int32_t> h_gang_rank;  // component ranks of the componentwise gang SCCs (host)
  std::vector<std::pair<int32_t, int32_t>> h_gang_sccs;  // per gang: its range in the GangScc table
  std::vector<int64_t> h_gang_hint;  // per gang and tail mode (index tail * n_gangs + gang): most terms any
                                     // solve of this plan needed (0: none yet)
  int64_t n_ghubs = 0, n_gpieces = 0;
  int32_t* gdone = nullptr;       // [n_gscc + 1] iterations when converged, -1 while running
  std::vector<uint32_t> h_int_ptr, h_full_ptr;
  // host copies used for scheduling and stats
  std::vector<int32_t> h_comp_vbeg;          // [K+1]
  std::vector<uint8_t> h_comp_class;         // [K] by rank: 0 SCC, 1 CAC(>=2), 2 singleton
  std::vector<int32_t> h_comp_level;         // [K] by rank
  std::vector<int64_t> h_comp_int_edges;     // [K] by rank
  std::vector<int32_t> h_comp_id_of_rank;    // [K]
  // per-solve work areas
  double* x = nullptr;            // [n] c R_v / outdeg(v), a quiet NaN until final
  double* R = nullptr;            // [n] rank in plan order (teams)
  double* wprime = nullptr;       // [n] W' in plan order (debug / features)
  void* y0 = nullptr;             // [n] series terms (float or double), ping
  void* y1 = nullptr;             // [n] pong
  unsigned long long* wgstats = nullptr;  // [grid * kWgStats]
  unsigned long long* trace = nullptr;    // [n_items * 4] optional item timeline
  hipStream_t cap_stream = nullptr;       // stream used to capture the hipGraph
  int32_t* iters = nullptr;       // [K] by rank
  double* lastnorm = nullptr;     // [K] by rank
  unsigned long long* counters = nullptr;  // [16] queue head, stats
  double* red = nullptr;          // [64] reduction scratch
  // captured launch sequences by key (solve options, buffers, gang budgets),
  // least recently used dropped beyond kGraphCache entries
  struct GraphEntry {
    uint64_t key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  static constexpr size_t kGraphCache = 8;
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  void drop_graphs();
  // FP64 residual certificate: per-workgroup partial sums; refinement: the
  // residual in the caller's order and the correction (allocated on first use)
  double* res_part = nullptr;
  double* res_w = nullptr;
  double* res_d = nullptr;
  std::vector<hipEvent_t> kev;  // per-launch timing events (kernel_timing)
  double* warm_buf = nullptr;   // starting-guess scratch (allocated on first use)
  int32_t* warm_gws = nullptr;  // [n_gscc] per gang SCC: guess kept / not / none
  ~Levels();
};

// ------------------------------------------------------ starting guesses
struct Mlp {
  int device = 0;
  float* master = nullptr;     // [kMlpParams] FP32 weights (flat, see mlp_dev.h)
  float* mom1 = nullptr;       // Adam first moments
  float* mom2 = nullptr;       // Adam second moments
  float* grad = nullptr;       // last batch gradient
  double* loss = nullptr;      // last batch sum of squared errors
  MlpPacked* packed = nullptr; // BF16 fragments used by every kernel
  float* gpart = nullptr;      // per-wavefront partial gradients
  double* lpart = nullptr;
  int64_t gpart_cap = 0;
  int64_t step = 0;
  ~Mlp();
};
void mlp_destroy(void* h);

int32_t build_levels(const Partition& p, const int64_t* row_ptr, const int32_t* col, const double* weight,
                     const pr_build_opts& opts, hipStream_t stream, Levels& lv);
uint64_t hash_weights(int64_t m, const double* weight);
int32_t make_schedule(Levels& lv, hipStream_t stream);
int32_t autotune_levels(Levels& lv, hipStream_t stream);
int32_t solve_levels(Levels& lv, double c, const double* W, double* R, const pr_solve_opts& o,
                     hipStream_t stream, pr_solve_stats* st);
int32_t solve_grid_size(int precision, int* grid);

}  // namespace prlib
