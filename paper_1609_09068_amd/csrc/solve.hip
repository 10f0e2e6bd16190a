// The PageRank step of Sec. 4.3 on the device.
//
// The plan (plan.hip) orders vertices level by level from the highest level
// down, components within a level by class and size, CAC vertices in
// topological order.  It splits the solve into phases:
//
//  * segment  one persistent kernel works through a run of items in plan
//             order; workgroups pop items from an atomic counter.
//      ITEM_VERTS   up to 256 consecutive one-vertex components or CAC
//                   vertices.  Every in-edge of such a vertex comes from a
//                   higher level or from earlier in its CAC's topological
//                   order, so R_v = W_v + sum_{u -> v} x_u with
//                   x_u = c R_u / outdeg(u) is exact in one pass (eq.
//                   PR:levels, Sec. 4.3.1).
//      ITEM_SMALL   up to four SCCs, one wavefront each, terms kept in LDS
//                   and registers.
//      ITEM_MEDIUM  one SCC per workgroup, rows staged in LDS when they fit.
//             SCC items gather W'_C (eq. PR:levels), then run the power
//             series P_0 = W'_C, P_{k+1} = c A_CC^T P_k, R_C = sum_k P_k
//             (Sec. 4.3.2) until the stop rule holds.
//  * gang     the SCCs of a level with many internal edges (and, for the
//             plain method, the whole graph) are iterated by every
//             workgroup, one launch per term; each launch also reads the
//             per-workgroup partial norms of the previous term to decide
//             the stop, in a fixed order.  Rows with very many in-edges are
//             summed in pieces and combined by a small launch per term.
//
// Dependencies inside a segment are data driven: x starts as a quiet NaN
// ("not ready"; a correction solve's x can have either sign) and every x_u
// is written once, with an agent-scope store, after R_u is final; readers
// poll with agent-scope loads.  Items are popped in
// plan order, so every item an item waits for went to a running workgroup.
// Inside a level the order is free (no edges join components of one level):
// the vertex items come first, then the workgroup and wavefront SCCs, so the
// pipelines of the large CACs start before the SCC items fill the machine.
//
// Precision: series terms y_k = c P_k / outdeg and their row sums are FP32
// (PR_PREC_MIXED) or FP64; R, W', x, the norms and every sum across rows are
// FP64.  All reductions use a fixed order (butterflies, fixed trees, and
// per-workgroup partials summed in workgroup order), so a solve is bitwise
// reproducible.
#include "solve_dev.h"

namespace prlib {

namespace {

template <typename T>
int32_t dalloc(T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1));
  if (e != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EHIP;
  }
  return PR_OK;
}

using GangFn = void (*)(SolveParams, int, int, int);

template <typename YT, bool WT>
GangFn gang_kernel(int rpw) {
  switch (rpw) {
    case 64: return k_gang<YT, 64, WT>;
    case 16: return k_gang<YT, 16, WT>;
    case 4: return k_gang<YT, 4, WT>;
    default: return k_gang<YT, 1, WT>;
  }
}
using HubFn = void (*)(SolveParams, int, int);
HubFn pick_hubs(int precision) {
  return precision == PR_PREC_FP64 ? (HubFn)k_gang_hubs<double> : (HubFn)k_gang_hubs<float>;
}
using WarmGangFn = void (*)(SolveParams, int, int);
template <typename YT>
WarmGangFn gang_warm_kernel(int rpw) {
  switch (rpw) {
    case 64: return k_gang_warm<YT, 64>;
    case 16: return k_gang_warm<YT, 16>;
    case 4: return k_gang_warm<YT, 4>;
    default: return k_gang_warm<YT, 1>;
  }
}
WarmGangFn pick_gang_warm(int precision, int rpw) {
  return precision == PR_PREC_FP64 ? gang_warm_kernel<double>(rpw) : gang_warm_kernel<float>(rpw);
}
SegFn pick_segment(int precision, int rpw, bool warm = false, bool tail = false, bool weighted = false) {
  const void* f = weighted ? (precision == PR_PREC_FP64 ? seg_kernel_w64(rpw, tail) : seg_kernel_w32(rpw, tail))
                  : precision == PR_PREC_FP64
                      ? (tail ? seg_kernel_f64_tail(rpw, warm) : seg_kernel_f64(rpw, warm))
                      : (tail ? seg_kernel_f32_tail(rpw, warm) : seg_kernel_f32(rpw, warm));
  return reinterpret_cast<SegFn>(const_cast<void*>(f));
}
GangFn pick_gang(int precision, int rpw, bool weighted = false) {
  if (weighted) return precision == PR_PREC_FP64 ? gang_kernel<double, true>(rpw) : gang_kernel<float, true>(rpw);
  return precision == PR_PREC_FP64 ? gang_kernel<double, false>(rpw) : gang_kernel<float, false>(rpw);
}

}  // namespace


// launch sizes: a segment uses every workgroup slot the device keeps
// resident; a gang launch up to eight workgroups per compute unit
static int32_t grid_for(int rpw, int* grid, int* ggrid) {
  int dev, cus;
  PR_HIP_CHECK(hipGetDevice(&dev));
  PR_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int seg = 1 << 30, gang = 1 << 30;
  for (int prec = 0; prec < 2; ++prec) {
    int occ = 0;
    PR_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)pick_segment(prec, rpw), kThreads, 0));
    seg = std::min(seg, occ);
    PR_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)pick_gang(prec, rpw), kThreads, 0));
    gang = std::min(gang, occ);
  }
  if (seg < 1 || gang < 1) {
    set_error("solve kernels cannot be resident (occupancy 0)");
    return PR_EHIP;
  }
  *grid = std::min(seg, 4) * cus;
  *ggrid = std::min(gang, 8) * cus;
  return PR_OK;
}

// edge-balanced split of rows [vb, ve) into G workgroup ranges; a hub row
// (summed in pieces) counts as one unit
static void balanced_bounds(const std::vector<uint32_t>& ptr, int vb, int ve, int G, int32_t* out) {
  auto w = [&](int r) -> int64_t {
    const uint32_t d = ptr[r + 1] - ptr[r];
    return (d > kHubRow ? 0 : (int64_t)d) + 1;
  };
  int64_t total = 0;
  for (int r = vb; r < ve; ++r) total += w(r);
  out[0] = vb;
  out[G] = ve;
  int r = vb;
  int64_t acc = 0;
  for (int g = 1; g < G; ++g) {
    const int64_t target = total * g / G;
    while (r < ve && acc < target) acc += w(r++);
    out[g] = r;
  }
}

struct GangTables {
  std::vector<GangDesc> gangs;
  std::vector<GangScc> sccs;
  std::vector<int32_t> bounds;
  std::vector<GangHub> hubs;
  std::vector<GangPiece> pieces;
  std::vector<int32_t> piece_ptr;
  std::vector<int32_t> hub_pieces;  // per hub, its piece positions in edge order
  int32_t slots = 0;
};

static void add_gang(const std::vector<uint32_t>& ptr, int G, int vb, int ve, const std::vector<int64_t>& ranks,
                     const std::vector<int32_t>& cvbeg, GangTables& T) {
  GangDesc gd{};
  gd.vbeg = vb;
  gd.vend = ve;
  gd.s0 = (int32_t)T.sccs.size();
  gd.boff = (int32_t)T.bounds.size();
  gd.h0 = (int32_t)T.hubs.size();
  T.bounds.resize(T.bounds.size() + G + 1);
  int32_t* b = T.bounds.data() + gd.boff;
  balanced_bounds(ptr, vb, ve, G, b);
  // pieces per workgroup of this gang, filled below
  std::vector<std::vector<GangPiece>> per_wg(G);
  int rot = 0;
  for (int64_t q : ranks) {
    GangScc sc{};
    sc.rank = (int32_t)q;
    sc.vbeg = q >= 0 ? cvbeg[q] : vb;
    sc.vend = q >= 0 ? cvbeg[q + 1] : ve;
    int f = 0;
    while (f < G && !(b[f + 1] > sc.vbeg && b[f] < b[f + 1])) ++f;
    int l = f;
    while (l + 1 < G && b[l + 1] < sc.vend) ++l;
    sc.wg_first = f;
    sc.wg_last = l;
    sc.pbase = T.slots;
    sc.gidx = (int32_t)T.sccs.size();
    const int nw = l - f + 1;
    int nh = 0;
    for (int r = sc.vbeg; r < sc.vend; ++r) {
      const uint32_t d = ptr[r + 1] - ptr[r];
      if (d <= kHubRow) continue;
      GangHub hb{};
      hb.row = r;
      hb.scc = sc.gidx;
      hb.slot = sc.pbase + nw + nh;
      const int hidx = (int)T.hubs.size();
      const uint32_t np = (d + kHubPiece - 1) / kHubPiece;
      hb.p0 = (int32_t)np;  // piece count for now; turned into a range below
      for (uint32_t j = 0; j < np; ++j) {
        GangPiece pc{};
        pc.ebeg = ptr[r] + j * kHubPiece;
        pc.eend = std::min(ptr[r + 1], pc.ebeg + kHubPiece);
        pc.hub = hidx;
        pc.pad = (int32_t)j;
        per_wg[f + (rot++ % nw)].push_back(pc);
      }
      T.hubs.push_back(hb);
      ++nh;
    }
    sc.nslot = nw + nh;
    T.slots += sc.nslot;
    T.sccs.push_back(sc);
  }
  gd.s1 = (int32_t)T.sccs.size();
  gd.h1 = (int32_t)T.hubs.size();
  // lay the pieces out by workgroup, and give each hub the positions of its
  // pieces in edge order (the combine sums them in that fixed order)
  for (int h = gd.h0; h < gd.h1; ++h) {
    const int32_t np = T.hubs[h].p0;
    T.hubs[h].p0 = (int32_t)T.hub_pieces.size();
    T.hubs[h].p1 = T.hubs[h].p0 + np;
    T.hub_pieces.resize(T.hub_pieces.size() + np);
  }
  gd.poff = (int32_t)T.piece_ptr.size();
  T.piece_ptr.push_back((int32_t)T.pieces.size());
  for (int g = 0; g < G; ++g) {
    for (const GangPiece& pc : per_wg[g]) {
      T.hub_pieces[T.hubs[pc.hub].p0 + pc.pad] = (int32_t)T.pieces.size();
      T.pieces.push_back(pc);
    }
    T.piece_ptr.push_back((int32_t)T.pieces.size());
  }
  T.gangs.push_back(gd);
}
// Plan of the CAC sweep inside each vertex item.  The item's vertices are in
// topological order (sub-levels), so one pass in that order gives each
// vertex's depth (the longest chain of in-item CAC edges ending there; the
// item's longest goes to Item.c) and a cover of the item by vertex-disjoint
// paths: a vertex continues the path of its deepest in-item predecessor that
// no other vertex continues yet (the first such in edge order), else it starts
// a path.  vpath lists the item's vertices path after path, each path in
// order (local index in bits 0-9, kVStart where a path starts), so that one
// lane can walk a whole path with the running value in a register.
// k_item_early then sets bit 16 of vpath[u] for every vertex u with a CAC
// edge into a later vertex item: those publish x the moment they are final,
// the others when their item ends.
__global__ __launch_bounds__(64) void k_item_paths(Item* items, int64_t n_items, const uint32_t* int_ptr,
                                                    const int32_t* int_src, uint32_t* vpath) {
  __shared__ int32_t depth[kVertMax];
  __shared__ int16_t succ[kVertMax];
  __shared__ uint8_t head[kVertMax];
  for (int64_t q = blockIdx.x; q < n_items; q += gridDim.x) {
    const Item it = items[q];
    if (it.kind != ITEM_VERTS) continue;
    if (threadIdx.x == 0) {
      const int nv = it.b - it.a;
      int32_t best = 0;
      for (int i = 0; i < nv; ++i) succ[i] = -1;
      for (int i = 0; i < nv; ++i) {
        const int v = it.a + i;
        int32_t d = 1, pd = 0;
        int pick = -1;
        for (uint32_t e = int_ptr[v]; e < int_ptr[v + 1]; ++e) {
          const int u = int_src[e] - it.a;
          if (u < 0 || u >= i) continue;
          d = max(d, depth[u] + 1);
          if (succ[u] < 0 && depth[u] > pd) {
            pd = depth[u];
            pick = u;
          }
        }
        depth[i] = d;
        head[i] = pick < 0 ? 1 : 0;
        if (pick >= 0) succ[pick] = (int16_t)i;
        best = max(best, d);
      }
      items[q].c = best;
      int pos = 0;
      for (int h = 0; h < nv; ++h) {
        if (!head[h]) continue;
        for (int i = h; i >= 0; i = succ[i]) vpath[it.a + pos++] = (uint32_t)i | (i == h ? kVStart : 0u);
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_item_early(const Item* items, int64_t n_items, const uint32_t* int_ptr,
                                                    const int32_t* int_src, uint32_t* vpath) {
  for (int64_t q = blockIdx.x; q < n_items; q += gridDim.x) {
    const Item it = items[q];
    if (it.kind != ITEM_VERTS) continue;
    for (int v = it.a + (int)threadIdx.x; v < it.b; v += 64)
      for (uint32_t e = int_ptr[v]; e < int_ptr[v + 1]; ++e) {
        const int u = int_src[e];
        if (u < it.a) atomicOr(&vpath[u], kVEarly);
      }
  }
}

// Slots of the rows of workgroup SCCs: each row's in-edges inside its SCC
// cut into groups of up to eight, each group stored as eight 16-bit source
// ids local to the SCC (two per word; the SCC's size pads a short group).
// One 16-byte load gives a thread a whole slot.  A weighted plan also gets
// the eight edge weights of every slot (zero for the pad), in FP64 and FP32.
__global__ __launch_bounds__(256) void k_medium_slots(const Item* items, int64_t n_items, const int32_t* comp_vbeg,
                                                      const uint32_t* int_ptr, const int32_t* int_src,
                                                      const uint32_t* mslot_ptr, uint4* mslot_src,
                                                      const double* int_w, double* mslot_w64, float* mslot_w32) {
  for (int64_t q = blockIdx.x; q < n_items; q += gridDim.x) {
    const Item it = items[q];
    if (it.kind != ITEM_MEDIUM) continue;
    const int vb = comp_vbeg[it.a], ve = comp_vbeg[it.a + 1];
    const uint32_t pad = (uint32_t)(ve - vb);
    if (pad > 65535u) continue;
    for (int v = vb + (int)threadIdx.x; v < ve; v += blockDim.x) {
      const uint32_t e0 = int_ptr[v], e1 = int_ptr[v + 1];
      uint32_t sl = mslot_ptr[v];
      for (uint32_t e = e0; e < e1; e += 8, ++sl) {
        uint32_t w[4];
        for (int m = 0; m < 4; ++m) {
          const uint32_t a0 = e + 2 * m < e1 ? (uint32_t)(int_src[e + 2 * m] - vb) : pad;
          const uint32_t a1 = e + 2 * m + 1 < e1 ? (uint32_t)(int_src[e + 2 * m + 1] - vb) : pad;
          w[m] = a0 | (a1 << 16);
        }
        mslot_src[sl] = make_uint4(w[0], w[1], w[2], w[3]);
        if (int_w) {
          for (int m = 0; m < 8; ++m) {
            const double wt = e + m < e1 ? int_w[e + m] : 0.0;
            mslot_w64[8 * (size_t)sl + m] = wt;
            mslot_w32[8 * (size_t)sl + m] = (float)wt;
          }
        }
      }
    }
  }
}

int32_t make_schedule(Levels& lv, hipStream_t s) {
  PR_TRY(grid_for(lv.opts.rows_per_wave, &lv.grid, &lv.ggrid));
  lv.sgrid = std::max(lv.grid, lv.ggrid);
  const int G = lv.ggrid;  // gang row bounds are per gang workgroup
  const int64_t K = lv.n_comp;
  std::vector<Item> items;
  GangTables T;
  std::vector<Phase> phases;
  int64_t seg_start = 0;
  int64_t r = 0;
  while (r < K) {
    const int lev = lv.h_comp_level[r];
    int64_t e = r;
    while (e < K && lv.h_comp_level[e] == lev) ++e;
    int64_t sc = r;
    while (sc < e && lv.h_comp_class[sc] == 0) ++sc;
    std::vector<int64_t> small, large;
    // vertex items first: the CAC pipelines carry the longest chains
    if (sc < e) {
      const int32_t v0 = lv.h_comp_vbeg[sc], v1 = lv.h_comp_vbeg[e];
      const int32_t vstep = lv.weighted ? kVertMaxW : kVertMax;
      for (int32_t v = v0; v < v1; v += vstep) items.push_back(Item{ITEM_VERTS, v, std::min(v1, v + vstep), 0});
    }
    for (int64_t q = r; q < sc; ++q) {
      const int32_t nv = lv.h_comp_vbeg[q + 1] - lv.h_comp_vbeg[q];
      if (nv <= lv.opts.small_cutoff) small.push_back(q);
      else if (lv.h_comp_int_edges[q] > lv.opts.team_edges) large.push_back(q);
      else items.push_back(Item{ITEM_MEDIUM, (int32_t)q, 0, 0});
    }
    for (size_t i = 0; i < small.size(); i += kWaves) {
      const int64_t a = small[i];
      const int64_t b = small[std::min(small.size() - 1, i + kWaves - 1)] + 1;
      items.push_back(Item{ITEM_SMALL, (int32_t)a, (int32_t)b, 0});
    }
    if (!large.empty()) {
      if ((int64_t)items.size() > seg_start) phases.push_back(Phase{0, (int32_t)seg_start, (int32_t)items.size()});
      seg_start = (int64_t)items.size();
      const int vb = lv.h_comp_vbeg[large.front()], ve = lv.h_comp_vbeg[large.back() + 1];
      phases.push_back(Phase{1, (int32_t)T.gangs.size(), 0});
      add_gang(lv.h_int_ptr, G, vb, ve, large, lv.h_comp_vbeg, T);
    }
    r = e;
  }
  if ((int64_t)items.size() > seg_start) phases.push_back(Phase{0, (int32_t)seg_start, (int32_t)items.size()});
  lv.n_items = (int64_t)items.size();
  lv.n_gangs = (int64_t)T.gangs.size();
  const int64_t n_gscc_cw = (int64_t)T.sccs.size();
  lv.h_gang_rank.clear();
  for (const GangScc& g : T.sccs) lv.h_gang_rank.push_back(g.rank);
  // the whole-graph gang of method PLAIN comes last
  if (!lv.h_full_ptr.empty()) add_gang(lv.h_full_ptr, G, 0, (int)lv.n, std::vector<int64_t>{-1}, lv.h_comp_vbeg, T);
  lv.n_gscc = (int64_t)T.sccs.size();
  lv.n_gslots = T.slots;
  lv.n_ghubs = (int64_t)T.hubs.size();
  lv.n_gpieces = (int64_t)T.pieces.size();
  lv.h_gang_nhub.clear();
  lv.h_gang_sccs.clear();
  for (const GangDesc& gd : T.gangs) {
    lv.h_gang_nhub.push_back(gd.h1 - gd.h0);
    lv.h_gang_sccs.push_back({gd.s0, gd.s1});
  }
  lv.h_gang_hint.assign(2 * T.gangs.size(), 0);
  lv.phases = phases;
  // device copies
  void* old[] = {lv.items, lv.gangs, lv.gsccs, lv.gbounds, lv.gpart, lv.gpmx, lv.gwsum, lv.gdone, lv.wgstats, lv.gpdiff, lv.gnhist,
                 lv.trace, lv.seg_heads, lv.ghubs, lv.gpieces, lv.gpiece_ptr, lv.gpiece_part, lv.ghub_pieces,
                 lv.warm_buf, lv.warm_gws, lv.mslot_ptr, lv.mslot_src, lv.mslot_w64, lv.mslot_w32};
  for (void* q : old)
    if (q) (void)hipFree(q);
  lv.mslot_ptr = nullptr;
  lv.mslot_src = nullptr;
  lv.mslot_w64 = nullptr;
  lv.mslot_w32 = nullptr;
  lv.warm_buf = nullptr;  // sized by the schedule: allocated again on first use
  lv.warm_gws = nullptr;
  lv.items = nullptr;
  lv.gangs = nullptr;
  lv.gsccs = nullptr;
  lv.gbounds = nullptr;
  lv.gpart = nullptr;
  lv.gpmx = nullptr;
  lv.gwsum = nullptr;
  lv.gpdiff = nullptr;
  lv.gnhist = nullptr;
  lv.gdone = nullptr;
  lv.wgstats = nullptr;
  lv.trace = nullptr;
  lv.seg_heads = nullptr;
  lv.ghubs = nullptr;
  lv.gpieces = nullptr;
  lv.gpiece_ptr = nullptr;
  lv.gpiece_part = nullptr;
  lv.ghub_pieces = nullptr;
  auto upload = [&](auto** dst, const auto& vec) -> int32_t {
    using T0 = typename std::remove_reference<decltype(vec)>::type::value_type;
    PR_TRY(dalloc(reinterpret_cast<T0**>(dst), vec.size()));
    if (!vec.empty())
      PR_HIP_CHECK(hipMemcpyAsync(*dst, vec.data(), sizeof(T0) * vec.size(), hipMemcpyHostToDevice, s));
    return PR_OK;
  };
  PR_TRY(upload(&lv.items, items));
  if (!lv.vpath) PR_TRY(dalloc(&lv.vpath, (size_t)std::max<int64_t>(lv.n, 1)));
  if (!items.empty()) {
    const unsigned ng = (unsigned)std::min<size_t>(items.size(), 4096);
    k_item_paths<<<ng, 64, 0, s>>>(lv.items, (int64_t)items.size(), lv.int_ptr, lv.int_src, lv.vpath);
    PR_HIP_CHECK(hipGetLastError());
    k_item_early<<<ng, 64, 0, s>>>(lv.items, (int64_t)items.size(), lv.int_ptr, lv.int_src, lv.vpath);
    PR_HIP_CHECK(hipGetLastError());
  }
  {
    // slot offsets of the rows of workgroup SCCs (every other row owns none)
    std::vector<uint32_t> msp((size_t)lv.n + 1);
    std::vector<std::pair<int32_t, int32_t>> med;
    for (const Item& it : items)
      if (it.kind == ITEM_MEDIUM) med.push_back({lv.h_comp_vbeg[it.a], lv.h_comp_vbeg[it.a + 1]});
    std::sort(med.begin(), med.end());
    uint64_t run = 0;
    size_t mi = 0;
    for (int64_t v = 0; v < lv.n; ++v) {
      while (mi < med.size() && med[mi].second <= v) ++mi;
      msp[v] = (uint32_t)run;
      if (mi < med.size() && med[mi].first <= v && med[mi].second - med[mi].first <= 65535)
        run += (lv.h_int_ptr[v + 1] - lv.h_int_ptr[v] + 7) / 8;
    }
    msp[lv.n] = (uint32_t)run;
    if (run >= (1ull << 32)) {
      set_error("too many SCC slots (%llu)", (unsigned long long)run);
      return PR_EINVAL;
    }
    lv.n_mslots = (int64_t)run;
    PR_TRY(upload(&lv.mslot_ptr, msp));
    PR_TRY(dalloc(&lv.mslot_src, std::max<size_t>(run, 1)));
    if (lv.weighted) {
      PR_TRY(dalloc(&lv.mslot_w64, 8 * std::max<size_t>(run, 1)));
      PR_TRY(dalloc(&lv.mslot_w32, 8 * std::max<size_t>(run, 1)));
    }
    if (run > 0) {
      k_medium_slots<<<(unsigned)std::min<size_t>(items.size(), 4096), 256, 0, s>>>(
          lv.items, (int64_t)items.size(), lv.comp_vbeg, lv.int_ptr, lv.int_src, lv.mslot_ptr, lv.mslot_src,
          lv.weighted ? lv.int_w64 : nullptr, lv.mslot_w64, lv.mslot_w32);
      PR_HIP_CHECK(hipGetLastError());
    }
  }
  PR_TRY(upload(&lv.gangs, T.gangs));
  PR_TRY(upload(&lv.gsccs, T.sccs));
  PR_TRY(upload(&lv.gbounds, T.bounds));
  PR_TRY(upload(&lv.ghubs, T.hubs));
  PR_TRY(upload(&lv.gpieces, T.pieces));
  PR_TRY(upload(&lv.gpiece_ptr, T.piece_ptr));
  PR_TRY(upload(&lv.ghub_pieces, T.hub_pieces));
  PR_TRY(dalloc(&lv.gpiece_part, T.pieces.size()));
  PR_TRY(dalloc(&lv.gpart, 2 * (size_t)T.slots));
  PR_TRY(dalloc(&lv.gpmx, 2 * (size_t)T.slots));
  PR_TRY(dalloc(&lv.gwsum, T.sccs.size()));
  PR_TRY(dalloc(&lv.gpdiff, 2 * (size_t)T.slots));
  PR_TRY(dalloc(&lv.gnhist, 3 * T.sccs.size()));
  PR_TRY(dalloc(&lv.gdone, T.sccs.size()));
  PR_TRY(dalloc(&lv.wgstats, (size_t)lv.sgrid * kWgStats));
  PR_TRY(dalloc(&lv.seg_heads, std::max<size_t>(phases.size(), 1)));
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
    PR_TRY(dalloc(&lv.res_part, 2 * kResBlocks + 8));
  }
  PR_HIP_CHECK(hipStreamSynchronize(s));
  pr_levels_info& I = lv.info;
  I.n_items = lv.n_items;
  I.n_gangs = lv.n_gangs;
  I.n_gang_scc = n_gscc_cw;
  I.v_gang = I.m_gang_internal = I.m_gang_between = 0;
  // the gang SCCs' own rows: a level's gang range can also span smaller
  // SCCs sorted between them (more vertices, fewer internal edges), which
  // their items iterate and the gang skips
  for (const int32_t q : lv.h_gang_rank) {
    const int32_t a = lv.h_comp_vbeg[q], z = lv.h_comp_vbeg[q + 1];
    uint32_t b[2];
    PR_HIP_CHECK(hipMemcpy(&b[0], lv.bnd_ptr + a, sizeof(uint32_t), hipMemcpyDeviceToHost));
    PR_HIP_CHECK(hipMemcpy(&b[1], lv.bnd_ptr + z, sizeof(uint32_t), hipMemcpyDeviceToHost));
    I.v_gang += z - a;
    I.m_gang_internal += lv.h_int_ptr[z] - lv.h_int_ptr[a];
    I.m_gang_between += b[1] - b[0];
  }
  I.n_phases = (int64_t)phases.size();
  I.n_hubs = lv.n_ghubs;
  I.rows_per_wave = lv.opts.rows_per_wave;
  I.small_cutoff = lv.opts.small_cutoff;
  I.team_edges = lv.opts.team_edges;
  I.grid_wgs = lv.sgrid;
  // the three-workgroup tail kernel exists for unweighted plans at 16 or 64
  // rows per wavefront; every other plan runs the two-workgroup one
  const bool w3 = lv.opts.seg_waves == 3 && !lv.weighted && (lv.opts.rows_per_wave == 16 || lv.opts.rows_per_wave == 64);
  I.seg_waves = w3 ? 3 : 2;
  // a new schedule invalidates a captured graph
  lv.drop_graphs();
  // the uploads above read host vectors that end with this function
  PR_HIP_CHECK(hipStreamSynchronize(s));
  return PR_OK;
}

static uint64_t mix64(uint64_t h, uint64_t x) {
  h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

// number of series terms after which every SCC has met the stop rule in
// exact arithmetic: ||P_k||_1 <= c^k ||W'_C||_1 (Sec. 4.4), plus slack for
// rounding; the paper rule uses max(P_k) <= ||P_k||_1 and ||W'_C||_1 <= sumW/(1-c)
static int64_t term_bound(const pr_solve_opts& o, double c, double sumW) {
  double k;
  if (o.stop == PR_STOP_CERT_L1) {
    k = std::ceil(std::log(o.eps * (1.0 - c)) / std::log(c));
  } else {
    const double top = sumW / (1.0 - c);
    k = top <= o.tol ? 1.0 : std::ceil(std::log(o.tol / top) / std::log(c));
  }
  if (!(k >= 1.0)) k = 1.0;
  k += 8.0;
  if (k > (double)o.max_iter) k = (double)o.max_iter;
  return (int64_t)k;
}

// the features of the guess (float4 per vertex) follow the other scratch of
// warm_buf, on a 16-byte boundary
static size_t warm_feat_off(const Levels& lv) {
  const size_t off = 3 * (size_t)lv.n + 3 * (size_t)lv.n_gslots + 2 * (size_t)lv.n_gscc;
  return (off + 1) & ~(size_t)1;
}

// the kernels' view of the plan for the FP64 residual: every edge once, in
// the between-component and inside-component rows, whatever the method
static SolveParams residual_params(const Levels& lv, double c, const double* W) {
  SolveParams q{};
  q.n = (int32_t)lv.n;
  q.c = c;
  q.W = W;
  q.perm = lv.perm;
  q.bnd_ptr = lv.bnd_ptr;
  q.bnd_src = lv.bnd_src;
  q.int_ptr = lv.int_ptr;
  q.int_src = lv.int_src;
  q.inv64 = lv.inv_deg64;
  q.bnd_w = lv.bnd_w64;
  q.int_w64 = lv.int_w64;
  return q;
}

static unsigned residual_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kResBlocks, (n + kThreads - 1) / kThreads));
}

// r = W - (I - c A^T) R in FP64 (R in the caller's order): sum |r| and sum
// |R| to out[0..1], and r itself in the caller's order to rw when not null
static void launch_residual(const Levels& lv, double c, const double* W, const double* R, double* rw, double* out,
                            hipStream_t s) {
  const unsigned g = residual_grid(lv.n);
  k_res_prep<<<g, kThreads, 0, s>>>(R, lv.perm, lv.inv_deg64, lv.n, lv.R, lv.x);
  if (lv.weighted) k_residual<true><<<g, kThreads, 0, s>>>(residual_params(lv, c, W), lv.R, lv.x, rw, lv.res_part);
  else k_residual<false><<<g, kThreads, 0, s>>>(residual_params(lv, c, W), lv.R, lv.x, rw, lv.res_part);
  k_res_sum<<<1, kThreads, 0, s>>>(lv.res_part, (int)g, out);
}

// One solve of the method (no refinement).  signed_w: W is a residual (a
// correction solve).  residual: end with the FP64 residual pass, its sums in
// lv.red[2..3].
static int32_t solve_once(Levels& lv, double c, const double* W, double* R, const pr_solve_opts& o,
                          hipStream_t s, pr_solve_stats* st, bool signed_w, bool residual) {
  int dev;
  PR_HIP_CHECK(hipGetDevice(&dev));
  if (dev != lv.device) {
    set_error("plan lives on device %d but device %d is current", lv.device, dev);
    return PR_EINVAL;
  }
  const auto host_t0 = std::chrono::steady_clock::now();
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
  p.bnd_w = lv.bnd_w64;
  p.int_w64 = plain ? lv.full_w64 : lv.int_w64;
  p.int_w32 = plain ? lv.full_w32 : lv.int_w32;
  p.vpath = lv.vpath;
  p.direct_max = plain ? 0 : o.small_direct;
  p.tail = (o.tail_estimate && o.stop == PR_STOP_CERT_L1) ? 1 : 0;
  p.signed_w = signed_w ? 1 : 0;
  p.gs_blocks = plain ? 0 : o.gs_blocks;
  p.mslot_ptr = lv.mslot_ptr;
  p.mslot_src = lv.mslot_src;
  p.mslot_w64 = lv.mslot_w64;
  p.mslot_w32 = lv.mslot_w32;
  p.inv32 = lv.inv_deg32;
  p.inv64 = lv.inv_deg64;
  p.x = lv.x;
  p.R = lv.R;
  p.wprime = lv.wprime;
  p.y0 = lv.y0;
  p.y1 = lv.y1;
  p.comp_vbeg = lv.comp_vbeg;
  p.iters = lv.iters;
  p.lastnorm = lv.lastnorm;
  p.counters = lv.counters;
  p.wgstats = lv.wgstats;
  p.gangs = lv.gangs;
  p.gscc = lv.gsccs;
  p.gbounds = lv.gbounds;
  p.gpart = lv.gpart;
  p.gpmx = lv.gpmx;
  p.gwsum = lv.gwsum;
  p.gpdiff = lv.gpdiff;
  p.gnhist = lv.gnhist;
  p.gdone = lv.gdone;
  p.ghubs = lv.ghubs;
  p.gpieces = lv.gpieces;
  p.gpiece_ptr = lv.gpiece_ptr;
  p.ghub_pieces = lv.ghub_pieces;
  p.gpiece_part = lv.gpiece_part;
  p.n_gslots = lv.n_gslots;
  p.timeout = (unsigned long long)clock_khz * 1000ull * 30ull;  // 30 s
  if (o.warm_start && !plain && lv.weighted) {
    set_error("warm_start is not available for a weighted plan (the network's features are those of unweighted graphs)");
    return PR_EINVAL;
  }
  if (o.warm_start && !plain) {
    const Mlp* m = reinterpret_cast<const Mlp*>(o.warm_start);
    if (m->device != lv.device) {
      set_error("the warm-start network lives on device %d, the plan on device %d", m->device, lv.device);
      return PR_EINVAL;
    }
    if (!lv.warm_buf) {
      PR_TRY(dalloc(&lv.warm_buf, warm_feat_off(lv) + 2 * (size_t)lv.n));
      PR_TRY(dalloc(&lv.warm_gws, std::max<int64_t>(lv.n_gscc, 1)));
    }
    p.gmlp = m->packed;
    if (o.warm_scope == 1) p.mlp = m->packed;  // every SCC, not only the gangs'
    p.wr0 = lv.warm_buf;
    p.wx = lv.warm_buf + lv.n;
    p.wres = lv.warm_buf + 2 * lv.n;
    p.gwp1 = lv.warm_buf + 3 * lv.n;
    p.gwr0 = p.gwp1 + lv.n_gslots;
    p.gwm0 = p.gwr0 + lv.n_gslots;
    p.gwn = p.gwm0 + lv.n_gslots;
    p.gwm = p.gwn + lv.n_gscc;
    p.gws = lv.warm_gws;
    p.wfeat = reinterpret_cast<float4*>(lv.warm_buf + warm_feat_off(lv));
  }
  if (o.trace == 1) {  // timeline of the segment items (tests / profiling)
    if (!lv.trace) {
      hipError_t e = hipMalloc(&lv.trace, sizeof(unsigned long long) * 4 * std::max<int64_t>(lv.n_items, 1));
      if (e != hipSuccess) {
        set_error("hipMalloc(trace) failed: %s", hipGetErrorString(e));
        return PR_ENOMEM;
      }
    }
    p.trace = lv.trace;
  }
  const int64_t K = std::max<int64_t>(lv.n_comp, 1);
  const unsigned init_blocks = (unsigned)std::min<int64_t>(4096, (lv.n + kThreads - 1) / kThreads + 1);

  // weights must be non-negative and finite (a negative x would read as "not
  // ready"); checked, and summed for the term bound, before the solve runs
  k_zero_counters<<<1, 64, 0, s>>>(lv.counters);
  k_init<<<init_blocks, kThreads, 0, s>>>(p, K, lv.n_gscc, (int64_t)lv.sgrid * kWgStats, lv.seg_heads,
                                              (int64_t)lv.phases.size());
  k_reduce1<<<kRedBlocks, kThreads, 0, s>>>(W, lv.n, lv.lastnorm, 0, lv.red + 8);
  PR_HIP_CHECK(hipGetLastError());
  unsigned long long badw = 0;
  std::vector<double> wparts(2 * kRedBlocks);
  PR_HIP_CHECK(hipMemcpyAsync(&badw, lv.counters + C_BAD_W, sizeof(badw), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipMemcpyAsync(wparts.data(), lv.red + 8, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  if (badw) {
    set_error("W has a negative or non-finite entry");
    return PR_EINVAL;
  }
  double sumW = 0.0;
  for (int i = 0; i < kRedBlocks; ++i) sumW += wparts[2 * i];
  const int64_t kb = term_bound(o, c, sumW);
  SegFn seg = pick_segment(o.precision, lv.opts.rows_per_wave, p.mlp != nullptr, p.tail != 0, lv.weighted);
  if (p.tail && !p.mlp && !lv.weighted && lv.opts.seg_waves == 3) {
    const void* f3 = seg_kernel_tail_w3(lv.opts.rows_per_wave, o.precision == PR_PREC_FP64);
    if (f3) seg = reinterpret_cast<SegFn>(const_cast<void*>(f3));
  }
  if (p.gs_blocks > 0)
    seg = reinterpret_cast<SegFn>(const_cast<void*>(seg_kernel_gs(lv.opts.rows_per_wave, o.precision == PR_PREC_FP64)));
  // the variants with the starting guess, the tail estimate or edge weights
  // need more registers: size their grid to what stays resident
  unsigned seg_grid = (unsigned)lv.grid;
  if (p.mlp || p.tail || lv.weighted || p.gs_blocks) {
    int occ = 0, cus = 0;
    PR_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)seg, kThreads, 0));
    PR_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, lv.device));
    seg_grid = (unsigned)std::max(1, std::min(lv.grid, std::max(occ, 1) * cus));
  }
  const GangFn gk = pick_gang(o.precision, lv.opts.rows_per_wave, lv.weighted);
  hipEvent_t ev0, ev1;
  PR_HIP_CHECK(hipEventCreate(&ev0));
  PR_HIP_CHECK(hipEventCreate(&ev1));
  const HubFn hk = pick_hubs(o.precision);
  // optional per-launch timing: an event after every launch, so launch i
  // spans events i and i+1 on the solve's stream
  const bool timing = o.kernel_timing == 1 && !o.use_graph;
  std::vector<int> fam;
  auto mark = [&](int f) -> int32_t {
    if (!timing) return PR_OK;
    const size_t i = fam.size() + 1;
    while (lv.kev.size() <= i) {
      hipEvent_t e;
      PR_HIP_CHECK(hipEventCreate(&e));
      lv.kev.push_back(e);
    }
    PR_HIP_CHECK(hipEventRecord(lv.kev[i], s));
    fam.push_back(f);
    return PR_OK;
  };
  const WarmGangFn wk = pick_gang_warm(o.precision, lv.opts.rows_per_wave);
  // A gang runs one launch per term up to a bound fixed before the solve
  // (the launches after its SCCs stop return at once).  Once a solve of this
  // plan has shown how many terms a gang needs, later solves launch that many
  // plus a margin instead of the worst case; a solve whose gang reaches the
  // shorter bound without its stop rule is run again with the worst case, so
  // results never depend on the bound.
  auto hint_at = [&](int gang) -> size_t { return (size_t)(p.tail ? 1 : 0) * lv.h_gang_sccs.size() + gang; };
  auto budget = [&](int gang) -> int64_t {
    if (o.cold) return kb;
    const int64_t h = lv.h_gang_hint[hint_at(gang)];
    return h > 0 ? std::min(kb, h + std::max<int64_t>(4, h / 4)) : kb;
  };
  std::vector<int> gangs_run;
  if (plain) {
    gangs_run.push_back((int)lv.n_gangs);
  } else {
    for (const Phase& ph : lv.phases)
      if (ph.kind == 1) gangs_run.push_back(ph.a);
  }
  auto launch_gang = [&](int gang) -> int32_t {
    const int nh = lv.h_gang_nhub[gang];
    const int64_t kg = budget(gang);
    for (int64_t k = 0; k <= kg + 1; ++k) {
      const int fin = k == kg + 1 ? 1 : 0;
      hipLaunchKernelGGL(gk, dim3(lv.ggrid), dim3(kThreads), 0, s, p, gang, (int)k, fin);
      PR_TRY(mark(1));
      if (nh > 0 && !fin) {
        hipLaunchKernelGGL(hk, dim3((nh + kWaves - 1) / kWaves), dim3(kThreads), 0, s, p, gang, (int)k);
        PR_TRY(mark(2));
      }
      if (k == 0 && p.gmlp) {  // the starting guess of the gang's SCCs
        for (int step = 0; step < 3; ++step) {
          hipLaunchKernelGGL(wk, dim3(lv.ggrid), dim3(kThreads), 0, s, p, gang, step);
          PR_TRY(mark(1));
          if (step == 0) {
            hipLaunchKernelGGL(k_gang_warm_net, dim3(lv.ggrid), dim3(kThreads), 0, s, p, gang);
            PR_TRY(mark(1));
          }
        }
      }
    }
    return PR_OK;
  };
  auto launch_all = [&](bool graph_mode) -> int32_t {
    if (graph_mode) {
      k_zero_counters<<<1, 64, 0, s>>>(lv.counters);
      k_init<<<init_blocks, kThreads, 0, s>>>(p, K, lv.n_gscc, (int64_t)lv.sgrid * kWgStats, lv.seg_heads,
                                              (int64_t)lv.phases.size());
    }
    if (plain) {
      PR_TRY(launch_gang((int)lv.n_gangs));  // the whole-graph gang
    } else {
      for (size_t pi = 0; pi < lv.phases.size(); ++pi) {
        const Phase& ph = lv.phases[pi];
        if (ph.kind == 1) {
          PR_TRY(launch_gang(ph.a));
        } else {
          SolveParams q = p;
          q.items = lv.items + ph.a;
          q.n_items = ph.b - ph.a;
          q.item_base = ph.a;
          q.seg_head = lv.seg_heads + pi;
          void* args[] = {&q};
          PR_HIP_CHECK(hipLaunchKernel((const void*)seg, dim3(seg_grid), dim3(kThreads), args, 0, s));
          PR_TRY(mark(0));
        }
      }
    }
    k_reduce1<<<kRedBlocks, kThreads, 0, s>>>(R, lv.n, lv.lastnorm, plain ? 1 : lv.n_comp, lv.red + 8);
    k_reduce2<<<1, kThreads, 0, s>>>(lv.red + 8, lv.red, lv.wgstats, lv.sgrid, lv.counters);
    if (residual) launch_residual(lv, c, W, R, nullptr, lv.red + 2, s);
    PR_HIP_CHECK(hipGetLastError());
    PR_TRY(mark(3));
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
    key = mix64(key, (uint64_t)kb);
    key = mix64(key, (uint64_t)(o.stop * 16 + o.precision * 4 + o.method));
    key = mix64(key, (uint64_t)o.small_direct);
    key = mix64(key, (uint64_t)o.tail_estimate);
    key = mix64(key, (uint64_t)(uintptr_t)seg);  // the segment kernel variant (seg_waves)
    key = mix64(key, (uint64_t)o.gs_blocks);
    key = mix64(key, (uint64_t)(o.trace == 1));
    key = mix64(key, (uint64_t)(uintptr_t)p.mlp);
    key = mix64(key, (uint64_t)(uintptr_t)p.gmlp);
    key = mix64(key, (uint64_t)(signed_w ? 2 : 0) + (residual ? 1 : 0));
    for (int gg : gangs_run) key = mix64(key, (uint64_t)budget(gg));
    Levels::GraphEntry* ge = nullptr;
    for (Levels::GraphEntry& e : lv.graphs)
      if (e.key == key) ge = &e;
    if (!ge) {
      if (lv.graphs.size() >= Levels::kGraphCache) {  // drop the least recently used
        auto old = std::min_element(lv.graphs.begin(), lv.graphs.end(),
                                    [](const Levels::GraphEntry& a, const Levels::GraphEntry& b) {
                                      return a.last_use < b.last_use;
                                    });
        if (old->exec) (void)hipGraphExecDestroy(old->exec);
        if (old->graph) (void)hipGraphDestroy(old->graph);
        lv.graphs.erase(old);
      }
      if (!lv.cap_stream) PR_HIP_CHECK(hipStreamCreateWithFlags(&lv.cap_stream, hipStreamNonBlocking));
      const hipStream_t caller = s;
      s = lv.cap_stream;
      PR_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      rc = launch_all(true);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(s, &g);
      s = caller;
      if (rc) return rc;
      if (ce != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ce));
        return PR_EHIP;
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
        return PR_EHIP;
      }
      lv.graphs.push_back({key, g, ex, 0});
      ge = &lv.graphs.back();
    }
    ge->last_use = ++lv.graph_clock;
    PR_HIP_CHECK(hipEventRecord(ev0, s));
    PR_HIP_CHECK(hipGraphLaunch(ge->exec, s));
    PR_HIP_CHECK(hipEventRecord(ev1, s));
  } else {
    PR_HIP_CHECK(hipEventRecord(ev0, s));
    if (timing) {
      if (lv.kev.empty()) {
        hipEvent_t e;
        PR_HIP_CHECK(hipEventCreate(&e));
        lv.kev.push_back(e);
      }
      PR_HIP_CHECK(hipEventRecord(lv.kev[0], s));
    }
    rc = launch_all(false);
    if (rc) return rc;
    PR_HIP_CHECK(hipEventRecord(ev1, s));
  }
  unsigned long long cnt[C_COUNT];
  double red[4] = {0.0, 0.0, 0.0, 0.0};
  PR_HIP_CHECK(hipMemcpyAsync(cnt, lv.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipMemcpyAsync(red, lv.red, sizeof(red), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  float ms = 0.f;
  PR_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (cnt[C_ERROR] == 1ull) {
    set_error("internal: a dependency wait timed out");
    return PR_EHIP;
  }
  if (cnt[C_ERROR] || cnt[C_BAD_W] > 1ull) {
    // the kernels only OR 1 into these slots: anything else was written by
    // something that does not own them (a counter-layout error)
    set_error("internal: counter layout error (error slot %llu, weight slot %llu)", cnt[C_ERROR], cnt[C_BAD_W]);
    return PR_EHIP;
  }
  if (!gangs_run.empty()) {
    // terms each gang needed; a gang cut by a shortened bound is run again
    std::vector<int32_t> gd((size_t)std::max<int64_t>(lv.n_gscc, 1));
    PR_HIP_CHECK(hipMemcpy(gd.data(), lv.gdone, sizeof(int32_t) * gd.size(), hipMemcpyDeviceToHost));
    bool cut = false;
    for (int gg : gangs_run) {
      int64_t need = 0;
      for (int32_t si = lv.h_gang_sccs[gg].first; si < lv.h_gang_sccs[gg].second; ++si)
        need = std::max<int64_t>(need, gd[si]);
      if (budget(gg) < kb && need >= budget(gg)) {
        lv.h_gang_hint[hint_at(gg)] = 0;
        cut = true;
      } else {
        lv.h_gang_hint[hint_at(gg)] = std::max(lv.h_gang_hint[hint_at(gg)], need);
      }
    }
    if (cut) return solve_once(lv, c, W, R, o, s, st, signed_w, residual);
  }
  local.edge_iters = (int64_t)cnt[S_EDGE_ITERS] + (plain ? 0 : (lv.info.m_between + lv.info.m_cac_internal));
  local.iters_max = (int64_t)cnt[S_ITERS_MAX];
  local.iters_sum = (int64_t)cnt[S_ITERS_SUM];
  local.n_iterated = (int64_t)cnt[S_N_ITERATED];
  local.n_not_converged = (int64_t)cnt[S_NOT_CONV];
  local.ws_accepted = (int64_t)cnt[S_WS_ACC];
  local.ws_rejected = (int64_t)cnt[S_WS_REJ];
  local.r_sum = red[0];
  local.cert_abs = c / (1.0 - c) * red[1];
  local.cert_rel = red[0] > 0.0 ? local.cert_abs / red[0] : 0.0;
  local.cert_trunc_rel = local.cert_rel;
  if (residual) {  // the FP64 residual bound replaces the truncation bound
    local.res_l1 = red[2];
    local.cert_abs = red[2] / (1.0 - c);
    local.cert_rel = red[3] > 0.0 ? local.cert_abs / red[3] : (red[2] > 0.0 ? INFINITY : 0.0);
  }
  local.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host_t0).count();
  local.kernel_ms = ms;
  local.vert_iters = (int64_t)cnt[S_VERT_ITERS] + (plain ? 0 : (lv.n - lv.info.v_scc));
  if (timing && !plain && !lv.h_gang_rank.empty()) {
    std::vector<int32_t> it(lv.n_comp);
    PR_HIP_CHECK(hipMemcpy(it.data(), lv.iters, sizeof(int32_t) * lv.n_comp, hipMemcpyDeviceToHost));
    for (int32_t r : lv.h_gang_rank) {
      local.gang_edge_iters += (int64_t)it[r] * lv.h_comp_int_edges[r];
      local.gang_vert_iters += (int64_t)it[r] * (lv.h_comp_vbeg[r + 1] - lv.h_comp_vbeg[r]);
    }
  }
  for (size_t i = 0; i < fam.size(); ++i) {
    float d = 0.f;
    PR_HIP_CHECK(hipEventElapsedTime(&d, lv.kev[i], lv.kev[i + 1]));
    local.kt_ms[fam[i]] += d;
    local.kt_count[fam[i]] += 1;
  }
  if (st) *st = local;
  return local.n_not_converged ? PR_NOT_CONVERGED : PR_OK;
}

// The solve of pr_solve: one solve of the method, then (refine >= 0) the FP64
// residual certificate, and while that bound exceeds eps (CERT rule) up to
// `refine` rounds of iterative refinement: the residual r in the caller's
// order, a correction solve (I - c A^T) d = r by the same method and
// precision to the looser target 0.25 eps / cert (its FP32 rounding is
// relative to d, which is about cert times smaller than R), R += d, and the
// residual again (Sec. 4.4: ||R - R*||_1 <= ||r||_1 / (1 - c)).
int32_t solve_levels(Levels& lv, double c, const double* W, double* R, const pr_solve_opts& o_in,
                     hipStream_t s, pr_solve_stats* st) {
  const auto host_t0 = std::chrono::steady_clock::now();
  pr_solve_opts o = o_in;
  if (o.precision == PR_PREC_AUTO)  // FP32 terms leave about 2^-24 / (1 - c) of relative error
    o.precision = (o.stop != PR_STOP_CERT_L1 || o.eps >= std::ldexp(1.0, -23) / (1.0 - c)) ? PR_PREC_MIXED
                                                                                         : PR_PREC_FP64;
  const bool residual = o.refine >= 0 && lv.n > 0;
  pr_solve_stats a{};
  int32_t rc = solve_once(lv, c, W, R, o, s, &a, false, residual);
  if (rc < 0) return rc;
  const int rounds = o.refine == 0 ? 2 : std::max(o.refine, 0);
  bool refined_to_eps = true;
  if (residual && o.stop == PR_STOP_CERT_L1) {
    while (a.cert_rel > o.eps && a.res_l1 > 0.0 && a.refine_rounds < rounds) {
      if (!lv.res_w) {
        PR_TRY(dalloc(&lv.res_w, (size_t)lv.n));
        PR_TRY(dalloc(&lv.res_d, (size_t)lv.n));
      }
      launch_residual(lv, c, W, R, lv.res_w, lv.red + 2, s);
      PR_HIP_CHECK(hipGetLastError());
      pr_solve_opts oc = o;
      oc.warm_start = nullptr;
      oc.trace = 0;
      oc.refine = -1;
      oc.eps = std::min(0.5, 0.25 * o.eps / a.cert_rel);
      pr_solve_stats b{};
      rc = solve_once(lv, c, lv.res_w, lv.res_d, oc, s, &b, true, false);
      if (rc < 0) return rc;
      k_add<<<residual_grid(lv.n), kThreads, 0, s>>>(R, lv.res_d, lv.n);
      launch_residual(lv, c, W, R, nullptr, lv.red + 2, s);
      PR_HIP_CHECK(hipGetLastError());
      double red[4];
      PR_HIP_CHECK(hipMemcpyAsync(red, lv.red, sizeof(red), hipMemcpyDeviceToHost, s));
      PR_HIP_CHECK(hipStreamSynchronize(s));
      a.edge_iters += b.edge_iters;
      a.vert_iters += b.vert_iters;
      a.iters_sum += b.iters_sum;
      a.iters_max = std::max(a.iters_max, b.iters_max);
      a.n_iterated += b.n_iterated;
      a.n_not_converged += b.n_not_converged;
      a.kernel_ms += b.kernel_ms;
      for (int f = 0; f < 4; ++f) {
        a.kt_ms[f] += b.kt_ms[f];
        a.kt_count[f] += b.kt_count[f];
      }
      a.gang_edge_iters += b.gang_edge_iters;
      a.gang_vert_iters += b.gang_vert_iters;
      a.res_l1 = red[2];
      a.r_sum = red[3];
      a.cert_abs = red[2] / (1.0 - c);
      a.cert_rel = red[3] > 0.0 ? a.cert_abs / red[3] : INFINITY;
      a.refine_rounds += 1;
    }
    refined_to_eps = !(a.cert_rel > o.eps);
  }
  a.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host_t0).count();
  a.precision_used = o.precision;
  if (st) *st = a;
  return (a.n_not_converged || !refined_to_eps) ? PR_NOT_CONVERGED : PR_OK;
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
  if (what == 4) {  // item timeline of the last traced solve: n_items x {wg | kind << 32, start, ready, end}
    if (!lv.trace) {
      set_error("no traced solve yet");
      return PR_EINVAL;
    }
    if (lv.n_items)
      PR_HIP_CHECK(hipMemcpy(host_out, lv.trace, sizeof(unsigned long long) * 4 * lv.n_items, hipMemcpyDeviceToHost));
    return PR_OK;
  }
  if (what == 3) {  // per-workgroup counters of the last solve: grid_wgs x 16 uint64
    PR_HIP_CHECK(hipMemcpy(host_out, lv.wgstats, sizeof(unsigned long long) * kWgStats * lv.sgrid,
                           hipMemcpyDeviceToHost));
    return PR_OK;
  }
  if (what == 5) {  // the plan's items: n_items x {kind, a, b, c} (int32)
    if (lv.n_items)
      PR_HIP_CHECK(hipMemcpy(host_out, lv.items, sizeof(Item) * lv.n_items, hipMemcpyDeviceToHost));
    return PR_OK;
  }
  if (what == 6) {  // per component rank: first plan position (int32[n_comp + 1])
    memcpy(host_out, lv.h_comp_vbeg.data(), sizeof(int32_t) * (K + 1));
    return PR_OK;
  }
  if (what == 7) {  // per component rank: the partition's component id (int32[n_comp])
    if (K) memcpy(host_out, lv.h_comp_id_of_rank.data(), sizeof(int32_t) * K);
    return PR_OK;
  }
  set_error("unknown debug array %d", what);
  return PR_EINVAL;
}
