// The intermediate step of Sec. 4.2 on the device: component order, vertex
// renumbering, split of the edges into "between components" and "inside a
// component" pull CSRs, 1/outdeg, and the work list of the solve kernel.
//
// Component order (Sec. 4.2): level descending, then kind (SCC, CAC with two
// or more vertices, one-vertex component), then size descending, ties by
// component id.  Vertices are laid out component by component in that
// order.  Inside a CAC they follow the reverse of the order in which the
// depth-first search closed their SCCs, which is a topological order of the
// CAC's edges (Sec. 4.3.1 needs every in-edge of a vertex used before the
// vertex itself).  Inside an SCC, where any order is valid, they are sorted
// by out-degree, highest first, so the most-gathered terms share cache
// lines.  Because levels are laid out from the highest down,
// every edge between components points from a lower position to a higher
// one, and inside a pull row the sources from other components (all at
// higher levels) come before the sources of the vertex's own component.
#include <algorithm>
#include <cstring>

#include "devsort.h"

namespace prlib {

namespace {

constexpr int kB = 256;

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kB - 1) / kB); }

__global__ void k_comp_key_size(const int32_t* size, int64_t K, uint32_t maxsize, uint32_t* key, uint32_t* val) {
  int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (k >= K) return;
  key[k] = maxsize - (uint32_t)size[k];
  val[k] = (uint32_t)k;
}

__global__ void k_comp_key_level(const int32_t* level, const uint8_t* type, const int32_t* size,
                                 const uint32_t* val, int64_t K, int32_t maxlevel, uint32_t* key) {
  int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (r >= K) return;
  const uint32_t k = val[r];
  const uint32_t cls = type[k] ? 0u : (size[k] >= 2 ? 1u : 2u);
  key[r] = (uint32_t)(maxlevel - level[k]) * 3u + cls;
}

__global__ void k_comp_rank(const uint32_t* id_of_rank, int64_t K, const int32_t* size, int32_t* rank_of_id,
                            uint32_t* size_by_rank) {
  int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (r >= K) return;
  const uint32_t k = id_of_rank[r];
  rank_of_id[k] = (int32_t)r;
  size_by_rank[r] = (uint32_t)size[k];
}

__global__ void k_topo_list(const int32_t* emit_pos, int64_t n, uint32_t* list) {
  int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (v >= n) return;
  list[n - 1 - emit_pos[v]] = (uint32_t)v;
}

// secondary vertex key: inside an SCC, out-degree descending (the vertices
// gathered most often end up next to each other, so their terms share cache
// lines); every other vertex keeps its topological position (key 0)
constexpr uint32_t kDegKeyMax = (1u << 20) - 1;
__global__ void k_vertex_degkey(const uint32_t* list, int64_t n, const int64_t* row_ptr, const int32_t* comp,
                                const uint8_t* ctype, uint32_t* key) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = list[i];
  if (!ctype[comp[v]]) {
    key[i] = 0u;
    return;
  }
  const int64_t d = row_ptr[v + 1] - row_ptr[v];
  key[i] = kDegKeyMax - (uint32_t)(d < (int64_t)kDegKeyMax ? d : (int64_t)kDegKeyMax);
}

__global__ void k_vertex_key(const uint32_t* list, int64_t n, const int32_t* comp, const int32_t* rank_of_id,
                             uint32_t* key) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  key[i] = (uint32_t)rank_of_id[comp[list[i]]];
}

__global__ void k_perm_inverse(const uint32_t* perm, int64_t n, int32_t* perm_out, int32_t* iperm) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = perm[i];
  perm_out[i] = (int32_t)v;
  iperm[v] = (int32_t)i;
}

// out-degree without self-loops, in plan order, and its reciprocals
__global__ void k_degrees(const int64_t* row_ptr, const int32_t* col, const int32_t* perm, int64_t n,
                          int32_t keep_loops, uint32_t* odeg, float* inv32, double* inv64) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int32_t u = perm[i];
  uint32_t d = 0;
  for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) d += (col[e] != u || keep_loops);
  odeg[i] = d;
  inv64[i] = d ? 1.0 / (double)d : 0.0;
  inv32[i] = d ? (float)(1.0 / (double)d) : 0.0f;
}

// edges in plan-source order: key = plan destination, value = plan source
__global__ void k_emit_edges(const int64_t* row_ptr, const int32_t* col, const int32_t* perm,
                             const int32_t* iperm, const uint32_t* optr, int64_t n, int32_t keep_loops,
                             uint32_t* dkey, uint32_t* sval) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int32_t u = perm[i];
  uint32_t pos = optr[i];
  for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
    const int32_t w = col[e];
    if (w == u && !keep_loops) continue;
    dkey[pos] = (uint32_t)iperm[w];
    sval[pos] = (uint32_t)i;
    ++pos;
  }
}

// weighted graph (Def. 3.4): s_u = total weight of u's out-edges (loops only
// with keep_loops) and 1/s_u; a vertex whose out-edges all weigh zero acts
// as dangling (1/s_u = 0).  odeg keeps the number of edges.
__global__ void k_degrees_w(const int64_t* row_ptr, const int32_t* col, const double* w, const int32_t* perm,
                            int64_t n, int32_t keep_loops, uint32_t* odeg, float* inv32, double* inv64) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int32_t u = perm[i];
  uint32_t d = 0;
  double sw = 0.0;
  for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
    if (col[e] != u || keep_loops) {
      ++d;
      sw += w[e];
    }
  }
  odeg[i] = d;
  inv64[i] = sw > 0.0 ? 1.0 / sw : 0.0;
  inv32[i] = sw > 0.0 ? (float)(1.0 / sw) : 0.0f;
}

// weighted graph: as k_emit_edges, with the edge's position in plan-source
// order as the sort value and the source and weight stored by position
__global__ void k_emit_edges_w(const int64_t* row_ptr, const int32_t* col, const double* w, const int32_t* perm,
                               const int32_t* iperm, const uint32_t* optr, int64_t n, int32_t keep_loops,
                               uint32_t* dkey, uint32_t* pval, uint32_t* spos, double* wpos) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int32_t u = perm[i];
  uint32_t pos = optr[i];
  for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
    const int32_t v = col[e];
    if (v == u && !keep_loops) continue;
    dkey[pos] = (uint32_t)iperm[v];
    pval[pos] = pos;
    spos[pos] = (uint32_t)i;
    wpos[pos] = w[e];
    ++pos;
  }
}

// after the stable sort by destination: source and weight of every edge
__global__ void k_edge_gather(const uint32_t* pval, const uint32_t* spos, const double* wpos, int64_t m,
                              uint32_t* sval, double* wsort) {
  int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e >= m) return;
  const uint32_t q = pval[e];
  sval[e] = spos[q];
  wsort[e] = wpos[q];
}

__global__ void k_split_copy_w(const uint32_t* full_ptr, const double* wsort, const uint32_t* bptr,
                               const uint32_t* iptr, int64_t n, double* bw, double* iw64, float* iw32) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const uint32_t lo = full_ptr[i];
  const uint32_t nb = bptr[i + 1] - bptr[i];
  for (uint32_t j = 0; j < nb; ++j) bw[bptr[i] + j] = wsort[lo + j];
  const uint32_t ni = iptr[i + 1] - iptr[i];
  for (uint32_t j = 0; j < ni; ++j) {
    const double v = wsort[lo + nb + j];
    iw64[iptr[i] + j] = v;
    iw32[iptr[i] + j] = (float)v;
  }
}

__global__ void k_to_f32(const double* a, int64_t m, float* b) {
  int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < m) b[e] = (float)a[e];
}

__global__ void k_count_rows(const uint32_t* dkey, int64_t m, uint32_t* cnt) {
  int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e >= m) return;
  atomicAdd(&cnt[dkey[e]], 1u);
}

__global__ void k_vertex_comp_begin(const uint32_t* perm, const int32_t* comp, const int32_t* rank_of_id,
                                    const int32_t* comp_vbeg, int64_t n, int32_t* vbeg_of) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  vbeg_of[i] = comp_vbeg[rank_of_id[comp[perm[i]]]];
}

// rows are sorted by source; sources before the row's component start are
// in other components (higher levels), the rest are inside the component
__global__ void k_split_count(const uint32_t* full_ptr, const uint32_t* src, const int32_t* vbeg_of, int64_t n,
                              uint32_t* bcnt, uint32_t* icnt) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const uint32_t lo = full_ptr[i], hi = full_ptr[i + 1];
  const uint32_t cut = (uint32_t)vbeg_of[i];
  uint32_t a = lo, b = hi;  // first position with src >= cut
  while (a < b) {
    uint32_t mid = a + (b - a) / 2;
    if (src[mid] < cut) a = mid + 1;
    else b = mid;
  }
  bcnt[i] = a - lo;
  icnt[i] = hi - a;
}

__global__ void k_split_copy(const uint32_t* full_ptr, const uint32_t* src, const uint32_t* bptr,
                             const uint32_t* iptr, int64_t n, int32_t* bsrc, int32_t* isrc) {
  int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const uint32_t lo = full_ptr[i];
  const uint32_t nb = bptr[i + 1] - bptr[i];
  for (uint32_t j = 0; j < nb; ++j) bsrc[bptr[i] + j] = (int32_t)src[lo + j];
  const uint32_t ni = iptr[i + 1] - iptr[i];
  for (uint32_t j = 0; j < ni; ++j) isrc[iptr[i] + j] = (int32_t)src[lo + nb + j];
}

__global__ void k_comp_int_edges(const uint32_t* iptr, const int32_t* comp_vbeg, int64_t K, uint32_t* out) {
  int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (r >= K) return;
  out[r] = iptr[comp_vbeg[r + 1]] - iptr[comp_vbeg[r]];
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

}  // namespace


void Levels::drop_graphs() {
  for (GraphEntry& g : graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  graphs.clear();
}

Levels::~Levels() {
  void* ps[] = {perm, comp_vbeg, comp_rank_of_id, comp_id_of_rank, bnd_ptr, bnd_src, int_ptr, int_src,
                full_ptr, full_src, inv_deg32, inv_deg64, items, gangs, gsccs, gbounds, gpart, gpmx, gpdiff, gnhist,
                gwsum, gdone, x, R, wprime, y0, y1, iters, lastnorm, counters, red, wgstats, trace,
                seg_heads, ghubs, gpieces, gpiece_ptr, gpiece_part, ghub_pieces, warm_buf, warm_gws, vpath,
                mslot_ptr, mslot_src, res_part, res_w, res_d, bnd_w64, int_w64, int_w32, full_w64, full_w32,
                mslot_w64, mslot_w32};
  drop_graphs();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (hipEvent_t e : kev) (void)hipEventDestroy(e);
  for (void* p : ps)
    if (p) (void)hipFree(p);
}

int32_t build_levels(const Partition& P, const int64_t* h_row_ptr, const int32_t* h_col, const double* h_weight,
                     const pr_build_opts& opts, hipStream_t s, Levels& lv) {
  const int64_t n = P.n;
  const int64_t K = P.n_comp;
  const int64_t m_in = h_row_ptr[n];
  PR_HIP_CHECK(hipGetDevice(&lv.device));
  lv.n = n;
  lv.n_comp = K;
  lv.n_levels = P.n_levels;
  lv.opts = opts;
  lv.graph_hash = P.graph_hash;
  lv.weighted = h_weight != nullptr;
  if (lv.weighted) lv.weight_hash = hash_weights(m_in, h_weight);
  DevScratch scr;
  // ---- uploads
  int64_t* d_rp;
  int32_t *d_col, *d_comp, *d_clevel, *d_csize, *d_emit;
  uint8_t* d_ctype;
  PR_TRY(scr.get(sizeof(int64_t) * (n + 1), (void**)&d_rp));
  PR_TRY(scr.get(sizeof(int32_t) * m_in, (void**)&d_col));
  PR_TRY(scr.get(sizeof(int32_t) * n, (void**)&d_comp));
  PR_TRY(scr.get(sizeof(int32_t) * K, (void**)&d_clevel));
  PR_TRY(scr.get(sizeof(int32_t) * K, (void**)&d_csize));
  PR_TRY(scr.get(sizeof(uint8_t) * K, (void**)&d_ctype));
  PR_TRY(scr.get(sizeof(int32_t) * n, (void**)&d_emit));
  PR_HIP_CHECK(hipMemcpyAsync(d_rp, h_row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
  if (m_in) PR_HIP_CHECK(hipMemcpyAsync(d_col, h_col, sizeof(int32_t) * m_in, hipMemcpyHostToDevice, s));
  double* d_w = nullptr;
  if (lv.weighted) {
    PR_TRY(scr.get(sizeof(double) * m_in, (void**)&d_w));
    if (m_in) PR_HIP_CHECK(hipMemcpyAsync(d_w, h_weight, sizeof(double) * m_in, hipMemcpyHostToDevice, s));
  }
  if (n) {
    PR_HIP_CHECK(hipMemcpyAsync(d_comp, P.comp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    PR_HIP_CHECK(hipMemcpyAsync(d_emit, P.emit_pos.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    PR_HIP_CHECK(hipMemcpyAsync(d_clevel, P.comp_level.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s));
    PR_HIP_CHECK(hipMemcpyAsync(d_csize, P.comp_size.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s));
    PR_HIP_CHECK(hipMemcpyAsync(d_ctype, P.comp_type.data(), K, hipMemcpyHostToDevice, s));
  }
  int32_t maxsize = 0;
  for (int64_t k = 0; k < K; ++k) maxsize = std::max(maxsize, P.comp_size[k]);
  const int32_t maxlevel = std::max(0, P.n_levels - 1);

  // ---- component order
  uint32_t *ckey, *cval, *csz_rank;
  PR_TRY(scr.get(sizeof(uint32_t) * K, (void**)&ckey));
  PR_TRY(scr.get(sizeof(uint32_t) * K, (void**)&cval));
  PR_TRY(scr.get(sizeof(uint32_t) * K, (void**)&csz_rank));
  PR_TRY(dalloc(&lv.comp_vbeg, K + 1));
  PR_TRY(dalloc(&lv.comp_rank_of_id, K));
  PR_TRY(dalloc(&lv.comp_id_of_rank, K));
  if (K) {
    k_comp_key_size<<<nblk(K), kB, 0, s>>>(d_csize, K, (uint32_t)maxsize, ckey, cval);
    PR_TRY(radix_sort_pairs(ckey, cval, K, bit_length((uint64_t)maxsize), s));
    k_comp_key_level<<<nblk(K), kB, 0, s>>>(d_clevel, d_ctype, d_csize, cval, K, maxlevel, ckey);
    PR_TRY(radix_sort_pairs(ckey, cval, K, bit_length((uint64_t)maxlevel * 3 + 2), s));
    k_comp_rank<<<nblk(K), kB, 0, s>>>(cval, K, d_csize, lv.comp_rank_of_id, csz_rank);
    PR_HIP_CHECK(hipMemcpyAsync(lv.comp_id_of_rank, cval, sizeof(int32_t) * K, hipMemcpyDeviceToDevice, s));
    PR_TRY(scan_u32(csz_rank, (uint32_t*)lv.comp_vbeg, K, s));
  } else {
    PR_HIP_CHECK(hipMemsetAsync(lv.comp_vbeg, 0, sizeof(int32_t), s));
  }

  // ---- vertex order
  uint32_t *vlist, *vkey;
  int32_t* iperm;
  PR_TRY(scr.get(sizeof(uint32_t) * n, (void**)&vlist));
  PR_TRY(scr.get(sizeof(uint32_t) * n, (void**)&vkey));
  PR_TRY(scr.get(sizeof(int32_t) * n, (void**)&iperm));
  PR_TRY(dalloc(&lv.perm, n));
  if (n) {
    k_topo_list<<<nblk(n), kB, 0, s>>>(d_emit, n, vlist);
    k_vertex_degkey<<<nblk(n), kB, 0, s>>>(vlist, n, d_rp, d_comp, d_ctype, vkey);
    PR_TRY(radix_sort_pairs(vkey, vlist, n, 20, s));
    k_vertex_key<<<nblk(n), kB, 0, s>>>(vlist, n, d_comp, lv.comp_rank_of_id, vkey);
    PR_TRY(radix_sort_pairs(vkey, vlist, n, bit_length((uint64_t)std::max<int64_t>(K - 1, 0)), s));
    k_perm_inverse<<<nblk(n), kB, 0, s>>>(vlist, n, lv.perm, iperm);
  }

  // ---- degrees
  uint32_t *odeg, *optr;
  PR_TRY(scr.get(sizeof(uint32_t) * n, (void**)&odeg));
  PR_TRY(scr.get(sizeof(uint32_t) * (n + 1), (void**)&optr));
  PR_TRY(dalloc(&lv.inv_deg32, n));
  PR_TRY(dalloc(&lv.inv_deg64, n));
  if (n && lv.weighted)
    k_degrees_w<<<nblk(n), kB, 0, s>>>(d_rp, d_col, d_w, lv.perm, n, opts.keep_loops, odeg, lv.inv_deg32,
                                       lv.inv_deg64);
  else if (n)
    k_degrees<<<nblk(n), kB, 0, s>>>(d_rp, d_col, lv.perm, n, opts.keep_loops, odeg, lv.inv_deg32, lv.inv_deg64);
  PR_TRY(scan_u32(odeg, optr, n, s));
  uint32_t m32 = 0;
  PR_HIP_CHECK(hipMemcpyAsync(&m32, optr + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  const int64_t m = m32;
  lv.m = m;

  // ---- edges: plan-source order, then stable sort by plan destination
  uint32_t *dkey, *sval, *rcnt;
  PR_TRY(scr.get(sizeof(uint32_t) * m, (void**)&dkey));
  PR_TRY(scr.get(sizeof(uint32_t) * m, (void**)&sval));
  PR_TRY(scr.get(sizeof(uint32_t) * n, (void**)&rcnt));
  double* wsort = nullptr;
  if (lv.weighted) {
    // sort the edges' positions, then fetch source and weight by position
    uint32_t *pval, *spos;
    double* wpos;
    PR_TRY(scr.get(sizeof(uint32_t) * m, (void**)&pval));
    PR_TRY(scr.get(sizeof(uint32_t) * m, (void**)&spos));
    PR_TRY(scr.get(sizeof(double) * m, (void**)&wpos));
    PR_TRY(scr.get(sizeof(double) * m, (void**)&wsort));
    if (n)
      k_emit_edges_w<<<nblk(n), kB, 0, s>>>(d_rp, d_col, d_w, lv.perm, iperm, optr, n, opts.keep_loops, dkey, pval,
                                            spos, wpos);
    PR_TRY(radix_sort_pairs(dkey, pval, m, bit_length((uint64_t)std::max<int64_t>(n - 1, 0)), s));
    if (m) k_edge_gather<<<nblk(m), kB, 0, s>>>(pval, spos, wpos, m, sval, wsort);
  } else {
    if (n) k_emit_edges<<<nblk(n), kB, 0, s>>>(d_rp, d_col, lv.perm, iperm, optr, n, opts.keep_loops, dkey, sval);
    PR_TRY(radix_sort_pairs(dkey, sval, m, bit_length((uint64_t)std::max<int64_t>(n - 1, 0)), s));
  }
  uint32_t* fptr;
  PR_TRY(scr.get(sizeof(uint32_t) * (n + 1), (void**)&fptr));
  if (n) PR_HIP_CHECK(hipMemsetAsync(rcnt, 0, sizeof(uint32_t) * n, s));
  if (m) k_count_rows<<<nblk(m), kB, 0, s>>>(dkey, m, rcnt);
  PR_TRY(scan_u32(rcnt, fptr, n, s));

  // ---- split into between-component and inside-component rows
  int32_t* vbeg_of;
  uint32_t *bcnt, *icnt;
  PR_TRY(scr.get(sizeof(int32_t) * n, (void**)&vbeg_of));
  PR_TRY(scr.get(sizeof(uint32_t) * n, (void**)&bcnt));
  PR_TRY(scr.get(sizeof(uint32_t) * n, (void**)&icnt));
  PR_TRY(dalloc(&lv.bnd_ptr, n + 1));
  PR_TRY(dalloc(&lv.int_ptr, n + 1));
  if (n) {
    k_vertex_comp_begin<<<nblk(n), kB, 0, s>>>((const uint32_t*)lv.perm, d_comp, lv.comp_rank_of_id,
                                                lv.comp_vbeg, n, vbeg_of);
    k_split_count<<<nblk(n), kB, 0, s>>>(fptr, sval, vbeg_of, n, bcnt, icnt);
  }
  PR_TRY(scan_u32(bcnt, lv.bnd_ptr, n, s));
  PR_TRY(scan_u32(icnt, lv.int_ptr, n, s));
  uint32_t mb = 0, mi = 0;
  PR_HIP_CHECK(hipMemcpyAsync(&mb, lv.bnd_ptr + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipMemcpyAsync(&mi, lv.int_ptr + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PR_HIP_CHECK(hipStreamSynchronize(s));
  PR_TRY(dalloc(&lv.bnd_src, mb));
  PR_TRY(dalloc(&lv.int_src, mi));
  if (n) k_split_copy<<<nblk(n), kB, 0, s>>>(fptr, sval, lv.bnd_ptr, lv.int_ptr, n, lv.bnd_src, lv.int_src);
  if (lv.weighted) {
    PR_TRY(dalloc(&lv.bnd_w64, mb));
    PR_TRY(dalloc(&lv.int_w64, mi));
    PR_TRY(dalloc(&lv.int_w32, mi));
    if (n)
      k_split_copy_w<<<nblk(n), kB, 0, s>>>(fptr, wsort, lv.bnd_ptr, lv.int_ptr, n, lv.bnd_w64, lv.int_w64,
                                            lv.int_w32);
  }
  if (opts.build_plain) {
    PR_TRY(dalloc(&lv.full_ptr, n + 1));
    PR_TRY(dalloc(&lv.full_src, m));
    PR_HIP_CHECK(hipMemcpyAsync(lv.full_ptr, fptr, sizeof(uint32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (m) PR_HIP_CHECK(hipMemcpyAsync(lv.full_src, sval, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, s));
    if (lv.weighted) {
      PR_TRY(dalloc(&lv.full_w64, m));
      PR_TRY(dalloc(&lv.full_w32, m));
      if (m) {
        PR_HIP_CHECK(hipMemcpyAsync(lv.full_w64, wsort, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
        k_to_f32<<<nblk(m), kB, 0, s>>>(wsort, m, lv.full_w32);
      }
    }
  }

  // ---- host copies of the pull row pointers (gang row bounds)
  lv.h_int_ptr.resize(n + 1);
  PR_HIP_CHECK(hipMemcpyAsync(lv.h_int_ptr.data(), lv.int_ptr, sizeof(uint32_t) * (n + 1), hipMemcpyDeviceToHost, s));
  if (opts.build_plain) {
    lv.h_full_ptr.resize(n + 1);
    PR_HIP_CHECK(hipMemcpyAsync(lv.h_full_ptr.data(), fptr, sizeof(uint32_t) * (n + 1), hipMemcpyDeviceToHost, s));
  }

  // ---- host copies for scheduling
  uint32_t* cint;
  PR_TRY(scr.get(sizeof(uint32_t) * K, (void**)&cint));
  if (K) k_comp_int_edges<<<nblk(K), kB, 0, s>>>(lv.int_ptr, lv.comp_vbeg, K, cint);
  std::vector<uint32_t> h_cint(K), h_idr(K);
  lv.h_comp_vbeg.resize(K + 1);
  PR_HIP_CHECK(hipMemcpyAsync(lv.h_comp_vbeg.data(), lv.comp_vbeg, sizeof(int32_t) * (K + 1), hipMemcpyDeviceToHost, s));
  if (K) {
    PR_HIP_CHECK(hipMemcpyAsync(h_cint.data(), cint, sizeof(uint32_t) * K, hipMemcpyDeviceToHost, s));
    PR_HIP_CHECK(hipMemcpyAsync(h_idr.data(), lv.comp_id_of_rank, sizeof(uint32_t) * K, hipMemcpyDeviceToHost, s));
  }
  PR_HIP_CHECK(hipStreamSynchronize(s));
  lv.h_comp_class.resize(K);
  lv.h_comp_level.resize(K);
  lv.h_comp_int_edges.resize(K);
  lv.h_comp_id_of_rank.resize(K);
  pr_levels_info& I = lv.info;
  memset(&I, 0, sizeof(I));
  I.n = n;
  I.m = m;
  I.n_comp = K;
  I.n_levels = P.n_levels;
  for (int64_t r = 0; r < K; ++r) {
    const uint32_t k = h_idr[r];
    const uint8_t cls = P.comp_type[k] ? 0 : (P.comp_size[k] >= 2 ? 1 : 2);
    lv.h_comp_id_of_rank[r] = (int32_t)k;
    lv.h_comp_class[r] = cls;
    lv.h_comp_level[r] = P.comp_level[k];
    lv.h_comp_int_edges[r] = h_cint[r];
    const int64_t sz = P.comp_size[k];
    if (cls == 0) {
      I.n_scc++;
      I.v_scc += sz;
      I.m_scc_internal += h_cint[r];
    } else if (cls == 1) {
      I.n_cac++;
      I.v_cac += sz;
      I.m_cac_internal += h_cint[r];
    } else {
      I.n_singleton++;
      I.v_singleton += sz;
      I.m_cac_internal += h_cint[r];  // self-loops of a one-vertex component (keep_loops)
    }
    // sanity: plan order must be level-descending
    if (r > 0 && lv.h_comp_level[r] > lv.h_comp_level[r - 1]) {
      set_error("internal: component order is not level-descending at rank %lld", (long long)r);
      return PR_EHIP;
    }
  }
  I.m_between = mb;
  if ((int64_t)mi != I.m_scc_internal + I.m_cac_internal) {
    set_error("internal: edge split mismatch (%u inside vs %lld)", mi,
              (long long)(I.m_scc_internal + I.m_cac_internal));
    return PR_EHIP;
  }
  PR_TRY(make_schedule(lv, s));
  if (opts.autotune) PR_TRY(autotune_levels(lv, s));
  return PR_OK;
}

}  // namespace prlib
