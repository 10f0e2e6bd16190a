// C ABI entry points, error reporting and the handle registry.
#include <cmath>
#include <cstdio>
#include <mutex>
#include <new>
#include <unordered_map>

#include "internal.h"

namespace prlib {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

static std::mutex g_reg_mu;
static std::unordered_map<const void*, HandleKind>& registry() {
  static std::unordered_map<const void*, HandleKind> r;
  return r;
}

void registry_add(void* h, HandleKind k) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  registry()[h] = k;
}

bool registry_has(const void* h, HandleKind k) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  auto it = registry().find(h);
  return it != registry().end() && it->second == k;
}

bool registry_remove(void* h, HandleKind* k) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  auto it = registry().find(h);
  if (it == registry().end()) return false;
  *k = it->second;
  registry().erase(it);
  return true;
}

}  // namespace prlib

using namespace prlib;


extern "C" {

const char* pr_last_error(void) { return g_last_error.c_str(); }

const char* pr_version(void) { return "componentwise-pagerank-mi355x 0.2 (gfx950)"; }

void pr_free(void* handle) {
  if (!handle) return;
  HandleKind k;
  if (!registry_remove(handle, &k)) return;
  switch (k) {
    case KIND_PARTITION:
      delete static_cast<Partition*>(handle);
      break;
    case KIND_LEVELS:
      delete static_cast<Levels*>(handle);
      break;
    case KIND_MLP:
      mlp_destroy(handle);
      break;
  }
}

int32_t pr_partition(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, uint32_t flags,
                     pr_partition_t** out) {
  if (!out) {
    set_error("out is NULL");
    return PR_EINVAL;
  }
  if (flags != 0) {
    set_error("flags must be 0 (got %u)", flags);
    return PR_EINVAL;
  }
  int32_t rc = validate_csr(n, row_ptr, col_idx);
  if (rc) return rc;
  Partition* p = new (std::nothrow) Partition();
  if (!p) {
    set_error("out of host memory");
    return PR_ENOMEM;
  }
  rc = run_partition(n, row_ptr, col_idx, *p);
  if (rc) {
    delete p;
    return rc;
  }
  p->graph_hash = hash_csr(n, row_ptr, col_idx);
  registry_add(p, KIND_PARTITION);
  *out = reinterpret_cast<pr_partition_t*>(p);
  return PR_OK;
}

int32_t pr_partition_get(const pr_partition_t* ph, int32_t* comp, int32_t* comp_level,
                         uint8_t* comp_type, int32_t* comp_size, int64_t* n_comp,
                         int32_t* n_levels) {
  if (!registry_has(ph, KIND_PARTITION)) {
    set_error("not a live pr_partition handle");
    return PR_EHANDLE;
  }
  const Partition* p = reinterpret_cast<const Partition*>(ph);
  if (comp && p->n) memcpy(comp, p->comp.data(), sizeof(int32_t) * p->n);
  if (comp_level && p->n_comp) memcpy(comp_level, p->comp_level.data(), sizeof(int32_t) * p->n_comp);
  if (comp_type && p->n_comp) memcpy(comp_type, p->comp_type.data(), p->n_comp);
  if (comp_size && p->n_comp) memcpy(comp_size, p->comp_size.data(), sizeof(int32_t) * p->n_comp);
  if (n_comp) *n_comp = p->n_comp;
  if (n_levels) *n_levels = p->n_levels;
  return PR_OK;
}

void pr_default_build_opts(pr_build_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->small_cutoff = 64;
  o->team_edges = 65536;
  o->rows_per_wave = 16;
  o->build_plain = 1;
  o->autotune = 0;
}

void pr_default_solve_opts(pr_solve_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->method = PR_METHOD_COMPONENTWISE;
  o->stop = PR_STOP_CERT_L1;
  o->precision = PR_PREC_MIXED;
  o->use_graph = 0;
  o->eps = 1e-6;
  o->tol = 1e-9;
  o->max_iter = 100000;
  o->warm_start = nullptr;
}

// pr_build_levels and pr_build_levels_weighted (weight null for the former)
static int32_t build_plan(const pr_partition_t* ph, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                          const double* weight, const pr_build_opts* opts, void* hip_stream, pr_levels_t** out) {
  if (!out) {
    set_error("out is NULL");
    return PR_EINVAL;
  }
  if (!registry_has(ph, KIND_PARTITION)) {
    set_error("not a live pr_partition handle");
    return PR_EHANDLE;
  }
  const Partition* p = reinterpret_cast<const Partition*>(ph);
  if (p->n != n) {
    set_error("partition has n = %lld but the graph has n = %lld", (long long)p->n, (long long)n);
    return PR_EINVAL;
  }
  int32_t rc = validate_csr(n, row_ptr, col_idx);
  if (rc) return rc;
  if (row_ptr[n] > (int64_t)INT32_MAX) {
    set_error("m = %lld edges; the device plan needs m < 2^31", (long long)row_ptr[n]);
    return PR_EINVAL;
  }
  if (hash_csr(n, row_ptr, col_idx) != p->graph_hash) {
    set_error("the partition was computed on a different graph");
    return PR_EINVAL;
  }
  if (weight) {
    const int64_t m = row_ptr[n];
    for (int64_t e = 0; e < m; ++e) {
      if (!(weight[e] >= 0.0) || !std::isfinite(weight[e])) {
        set_error("weight[%lld] = %g: edge weights must be finite and non-negative", (long long)e, weight[e]);
        return PR_EINVAL;
      }
    }
  }
  pr_build_opts o;
  pr_default_build_opts(&o);
  if (opts) {
    o = *opts;
    pr_build_opts d;
    pr_default_build_opts(&d);
    if (o.small_cutoff <= 0) o.small_cutoff = d.small_cutoff;
    if (o.team_edges <= 0) o.team_edges = d.team_edges;
    if (o.rows_per_wave <= 0) o.rows_per_wave = d.rows_per_wave;
  }
  if (o.small_cutoff > 256) {
    set_error("small_cutoff = %d exceeds 256", o.small_cutoff);
    return PR_EINVAL;
  }
  if (o.seg_waves != 0 && o.seg_waves != 2 && o.seg_waves != 3) {
    set_error("seg_waves = %d, expected 0, 2 or 3", o.seg_waves);
    return PR_EINVAL;
  }
  if (o.autotune < 0 || o.autotune > 2) {
    set_error("autotune = %d, expected 0, 1 or 2", o.autotune);
    return PR_EINVAL;
  }
  if (o.rows_per_wave != 1 && o.rows_per_wave != 4 && o.rows_per_wave != 16 && o.rows_per_wave != 64) {
    set_error("rows_per_wave = %d, expected 1, 4, 16 or 64", o.rows_per_wave);
    return PR_EINVAL;
  }
  Levels* lv = new (std::nothrow) Levels();
  if (!lv) {
    set_error("out of host memory");
    return PR_ENOMEM;
  }
  rc = build_levels(*p, row_ptr, col_idx, weight, o, (hipStream_t)hip_stream, *lv);
  if (rc) {
    delete lv;
    return rc;
  }
  registry_add(lv, KIND_LEVELS);
  *out = reinterpret_cast<pr_levels_t*>(lv);
  return PR_OK;
}

int32_t pr_build_levels(const pr_partition_t* ph, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                        const pr_build_opts* opts, void* hip_stream, pr_levels_t** out) {
  return build_plan(ph, n, row_ptr, col_idx, nullptr, opts, hip_stream, out);
}

int32_t pr_build_levels_weighted(const pr_partition_t* ph, int64_t n, const int64_t* row_ptr,
                                 const int32_t* col_idx, const double* weight, const pr_build_opts* opts,
                                 void* hip_stream, pr_levels_t** out) {
  if (!weight) {
    set_error("weight is NULL");
    return PR_EINVAL;
  }
  return build_plan(ph, n, row_ptr, col_idx, weight, opts, hip_stream, out);
}

int32_t pr_levels_get_info(const pr_levels_t* lh, pr_levels_info* info) {
  if (!registry_has(lh, KIND_LEVELS)) {
    set_error("not a live pr_levels handle");
    return PR_EHANDLE;
  }
  if (!info) {
    set_error("info is NULL");
    return PR_EINVAL;
  }
  *info = reinterpret_cast<const Levels*>(lh)->info;
  return PR_OK;
}

int32_t pr_solve(pr_levels_t* lh, double c, const void* W_dev, void* R_dev, const pr_solve_opts* opts,
                 void* hip_stream, pr_solve_stats* stats) {
  if (!registry_has(lh, KIND_LEVELS)) {
    set_error("not a live pr_levels handle");
    return PR_EHANDLE;
  }
  Levels* lv = reinterpret_cast<Levels*>(lh);
  pr_solve_opts o;
  pr_default_solve_opts(&o);
  if (opts) o = *opts;
  if (!(c > 0.0 && c < 1.0)) {
    set_error("damping c = %g outside (0, 1)", c);
    return PR_EINVAL;
  }
  if (o.stop == PR_STOP_CERT_L1 && !(o.eps > 0.0)) {
    set_error("eps = %g must be > 0", o.eps);
    return PR_EINVAL;
  }
  if (o.stop == PR_STOP_PAPER_MAXABS && !(o.tol > 0.0)) {
    set_error("tol = %g must be > 0", o.tol);
    return PR_EINVAL;
  }
  if (o.stop != PR_STOP_CERT_L1 && o.stop != PR_STOP_PAPER_MAXABS) {
    set_error("unknown stop rule %d", o.stop);
    return PR_EINVAL;
  }
  if (o.method != PR_METHOD_COMPONENTWISE && o.method != PR_METHOD_PLAIN) {
    set_error("unknown method %d", o.method);
    return PR_EINVAL;
  }
  if (o.precision != PR_PREC_MIXED && o.precision != PR_PREC_FP64 && o.precision != PR_PREC_AUTO) {
    set_error("unknown precision %d", o.precision);
    return PR_EINVAL;
  }
  if (o.max_iter <= 0) {
    set_error("max_iter = %lld must be > 0", (long long)o.max_iter);
    return PR_EINVAL;
  }
  if (o.method == PR_METHOD_PLAIN && !lv->full_ptr) {
    set_error("method PLAIN needs a plan built with build_plain = 1");
    return PR_EINVAL;
  }
  if (lv->n > 0 && (!W_dev || !R_dev)) {
    set_error("W_dev / R_dev is NULL");
    return PR_EINVAL;
  }
  if (o.warm_scope != 0 && o.warm_scope != 1) {
    set_error("warm_scope = %d, expected 0 or 1", o.warm_scope);
    return PR_EINVAL;
  }
  if (o.tail_estimate != 0 && o.tail_estimate != 1) {
    set_error("tail_estimate = %d, expected 0 or 1", o.tail_estimate);
    return PR_EINVAL;
  }
  if (o.cold != 0 && o.cold != 1) {
    set_error("cold = %d, expected 0 or 1", o.cold);
    return PR_EINVAL;
  }
  if (o.refine < -1 || o.refine > 16) {
    set_error("refine = %d, expected -1 (no residual pass), 0 (default) or 1..16 rounds", o.refine);
    return PR_EINVAL;
  }
  if (o.gs_blocks < 0 || o.gs_blocks > 8) {
    set_error("gs_blocks = %d, expected 0..8", o.gs_blocks);
    return PR_EINVAL;
  }
  if (o.gs_blocks > 0 && (o.tail_estimate || o.warm_start || lv->weighted)) {
    set_error("gs_blocks > 0 does not combine with tail_estimate, warm_start or a weighted plan");
    return PR_EINVAL;
  }
  if (o.small_direct < 0 || o.small_direct > 80) {
    set_error("small_direct = %d, expected 0..80", o.small_direct);
    return PR_EINVAL;
  }
  if (o.warm_start && !registry_has(o.warm_start, KIND_MLP)) {
    set_error("warm_start is not a live pr_mlp handle");
    return PR_EHANDLE;
  }
  return solve_levels(*lv, c, (const double*)W_dev, (double*)R_dev, o, (hipStream_t)hip_stream, stats);
}

}  // extern "C"
