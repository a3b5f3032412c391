// kc_api.hip -- the C interface of the library (include/kclique.h).
//
// A call runs, in stream order on one GPU: CSR validation, Pre-Core and
// Pre-List (Sec. 5), the orientation (Sec. 6.2 or 7.4), the root filter
// d+ >= k-1 (Alg. 5 and Alg. 6), and the listing of SDegree or BitCol.  The
// total is the Pre-List count plus the listing count.  Host pointers are
// staged to the device first; device pointers are used in place.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <vector>

#include "kc_internal.h"

extern "C" void kc_options_init(kc_options* opt) {
  if (opt) memset(opt, 0, sizeof(*opt));
}

extern "C" const char* kc_status_string(int status) {
  switch (status) {
    case KC_OK: return "ok";
    case KC_EINVAL: return "invalid argument or malformed graph";
    case KC_ENOMEM: return "device memory allocation failed";
    case KC_EOVERFLOW: return "count does not fit in 64 bits";
    case KC_EDEVICE: return "HIP runtime error";
    case KC_EUNSUPPORTED: return "local subgraph larger than supported";
  }
  return "unknown status";
}

__global__ void k_roots(int32_t n, const int32_t* __restrict__ drp, int32_t km1, const int32_t* vk, int32_t* roots,
                        int32_t* nroots, int32_t* max_dplus) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t d = u < n ? drp[u + 1] - drp[u] : 0;
  bool take = u < n && d >= kc_vk(vk, u, km1 + 1) - 1;
  uint64_t m = kc_ballot(take);
  int base = 0;
  if (kc_lane() == 0 && m) base = atomicAdd(nroots, __popcll(m));
  base = __shfl(base, 0, 64);
  if (take) roots[base + kc_mbcnt(m)] = u;
  int mx = kc_wave_max_i32(take ? d : 0);
  if (kc_lane() == 0 && mx > 0) atomicMax(max_dplus, mx);
}

// k = 1 and k = 2: every vertex, every edge (linear cases, Sec. 8).
__global__ void k_small_k(int32_t n, const int32_t* __restrict__ rp, int32_t k, unsigned long long* pv) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  pv[v] = k == 1 ? 1ull : (unsigned long long)(rp[v + 1] - rp[v]);
}

struct HostEvents {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  ~HostEvents() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

static int count_impl(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                      const kc_options* opt_in, uint64_t* count_out, uint64_t* pv_out) {
  kc_options defaults;
  memset(&defaults, 0, sizeof(defaults));
  const kc_options* opt = opt_in ? opt_in : &defaults;
  if (n < 0 || k < 1 || !count_out) return KC_EINVAL;
  if (order != KC_ORDER_DEGREE && order != KC_ORDER_COLOR) return KC_EINVAL;
  if (opt->schedule != KC_SCHED_DEGREE && opt->schedule != KC_SCHED_LEARNED) return KC_EINVAL;
  if (n > 0 && !row_ptr) return KC_EINVAL;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return KC_EDEVICE;
  hipStream_t s = (hipStream_t)opt->stream;
  kc_stats* stats = opt->stats;
  if (stats) memset(stats, 0, sizeof(*stats));
  HostEvents ev;
  for (auto& x : ev.e) KC_HIP(hipEventCreate(&x));
  KC_HIP(hipEventRecord(ev.e[0], s));

  kc_scratch scr(s);
  // ---- graph on the device
  kc_dev_graph g;
  g.n = n;
  int32_t nnz32 = 0;
  if (n > 0) {
    if (opt->device_ptrs) {
      KC_HIP(hipMemcpyAsync(&nnz32, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      KC_HIP(hipStreamSynchronize(s));
    } else {
      nnz32 = row_ptr[n];
    }
  }
  if (nnz32 < 0) return KC_EINVAL;
  g.nnz = nnz32;
  if (n > 0 && nnz32 > 0 && !col_idx) return KC_EINVAL;
  if (opt->device_ptrs) {
    g.rp = row_ptr;
    g.col = col_idx;
  } else {
    int32_t *rp_d = nullptr, *col_d = nullptr;
    KC_TRY(scr.get(&rp_d, (size_t)n + 1));
    KC_TRY(scr.get(&col_d, (size_t)nnz32 + 1));
    KC_HIP(hipMemcpyAsync(rp_d, row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
    if (nnz32 > 0) KC_HIP(hipMemcpyAsync(col_d, col_idx, sizeof(int32_t) * (size_t)nnz32, hipMemcpyHostToDevice, s));
    g.rp = rp_d;
    g.col = col_d;
  }
  // ---- device state
  int* flags;
  unsigned long long *count_d, *prelist_d, *counters;
  KC_TRY(scr.get(&flags, 4));
  KC_TRY(scr.get(&count_d, 2));
  KC_TRY(scr.get(&prelist_d, 2));
  KC_TRY(scr.get(&counters, 8));
  KC_HIP(hipMemsetAsync(flags, 0, sizeof(int) * 4, s));
  KC_HIP(hipMemsetAsync(count_d, 0, sizeof(unsigned long long) * 2, s));
  KC_HIP(hipMemsetAsync(prelist_d, 0, sizeof(unsigned long long) * 2, s));
  KC_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * 8, s));
  unsigned long long* pv_d = nullptr;
  if (pv_out) {
    if (opt->device_ptrs) pv_d = (unsigned long long*)pv_out;
    else KC_TRY(scr.get(&pv_d, (size_t)n + 1));
    if (n > 0) KC_HIP(hipMemsetAsync(pv_d, 0, sizeof(unsigned long long) * (size_t)n, s));
  }
  if (n > 0) {
    if (opt->root_count) KC_HIP(hipMemsetAsync(opt->root_count, 0, sizeof(uint64_t) * (size_t)n, s));
    if (opt->root_work) KC_HIP(hipMemsetAsync(opt->root_work, 0, sizeof(uint64_t) * (size_t)n, s));
    if (opt->root_isect) KC_HIP(hipMemsetAsync(opt->root_isect, 0, sizeof(uint64_t) * (size_t)n, s));
    if (opt->root_features) KC_HIP(hipMemsetAsync(opt->root_features, 0, sizeof(float) * 4 * (size_t)n, s));
  }

  // ---- validation
  int hflags = 0;
  if (!opt->trusted_input) {
    KC_TRY(kc_validate_graph(g, flags, s));
    KC_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    if (hflags & KC_FLAG_BADGRAPH) return KC_EINVAL;
  }

  uint64_t total = 0;
  const int32_t* vk = opt->vertex_k;
  if (vk && !opt->device_ptrs) return KC_EINVAL;
  if (vk && k < 3) return KC_EUNSUPPORTED;
  if (k <= 2 || (k > n && !vk)) {
    // linear cases and the empty answer
    if (k == 1) total = (uint64_t)n;
    else if (k == 2) total = (uint64_t)nnz32 / 2;
    if (pv_d && n > 0 && k <= 2) {
      k_small_k<<<(n + 255) / 256, 256, 0, s>>>(n, g.rp, k, pv_d);
      KC_HIP(hipGetLastError());
    }
    KC_HIP(hipEventRecord(ev.e[1], s));
    KC_HIP(hipEventRecord(ev.e[2], s));
  } else {
    if (k > KC_KMAX_LIMIT) return KC_EUNSUPPORTED;
    kc_prep_out prep;
    KC_TRY(kc_preprocess(g, k, vk, order, prelist_d, pv_d, (unsigned long long*)opt->root_count, flags, &prep,
                         scr, s));
    KC_HIP(hipEventRecord(ev.e[1], s));
    int32_t *roots, *rinfo;
    KC_TRY(scr.get(&roots, (size_t)n + 1));
    KC_TRY(scr.get(&rinfo, 4));
    KC_HIP(hipMemsetAsync(rinfo, 0, sizeof(int32_t) * 4, s));
    k_roots<<<(n + 255) / 256, 256, 0, s>>>(n, prep.drp, k - 1, vk, roots, rinfo, rinfo + 1);
    KC_HIP(hipGetLastError());
    int32_t hr[2] = {0, 0};
    KC_HIP(hipMemcpyAsync(hr, rinfo, sizeof(hr), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    kc_list_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n;
    c.k = k;
    c.vk = vk;
    c.root_count = (unsigned long long*)opt->root_count;
    c.drp = prep.drp;
    c.dcol = prep.dcol;
    c.core = prep.core;
    c.nroots = hr[0];
    c.roots = roots;
    c.count = count_d;
    c.pv = pv_d;
    c.flags = flags;
    c.root_work = opt->root_work;
    c.root_isect = opt->root_isect;
    c.root_features = opt->root_features;
    c.counters = counters;
    c.opt = opt;
    c.stats = stats;
    KC_HIP(hipEventRecord(ev.e[2], s));
    if (order == KC_ORDER_DEGREE) KC_TRY(kc_list_sdegree(c, scr, s));
    else KC_TRY(kc_list_bitcol(c, scr, s));
    if (stats) {
      stats->n_roots = hr[0];
      stats->max_out_degree = hr[1];
      stats->max_core = prep.max_core;
    }
  }
  KC_HIP(hipEventRecord(ev.e[3], s));
  // ---- results
  unsigned long long hres[2] = {0, 0}, hcnt[8];
  KC_HIP(hipMemcpyAsync(hres, count_d, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(hres + 1, prelist_d, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(hcnt, counters, sizeof(hcnt), hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  if (pv_out && !opt->device_ptrs && n > 0)
    KC_HIP(hipMemcpyAsync(pv_out, pv_d, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  if (hflags & KC_FLAG_OVERFLOW) return KC_EOVERFLOW;
  if (hflags & KC_FLAG_TOOBIG) return KC_EUNSUPPORTED;
  if (k > 2 && (k <= n || vk)) {
    total = hres[0] + hres[1];
    if (total < hres[0]) return KC_EOVERFLOW;
  }
  *count_out = total;
  if (stats) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev.e[0], ev.e[3]) == hipSuccess) stats->total_ms = t;
    if (hipEventElapsedTime(&t, ev.e[0], ev.e[1]) == hipSuccess) stats->prep_ms = t;
    stats->prelist_count = hres[1];
    stats->nodes = hcnt[0];
    stats->isect = hcnt[1];
    stats->work = hcnt[2];
    stats->stage_bytes = hcnt[3];
    stats->isect_wide = hcnt[4];
    stats->isect_compressed = hcnt[5];
  }
  return KC_OK;
}

extern "C" int kclique_count_ex(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                                const kc_options* opt, uint64_t* count_out, uint64_t* per_vertex_out) {
  return count_impl(n, row_ptr, col_idx, k, order, opt, count_out, per_vertex_out);
}

extern "C" int kclique_count(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                             uint64_t* count_out) {
  return count_impl(n, row_ptr, col_idx, k, order, nullptr, count_out, nullptr);
}

extern "C" int kclique_list_per_vertex(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k,
                                       int32_t order, uint64_t* per_vertex_out, uint64_t* count_out) {
  uint64_t c = 0;
  if (!per_vertex_out && n > 0) return KC_EINVAL;
  int st = count_impl(n, row_ptr, col_idx, k, order, nullptr, &c, per_vertex_out);
  if (st == KC_OK && count_out) *count_out = c;
  return st;
}

// Batched counting: the graphs become one disjoint union (vertex ids shifted
// by the preceding graphs' sizes) with a k per vertex, counted by a single call
// -- one preprocessing pass, one staging pass and one persistent listing
// launch per word class for all graphs -- and the per-root attribution is
// summed per graph.
__global__ void k_union_rows(int32_t ng, const int32_t* __restrict__ n, const int64_t* __restrict__ voff,
                             const int64_t* __restrict__ row_off, const int64_t* __restrict__ eoff,
                             const int32_t* __restrict__ rp_cat, int32_t* rp_out, int32_t* vk_out,
                             const int32_t* __restrict__ kk, int32_t* gid) {
  int32_t g = blockIdx.y;
  if (g >= ng) return;
  const int32_t ng_v = n[g];
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < ng_v; v += gridDim.x * blockDim.x) {
    const int64_t gv = voff[g] + v;
    rp_out[gv] = (int32_t)(eoff[g] + rp_cat[row_off[g] + v]);
    vk_out[gv] = kk[g];
    gid[gv] = g;
  }
}

__global__ void k_union_cols(int32_t ng, const int32_t* __restrict__ n, const int64_t* __restrict__ voff,
                             const int64_t* __restrict__ row_off, const int64_t* __restrict__ col_off,
                             const int64_t* __restrict__ eoff, const int32_t* __restrict__ rp_cat,
                             const int32_t* __restrict__ col_cat, int32_t* col_out) {
  int32_t g = blockIdx.y;
  if (g >= ng) return;
  const int64_t m = rp_cat[row_off[g] + n[g]];
  const int32_t shift = (int32_t)voff[g];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    col_out[eoff[g] + i] = col_cat[col_off[g] + i] + shift;
}

__global__ void k_graph_sums(int32_t nv, const int32_t* __restrict__ gid, const unsigned long long* __restrict__ rc,
                             unsigned long long* out) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const unsigned long long c = rc[v];
  if (c) atomicAdd(&out[gid[v]], c);
}

extern "C" int kclique_count_batched(int32_t num_graphs, const int32_t* n, const int64_t* row_off,
                                     const int64_t* col_off, const int32_t* row_ptr_cat, const int32_t* col_idx_cat,
                                     const int32_t* k, int32_t order, const kc_options* opt, uint64_t* counts_out) {
  if (num_graphs < 0 || (num_graphs > 0 && (!n || !row_off || !col_off || !k || !counts_out))) return KC_EINVAL;
  if (num_graphs == 0) return KC_OK;
  kc_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof(o));
  hipStream_t s = (hipStream_t)o.stream;
  const bool dev_in = o.device_ptrs != 0;
  // sizes (host): vertex and edge offsets of the union, largest k
  std::vector<int64_t> voff(num_graphs + 1), eoff(num_graphs + 1);
  std::vector<int32_t> m(num_graphs);
  int32_t kmax = 0;
  for (int32_t g = 0; g < num_graphs; ++g) {
    if (n[g] < 0 || k[g] < 1) return KC_EINVAL;
    if (dev_in) {
      KC_HIP(hipMemcpy(&m[g], row_ptr_cat + row_off[g] + n[g], sizeof(int32_t), hipMemcpyDeviceToHost));
    } else {
      m[g] = row_ptr_cat[row_off[g] + n[g]];
    }
    kmax = k[g] > kmax ? k[g] : kmax;
  }
  voff[0] = eoff[0] = 0;
  for (int32_t g = 0; g < num_graphs; ++g) {
    voff[g + 1] = voff[g] + n[g];
    eoff[g + 1] = eoff[g] + m[g];
  }
  const int64_t NV = voff[num_graphs], NE = eoff[num_graphs];
  if (NV >= INT32_MAX || NE >= INT32_MAX) return KC_EUNSUPPORTED;
  // graphs with k < 3 are answered directly; the rest join the union (their
  // k must be at least 3 for the listing path), with small k lifted out
  std::vector<uint64_t> result(num_graphs, 0);
  bool any_small = false;
  for (int32_t g = 0; g < num_graphs; ++g)
    if (k[g] <= 2) any_small = true;
  kc_scratch scr(s);
  int32_t *rp_u, *col_u, *vk_u, *gid, *kk_d, *n_d;
  int64_t *voff_d, *eoff_d, *roff_d, *coff_d;
  unsigned long long *rc, *sums;
  KC_TRY(scr.get(&rp_u, (size_t)NV + 1));
  KC_TRY(scr.get(&col_u, (size_t)NE + 1));
  KC_TRY(scr.get(&vk_u, (size_t)NV + 1));
  KC_TRY(scr.get(&gid, (size_t)NV + 1));
  KC_TRY(scr.get(&rc, (size_t)NV + 1));
  KC_TRY(scr.get(&sums, (size_t)num_graphs));
  KC_TRY(scr.get(&kk_d, (size_t)num_graphs));
  KC_TRY(scr.get(&n_d, (size_t)num_graphs));
  KC_TRY(scr.get(&voff_d, (size_t)num_graphs + 1));
  KC_TRY(scr.get(&eoff_d, (size_t)num_graphs + 1));
  KC_TRY(scr.get(&roff_d, (size_t)num_graphs));
  KC_TRY(scr.get(&coff_d, (size_t)num_graphs));
  std::vector<int32_t> kk(num_graphs);
  for (int32_t g = 0; g < num_graphs; ++g) kk[g] = k[g] < 3 ? 3 : k[g];
  KC_HIP(hipMemcpyAsync(kk_d, kk.data(), sizeof(int32_t) * num_graphs, hipMemcpyHostToDevice, s));
  KC_HIP(hipMemcpyAsync(n_d, n, sizeof(int32_t) * num_graphs, hipMemcpyHostToDevice, s));
  KC_HIP(hipMemcpyAsync(voff_d, voff.data(), sizeof(int64_t) * (num_graphs + 1), hipMemcpyHostToDevice, s));
  KC_HIP(hipMemcpyAsync(eoff_d, eoff.data(), sizeof(int64_t) * (num_graphs + 1), hipMemcpyHostToDevice, s));
  KC_HIP(hipMemcpyAsync(roff_d, row_off, sizeof(int64_t) * num_graphs, hipMemcpyHostToDevice, s));
  KC_HIP(hipMemcpyAsync(coff_d, col_off, sizeof(int64_t) * num_graphs, hipMemcpyHostToDevice, s));
  const int32_t* rp_src = row_ptr_cat;
  const int32_t* col_src = col_idx_cat;
  if (!dev_in) {
    // stage the concatenated host arrays
    int64_t rtot = 0, ctot = 0;
    for (int32_t g = 0; g < num_graphs; ++g) {
      rtot = row_off[g] + n[g] + 1 > rtot ? row_off[g] + n[g] + 1 : rtot;
      ctot = col_off[g] + m[g] > ctot ? col_off[g] + m[g] : ctot;
    }
    int32_t *r_d, *c_d;
    KC_TRY(scr.get(&r_d, (size_t)rtot + 1));
    KC_TRY(scr.get(&c_d, (size_t)ctot + 1));
    KC_HIP(hipMemcpyAsync(r_d, row_ptr_cat, sizeof(int32_t) * rtot, hipMemcpyHostToDevice, s));
    if (ctot > 0) KC_HIP(hipMemcpyAsync(c_d, col_idx_cat, sizeof(int32_t) * ctot, hipMemcpyHostToDevice, s));
    rp_src = r_d;
    col_src = c_d;
  }
  dim3 grid_r(64, num_graphs), grid_c(256, num_graphs);
  k_union_rows<<<grid_r, 256, 0, s>>>(num_graphs, n_d, voff_d, roff_d, eoff_d, rp_src, rp_u, vk_u, kk_d, gid);
  k_union_cols<<<grid_c, 256, 0, s>>>(num_graphs, n_d, voff_d, roff_d, coff_d, eoff_d, rp_src, col_src, col_u);
  KC_HIP(hipGetLastError());
  int32_t last = (int32_t)NE;
  KC_HIP(hipMemcpyAsync(rp_u + NV, &last, sizeof(int32_t), hipMemcpyHostToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  kc_options u = o;
  u.device_ptrs = 1;
  u.vertex_k = vk_u;
  u.root_count = (uint64_t*)rc;
  u.root_work = nullptr;
  u.root_isect = nullptr;
  u.root_features = nullptr;
  uint64_t total = 0;
  KC_TRY(count_impl((int32_t)NV, rp_u, col_u, kmax < 3 ? 3 : kmax, order, &u, &total, nullptr));
  KC_HIP(hipMemsetAsync(sums, 0, sizeof(unsigned long long) * num_graphs, s));
  k_graph_sums<<<(unsigned)((NV + 255) / 256), 256, 0, s>>>((int32_t)NV, gid, rc, sums);
  KC_HIP(hipGetLastError());
  KC_HIP(hipMemcpyAsync(result.data(), sums, sizeof(uint64_t) * num_graphs, hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  // k = 1 and k = 2 directly
  if (any_small)
    for (int32_t g = 0; g < num_graphs; ++g)
      if (k[g] == 1) result[g] = (uint64_t)n[g];
      else if (k[g] == 2) result[g] = (uint64_t)m[g] / 2;
  if (dev_in) {
    KC_HIP(hipMemcpyAsync(counts_out, result.data(), sizeof(uint64_t) * num_graphs, hipMemcpyHostToDevice, s));
    KC_HIP(hipStreamSynchronize(s));
  } else {
    memcpy(counts_out, result.data(), sizeof(uint64_t) * num_graphs);
  }
  return KC_OK;
}
