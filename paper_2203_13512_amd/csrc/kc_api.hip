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

#include <mutex>
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
    case KC_EWORKSPACE: return "workspace smaller than the call needs (see kclique_workspace_size)";
  }
  return "unknown status";
}

__global__ void k_roots(int32_t n, const int32_t* __restrict__ drp, int32_t km1, const int32_t* vk,
                        const uint8_t* __restrict__ mask, int32_t* roots, int32_t* nroots, int32_t* max_dplus) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t d = u < n ? drp[u + 1] - drp[u] : 0;
  bool take = u < n && d >= kc_vk(vk, u, km1 + 1) - 1 && (!mask || mask[u]);
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

// Listing output for k = 1 (every vertex) and k = 2 (every edge, as (u, v)
// with u < v; rows of vertex u start at the prefix sum of the higher
// neighbour counts).
__global__ void k_emit_k1(int32_t n, kc_emit e) {
  const int64_t T = n < e.cap ? n : e.cap;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T; v += (int64_t)gridDim.x * blockDim.x)
    e.out[v] = (int32_t)v;
}
__global__ void k_higher_deg(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t* hd) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= n) return;
  const int32_t u = (int32_t)wave;
  int32_t c = 0;
  for (int32_t i = rp[u] + kc_lane(); i < rp[u + 1]; i += KC_WAVE) c += col[i] > u;
  c = (int32_t)kc_wave_sum_u32((uint32_t)c);
  if (kc_lane() == 0) hd[u] = c;
}
__global__ void k_emit_k2(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const int32_t* __restrict__ off, kc_emit e) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= n) return;
  const int32_t u = (int32_t)wave;
  int64_t o = off[u];
  const int32_t b = rp[u], en = rp[u + 1];
  for (int32_t base = b; base < en; base += KC_WAVE) {
    const int32_t i = base + kc_lane();
    const int32_t v = i < en ? col[i] : -1;
    const bool take = v > u;
    const uint64_t m = kc_ballot(take);
    const int64_t row = o + kc_mbcnt(m);
    if (take && row < e.cap) {
      e.out[2 * row] = u;
      e.out[2 * row + 1] = v;
    }
    o += __popcll(m);
  }
}

// Timing events of a call, created only when statistics are asked for.
struct HostEvents {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  int init(bool want) {
    on = want;
    if (on)
      for (auto& x : e) KC_HIP(hipEventCreate(&x));
    return KC_OK;
  }
  int record(int i, hipStream_t s) {
    if (on) KC_HIP(hipEventRecord(e[i], s));
    return KC_OK;
  }
  ~HostEvents() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

// With `cap` the call is prepared only: everything up to the listing phase
// runs (in `ext_scr`, which the caller keeps), and the listing phase is handed
// over in `cap` instead of being launched (BitCol counting only).  With
// `size_out` the call runs up to the listing phase on scratch it allocates
// itself and reports the workspace an identical call needs.
static int count_impl(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                      const kc_options* opt_in, uint64_t* count_out, uint64_t* pv_out,
                      kc_scratch* ext_scr = nullptr, kc_capture* cap = nullptr, size_t* size_out = nullptr,
                      bool size_pv = false, int32_t* list_out = nullptr, int64_t list_cap = 0,
                      int64_t* written_out = nullptr) {
  kc_options defaults;
  memset(&defaults, 0, sizeof(defaults));
  const kc_options* opt = opt_in ? opt_in : &defaults;
  if (n < 0 || k < 1 || !count_out) return KC_EINVAL;
  if (cap && (!ext_scr || order != KC_ORDER_COLOR || pv_out)) return KC_EUNSUPPORTED;
  if (order < KC_ORDER_DEGREE || order > KC_ORDER_CORE_REDUCED) return KC_EINVAL;
  // the reduced SDegree orders orient the graph as their base order does
  const bool reduce = order == KC_ORDER_DEGREE_REDUCED || order == KC_ORDER_CORE_REDUCED;
  if (order == KC_ORDER_DEGREE_REDUCED) order = KC_ORDER_DEGREE;
  if (order == KC_ORDER_CORE_REDUCED) order = KC_ORDER_CORE;
  if (opt->disable & ~(KC_NO_PRECORE | KC_NO_PRELIST | KC_NO_PRUNE)) return KC_EINVAL;
  if (opt->schedule != KC_SCHED_DEGREE && opt->schedule != KC_SCHED_LEARNED) return KC_EINVAL;
  if (n > 0 && !row_ptr) return KC_EINVAL;
  if (opt->workspace && !ext_scr && !size_out && opt->workspace_bytes == 0) return KC_EWORKSPACE;
  const bool listing = written_out != nullptr;
  if (listing && (pv_out || cap || opt->vertex_k || list_cap < 0 || (list_cap > 0 && !list_out))) return KC_EINVAL;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return KC_EDEVICE;
  hipStream_t s = (hipStream_t)opt->stream;
  kc_stats* stats = opt->stats;
  if (stats) memset(stats, 0, sizeof(*stats));
  HostEvents ev;
  KC_TRY(ev.init(stats != nullptr && !size_out));
  KC_TRY(ev.record(0, s));

  const bool own_arena = opt->workspace && !ext_scr && !size_out;
  kc_scratch local_scr(s, own_arena ? opt->workspace : nullptr, own_arena ? opt->workspace_bytes : 0);
  kc_scratch& scr = ext_scr ? *ext_scr : local_scr;
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
  kc_scratch pv_standin(s);  // a size query's stand-in for the caller's device array (not counted)
  if (pv_out || size_pv) {
    if (opt->device_ptrs && pv_out) pv_d = (unsigned long long*)pv_out;
    else if (opt->device_ptrs) KC_TRY(pv_standin.get(&pv_d, (size_t)n + 1));
    else KC_TRY(scr.get(&pv_d, (size_t)n + 1));
    if (n > 0) KC_HIP(hipMemsetAsync(pv_d, 0, sizeof(unsigned long long) * (size_t)n, s));
  }
  kc_emit em;
  unsigned long long small_rows = 0;  // rows of the k <= 2 output (host source of a copy)
  if (listing) {
    em.cap = list_cap;
    KC_TRY(scr.get(&em.pos, 2));
    KC_HIP(hipMemsetAsync(em.pos, 0, sizeof(unsigned long long), s));
    if (opt->device_ptrs) em.out = list_out;
    else if (list_cap > 0) KC_TRY(scr.get(&em.out, (size_t)list_cap * (size_t)k));
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
  const uint8_t* mask = opt->root_mask;
  if (mask && !opt->device_ptrs) return KC_EINVAL;
  if (mask && k < 3) return KC_EUNSUPPORTED;
  if (k <= 2 || (k > n && !vk)) {
    if (cap) return KC_EUNSUPPORTED;
    // linear cases and the empty answer
    if (k == 1) total = (uint64_t)n;
    else if (k == 2) total = (uint64_t)nnz32 / 2;
    if (pv_d && n > 0 && k <= 2) {
      k_small_k<<<(n + 255) / 256, 256, 0, s>>>(n, g.rp, k, pv_d);
      KC_HIP(hipGetLastError());
    }
    if (listing && n > 0 && k <= 2 && list_cap > 0) {
      if (k == 1) {
        k_emit_k1<<<1024, 256, 0, s>>>(n, em);
      } else {
        int32_t *hd, *off;
        KC_TRY(scr.get(&hd, (size_t)n + 1));
        KC_TRY(scr.get(&off, (size_t)n + 1));
        k_higher_deg<<<(unsigned)(((int64_t)n * KC_WAVE + 255) / 256), 256, 0, s>>>(n, g.rp, g.col, hd);
        KC_HIP(hipGetLastError());
        KC_TRY(kc_scan_i32(hd, off, n, nullptr, scr, s));
        k_emit_k2<<<(unsigned)(((int64_t)n * KC_WAVE + 255) / 256), 256, 0, s>>>(n, g.rp, g.col, off, em);
      }
      KC_HIP(hipGetLastError());
    }
    if (listing) {
      small_rows = k <= 2 ? (unsigned long long)total : 0ull;
      KC_HIP(hipMemcpyAsync(em.pos, &small_rows, sizeof(small_rows), hipMemcpyHostToDevice, s));
    }
    KC_TRY(ev.record(1, s));
    KC_TRY(ev.record(2, s));
  } else {
    if (k > KC_KMAX_LIMIT) return KC_EUNSUPPORTED;
    kc_prep_out prep;
    KC_TRY(kc_preprocess(g, k, vk, order, prelist_d, pv_d, (unsigned long long*)opt->root_count, flags, &prep,
                         scr, s, listing ? &em : nullptr, opt->disable, mask));
    KC_TRY(ev.record(1, s));
    int32_t *roots, *rinfo;
    KC_TRY(scr.get(&roots, (size_t)n + 1));
    KC_TRY(scr.get(&rinfo, 4));
    KC_HIP(hipMemsetAsync(rinfo, 0, sizeof(int32_t) * 4, s));
    k_roots<<<(n + 255) / 256, 256, 0, s>>>(n, prep.drp, k - 1, vk, mask, roots, rinfo, rinfo + 1);
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
    c.capture = cap;
    c.size_only = size_out != nullptr;
    c.emit = listing ? &em : nullptr;
    c.reduce = reduce;
    KC_TRY(ev.record(2, s));
    if (order == KC_ORDER_COLOR) KC_TRY(kc_list_bitcol(c, scr, s));
    else KC_TRY(kc_list_sdegree(c, scr, s));
    if (size_out) {
      KC_HIP(hipStreamSynchronize(s));
      *size_out = scr.need;
      return KC_OK;
    }
    if (cap) {
      KC_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
      KC_HIP(hipStreamSynchronize(s));
      if (hflags & KC_FLAG_OVERFLOW) return KC_EOVERFLOW;
      if (hflags & KC_FLAG_TOOBIG) return KC_EUNSUPPORTED;
      cap->count_d = count_d;
      cap->flags = flags;
      return KC_OK;
    }
    if (stats) {
      stats->n_roots = hr[0];
      stats->max_out_degree = hr[1];
      stats->max_core = prep.max_core;
    }
  }
  if (size_out) {  // k <= 2 or k > n: nothing to list
    *size_out = scr.need;
    return KC_OK;
  }
  KC_TRY(ev.record(3, s));
  // ---- results
  unsigned long long hres[2] = {0, 0}, hcnt[8];
  KC_HIP(hipMemcpyAsync(hres, count_d, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(hres + 1, prelist_d, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(hcnt, counters, sizeof(hcnt), hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  if (pv_out && !opt->device_ptrs && n > 0)
    KC_HIP(hipMemcpyAsync(pv_out, pv_d, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  unsigned long long reserved = 0;
  if (listing) KC_HIP(hipMemcpyAsync(&reserved, em.pos, sizeof(reserved), hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  if (listing) {
    const int64_t written = (int64_t)(reserved < (unsigned long long)list_cap ? reserved : (unsigned long long)list_cap);
    *written_out = written;
    if (!opt->device_ptrs && written > 0) {
      KC_HIP(hipMemcpyAsync(list_out, em.out, sizeof(int32_t) * (size_t)written * (size_t)k, hipMemcpyDeviceToHost,
                            s));
      KC_HIP(hipStreamSynchronize(s));
    }
  }
  if (hflags & KC_FLAG_OVERFLOW) return KC_EOVERFLOW;
  if (hflags & KC_FLAG_TOOBIG) return KC_EUNSUPPORTED;
  if (k > 2 && (k <= n || vk)) {
    total = hres[0] + hres[1];
    if (total < hres[0]) return KC_EOVERFLOW;
  }
  *count_out = total;
  if (stats) {
    float t = 0.f;
    if (ev.on && hipEventElapsedTime(&t, ev.e[0], ev.e[3]) == hipSuccess) stats->total_ms = t;
    if (ev.on && hipEventElapsedTime(&t, ev.e[0], ev.e[1]) == hipSuccess) stats->prep_ms = t;
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

extern "C" int kclique_list(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                            const kc_options* opt, int32_t* cliques_out, int64_t capacity, int64_t* written_out,
                            uint64_t* count_out) {
  if (!written_out || !count_out) return KC_EINVAL;
  *written_out = 0;
  kc_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof(o));
  // the schedule and the per-root logs do not apply to the output pass
  o.root_work = nullptr;
  o.root_isect = nullptr;
  o.root_features = nullptr;
  return count_impl(n, row_ptr, col_idx, k, order, &o, count_out, nullptr, nullptr, nullptr, nullptr, false,
                    cliques_out, capacity, written_out);
}

// ------------------------------------------------ allocation-free entry point
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid it): every byte of a call's
// scratch comes from `scratch`, a fixed array in the library's device code
// that each GPU the library runs on holds until the process ends.  Its device
// address is looked up once per device (the host-side name of the array is
// not a device address).  Calls on one GPU share the array: overlapping calls
// on one GPU race, so the caller serialises them.
#define KC_NOALLOC_BYTES ((size_t)256 << 20)
#define KC_NOALLOC_DEVICES 64
static __device__ __align__(256) unsigned char scratch[KC_NOALLOC_BYTES];
static void* g_scratch_ptr[KC_NOALLOC_DEVICES];
static std::mutex g_scratch_mu;

static int noalloc_scratch(void** out) {
  int dev = -1;
  KC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= KC_NOALLOC_DEVICES) return KC_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    KC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return KC_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KC_OK;
}

extern "C" int kclique_count_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k,
                                     int32_t order, const kc_options* opt, uint64_t* count_out,
                                     uint64_t* per_vertex_out) {
  void* ws = nullptr;
  KC_TRY(noalloc_scratch(&ws));
  kc_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof(o));
  o.workspace = ws;
  o.workspace_bytes = KC_NOALLOC_BYTES;
  o.class_streams = 1;  // no streams or events are created either
  o.stats = nullptr;
  return count_impl(n, row_ptr, col_idx, k, order, &o, count_out, per_vertex_out);
}

extern "C" int kclique_workspace_size(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k,
                                      int32_t order, int32_t per_vertex, const kc_options* opt, size_t* bytes) {
  if (!bytes) return KC_EINVAL;
  *bytes = 0;
  kc_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof(o));
  o.workspace = nullptr;
  o.workspace_bytes = 0;
  o.stats = nullptr;
  o.root_work = nullptr;
  o.root_isect = nullptr;
  o.root_features = nullptr;
  o.root_count = nullptr;
  uint64_t unused = 0;
  return count_impl(n, row_ptr, col_idx, k, order, &o, &unused, nullptr, nullptr, nullptr, bytes, per_vertex != 0);
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

// The union of a batch of graphs on the device (vertex ids shifted by the
// preceding graphs' sizes), with each vertex's k (graphs with k < 3 are
// answered directly and take part with k = 3) and its graph's index.
struct BatchUnion {
  int32_t ng = 0;
  int64_t NV = 0, NE = 0;
  int32_t kmax = 0;
  std::vector<int32_t> n, m, k;  // per graph: vertices, adjacency entries, requested k
  int32_t *rp = nullptr, *col = nullptr, *vk = nullptr, *gid = nullptr;
};

static int build_union(int32_t num_graphs, const int32_t* n, const int64_t* row_off, const int64_t* col_off,
                       const int32_t* row_ptr_cat, const int32_t* col_idx_cat, const int32_t* k, bool dev_in,
                       kc_scratch& scr, hipStream_t s, BatchUnion* U) {
  U->ng = num_graphs;
  U->n.assign(n, n + num_graphs);
  U->k.assign(k, k + num_graphs);
  U->m.assign(num_graphs, 0);
  std::vector<int64_t> voff(num_graphs + 1), eoff(num_graphs + 1);
  U->kmax = 0;
  for (int32_t g = 0; g < num_graphs; ++g) {
    if (n[g] < 0 || k[g] < 1) return KC_EINVAL;
    if (dev_in) {
      KC_HIP(hipMemcpy(&U->m[g], row_ptr_cat + row_off[g] + n[g], sizeof(int32_t), hipMemcpyDeviceToHost));
    } else {
      U->m[g] = row_ptr_cat[row_off[g] + n[g]];
    }
    if (U->m[g] < 0) return KC_EINVAL;
    U->kmax = k[g] > U->kmax ? k[g] : U->kmax;
  }
  voff[0] = eoff[0] = 0;
  for (int32_t g = 0; g < num_graphs; ++g) {
    voff[g + 1] = voff[g] + n[g];
    eoff[g + 1] = eoff[g] + U->m[g];
  }
  U->NV = voff[num_graphs];
  U->NE = eoff[num_graphs];
  if (U->NV >= INT32_MAX || U->NE >= INT32_MAX) return KC_EUNSUPPORTED;
  int32_t *kk_d, *n_d;
  int64_t *voff_d, *eoff_d, *roff_d, *coff_d;
  KC_TRY(scr.get(&U->rp, (size_t)U->NV + 1));
  KC_TRY(scr.get(&U->col, (size_t)U->NE + 1));
  KC_TRY(scr.get(&U->vk, (size_t)U->NV + 1));
  KC_TRY(scr.get(&U->gid, (size_t)U->NV + 1));
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
      ctot = col_off[g] + U->m[g] > ctot ? col_off[g] + U->m[g] : ctot;
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
  k_union_rows<<<grid_r, 256, 0, s>>>(num_graphs, n_d, voff_d, roff_d, eoff_d, rp_src, U->rp, U->vk, kk_d, U->gid);
  k_union_cols<<<grid_c, 256, 0, s>>>(num_graphs, n_d, voff_d, roff_d, coff_d, eoff_d, rp_src, col_src, U->col);
  KC_HIP(hipGetLastError());
  int32_t last = (int32_t)U->NE;
  KC_HIP(hipMemcpyAsync(U->rp + U->NV, &last, sizeof(int32_t), hipMemcpyHostToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

// Options of the union's call: per-vertex k and per-root attribution.
static kc_options union_options(const kc_options& o, const BatchUnion& U, unsigned long long* rc) {
  kc_options u = o;
  u.device_ptrs = 1;
  u.workspace = nullptr;  // batched calls and plans allocate their own scratch
  u.workspace_bytes = 0;
  u.vertex_k = U.vk;
  u.root_mask = nullptr;
  u.root_count = (uint64_t*)rc;
  u.root_work = nullptr;
  u.root_isect = nullptr;
  u.root_features = nullptr;
  u.stats = nullptr;
  return u;
}

// Per-graph results: the union's per-graph sums, with k = 1 and k = 2 answered
// directly; written to host or device memory.
static int finish_batch(const BatchUnion& U, const uint64_t* sums_host, bool dev_out, uint64_t* counts_out,
                        hipStream_t s) {
  std::vector<uint64_t> result(sums_host, sums_host + U.ng);
  for (int32_t g = 0; g < U.ng; ++g)
    if (U.k[g] == 1) result[g] = (uint64_t)U.n[g];
    else if (U.k[g] == 2) result[g] = (uint64_t)U.m[g] / 2;
  if (dev_out) {
    KC_HIP(hipMemcpyAsync(counts_out, result.data(), sizeof(uint64_t) * U.ng, hipMemcpyHostToDevice, s));
    KC_HIP(hipStreamSynchronize(s));
  } else {
    memcpy(counts_out, result.data(), sizeof(uint64_t) * U.ng);
  }
  return KC_OK;
}

extern "C" int kclique_count_batched(int32_t num_graphs, const int32_t* n, const int64_t* row_off,
                                     const int64_t* col_off, const int32_t* row_ptr_cat, const int32_t* col_idx_cat,
                                     const int32_t* k, int32_t order, const kc_options* opt, uint64_t* counts_out) {
  if (num_graphs < 0 || (num_graphs > 0 && (!n || !row_off || !col_off || !k || !counts_out))) return KC_EINVAL;
  if (num_graphs == 0) return KC_OK;
  kc_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof(o));
  if (o.root_mask) return KC_EINVAL;  // a mask over the union's vertices is not offered
  hipStream_t s = (hipStream_t)o.stream;
  const bool dev_in = o.device_ptrs != 0;
  kc_scratch scr(s);
  BatchUnion U;
  KC_TRY(build_union(num_graphs, n, row_off, col_off, row_ptr_cat, col_idx_cat, k, dev_in, scr, s, &U));
  unsigned long long *rc, *sums;
  KC_TRY(scr.get(&rc, (size_t)U.NV + 1));
  KC_TRY(scr.get(&sums, (size_t)num_graphs));
  kc_options u = union_options(o, U, rc);
  uint64_t total = 0;
  KC_TRY(count_impl((int32_t)U.NV, U.rp, U.col, U.kmax < 3 ? 3 : U.kmax, order, &u, &total, nullptr));
  KC_HIP(hipMemsetAsync(sums, 0, sizeof(unsigned long long) * num_graphs, s));
  k_graph_sums<<<(unsigned)((U.NV + 255) / 256), 256, 0, s>>>((int32_t)U.NV, U.gid, rc, sums);
  KC_HIP(hipGetLastError());
  std::vector<uint64_t> hs(num_graphs);
  KC_HIP(hipMemcpyAsync(hs.data(), sums, sizeof(uint64_t) * num_graphs, hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  return finish_batch(U, hs.data(), dev_in, counts_out, s);
}

// ------------------------------------------------------------ plans
// A prepared batch: preprocessing, orientation, staging and scheduling ran
// once; the listing phase and the per-graph sums are a captured HIP graph that
// each execution replays.  The graph starts by restoring the state the
// listing phase starts from (totals and flags cleared, per-root attribution
// back to the Pre-List part), with kernels only.
__global__ void k_plan_reset(unsigned long long* count_d, int* flags, unsigned long long* rc,
                             const unsigned long long* __restrict__ rc_pre, int64_t nv, unsigned long long* sums,
                             int32_t ng) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < nv; i += stride) rc[i] = rc_pre[i];
  for (int64_t i = i0; i < ng; i += stride) sums[i] = 0;
  if (i0 == 0) {
    count_d[0] = 0;
    for (int j = 0; j < 4; ++j) flags[j] = 0;
  }
}

struct kc_plan {
  int device = 0;
  hipStream_t cs = nullptr;  // capture stream
  kc_scratch* scr = nullptr;
  kc_capture cap;
  BatchUnion U;
  unsigned long long *rc = nullptr, *rc_pre = nullptr, *sums = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool dev_out = false;
  ~kc_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamSynchronize(cs);
    delete scr;  // frees on its stream
    if (cs) {
      (void)hipStreamSynchronize(cs);
      (void)hipStreamDestroy(cs);
    }
  }
};

static int plan_batched(int32_t num_graphs, const int32_t* n, const int64_t* row_off, const int64_t* col_off,
                        const int32_t* row_ptr_cat, const int32_t* col_idx_cat, const int32_t* k, int32_t order,
                        const kc_options* opt, kc_plan* P) {
  kc_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof(o));
  if (o.root_mask) return KC_EINVAL;
  const bool dev_in = o.device_ptrs != 0;
  P->dev_out = dev_in;
  KC_HIP(hipGetDevice(&P->device));
  KC_HIP(hipStreamCreateWithFlags(&P->cs, hipStreamNonBlocking));
  hipStream_t s = P->cs;
  o.stream = (void*)s;
  P->scr = new kc_scratch(s);
  KC_TRY(build_union(num_graphs, n, row_off, col_off, row_ptr_cat, col_idx_cat, k, dev_in, *P->scr, s, &P->U));
  const BatchUnion& U = P->U;
  KC_TRY(P->scr->get(&P->rc, (size_t)U.NV + 1));
  KC_TRY(P->scr->get(&P->rc_pre, (size_t)U.NV + 1));
  KC_TRY(P->scr->get(&P->sums, (size_t)num_graphs));
  kc_options u = union_options(o, U, P->rc);
  u.class_streams = 1;  // one stream: the replay is a chain of kernels
  uint64_t unused = 0;
  KC_TRY(count_impl((int32_t)U.NV, U.rp, U.col, U.kmax < 3 ? 3 : U.kmax, order, &u, &unused, nullptr, P->scr,
                    &P->cap));
  // the attribution so far is Pre-List's; every replay starts from it
  KC_HIP(hipMemcpyAsync(P->rc_pre, P->rc, sizeof(unsigned long long) * (size_t)U.NV, hipMemcpyDeviceToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  KC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int st = KC_OK;
  {
    const int64_t nv = U.NV > num_graphs ? U.NV : num_graphs;
    const unsigned blocks = (unsigned)((nv + 255) / 256 < 4096 ? (nv + 255) / 256 : 4096);
    k_plan_reset<<<blocks > 0 ? blocks : 1, 256, 0, s>>>(P->cap.count_d, P->cap.flags, P->rc, P->rc_pre, U.NV,
                                                         P->sums, num_graphs);
    if (P->cap.launch) st = P->cap.launch(P->cap.state, s);
    if (st == KC_OK && U.NV > 0)
      k_graph_sums<<<(unsigned)((U.NV + 255) / 256), 256, 0, s>>>((int32_t)U.NV, U.gid, P->rc, P->sums);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  P->graph = g;
  if (st != KC_OK) return st;
  KC_HIP(e);
  KC_HIP(hipGetLastError());
  KC_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
  return KC_OK;
}

extern "C" int kclique_plan_batched(int32_t num_graphs, const int32_t* n, const int64_t* row_off,
                                    const int64_t* col_off, const int32_t* row_ptr_cat, const int32_t* col_idx_cat,
                                    const int32_t* k, int32_t order, const kc_options* opt, kc_plan** plan_out) {
  if (!plan_out) return KC_EINVAL;
  *plan_out = nullptr;
  if (num_graphs < 1 || !n || !row_off || !col_off || !k || !row_ptr_cat) return KC_EINVAL;
  if (order != KC_ORDER_COLOR) return KC_EUNSUPPORTED;
  kc_plan* P = new kc_plan;
  const int st = plan_batched(num_graphs, n, row_off, col_off, row_ptr_cat, col_idx_cat, k, order, opt, P);
  if (st != KC_OK) {
    delete P;
    return st;
  }
  *plan_out = P;
  return KC_OK;
}

extern "C" int kclique_plan_execute(kc_plan* P, void* stream, uint64_t* counts_out) {
  if (!P || !counts_out || !P->exec) return KC_EINVAL;
  int dev = -1;
  KC_HIP(hipGetDevice(&dev));
  if (dev != P->device) return KC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  KC_HIP(hipGraphLaunch(P->exec, s));
  std::vector<uint64_t> hs(P->U.ng);
  int hflags = 0;
  KC_HIP(hipMemcpyAsync(hs.data(), P->sums, sizeof(uint64_t) * P->U.ng, hipMemcpyDeviceToHost, s));
  KC_HIP(hipMemcpyAsync(&hflags, P->cap.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  if (hflags & KC_FLAG_OVERFLOW) return KC_EOVERFLOW;
  if (hflags & KC_FLAG_TOOBIG) return KC_EUNSUPPORTED;
  return finish_batch(P->U, hs.data(), P->dev_out, counts_out, s);
}

extern "C" int kclique_plan_destroy(kc_plan* P) {
  delete P;
  return KC_OK;
}
