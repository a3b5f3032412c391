// kc_prep.hip -- input validation, Pre-Core, Pre-List and orientations.
//
// Paper passages: Pre-Core is Alg. 3 (Sec. 5.1), Pre-List is Alg. 4
// (Sec. 5.2), the degree orientation is Sec. 6.2 (u -> v iff d_u < d_v, ties
// by id) and the degeneracy orientation is the one BitCol uses (Sec. 7.4).
//
// GPU design: every step is a data-parallel sweep over a frontier or over all
// vertices.  Pre-Core peels in frontier rounds: one decrement per incident
// edge, and the unique decrement that takes a degree from k-1 to k-2 enqueues
// the vertex (so each vertex enters the queue once, as in Alg. 3).  Pre-List
// finds components by lock-free union-find (hooking the larger root onto the
// smaller with compare-and-swap), then tallies vertices and degree sums per
// component.  The degeneracy order is a synchronous peel: at level c every
// live vertex of live degree <= c is removed in the same round; a round's
// number orders vertices (ties by id), so out-degrees never exceed core
// numbers.  DAG rows keep ascending id order (one wave per row, ballot
// compaction).
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include "kc_internal.h"

static char g_last_error[256];
void kc_set_hip_error(hipError_t e, const char* what, const char* file, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s failed (%s) at %s:%d", what, hipGetErrorString(e), file, line);
}

kc_scratch::~kc_scratch() {
  for (int i = 0; i < count; ++i) (void)hipFreeAsync(ptrs[i], stream);
  free(ptrs);
}
int kc_scratch::alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  bytes = (bytes + KC_SCRATCH_ALIGN - 1) & ~(size_t)(KC_SCRATCH_ALIGN - 1);
  const size_t at = need;
  need += bytes;
  if (arena) {
    if (need > arena_bytes) return KC_EWORKSPACE;
    *p = arena + at;
    return KC_OK;
  }
  if (count == cap) {
    const int ncap = cap ? 2 * cap : 64;
    void** np = (void**)realloc(ptrs, sizeof(void*) * (size_t)ncap);
    if (!np) return KC_ENOMEM;
    ptrs = np;
    cap = ncap;
  }
  hipError_t e = hipMallocAsync(p, bytes, stream);
  if (e != hipSuccess) {
    kc_set_hip_error(e, "hipMallocAsync", __FILE__, __LINE__);
    *p = nullptr;
    return KC_ENOMEM;
  }
  ptrs[count++] = *p;
  return KC_OK;
}

// ------------------------------------------------------------------- scan
#define SCAN_BLOCK 256
#define SCAN_ITEMS 8
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)

template <class T>
__global__ void k_scan_tiles(const T* in, T* out, int64_t n, T* tile_sums) {
  __shared__ T sh[SCAN_BLOCK];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    T x = idx < n ? in[idx] : (T)0;
    v[i] = run;
    run += x;
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele over the per-thread sums
  for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
    T y = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : (T)0;
    __syncthreads();
    sh[threadIdx.x] += y;
    __syncthreads();
  }
  T excl = threadIdx.x ? sh[threadIdx.x - 1] : (T)0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = v[i] + excl;
  }
  if (threadIdx.x == SCAN_BLOCK - 1) tile_sums[blockIdx.x] = sh[SCAN_BLOCK - 1];
}

template <class T>
__global__ void k_scan_add(T* out, int64_t n, const T* tile_offsets) {
  int64_t idx = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
  T add = tile_offsets[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i, idx += SCAN_BLOCK)
    if (idx < n) out[idx] += add;
}

template <class T>
__global__ void k_scan_total(const T* in, const T* out, int64_t n, T* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = n > 0 ? out[n - 1] + in[n - 1] : (T)0;
}

template <class T>
static int scan_impl(const T* in, T* out, int64_t n, T* total_dev, kc_scratch& scr, hipStream_t s) {
  if (n <= 0) {
    if (total_dev) KC_HIP(hipMemsetAsync(total_dev, 0, sizeof(T), s));
    return KC_OK;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  // the last input value is needed for the total; keep it before `out` may
  // overwrite an aliased `in`.  The temporaries live until the call ends.
  T* last = nullptr;
  KC_TRY(scr.get(&last, (size_t)tiles + 2));
  T* sums = last + 1;
  KC_HIP(hipMemcpyAsync(last, in + (n - 1), sizeof(T), hipMemcpyDeviceToDevice, s));
  k_scan_tiles<T><<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, out, n, sums);
  KC_HIP(hipGetLastError());
  if (tiles > 1) {
    T* sums_scanned = nullptr;
    KC_TRY(scr.get(&sums_scanned, (size_t)tiles + 1));
    KC_TRY(scan_impl<T>(sums, sums_scanned, tiles, (T*)nullptr, scr, s));
    k_scan_add<T><<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(out, n, sums_scanned);
    KC_HIP(hipGetLastError());
  }
  if (total_dev) {
    k_scan_total<T><<<1, 1, 0, s>>>(last, out + (n - 1), 1, total_dev);
    KC_HIP(hipGetLastError());
  }
  return KC_OK;
}

int kc_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev, kc_scratch& scr, hipStream_t s) {
  return scan_impl<int32_t>(in, out, n, total_dev, scr, s);
}
int kc_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total_dev, kc_scratch& scr, hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, total_dev, scr, s);
}

// -------------------------------------------------------------- validation
// One wave per vertex: rows ascending, ids in range, no loops, and the
// reverse of every entry present (binary search in the other row).
__global__ void k_validate(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           int64_t nnz, int* flags) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  int lane = kc_lane();
  if (wave > n) return;
  if (wave == n) {
    if (lane == 0 && ((n > 0 && rp[0] != 0) || (int64_t)rp[n] != nnz)) atomicOr(flags, KC_FLAG_BADGRAPH);
    return;
  }
  int32_t v = (int32_t)wave;
  int32_t b = rp[v], e = rp[v + 1];
  if (e < b || b < 0 || (int64_t)e > nnz) {
    if (lane == 0) atomicOr(flags, KC_FLAG_BADGRAPH);
    return;
  }
  bool bad = false;
  for (int32_t i = b + lane; i < e; i += KC_WAVE) {
    int32_t w = col[i];
    if (w < 0 || w >= n || w == v) { bad = true; continue; }
    if (i > b && col[i - 1] >= w) { bad = true; continue; }
    int32_t lo = rp[w], hi = rp[w + 1];
    if (lo < 0 || hi < lo || (int64_t)hi > nnz) { bad = true; continue; }
    while (lo < hi) {
      int32_t mid = lo + ((hi - lo) >> 1);
      if (col[mid] < v) lo = mid + 1; else hi = mid;
    }
    if (lo >= rp[w + 1] || col[lo] != v) bad = true;
  }
  if (kc_ballot(bad) && lane == 0) atomicOr(flags, KC_FLAG_BADGRAPH);
}

int kc_validate_graph(const kc_dev_graph& g, int* flags_dev, hipStream_t s) {
  int64_t waves = (int64_t)g.n + 1;
  int64_t threads = waves * KC_WAVE;
  unsigned blocks = (unsigned)((threads + 255) / 256);
  k_validate<<<blocks, 256, 0, s>>>(g.n, g.rp, g.col, g.nnz, flags_dev);
  KC_HIP(hipGetLastError());
  return KC_OK;
}

// ---------------------------------------------------------------- Pre-Core
__global__ void k_precore_init(int32_t n, const int32_t* __restrict__ rp, int32_t km1, const int32_t* vk,
                               int32_t* deg, uint8_t* removed, int32_t* F, int32_t* fcount, bool skip) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t d = rp[v + 1] - rp[v];
  deg[v] = d;
  bool rm = !skip && d < kc_vk(vk, v, km1 + 1) - 1;
  removed[v] = rm ? 1 : 0;
  if (rm) F[atomicAdd(fcount, 1)] = v;
}

// One wave per frontier vertex; every neighbour's degree drops by one and the
// decrement that crosses from km1 to km1-1 enqueues it.
__global__ void k_precore_peel(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t km1,
                               const int32_t* vk, const int32_t* __restrict__ F, int32_t nf, int32_t* deg,
                               uint8_t* removed, int32_t* Fnext, int32_t* fnext_count) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= nf) return;
  int lane = kc_lane();
  int32_t u = F[wave];
  for (int32_t i = rp[u] + lane; i < rp[u + 1]; i += KC_WAVE) {
    int32_t v = col[i];
    int32_t old = atomicSub(&deg[v], 1);
    if (old == kc_vk(vk, v, km1 + 1) - 1) {
      removed[v] = 1;
      Fnext[atomicAdd(fnext_count, 1)] = v;
    }
  }
}

// ---------------------------------------------------------------- Pre-List
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t v) {
  for (;;) {
    int32_t p = parent[v];
    if (p == v) return v;
    int32_t gp = parent[p];
    if (gp != p) parent[v] = gp;  // path halving (benign race: gp is an ancestor)
    v = p;
  }
}

__global__ void k_uf_init(int32_t n, const uint8_t* removed, int32_t* parent) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) parent[v] = v;
}

__global__ void k_uf_hook(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const uint8_t* __restrict__ removed, int32_t* parent) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= n) return;
  int32_t u = (int32_t)wave;
  if (removed[u]) return;
  int lane = kc_lane();
  for (int32_t i = rp[u] + lane; i < rp[u + 1]; i += KC_WAVE) {
    int32_t v = col[i];
    if (v <= u || removed[v]) continue;
    for (;;) {
      int32_t ru = uf_find(parent, u), rv = uf_find(parent, v);
      if (ru == rv) break;
      int32_t hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
      if (atomicCAS(&parent[hi], hi, lo) == hi) break;
    }
  }
}

__global__ void k_uf_stats(int32_t n, const uint8_t* removed, int32_t* parent, const int32_t* deg,
                           int32_t* comp_n, unsigned long long* comp_dsum) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || removed[v]) return;
  int32_t r = uf_find(parent, v);
  parent[v] = r;
  atomicAdd(&comp_n[r], 1);
  atomicAdd(&comp_dsum[r], (unsigned long long)deg[v]);
}

// A live root whose component's degree sum is n_c (n_c - 1) is a clique
// component: it contributes C(n_c, k) cliques.
__global__ void k_prelist_roots(int32_t n, int32_t k, const int32_t* vk, const uint8_t* removed,
                                const int32_t* parent, const int32_t* comp_n, const unsigned long long* comp_dsum,
                                uint8_t* is_clique, unsigned long long* prelist_count,
                                unsigned long long* root_count, int* flags, const uint8_t* mask) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  is_clique[v] = 0;
  if (removed[v] || parent[v] != v) return;
  uint64_t nc = (uint64_t)comp_n[v];
  if (comp_dsum[v] != nc * (nc - 1)) return;
  is_clique[v] = 1;
  if (mask && !mask[v]) return;  // reported by the share that holds the smallest vertex
  uint64_t c;
  if (!kc_binom(nc, (uint64_t)kc_vk(vk, v, k), &c)) { atomicOr(flags, KC_FLAG_OVERFLOW); return; }
  kc_add_checked(prelist_count, c, flags);
  if (root_count) kc_add_checked(&root_count[v], c, flags);  // v is the component's smallest vertex
}

__global__ void k_prelist_remove(int32_t n, int32_t k, const int32_t* vk, uint8_t* removed,
                                 const int32_t* parent, const int32_t* comp_n, const uint8_t* is_clique,
                                 unsigned long long* pv, int* flags, const uint8_t* mask) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || removed[v]) return;
  int32_t r = parent[v];
  if (!is_clique[r]) return;
  removed[v] = 1;
  if (pv && (!mask || mask[r])) {
    uint64_t c;
    if (!kc_binom((uint64_t)comp_n[r] - 1, (uint64_t)kc_vk(vk, v, k) - 1, &c)) {
      atomicOr(flags, KC_FLAG_OVERFLOW);
      return;
    }
    kc_add_checked(&pv[v], c, flags);
  }
}

// ------------------------------------------------- Pre-List output
// Listing mode: a clique component reports each of its C(n_c, k) k-subsets
// (Alg. 4).  Its members are gathered into one list per component; the
// components' subset counts (capped at the output capacity) are prefix-summed
// into row offsets, and row t of component c is the t-th k-subset of its
// member list in the combinatorial number system: the largest a_k with
// C(a_k, k) <= t, then the largest a_{k-1} < a_k with C(a_{k-1}, k-1) <=
// t - C(a_k, k), and so on.
__global__ void k_pl_sizes(int32_t n, int32_t k, const int32_t* vk, const uint8_t* __restrict__ removed,
                           const int32_t* __restrict__ parent, const uint8_t* __restrict__ is_clique,
                           const int32_t* __restrict__ comp_n, int64_t cap, const uint8_t* mask, int32_t* msz,
                           int64_t* tsz) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const bool root = !removed[v] && parent[v] == v && is_clique[v] && (!mask || mask[v]);
  uint64_t c = 0;
  if (root && !kc_binom((uint64_t)comp_n[v], (uint64_t)kc_vk(vk, v, k), &c)) c = ~0ull;
  msz[v] = root ? comp_n[v] : 0;
  tsz[v] = root ? (int64_t)(c < (uint64_t)cap ? c : (uint64_t)cap) : 0;
}

__global__ void k_pl_members(int32_t n, const uint8_t* __restrict__ removed, const int32_t* __restrict__ parent,
                             const uint8_t* __restrict__ is_clique, const uint8_t* mask,
                             const int32_t* __restrict__ moff, int32_t* fill, int32_t* members) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || removed[v]) return;
  const int32_t r = parent[v];
  if (!is_clique[r] || (mask && !mask[r])) return;
  members[moff[r] + atomicAdd(&fill[r], 1)] = v;
}

// true when C(c, j) <= x (a value past 64 bits is larger than any x)
__device__ __forceinline__ bool binom_le(uint64_t c, uint64_t j, uint64_t x, uint64_t* val) {
  return kc_binom(c, j, val) && *val <= x;
}

__global__ void k_pl_emit(int32_t n, int32_t k, const int32_t* vk, const int64_t* __restrict__ toff,
                          const int32_t* __restrict__ moff, const int32_t* __restrict__ comp_n,
                          const int32_t* __restrict__ members, const int64_t* __restrict__ total, kc_emit e) {
  const int64_t T = *total < e.cap ? *total : e.cap;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < T; t += (int64_t)gridDim.x * blockDim.x) {
    // the component whose row range holds t: the last vertex with offset <= t
    int32_t lo = 0, hi = n;
    while (lo < hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      if (toff[mid] <= t) lo = mid + 1; else hi = mid;
    }
    const int32_t c = lo - 1;
    uint64_t x = (uint64_t)(t - toff[c]);
    const int kc = kc_vk(vk, c, k);
    int32_t top = comp_n[c] - 1;
    int32_t* row = e.out + t * (int64_t)k;
    for (int j = kc; j >= 1; --j) {
      int32_t a = j - 1, b = top;
      uint64_t val = 0;
      while (a < b) {  // largest element a with C(a, j) <= x
        const int32_t mid = a + ((b - a + 1) >> 1);
        if (binom_le((uint64_t)mid, (uint64_t)j, x, &val)) a = mid; else b = mid - 1;
      }
      kc_binom((uint64_t)a, (uint64_t)j, &val);
      x -= val;
      row[kc - j] = members[moff[c] + a];
      top = a - 1;
    }
  }
}

// -------------------------------------------------------- degeneracy peel
// Level scan: compacts the still-live vertices of `A` into `Anext`, and
// records the minimum live degree.
__global__ void k_peel_compact(const int32_t* __restrict__ A, int32_t na, const uint8_t* __restrict__ peeled,
                               const int32_t* __restrict__ deg, int32_t* Anext, int32_t* nnext, int32_t* mindeg) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = false;
  int32_t v = 0, d = 0x7fffffff;
  if (i < na) {
    v = A[i];
    live = !peeled[v];
    if (live) d = deg[v];
  }
  uint64_t m = kc_ballot(live);
  int base = 0;
  if (kc_lane() == 0 && m) base = atomicAdd(nnext, __popcll(m));
  base = __shfl(base, 0, 64);
  if (live) Anext[base + kc_mbcnt(m)] = v;
  // wave min then one atomic
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    int y = __shfl_xor(d, off, 64);
    d = d < y ? d : y;
  }
  if (kc_lane() == 0 && m) atomicMin(mindeg, d);
}

__global__ void k_peel_select(const int32_t* __restrict__ A, int32_t na, const int32_t* __restrict__ deg,
                              const int32_t* __restrict__ level, int32_t* F, int32_t* fcount) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= na) return;
  int32_t v = A[i];
  if (deg[v] <= *level) F[atomicAdd(fcount, 1)] = v;
}

__global__ void k_peel_mark(const int32_t* __restrict__ F, int32_t nf, int32_t round, const int32_t* level,
                            uint8_t* peeled, int32_t* key, int32_t* core) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  int32_t v = F[i];
  peeled[v] = 1;
  key[v] = round;
  core[v] = *level;
}

// One wave per frontier vertex: decrement live neighbours; the decrement that
// takes a degree from level+1 to level puts the vertex in the next round.
__global__ void k_peel_dec(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ F, int32_t nf, const uint8_t* __restrict__ peeled,
                           const int32_t* level, int32_t* deg, int32_t* Fnext, int32_t* fnext_count) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= nf) return;
  int lane = kc_lane();
  int32_t u = F[wave];
  int32_t c = *level;
  for (int32_t i = rp[u] + lane; i < rp[u + 1]; i += KC_WAVE) {
    int32_t v = col[i];
    if (peeled[v]) continue;
    int32_t old = atomicSub(&deg[v], 1);
    if (old == c + 1) Fnext[atomicAdd(fnext_count, 1)] = v;
  }
}

// First level scan: the live list is implicitly 0..n-1.
__global__ void k_iota_compact(int32_t na, const uint8_t* peeled, const int32_t* deg, int32_t* Anext, int32_t* nnext,
                               int32_t* mindeg) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = false;
  int32_t d = 0x7fffffff;
  if (i < na) {
    live = !peeled[i];
    if (live) d = deg[i];
  }
  uint64_t m = kc_ballot(live);
  int base = 0;
  if (kc_lane() == 0 && m) base = atomicAdd(nnext, __popcll(m));
  base = __shfl(base, 0, 64);
  if (live) Anext[base + kc_mbcnt(m)] = i;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    int y = __shfl_xor(d, off, 64);
    d = d < y ? d : y;
  }
  if (kc_lane() == 0 && m) atomicMin(mindeg, d);
}

// ---------------------------------------------------------------- DAG build
__device__ __forceinline__ bool dag_before(int32_t ku, int32_t u, int32_t kv, int32_t v) {
  return ku < kv || (ku == kv && u < v);
}

__global__ void k_dag_count(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const uint8_t* __restrict__ removed, const int32_t* __restrict__ key, int32_t* dplus) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= n) return;
  int32_t u = (int32_t)wave;
  int lane = kc_lane();
  if (removed[u]) {
    if (lane == 0) dplus[u] = 0;
    return;
  }
  int32_t ku = key[u];
  int32_t cnt = 0;
  for (int32_t i = rp[u] + lane; i < rp[u + 1]; i += KC_WAVE) {
    int32_t v = col[i];
    bool out = !removed[v] && dag_before(ku, u, key[v], v);
    cnt += __popcll(kc_ballot(out));
  }
  if (lane == 0) dplus[u] = cnt;
}

__global__ void k_dag_fill(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const uint8_t* __restrict__ removed, const int32_t* __restrict__ key,
                           const int32_t* __restrict__ drp, int32_t* dcol) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE;
  if (wave >= n) return;
  int32_t u = (int32_t)wave;
  if (removed[u]) return;
  int lane = kc_lane();
  int32_t ku = key[u];
  int32_t o = drp[u];
  int32_t b = rp[u], e = rp[u + 1];
  for (int32_t base = b; base < e; base += KC_WAVE) {
    int32_t i = base + lane;
    int32_t v = i < e ? col[i] : 0;
    bool out = i < e && !removed[v] && dag_before(ku, u, key[v], v);
    uint64_t m = kc_ballot(out);
    if (out) dcol[o + kc_mbcnt(m)] = v;
    o += __popcll(m);
  }
}

static inline unsigned grid_for(int64_t threads, int block = 256) {
  return (unsigned)((threads + block - 1) / block);
}

static int read_i32(const int32_t* dev, int32_t* host, hipStream_t s) {
  KC_HIP(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

int kc_preprocess(const kc_dev_graph& g, int32_t k, const int32_t* vk, int32_t order,
                  unsigned long long* prelist_count_dev, unsigned long long* pv_dev, unsigned long long* root_count,
                  int* flags_dev, kc_prep_out* out, kc_scratch& scr, hipStream_t s, const kc_emit* emit,
                  int32_t disable, const uint8_t* mask) {
  const int32_t n = g.n;
  const int32_t km1 = k - 1;
  memset(out, 0, sizeof(*out));
  KC_TRY(scr.get(&out->removed, (size_t)n + 1));
  KC_TRY(scr.get(&out->deg, (size_t)n + 1));
  KC_TRY(scr.get(&out->key, (size_t)n + 1));
  KC_TRY(scr.get(&out->drp, (size_t)n + 2));
  int32_t *F0, *F1, *counters;
  KC_TRY(scr.get(&F0, (size_t)n + 1));
  KC_TRY(scr.get(&F1, (size_t)n + 1));
  KC_TRY(scr.get(&counters, 8));
  int32_t hcnt[16];  // host copies of device counters (pageable: the copies are synchronised)

  // ---- Pre-Core (Alg. 3)
  KC_HIP(hipMemsetAsync(counters, 0, 8 * sizeof(int32_t), s));
  if (n > 0) {
    k_precore_init<<<grid_for(n), 256, 0, s>>>(n, g.rp, km1, vk, out->deg, out->removed, F0, counters,
                                               (disable & KC_NO_PRECORE) != 0);
    KC_HIP(hipGetLastError());
  }
  KC_TRY(read_i32(counters, hcnt, s));
  int32_t nf = hcnt[0];
  while (nf > 0) {
    KC_HIP(hipMemsetAsync(counters + 1, 0, sizeof(int32_t), s));
    k_precore_peel<<<grid_for((int64_t)nf * KC_WAVE), 256, 0, s>>>(g.rp, g.col, km1, vk, F0, nf, out->deg,
                                                                    out->removed, F1, counters + 1);
    KC_HIP(hipGetLastError());
    KC_TRY(read_i32(counters + 1, hcnt, s));
    nf = hcnt[0];
    int32_t* t = F0; F0 = F1; F1 = t;
  }

  // ---- Pre-List (Alg. 4)
  if (!(disable & KC_NO_PRELIST)) {
    int32_t *parent, *comp_n;
    unsigned long long* comp_dsum;
    uint8_t* is_clique;
    KC_TRY(scr.get(&parent, (size_t)n + 1));
    KC_TRY(scr.get(&comp_n, (size_t)n + 1));
    KC_TRY(scr.get(&comp_dsum, (size_t)n + 1));
    KC_TRY(scr.get(&is_clique, (size_t)n + 1));
    if (n > 0) {
      KC_HIP(hipMemsetAsync(comp_n, 0, sizeof(int32_t) * (size_t)n, s));
      KC_HIP(hipMemsetAsync(comp_dsum, 0, sizeof(unsigned long long) * (size_t)n, s));
      k_uf_init<<<grid_for(n), 256, 0, s>>>(n, out->removed, parent);
      k_uf_hook<<<grid_for((int64_t)n * KC_WAVE), 256, 0, s>>>(n, g.rp, g.col, out->removed, parent);
      k_uf_stats<<<grid_for(n), 256, 0, s>>>(n, out->removed, parent, out->deg, comp_n, comp_dsum);
      k_prelist_roots<<<grid_for(n), 256, 0, s>>>(n, k, vk, out->removed, parent, comp_n, comp_dsum, is_clique,
                                                   prelist_count_dev, root_count, flags_dev, mask);
      KC_HIP(hipGetLastError());
    }
    if (emit) {
      // report the clique components' k-subsets; the listing's rows follow
      int32_t *msz, *moff, *fill, *members;
      int64_t *tsz, *toff, *ttot;
      KC_TRY(scr.get(&msz, (size_t)n + 1));
      KC_TRY(scr.get(&moff, (size_t)n + 1));
      KC_TRY(scr.get(&fill, (size_t)n + 1));
      KC_TRY(scr.get(&members, (size_t)n + 1));
      KC_TRY(scr.get(&tsz, (size_t)n + 1));
      KC_TRY(scr.get(&toff, (size_t)n + 1));
      KC_TRY(scr.get(&ttot, 2));
      if (n > 0) {
        k_pl_sizes<<<grid_for(n), 256, 0, s>>>(n, k, vk, out->removed, parent, is_clique, comp_n, emit->cap, mask, msz,
                                               tsz);
        KC_HIP(hipGetLastError());
      }
      KC_TRY(kc_scan_i32(msz, moff, n, nullptr, scr, s));
      KC_TRY(kc_scan_i64(tsz, toff, n, ttot, scr, s));
      if (n > 0) {
        KC_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * (size_t)n, s));
        k_pl_members<<<grid_for(n), 256, 0, s>>>(n, out->removed, parent, is_clique, mask, moff, fill, members);
        k_pl_emit<<<1024, 256, 0, s>>>(n, k, vk, toff, moff, comp_n, members, ttot, *emit);
        KC_HIP(hipGetLastError());
      }
      KC_HIP(hipMemcpyAsync(emit->pos, ttot, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    }
    if (n > 0) {
      k_prelist_remove<<<grid_for(n), 256, 0, s>>>(n, k, vk, out->removed, parent, comp_n, is_clique, pv_dev,
                                                    flags_dev, mask);
      KC_HIP(hipGetLastError());
    }
  }

  // ---- orientation
  if (order == KC_ORDER_DEGREE) {
    // key = degree in the reduced graph (Pre-List removes whole components,
    // so the Pre-Core degrees of the survivors are unchanged)
    if (n > 0) KC_HIP(hipMemcpyAsync(out->key, out->deg, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
  } else {
    // degeneracy order (BitCol, and SDegree on the degeneracy order)
    KC_TRY(scr.get(&out->core, (size_t)n + 1));
    int32_t *A0, *A1, *pdeg;
    uint8_t* peeled;
    KC_TRY(scr.get(&A0, (size_t)n + 1));
    KC_TRY(scr.get(&A1, (size_t)n + 1));
    KC_TRY(scr.get(&pdeg, (size_t)n + 1));
    KC_TRY(scr.get(&peeled, (size_t)n + 1));
    if (n > 0) {
      KC_HIP(hipMemcpyAsync(pdeg, out->deg, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
      KC_HIP(hipMemcpyAsync(peeled, out->removed, (size_t)n, hipMemcpyDeviceToDevice, s));
      KC_HIP(hipMemsetAsync(out->core, 0xff, sizeof(int32_t) * (size_t)n, s));
      KC_HIP(hipMemsetAsync(out->key, 0xff, sizeof(int32_t) * (size_t)n, s));
    }
    // all vertices start in the live list (implicitly 0..n-1); the first
    // compaction drops the removed ones
    int32_t na = n;
    int32_t round = 0;
    int32_t* level = counters + 4;  // current level c (device)
    int32_t* mind = counters + 5;
    KC_HIP(hipMemsetAsync(level, 0, sizeof(int32_t), s));
    int32_t max_core = 0;
    bool first = true;
    while (na > 0) {
      // level scan: compact live list, find min degree, select frontier
      KC_HIP(hipMemsetAsync(counters + 2, 0, sizeof(int32_t), s));
      KC_HIP(hipMemsetAsync(mind, 0x7f, sizeof(int32_t), s));
      if (first) {
        k_iota_compact<<<grid_for(na), 256, 0, s>>>(na, peeled, pdeg, A1, counters + 2, mind);
        first = false;
      } else {
        k_peel_compact<<<grid_for(na), 256, 0, s>>>(A0, na, peeled, pdeg, A1, counters + 2, mind);
      }
      KC_HIP(hipGetLastError());
      KC_TRY(read_i32(counters + 2, hcnt, s));
      na = hcnt[0];
      { int32_t* t = A0; A0 = A1; A1 = t; }
      if (na == 0) break;
      // level = max(level, mindeg)
      KC_HIP(hipMemcpyAsync(hcnt + 1, mind, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      KC_HIP(hipStreamSynchronize(s));
      int32_t c = hcnt[1];
      if (c > max_core) max_core = c;
      KC_HIP(hipMemcpyAsync(level, &hcnt[1], sizeof(int32_t), hipMemcpyHostToDevice, s));
      KC_HIP(hipMemsetAsync(counters + 3, 0, sizeof(int32_t), s));
      k_peel_select<<<grid_for(na), 256, 0, s>>>(A0, na, pdeg, level, F0, counters + 3);
      KC_HIP(hipGetLastError());
      KC_TRY(read_i32(counters + 3, hcnt, s));
      nf = hcnt[0];
      // rounds at this level
      while (nf > 0) {
        k_peel_mark<<<grid_for(nf), 256, 0, s>>>(F0, nf, round, level, peeled, out->key, out->core);
        KC_HIP(hipMemsetAsync(counters + 1, 0, sizeof(int32_t), s));
        k_peel_dec<<<grid_for((int64_t)nf * KC_WAVE), 256, 0, s>>>(g.rp, g.col, F0, nf, peeled, level, pdeg, F1,
                                                                    counters + 1);
        KC_HIP(hipGetLastError());
        round++;
        KC_TRY(read_i32(counters + 1, hcnt, s));
        nf = hcnt[0];
        int32_t* t = F0; F0 = F1; F1 = t;
      }
    }
    out->max_core = max_core;
  }

  // ---- DAG (out-neighbour lists in ascending id order)
  if (n > 0) {
    k_dag_count<<<grid_for((int64_t)n * KC_WAVE), 256, 0, s>>>(n, g.rp, g.col, out->removed, out->key, out->drp);
    KC_HIP(hipGetLastError());
  }
  KC_TRY(kc_scan_i32(out->drp, out->drp, n, out->drp + n, scr, s));
  int32_t dn = 0;
  KC_TRY(read_i32(out->drp + n, &hcnt[2], s));
  dn = hcnt[2];
  out->dnnz = dn;
  KC_TRY(scr.get(&out->dcol, (size_t)dn + 1));
  if (n > 0) {
    k_dag_fill<<<grid_for((int64_t)n * KC_WAVE), 256, 0, s>>>(n, g.rp, g.col, out->removed, out->key, out->drp,
                                                               out->dcol);
    KC_HIP(hipGetLastError());
  }
  return KC_OK;
}

