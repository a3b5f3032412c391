// kc_internal.h -- shared declarations of the k-clique library (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kclique.h"

#define KC_WAVE 64
// Largest k handled by the listing kernels (recursion depth k-1).
#define KC_KMAX_LIMIT 32

// ----------------------------------------------------------- error plumbing
#define KC_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) {                           \
      kc_set_hip_error(e_, #call, __FILE__, __LINE__); \
      return e_ == hipErrorOutOfMemory ? KC_ENOMEM : KC_EDEVICE; \
    }                                                 \
  } while (0)

#define KC_TRY(expr)        \
  do {                      \
    int st_ = (expr);       \
    if (st_ != KC_OK) return st_; \
  } while (0)

void kc_set_hip_error(hipError_t e, const char* what, const char* file, int line);

// Device flags set by kernels (bit mask in a device int).
#define KC_FLAG_BADGRAPH 1
#define KC_FLAG_OVERFLOW 2
#define KC_FLAG_TOOBIG 4

// ------------------------------------------------------ device-side helpers
__device__ __forceinline__ int kc_lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t kc_ballot(bool p) { return __ballot(p); }

// Exclusive count of set bits of `mask` below this lane.
__device__ __forceinline__ int kc_mbcnt(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int kc_readfirst(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t kc_readlane(uint32_t x, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

// Wave-wide sum of a 32-bit unsigned value (all lanes active).
__device__ __forceinline__ uint32_t kc_wave_sum_u32(uint32_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off, 64);
  return x;
}
__device__ __forceinline__ uint64_t kc_wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    lo = (uint32_t)__shfl_xor((int)lo, off, 64);
    hi = (uint32_t)__shfl_xor((int)hi, off, 64);
    x += ((uint64_t)hi << 32) | lo;
  }
  return x;
}
__device__ __forceinline__ int kc_wave_max_i32(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    int y = __shfl_xor(x, off, 64);
    x = x > y ? x : y;
  }
  return x;
}

// Orders LDS accesses of the lanes of one wave (a compiler-level barrier;
// the LDS unit processes one wave's requests in order).
__device__ __forceinline__ void kc_wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds x into *acc (device, 64-bit) and raises the overflow flag on wrap.
__device__ __forceinline__ void kc_add_checked(unsigned long long* acc, uint64_t x, int* flags) {
  if (x == 0) return;
  unsigned long long old = atomicAdd(acc, (unsigned long long)x);
  if (old + x < old) atomicOr(flags, KC_FLAG_OVERFLOW);
}

// C(n, k) exactly; returns false when the value does not fit in 64 bits.
// r_i = C(n-k+i, i) = r_{i-1} (n-k+i) / i; dividing i by gcd(r_{i-1}, i)
// first keeps every intermediate exact and within 64 bits.
__device__ __forceinline__ bool kc_binom(uint64_t n, uint64_t k, uint64_t* out) {
  if (k > n) { *out = 0; return true; }
  if (k > n - k) k = n - k;
  uint64_t r = 1;
  for (uint64_t i = 1; i <= k; ++i) {
    uint64_t a = r, b = i;
    while (b) { uint64_t t = a % b; a = b; b = t; }
    uint64_t g = a;
    uint64_t rr = r / g, ii = i / g;
    uint64_t x = (n - k + i) / ii;
    uint64_t p;
    if (__builtin_mul_overflow(rr, x, &p)) return false;
    r = p;
  }
  *out = r;
  return true;
}

// ------------------------------------------------------------- host side
struct kc_dev_graph {
  int32_t n;
  int64_t nnz;
  const int32_t* rp;
  const int32_t* col;
};

// Device scratch of one call.  Either stream-ordered allocations released at
// scope exit, or sub-allocations (256-byte aligned, bump pointer) of a
// caller-owned arena that is never freed here.  Every allocation of a call
// goes through one kc_scratch and none is released before the call ends, so
// the arena a call needs is the sum of its aligned requests (`need`), which a
// size query obtains by running the call's preparation (kc_list_ctx.size_only).
#define KC_SCRATCH_ALIGN 256
struct kc_scratch {
  hipStream_t stream = nullptr;
  void** ptrs = nullptr;   // stream-ordered allocations to free
  int count = 0, cap = 0;
  char* arena = nullptr;   // caller-owned memory (nullable)
  size_t arena_bytes = 0;
  size_t need = 0;         // bytes an arena would need for the requests so far
  explicit kc_scratch(hipStream_t s) : stream(s) {}
  kc_scratch(hipStream_t s, void* mem, size_t bytes) : stream(s), arena((char*)mem), arena_bytes(bytes) {}
  kc_scratch(const kc_scratch&) = delete;
  kc_scratch& operator=(const kc_scratch&) = delete;
  ~kc_scratch();
  int alloc(void** p, size_t bytes);
  template <class T>
  int get(T** p, size_t count_elems) {
    return alloc((void**)p, count_elems * sizeof(T) + 16);
  }
};

// Exclusive prefix sums on the device (n elements; out may alias in); the
// temporaries come from `scr`.
int kc_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev, kc_scratch& scr, hipStream_t s);
int kc_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total_dev, kc_scratch& scr, hipStream_t s);

// Listing output: rows of k vertex ids written to `out` (device, row-major),
// at most `cap` of them; `pos` (device) counts the rows reserved so far --
// rows at or beyond `cap` are counted but not written.
struct kc_emit {
  int32_t* out = nullptr;
  int64_t cap = 0;
  unsigned long long* pos = nullptr;
};

// Preprocessing (kc_prep.hip).
struct kc_prep_out {
  uint8_t* removed;   // [n] 1 = removed by Pre-Core or Pre-List
  int32_t* deg;       // [n] live degree after Pre-Core
  int32_t* key;       // [n] order key (degree or peel round)
  int32_t* core;      // [n] core number (degeneracy orders), else null
  int32_t* drp;       // [n+1] DAG row pointers
  int32_t* dcol;      // DAG columns (ascending id per row)
  int64_t dnnz;
  int32_t max_core;
};
int kc_validate_graph(const kc_dev_graph& g, int* flags_dev, hipStream_t s);
int kc_preprocess(const kc_dev_graph& g, int32_t k, const int32_t* vk, int32_t order,
                  unsigned long long* prelist_count_dev, unsigned long long* pv_dev, unsigned long long* root_count,
                  int* flags_dev, kc_prep_out* out, kc_scratch& scr, hipStream_t s, const kc_emit* emit = nullptr,
                  int32_t disable = 0, const uint8_t* root_mask = nullptr);

// Listing (kc_sdegree.hip, kc_bitcol.hip).
struct kc_list_ctx {
  int32_t n;
  int32_t k;               // maximum k
  const int32_t* vk;       // per-vertex k (nullable: uniform k)
  unsigned long long* root_count;  // per-vertex attribution (nullable)
  const int32_t* drp;
  const int32_t* dcol;
  const int32_t* core;
  int32_t nroots;
  int32_t* roots;          // [nroots] vertex id of each root
  unsigned long long* count;   // device total
  unsigned long long* pv;      // device per-vertex (nullable)
  int* flags;
  // logs (nullable device arrays indexed by vertex id)
  uint64_t* root_work;
  uint64_t* root_isect;
  float* root_features;
  // accumulated work counters (device, 4 x u64: nodes, isect, work, staged words)
  unsigned long long* counters;
  const kc_options* opt;
  kc_stats* stats;
  struct kc_capture* capture;  // non-null: prepare only, hand the listing phase over
  bool size_only;              // stop before the listing launches (workspace size query)
  const kc_emit* emit;         // non-null: write every clique listed (no schedule, no per-vertex output)
  bool reduce;                 // SDegree: out-neighbour reduction (Sec. 7.2)
};

// A prepared call's listing phase, to be captured into a HIP graph and
// replayed: `launch` enqueues it on a stream (kernels only).
struct kc_capture {
  unsigned long long* count_d = nullptr;  // the call's device total (listing part)
  int* flags = nullptr;                   // the call's device flags
  void* state = nullptr;
  int (*launch)(const void* state, hipStream_t s) = nullptr;
  void (*destroy)(void* state) = nullptr;
  ~kc_capture() {
    if (destroy && state) destroy(state);
  }
};
int kc_list_sdegree(kc_list_ctx& c, kc_scratch& scr, hipStream_t s);
int kc_list_bitcol(kc_list_ctx& c, kc_scratch& scr, hipStream_t s);

// MLP (kc_mlp.hip).
int kc_mlp_forward_dev(const float* params, const float* x, int32_t rows, float* y, hipStream_t s);

// Scheduling helpers (kc_sched.hip).
// Groups items 0..n-1 by bin (ascending bin order; order inside a bin is
// unspecified): out_dev[host_off[b] .. host_off[b+1]) holds bin b's items.
int kc_bin_sort(const int32_t* bin_dev, int32_t n, int32_t nbins, int32_t* out_dev, int32_t* host_off,
                kc_scratch& scr, hipStream_t s);
int kc_device_cus();
__device__ __forceinline__ int kc_vk(const int32_t* vk, int32_t v, int k) { return vk ? vk[v] : k; }

// Quantised schedule key (0..63, larger = heavier) from a work estimate in
// natural-log units.
__device__ __forceinline__ int kc_key_q(float logw) {
  float q = logw * 2.0f;
  return q <= 0.f ? 0 : (q >= 63.f ? 63 : (int)q);
}
