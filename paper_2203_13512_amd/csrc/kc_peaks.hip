// Microbenchmarks of the three rates the listing and staging kernels are
// bounded by, measured on the GPU they run on (the published figures are
// nominal): 32-bit integer VALU issue with the operations of a BitJoin
// (AND, population count with accumulate, XOR), LDS read bandwidth with
// conflict-free 16-byte reads, and HBM bandwidth of a plain vectorised copy.
// Built as its own library (libkcpeaks.so) for the benchmark; it is not part
// of the k-clique interface.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;

// Each thread runs `iters` rounds over kChains independent dependency chains;
// a round is 3 integer operations per chain.  The mask m is a run-time value
// so that nothing is folded.
__global__ __launch_bounds__(kThreads) void k_peak_valu(uint32_t m, int iters, uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
  uint32_t a[kChains], acc[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    a[i] = tid * 0x9e3779b9u + (uint32_t)i * 0x85ebca6bu;
    acc[i] = 0;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      const uint32_t t = a[i] & m;
      acc[i] = (uint32_t)__popc(t) + acc[i];
      a[i] = t ^ acc[i];
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) r ^= a[i] + acc[i];
  out[tid] = r;
}

// LDS reads: each wave reads 64 consecutive 16-byte words (1 KiB, every bank
// once per quarter), `iters` times over a 16 KiB buffer.  The step between
// reads is a run-time value, so the compiler cannot see the period of the
// sequence; the words are summed, so repeated reads do not cancel.
constexpr int kLdsWords = 1024;  // uint4 = 16 KiB

__global__ __launch_bounds__(kThreads) void k_peak_lds(int iters, int step, uint32_t* __restrict__ out) {
  __shared__ uint4 buf[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += kThreads)
    buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
  __syncthreads();
  uint4 x = make_uint4(0, 0, 0, 0);
  int p = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const uint4 v = buf[p];
    x.x += v.x;
    x.y += v.y;
    x.z += v.z;
    x.w += v.w;
    p = (p + step) & (kLdsWords - 1);
  }
  out[blockIdx.x * kThreads + threadIdx.x] = x.x ^ x.y ^ x.z ^ x.w;
}

// Plain copy of n16 16-byte words, grid-stride.
__global__ __launch_bounds__(kThreads) void k_peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// which: 0 = VALU (result in int32 operations), 1 = LDS (bytes read),
// 2 = HBM copy (bytes read + written; src/dst are device buffers of `bytes`
// bytes, a multiple of 16).  `scratch` is a device buffer of
// `scratch_bytes` >= blocks * 256 * 4 bytes for the VALU and LDS kernels.  Runs `reps` timed
// launches after one untimed one on the default stream and returns the mean
// duration of a launch in *ms and the work of one launch in *units.
// Returns 0, or -1 on invalid arguments, -4 on a HIP error.
int kcp_measure(int32_t which, int32_t blocks, int32_t iters, int32_t reps, void* scratch, int64_t scratch_bytes,
                const void* src, void* dst, int64_t bytes, double* ms, double* units) {
  if (blocks <= 0 || reps <= 0 || !ms || !units) return -1;
  if (which <= 1 && (!scratch || iters <= 0 || scratch_bytes < (int64_t)blocks * kThreads * 4)) return -1;
  if (which == 2 && (!src || !dst || bytes <= 0 || (bytes & 15))) return -1;
  if (which < 0 || which > 2) return -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -4;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -4;
  }
  auto launch = [&]() {
    if (which == 0)
      k_peak_valu<<<blocks, kThreads>>>(0x7fffbfffu, iters, (uint32_t*)scratch);
    else if (which == 1)
      k_peak_lds<<<blocks, kThreads>>>(iters, kThreads, (uint32_t*)scratch);
    else
      k_peak_copy<<<blocks, kThreads>>>((const uint4*)src, (uint4*)dst, bytes / 16);
  };
  launch();
  bool ok = hipGetLastError() == hipSuccess;
  ok = ok && hipEventRecord(e0, 0) == hipSuccess;
  for (int r = 0; r < reps && ok; ++r) {
    launch();
    ok = hipGetLastError() == hipSuccess;
  }
  ok = ok && hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  float t = 0.f;
  ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return -4;
  *ms = (double)t / reps;
  const double threads = (double)blocks * kThreads;
  if (which == 0)
    *units = threads * (double)iters * kChains * 3.0;
  else if (which == 1)
    *units = threads * (double)iters * 16.0;
  else
    *units = 2.0 * (double)bytes;
  return 0;
}

}  // extern "C"
