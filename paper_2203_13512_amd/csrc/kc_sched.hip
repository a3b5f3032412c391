// kc_sched.hip -- binning of work items for the persistent listing kernels.
//
// The persistent kernels take items from a queue in array order, so the
// schedule is the order of that array.  Items are grouped by a bin number
// (a bitmap class or candidate-list class, then a quantised work key in
// descending order) with a counting sort: histogram, exclusive scan,
// scatter.
#include <hip/hip_runtime.h>

#include <vector>

#include "kc_internal.h"

__global__ void k_bin_hist(const int32_t* __restrict__ bin, int32_t n, int32_t nbins, int32_t* hist) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t b = bin[i];
  if (b >= 0 && b < nbins) atomicAdd(&hist[b], 1);
}

__global__ void k_bin_scatter(const int32_t* __restrict__ bin, int32_t n, int32_t nbins, int32_t* cursor,
                              int32_t* out) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t b = bin[i];
  if (b >= 0 && b < nbins) out[atomicAdd(&cursor[b], 1)] = i;
}

int kc_bin_sort(const int32_t* bin_dev, int32_t n, int32_t nbins, int32_t* out_dev, int32_t* host_off,
                kc_scratch& scr, hipStream_t s) {
  int32_t* hist;
  KC_TRY(scr.get(&hist, (size_t)nbins + 1));
  KC_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * ((size_t)nbins + 1), s));
  if (n > 0) {
    k_bin_hist<<<(n + 255) / 256, 256, 0, s>>>(bin_dev, n, nbins, hist);
    KC_HIP(hipGetLastError());
  }
  KC_TRY(kc_scan_i32(hist, hist, nbins + 1, nullptr, scr, s));
  KC_HIP(hipMemcpyAsync(host_off, hist, sizeof(int32_t) * ((size_t)nbins + 1), hipMemcpyDeviceToHost, s));
  if (n > 0) {
    k_bin_scatter<<<(n + 255) / 256, 256, 0, s>>>(bin_dev, n, nbins, hist, out_dev);
    KC_HIP(hipGetLastError());
  }
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

int kc_device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 256;
    cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
  }
  return cus;
}
