// kc_mlp.hip -- the work predictor: an MLP 4 -> 64 -> 64 -> 1 with ReLU in
// FP32 (forward, backward, Adam), written as plain HIP kernels.
//
// Parameter block (row-major): W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3.
// Inference: one thread per row with the parameters staged in LDS (every lane
// reads the same weight at the same time, an LDS broadcast).  Training: a row
// kernel computes activations and the per-row gradients of the pre-activations;
// two reduction kernels form each parameter's gradient as a sum over the rows
// (partial sums per chunk of rows, then the partials in chunk order: a fixed
// summation order, so results are reproducible); an update kernel applies
// Adam.  Scratch (the per-row buffer and the partials) comes from the caller's
// workspace when one is given.
#include <hip/hip_runtime.h>

#include "kc_internal.h"

#define H KC_MLP_HIDDEN
#define NIN KC_MLP_IN
#define P_W1 0
#define P_B1 (P_W1 + H * NIN)
#define P_W2 (P_B1 + H)
#define P_B2 (P_W2 + H * H)
#define P_W3 (P_B2 + H)
#define P_B3 (P_W3 + H)
#define P_N (P_B3 + 1)
static_assert(P_N == KC_MLP_NPARAMS, "parameter layout");

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ x,
                                                     int32_t rows, float* __restrict__ y) {
  __shared__ float P[P_N];
  for (int i = threadIdx.x; i < P_N; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float in[NIN];
#pragma unroll
  for (int c = 0; c < NIN; ++c) in[c] = x[(int64_t)r * NIN + c];
  float h1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float z = P[P_B1 + j];
#pragma unroll
    for (int c = 0; c < NIN; ++c) z = fmaf(P[P_W1 + j * NIN + c], in[c], z);
    h1[j] = z > 0.f ? z : 0.f;
  }
  float out = P[P_B3];
  for (int j = 0; j < H; ++j) {
    float z = P[P_B2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) z = fmaf(P[P_W2 + j * H + i], h1[i], z);
    out = fmaf(P[P_W3 + j], z > 0.f ? z : 0.f, out);
  }
  y[r] = out;
}

int kc_mlp_forward_dev(const float* params, const float* x, int32_t rows, float* y, hipStream_t s) {
  if (rows <= 0) return KC_OK;
  k_mlp_forward<<<(rows + 255) / 256, 256, 0, s>>>(params, x, rows, y);
  KC_HIP(hipGetLastError());
  return KC_OK;
}

// Per-row forward and backward.  Stores h1, h2, dz1, dz2 (64 each), dy and
// the squared error of each row into `rowbuf` (rows x 258 floats).
#define ROWW (4 * H + 2)
__global__ __launch_bounds__(256) void k_mlp_rows(const float* __restrict__ params, const float* __restrict__ x,
                                                  const float* __restrict__ target, int32_t rows,
                                                  float* __restrict__ rowbuf) {
  __shared__ float P[P_N];
  for (int i = threadIdx.x; i < P_N; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float* o = rowbuf + (int64_t)r * ROWW;
  float in[NIN];
#pragma unroll
  for (int c = 0; c < NIN; ++c) in[c] = x[(int64_t)r * NIN + c];
  float h1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float z = P[P_B1 + j];
#pragma unroll
    for (int c = 0; c < NIN; ++c) z = fmaf(P[P_W1 + j * NIN + c], in[c], z);
    h1[j] = z > 0.f ? z : 0.f;
    o[j] = h1[j];
  }
  float yv = P[P_B3];
  for (int j = 0; j < H; ++j) {
    float z = P[P_B2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) z = fmaf(P[P_W2 + j * H + i], h1[i], z);
    float h2 = z > 0.f ? z : 0.f;
    o[H + j] = h2;
    o[3 * H + j] = z;  // z2 kept for the mask, replaced by dz2 below
    yv = fmaf(P[P_W3 + j], h2, yv);
  }
  const float err = yv - target[r];
  const float dy = 2.0f * err / (float)rows;
  o[4 * H] = dy;
  o[4 * H + 1] = err * err;
  // dz2 = dy * W3 * [z2 > 0]
  float dh1[H];
#pragma unroll
  for (int i = 0; i < H; ++i) dh1[i] = 0.f;
  for (int j = 0; j < H; ++j) {
    float z2 = o[3 * H + j];
    float dz2 = z2 > 0.f ? dy * P[P_W3 + j] : 0.f;
    o[3 * H + j] = dz2;
#pragma unroll
    for (int i = 0; i < H; ++i) dh1[i] = fmaf(P[P_W2 + j * H + i], dz2, dh1[i]);
  }
#pragma unroll
  for (int i = 0; i < H; ++i) o[2 * H + i] = h1[i] > 0.f ? dh1[i] : 0.f;  // dz1
}

// Gradients as sums over rows, in two passes with a fixed summation order
// (results are reproducible): each (parameter, chunk of MLP_CHUNK rows) pair
// is one thread's partial sum, then one thread per parameter adds its
// partials in chunk order.  Slot P_N carries the squared-error sum (loss).
#define MLP_CHUNK 256
__global__ __launch_bounds__(256) void k_mlp_grad_part(const float* __restrict__ x, const float* __restrict__ rowbuf,
                                                       int32_t rows, float* __restrict__ part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > P_N) return;
  const int32_t r0 = (int32_t)blockIdx.y * MLP_CHUNK;
  const int32_t r1 = r0 + MLP_CHUNK < rows ? r0 + MLP_CHUNK : rows;
  float g = 0.f;
  for (int32_t r = r0; r < r1; ++r) {
    const float* o = rowbuf + (int64_t)r * ROWW;
    float v;
    if (p < P_B1) {
      int j = p / NIN, c = p % NIN;
      v = o[2 * H + j] * x[(int64_t)r * NIN + c];
    } else if (p < P_W2) {
      v = o[2 * H + (p - P_B1)];
    } else if (p < P_B2) {
      int q = p - P_W2, j = q / H, i = q % H;
      v = o[3 * H + j] * o[i];
    } else if (p < P_W3) {
      v = o[3 * H + (p - P_B2)];
    } else if (p < P_B3) {
      v = o[4 * H] * o[H + (p - P_W3)];
    } else if (p == P_B3) {
      v = o[4 * H];
    } else {
      v = o[4 * H + 1];  // squared error of the row
    }
    g += v;
  }
  part[(int64_t)blockIdx.y * (P_N + 1) + p] = g;
}

__global__ __launch_bounds__(256) void k_mlp_grad_sum(const float* __restrict__ part, int32_t nchunks, int32_t rows,
                                                      float* __restrict__ grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > P_N) return;
  float g = 0.f;
  for (int32_t c = 0; c < nchunks; ++c) g += part[(int64_t)c * (P_N + 1) + p];
  if (p == P_N) *loss = g / (float)(rows > 0 ? rows : 1);
  else grad[p] = g;
}

static size_t mlp_align(size_t b) { return (b + 255) & ~(size_t)255; }
static size_t mlp_rowbuf_bytes(int32_t rows) { return mlp_align(sizeof(float) * (size_t)rows * ROWW); }
static size_t mlp_part_bytes(int32_t rows) {
  const size_t nchunks = ((size_t)rows + MLP_CHUNK - 1) / MLP_CHUNK;
  return mlp_align(sizeof(float) * nchunks * (P_N + 1));
}

__global__ void k_mlp_adam(float* __restrict__ params, const float* __restrict__ grad, float* __restrict__ m,
                           float* __restrict__ v, int32_t t, float lr) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P_N) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float g = grad[p];
  float mm = b1 * m[p] + (1.f - b1) * g;
  float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  float mh = mm / (1.f - powf(b1, (float)t));
  float vh = vv / (1.f - powf(b2, (float)t));
  params[p] -= lr * mh / (sqrtf(vh) + eps);
}

extern "C" int kc_mlp_forward(const float* params, const float* x, int32_t rows, float* y, void* stream) {
  if (rows < 0 || (rows > 0 && (!params || !x || !y))) return KC_EINVAL;
  return kc_mlp_forward_dev(params, x, rows, y, (hipStream_t)stream);
}

extern "C" int kc_mlp_workspace_size(int32_t rows, size_t* bytes) {
  if (!bytes || rows < 0) return KC_EINVAL;
  *bytes = mlp_rowbuf_bytes(rows) + mlp_part_bytes(rows);
  return KC_OK;
}

extern "C" int kc_mlp_train_step(float* params, const float* x, const float* target, int32_t rows, float* grad,
                                 float* loss_out, float* m, float* v, int32_t t, float lr, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  if (rows <= 0 || !params || !x || !target || !grad || !loss_out) return KC_EINVAL;
  if (lr > 0.f && (!m || !v || t < 1)) return KC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t need = mlp_rowbuf_bytes(rows) + mlp_part_bytes(rows);
  kc_scratch scr(s, workspace, workspace ? workspace_bytes : 0);
  if (workspace && workspace_bytes < need) return KC_EWORKSPACE;
  float *rowbuf = nullptr, *part = nullptr;
  KC_TRY(scr.alloc((void**)&rowbuf, mlp_rowbuf_bytes(rows)));
  KC_TRY(scr.alloc((void**)&part, mlp_part_bytes(rows)));
  const int32_t nchunks = (rows + MLP_CHUNK - 1) / MLP_CHUNK;
  const unsigned pblocks = (P_N + 1 + 255) / 256;
  k_mlp_rows<<<(rows + 255) / 256, 256, 0, s>>>(params, x, target, rows, rowbuf);
  k_mlp_grad_part<<<dim3(pblocks, (unsigned)nchunks), 256, 0, s>>>(x, rowbuf, rows, part);
  k_mlp_grad_sum<<<pblocks, 256, 0, s>>>(part, nchunks, rows, grad, loss_out);
  if (lr > 0.f) k_mlp_adam<<<(P_N + 255) / 256, 256, 0, s>>>(params, grad, m, v, t, lr);
  KC_HIP(hipGetLastError());
  return KC_OK;
}
