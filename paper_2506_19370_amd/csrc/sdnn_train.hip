// Training of the smoothness classifier (the network of Sec. 4 / Alg. 3,
// trained here on synthetic FC-filtered lines): forward pass, weighted
// softmax cross-entropy, backward pass and Adam, as hand-written kernels.
//
// Forward and the backward products use the forward's rounding: inputs,
// weight matrices and hidden activations rounded to bf16 (FP32 accumulation)
// unless the FP32-activation flag is set.  Per-sample forward/backward runs
// one thread per sample with the parameters in LDS and stores activations
// and back-propagated errors feature-major; the weight gradients are then
// batch reductions (one workgroup per parameter row), followed by Adam.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/fcsdnn.h"
#include "classify.h"
#include "sdnn_train.h"
#include "stage_kernels.h"

namespace fcs {

namespace {

constexpr int kIn = 16, kH = 64, kC = 3;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kC * kH, kNP = oB3 + kC;

__device__ __forceinline__ float rnd(float v, bool fp32) { return fp32 ? v : bf16_round(v); }

// Workspace (floats): X[16][B], A1[64][B], A2[64][B], G1[64][B], G2[64][B],
// G3[3][B], W[B] (per-sample loss weight), L[B] (per-sample loss).
__global__ __launch_bounds__(256) void k_train_fwd_bwd(const float* __restrict__ params, const float* __restrict__ x,
                                                       const int32_t* __restrict__ labels,
                                                       const float* __restrict__ cw, int B, float* __restrict__ ws,
                                                       int fp32) {
  __shared__ float P[kNP];
  for (int q = threadIdx.x; q < kNP; q += blockDim.x) {
    bool weight = q < oB1 || (q >= oW2 && q < oB2) || (q >= oW3 && q < oB3);
    P[q] = weight ? rnd(params[q], fp32) : params[q];
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  float* X = ws;
  float* A1 = X + kIn * B;
  float* A2 = A1 + kH * B;
  float* G1 = A2 + kH * B;
  float* G2 = G1 + kH * B;
  float* G3 = G2 + kH * B;
  float* SW = G3 + kC * B;
  float* SL = SW + B;
  float xi[kIn], z1[kH], a1[kH], z2[kH], a2[kH];
  for (int m = 0; m < kIn; ++m) {
    xi[m] = rnd(x[static_cast<int64_t>(i) * kIn + m], fp32);
    X[m * B + i] = xi[m];
  }
  for (int o = 0; o < kH; ++o) {
    float s = 0.0f;
    for (int m = 0; m < kIn; ++m) s = fmaf(P[oW1 + o * kIn + m], xi[m], s);
    z1[o] = s + P[oB1 + o];
    a1[o] = rnd(fmaxf(z1[o], 0.0f), fp32);
    A1[o * B + i] = a1[o];
  }
  for (int o = 0; o < kH; ++o) {
    float s = 0.0f;
    for (int m = 0; m < kH; ++m) s = fmaf(P[oW2 + o * kH + m], a1[m], s);
    z2[o] = s + P[oB2 + o];
    a2[o] = rnd(fmaxf(z2[o], 0.0f), fp32);
    A2[o * B + i] = a2[o];
  }
  float z3[kC];
  for (int o = 0; o < kC; ++o) {
    float s = 0.0f;
    for (int m = 0; m < kH; ++m) s = fmaf(P[oW3 + o * kH + m], a2[m], s);
    z3[o] = s + P[oB3 + o];
  }
  const int y = labels[i];
  float zm = fmaxf(z3[0], fmaxf(z3[1], z3[2]));
  float e[kC], se = 0.0f;
  for (int o = 0; o < kC; ++o) {
    e[o] = expf(z3[o] - zm);
    se += e[o];
  }
  const float w = cw[y];
  SW[i] = w;
  SL[i] = w * (logf(se) + zm - z3[y]);
  // errors are scaled by the per-sample weight; the 1 / sum(w) factor is
  // applied in the reductions
  float g3[kC];
  for (int o = 0; o < kC; ++o) {
    g3[o] = w * (e[o] / se - (o == y ? 1.0f : 0.0f));
    G3[o * B + i] = g3[o];
  }
  float g2[kH];
  for (int m = 0; m < kH; ++m) {
    float s = 0.0f;
    for (int o = 0; o < kC; ++o) s = fmaf(g3[o], P[oW3 + o * kH + m], s);
    g2[m] = z2[m] > 0.0f ? s : 0.0f;
    G2[m * B + i] = g2[m];
  }
  for (int m = 0; m < kH; ++m) {
    float s = 0.0f;
    for (int o = 0; o < kH; ++o) s = fmaf(g2[o], P[oW2 + o * kH + m], s);
    G1[m * B + i] = z1[m] > 0.0f ? s : 0.0f;
  }
}

// One workgroup per output row of a weight matrix (plus one for the loss):
// grad[o][m] = sum_i G[o][i] A[m][i] / sum_i w_i, bias grad = sum_i G[o][i] / sum_i w_i.
__global__ __launch_bounds__(256) void k_train_reduce(int B, const float* __restrict__ ws,
                                                      float* __restrict__ grads, float* __restrict__ loss) {
  __shared__ float red[256];
  const float* X = ws;
  const float* A1 = X + kIn * B;
  const float* A2 = A1 + kH * B;
  const float* G1 = A2 + kH * B;
  const float* G2 = G1 + kH * B;
  const float* G3 = G2 + kH * B;
  const float* SW = G3 + kC * B;
  const float* SL = SW + B;
  auto block_sum = [&](float v) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    float r = red[0];
    __syncthreads();
    return r;
  };
  float wsum = 0.0f;
  for (int i = threadIdx.x; i < B; i += blockDim.x) wsum += SW[i];
  wsum = block_sum(wsum);
  const float inv = 1.0f / wsum;
  int row = blockIdx.x;
  if (row == kH + kH + kC) {
    float l = 0.0f;
    for (int i = threadIdx.x; i < B; i += blockDim.x) l += SL[i];
    l = block_sum(l);
    if (threadIdx.x == 0) *loss = l * inv;
    return;
  }
  const float* G;
  const float* A;
  int nin, wofs, bofs, o;
  if (row < kH) {
    o = row;
    G = G1 + o * B;
    A = X;
    nin = kIn;
    wofs = oW1;
    bofs = oB1;
  } else if (row < 2 * kH) {
    o = row - kH;
    G = G2 + o * B;
    A = A1;
    nin = kH;
    wofs = oW2;
    bofs = oB2;
  } else {
    o = row - 2 * kH;
    G = G3 + o * B;
    A = A2;
    nin = kH;
    wofs = oW3;
    bofs = oB3;
  }
  for (int m = -1; m < nin; ++m) {
    float s = 0.0f;
    for (int i = threadIdx.x; i < B; i += blockDim.x) s += G[i] * (m < 0 ? 1.0f : A[m * B + i]);
    s = block_sum(s);
    if (threadIdx.x == 0) {
      if (m < 0)
        grads[bofs + o] = s * inv;
      else
        grads[wofs + o * nin + m] = s * inv;
    }
  }
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float c1, float c2) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float gg = g[q];
  float mm = 0.9f * m[q] + 0.1f * gg;
  float vv = 0.999f * v[q] + 0.001f * gg * gg;
  m[q] = mm;
  v[q] = vv;
  float mh = mm / c1, vh = vv / c2;
  p[q] = p[q] - lr * mh / (sqrtf(vh) + 1e-8f);
}

}  // namespace

// Library-owned scratch of the allocation-free training step: the per-sample
// activations and errors of a batch of at most FCS_SDNN_TRAIN_MAX_BATCH
// samples plus one gradient vector (9.1 MB).  Each GPU the library runs on
// holds its own copy until the process ends.
constexpr size_t kScratchFloats =
    static_cast<size_t>(FCS_SDNN_TRAIN_MAX_BATCH) * (kIn + 4 * kH + kC + 2) + kNP;
__device__ __align__(256) float scratch[kScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`, looked up once per
// device (host code must not pass the symbol itself to a kernel).
hipError_t scratch_for_current_device(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = static_cast<float*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}
}  // namespace

size_t sdnn_train_floats(int B) { return static_cast<size_t>(B) * (kIn + 4 * kH + kC + 2) + kNP; }

hipError_t launch_sdnn_train(float* params, float* m, float* v, int t, float lr, const float* x,
                             const int32_t* labels, const float* cw, int B, float* loss, float* grads_out,
                             float* ws, int fp32, hipStream_t s) {
  float* grads = grads_out ? grads_out : ws + static_cast<size_t>(B) * (kIn + 4 * kH + kC + 2);
  hipLaunchKernelGGL(k_train_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, s, params, x, labels, cw, B, ws, fp32);
  hipLaunchKernelGGL(k_train_reduce, dim3(2 * kH + kC + 1), dim3(256), 0, s, B, ws, grads, loss);
  double c1 = 1.0 - __builtin_pow(0.9, t), c2 = 1.0 - __builtin_pow(0.999, t);
  hipLaunchKernelGGL(k_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, params, m, v, grads, kNP, lr,
                     static_cast<float>(c1), static_cast<float>(c2));
  return hipGetLastError();
}

}  // namespace fcs

// Allocation-free form of fcs_sdnn_train_step: the same kernels on the
// library-owned scratch of the current GPU.  No slot of the scratch is read
// before the same call wrote it, so nothing is cleared between calls.
extern "C" fcs_status fcs_sdnn_train_step_noalloc(float* params, float* m, float* v, int32_t t, float lr,
                                                  const float* x, const int32_t* labels,
                                                  const float* class_weight, int32_t batch, float* loss,
                                                  float* grads, int32_t flags, void* stream) {
  if (!params || !m || !v || !x || !labels || !class_weight || !loss || batch <= 0 || t < 1) return FCS_EINVAL;
  if (batch > FCS_SDNN_TRAIN_MAX_BATCH) return FCS_EINVAL;
  float* ws = nullptr;
  if (fcs::scratch_for_current_device(&ws) != hipSuccess) return FCS_EHIP;
  return fcs::launch_sdnn_train(params, m, v, t, lr, x, labels, class_weight, batch, loss, grads, ws, flags & 1,
                                static_cast<hipStream_t>(stream)) == hipSuccess
             ? FCS_OK
             : FCS_EHIP;
}
