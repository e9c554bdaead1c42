// Device functions of the smoothness classification of a 16-point window
// of the proxy variable (Sec. 4 and Alg. 3): normalization, the SDNN
// (16-64-64-3 MLP, bf16 inputs / weights / hidden activations, FP32
// accumulation, argmax with ties to the higher class) and the modal-decay
// fallback (energy fraction of the modes of degree >= 8 in the orthonormal
// discrete polynomial basis; tau = 2 above 10^-1.5, 1 above 10^-3).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fcs {

__device__ __forceinline__ float bf16_round(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// (v - min) / (max - min); false when the window is flat (class 0).
__device__ __forceinline__ bool normalize_window(const double* v, double* x) {
  double lo = v[0], hi = v[0], am = fabs(v[0]);
  for (int m = 1; m < 16; ++m) {
    lo = fmin(lo, v[m]);
    hi = fmax(hi, v[m]);
    am = fmax(am, fabs(v[m]));
  }
  double range = hi - lo;
  if (range < 1e-3 * fmax(am, 1.0)) return false;
  for (int m = 0; m < 16; ++m) x[m] = (v[m] - lo) / range;
  return true;
}

__device__ __forceinline__ int classify_modal(const double* v, const double* basis) {
  double x[16];
  if (!normalize_window(v, x)) return 0;
  double e_all = 0.0, e_hi = 0.0;
  for (int c = 1; c < 16; ++c) {
    double s = 0.0;
    for (int m = 0; m < 16; ++m) s += x[m] * basis[m * 16 + c];
    e_all += s * s;
    if (c >= 8) e_hi += s * s;
  }
  double frac = e_hi / (e_all > 0 ? e_all : 1.0);
  return frac > 0.031622776601683791 ? 2 : (frac > 1e-3 ? 1 : 0);
}

// W: bf16-rounded weights and FP32 biases in the parameter-blob order.
__device__ __forceinline__ int classify_sdnn(const double* v, const float* W, float* logits = nullptr) {
  double xd[16];
  if (!normalize_window(v, xd)) {
    if (logits) logits[0] = logits[1] = logits[2] = 0.0f;
    return 0;
  }
  const float* W1 = W;
  const float* b1 = W1 + 64 * 16;
  const float* W2 = b1 + 64;
  const float* b2 = W2 + 64 * 64;
  const float* W3 = b2 + 64;
  const float* b3 = W3 + 3 * 64;
  float x[16], h1[64], h2[64], z[3];
  for (int m = 0; m < 16; ++m) x[m] = bf16_round(static_cast<float>(xd[m]));
  for (int o = 0; o < 64; ++o) {
    float s = 0.0f;
    for (int m = 0; m < 16; ++m) s = fmaf(W1[o * 16 + m], x[m], s);
    h1[o] = bf16_round(fmaxf(s + b1[o], 0.0f));
  }
  for (int o = 0; o < 64; ++o) {
    float s = 0.0f;
    for (int m = 0; m < 64; ++m) s = fmaf(W2[o * 64 + m], h1[m], s);
    h2[o] = bf16_round(fmaxf(s + b2[o], 0.0f));
  }
  for (int o = 0; o < 3; ++o) {
    float s = 0.0f;
    for (int m = 0; m < 64; ++m) s = fmaf(W3[o * 64 + m], h2[m], s);
    z[o] = s + b3[o];
  }
  if (logits)
    for (int o = 0; o < 3; ++o) logits[o] = z[o];
  int best = 2;
  if (z[1] > z[best]) best = 1;
  if (z[0] > z[best]) best = 0;
  return best;
}

// Load the parameter blob into LDS, rounding the weight matrices to bf16.
__device__ __forceinline__ void load_sdnn_params(const float* src, float* dst, int nparam) {
  const int w1 = 64 * 16, b1 = w1 + 64, w2 = b1 + 64 * 64, b2 = w2 + 64, w3 = b2 + 3 * 64;
  for (int q = threadIdx.x; q < nparam; q += blockDim.x) {
    bool weight = q < w1 || (q >= b1 && q < w2) || (q >= b2 && q < w3);
    dst[q] = weight ? bf16_round(src[q]) : src[q];
  }
}

}  // namespace fcs
