// Device functions of the smoothness classification of a 16-point window
// of the proxy variable (Sec. 4 and Alg. 3): normalization, the SDNN
// (16-64-64-3 MLP, bf16 inputs / weights / hidden activations, FP32
// accumulation, argmax with ties to the higher class) on the matrix cores,
// and the modal-decay fallback (energy fraction of the modes of degree >= 8 in the orthonormal
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

// ---------------------------------------------------------------------------
// SDNN inference on the matrix cores, 16 windows per wave.
//
// Lane l of a wave owns window l % 16 and its input features 4 g .. 4 g + 3
// (g = l / 16).  Layer k computes Z_k^T = W_k H_{k-1}^T (hidden units as MFMA
// rows, windows as columns), so lane l receives the pre-activations of
// hidden units 4 g + r (r < 4) of every 16-row tile for window l % 16.  Two
// such tiles form the B operand of the next 16x16x32 product directly: the
// sum over hidden units may run in any order, so the k slots of lane group g
// are taken as hidden units {4 g .. 4 g + 3} of the first tile and
// {4 g .. 4 g + 3} of the second, and the weight fragments are gathered in
// that same order.  Weights and biases stay in registers for the whole
// kernel.  Arithmetic: bf16 inputs, weights and hidden activations, FP32
// accumulation (the products' summation order differs from a sequential
// loop only by FP32 rounding).
typedef short sdnn_s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 sdnn_bf16x8 __attribute__((ext_vector_type(8)));
typedef float sdnn_f32x4 __attribute__((ext_vector_type(4)));

struct SdnnFrag {
  sdnn_s16x4 w1[4];       // layer 1, hidden tile ht
  sdnn_bf16x8 w2[4][2];   // layer 2, [output tile][input block]
  sdnn_bf16x8 w3[2];      // layer 3 (rows >= 3 zero), [input block]
  float b1[4][4], b2[4][4], b3[4];
};

// Hidden unit of k slot j of lane group g in input block kb.
__device__ __forceinline__ int sdnn_slot(int kb, int g, int j) { return 32 * kb + (j < 4 ? 4 * g + j : 12 + 4 * g + j); }

constexpr int kSdnnParams = 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3;

// Fragment table: the weights and biases each lane needs, lane-major, 84
// 32-bit words per lane (21 x 16 bytes):
//   0..7    layer-1 weights, tile ht: words 2 ht, 2 ht + 1 (4 bf16)
//   8..39   layer-2 weights, [output tile mt][input block kb]: 4 words each
//   40..47  layer-3 weights, [input block kb]: 4 words each
//   48..63  layer-1 biases of the lane's rows [ht][r] (FP32)
//   64..79  layer-2 biases [ht][r]
//   80..83  layer-3 biases of rows 4 g + r (zero beyond the 3 classes)
constexpr int kSdnnFragWords = 84;

// bf16 bit pattern of f, round to nearest even (the rounding the oracle
// applies).
__device__ __forceinline__ uint32_t bf16_bits(float f) { return __float_as_uint(bf16_round(f)) >> 16; }

__device__ __forceinline__ uint32_t bf16_pair(float a, float b) { return bf16_bits(a) | (bf16_bits(b) << 16); }

// Word w of lane `lane`'s fragment table, from the FP32 parameter blob.
__device__ __forceinline__ uint32_t sdnn_frag_word(const float* __restrict__ W, int lane, int w) {
  const float* W1 = W;
  const float* B1 = W1 + 64 * 16;
  const float* W2 = B1 + 64;
  const float* B2 = W2 + 64 * 64;
  const float* W3 = B2 + 64;
  const float* B3 = W3 + 3 * 64;
  const int g = lane >> 4, c = lane & 15;
  if (w < 8) {
    const int ht = w >> 1, j = 2 * (w & 1);
    const float* r = W1 + (16 * ht + c) * 16 + 4 * g + j;
    return bf16_pair(r[0], r[1]);
  }
  if (w < 40) {
    const int i = w - 8, mt = i >> 3, kb = (i >> 2) & 1, j = 2 * (i & 3);
    const float* r = W2 + (16 * mt + c) * 64;
    return bf16_pair(r[sdnn_slot(kb, g, j)], r[sdnn_slot(kb, g, j + 1)]);
  }
  if (w < 48) {
    const int i = w - 40, kb = i >> 2, j = 2 * (i & 3);
    if (c >= 3) return 0u;
    const float* r = W3 + c * 64;
    return bf16_pair(r[sdnn_slot(kb, g, j)], r[sdnn_slot(kb, g, j + 1)]);
  }
  float v;
  if (w < 64) {
    v = B1[16 * ((w - 48) >> 2) + 4 * g + ((w - 48) & 3)];
  } else if (w < 80) {
    v = B2[16 * ((w - 64) >> 2) + 4 * g + ((w - 64) & 3)];
  } else {
    const int row = 4 * g + (w - 80);
    v = row < 3 ? B3[row] : 0.0f;
  }
  return __float_as_uint(v);
}

// Unpacks this lane's fragments from a table (global memory or LDS).
__device__ __forceinline__ void load_sdnn_frag(const uint32_t* table, SdnnFrag& F) {
  const uint4* t = reinterpret_cast<const uint4*>(table + (threadIdx.x & 63) * kSdnnFragWords);
  uint4 q[21];
#pragma unroll
  for (int i = 0; i < 21; ++i) q[i] = t[i];
  const uint32_t* u = reinterpret_cast<const uint32_t*>(q);
#pragma unroll
  for (int ht = 0; ht < 4; ++ht) {
    const uint32_t lo = u[2 * ht], hi = u[2 * ht + 1];
    F.w1[ht] = sdnn_s16x4{static_cast<short>(lo & 0xFFFF), static_cast<short>(lo >> 16),
                          static_cast<short>(hi & 0xFFFF), static_cast<short>(hi >> 16)};
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) F.w2[mt][kb] = __builtin_bit_cast(sdnn_bf16x8, q[2 + 2 * mt + kb]);
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) F.w3[kb] = __builtin_bit_cast(sdnn_bf16x8, q[10 + kb]);
#pragma unroll
  for (int ht = 0; ht < 4; ++ht)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      F.b1[ht][r] = __uint_as_float(u[48 + 4 * ht + r]);
      F.b2[ht][r] = __uint_as_float(u[64 + 4 * ht + r]);
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) F.b3[r] = __uint_as_float(u[80 + r]);
}

// Builds the fragment table of a parameter blob in LDS (whole block).
__device__ __forceinline__ void build_sdnn_table(const float* __restrict__ W, uint32_t* table) {
  for (int q = threadIdx.x; q < 64 * kSdnnFragWords; q += blockDim.x)
    table[q] = sdnn_frag_word(W, q / kSdnnFragWords, q % kSdnnFragWords);
  __syncthreads();
}

// Two 16-row tiles of pre-activations -> bf16 ReLU activations as one B
// fragment (k slots in the order of sdnn_slot).
__device__ __forceinline__ sdnn_bf16x8 sdnn_act(const sdnn_f32x4& za, const float* ba, const sdnn_f32x4& zb,
                                                const float* bb) {
  sdnn_bf16x8 h;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    // v_cvt_pk_bf16_f32 rounds to nearest even, as bf16_round does
    h[j] = static_cast<__bf16>(fmaxf(za[j] + ba[j], 0.0f));
    h[4 + j] = static_cast<__bf16>(fmaxf(zb[j] + bb[j], 0.0f));
  }
  return h;
}

// One wave-wide evaluation of 16 windows.  x: this lane's four features
// (already bf16-rounded).  On return lanes 0..15 hold the three logits of
// window lane % 16 in z[0..2].
__device__ __forceinline__ void sdnn_mfma(const SdnnFrag& F, const float (&x)[4], float (&z)[3]) {
  sdnn_s16x4 xb;
#pragma unroll
  for (int j = 0; j < 4; ++j) xb[j] = static_cast<short>(__float_as_uint(x[j]) >> 16);  // x is bf16-exact
  const sdnn_f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  sdnn_f32x4 z1[4];
#pragma unroll
  for (int ht = 0; ht < 4; ++ht) z1[ht] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F.w1[ht], xb, zero, 0, 0, 0);
  sdnn_bf16x8 h1[2];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) h1[kb] = sdnn_act(z1[2 * kb], F.b1[2 * kb], z1[2 * kb + 1], F.b1[2 * kb + 1]);
  sdnn_f32x4 z2[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    z2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[mt][0], h1[0], zero, 0, 0, 0);
    z2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[mt][1], h1[1], z2[mt], 0, 0, 0);
  }
  sdnn_bf16x8 h2[2];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) h2[kb] = sdnn_act(z2[2 * kb], F.b2[2 * kb], z2[2 * kb + 1], F.b2[2 * kb + 1]);
  sdnn_f32x4 z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w3[0], h2[0], zero, 0, 0, 0);
  z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w3[1], h2[1], z3, 0, 0, 0);
#pragma unroll
  for (int o = 0; o < 3; ++o) z[o] = z3[o] + F.b3[o];
}

// Class from logits, ties to the higher class.
__device__ __forceinline__ int sdnn_argmax(const float (&z)[3]) {
  int best = 2;
  if (z[1] > z[best]) best = 1;
  if (z[0] > z[best]) best = 0;
  return best;
}

// Lane-distributed window normalisation: v holds this lane's 4 of the 16
// window values (lanes l, l ^ 16, l ^ 32, l ^ 48 share a window).  Returns
// false (flat window, class 0) when max - min < 1e-3 max(max |v|, 1).
__device__ __forceinline__ bool sdnn_features(const double (&v)[4], float (&x)[4]) {
  double lo = fmin(fmin(v[0], v[1]), fmin(v[2], v[3]));
  double hi = fmax(fmax(v[0], v[1]), fmax(v[2], v[3]));
  lo = fmin(lo, __shfl_xor(lo, 16));
  hi = fmax(hi, __shfl_xor(hi, 16));
  lo = fmin(lo, __shfl_xor(lo, 32));
  hi = fmax(hi, __shfl_xor(hi, 32));
  const double am = fmax(fabs(lo), fabs(hi));  // max |v| over the window
  const double range = hi - lo;
  const bool live = !(range < 1e-3 * fmax(am, 1.0));
  // one reciprocal per window; (v - lo) * (1 / range) and (v - lo) / range
  // differ by at most one FP64 ulp, far below the bf16 rounding that follows
  const double inv = live ? 1.0 / range : 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = live ? bf16_round(static_cast<float>((v[j] - lo) * inv)) : 0.0f;
  return live;
}

}  // namespace fcs
