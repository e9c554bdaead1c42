// Training of the smoothness classifier (the network of Sec. 4 / Alg. 3,
// trained here on synthetic FC-filtered lines): forward pass, weighted
// softmax cross-entropy, backward pass and Adam, as hand-written kernels.
//
// Default (BF16) mode, on the matrix cores: inputs, weight matrices and
// hidden activations rounded to bf16 (nearest even) wherever they enter a
// product, FP32 accumulation; the back-propagated errors (FP32) enter the
// products as the sum of two bf16 parts (hi + lo, 16 significant bits), so
// every product of an error with a bf16 operand is formed exactly.
//   k_train_mfma: forward and backward of 16 samples per wave (the inference
//     layout of classify.h, plus the transposed layer-2 product for the
//     errors), storing inputs, activations and errors feature-major;
//   k_train_grad_mfma: the weight and bias gradients of one 256-sample chunk
//     as 16 x 16 MFMA tiles over the chunk (errors as A rows, activations as
//     B columns, samples as the reduction index), one tile per wave;
//   k_train_finish: the chunk sums in a fixed order, the 1 / sum(w) factor
//     and Adam.
// FP32 mode (gradient-check, no bf16 rounding): one thread per sample for
// forward/backward, batch reductions per parameter row, then Adam.
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
static_assert(kNP == kSdnnParams, "parameter blob layout");
// Samples per gradient chunk; the workspace rows hold the batch padded to a
// multiple of it (padding samples carry zero weight and zero errors).
constexpr int kChunk = 256;
// Per chunk: the kNP gradient sums, the weight sum and the loss sum.
constexpr int kPart = kNP + 2;
// Gradient tiles of one chunk (one wave each): 16 of W2, 4 of W1, 4 of W3,
// 4 of b1, 4 of b2, 1 of b3, and the weight / loss sums.
constexpr int kGradJobs = 34;

__device__ __forceinline__ float rnd(float v, bool fp32) { return fp32 ? v : bf16_round(v); }

// Workspace rows (floats, row stride S = batch rounded up to kChunk):
// X[16][S], A1[64][S], A2[64][S], G1[64][S], G2[64][S], G3[3][S], W[S]
// (per-sample loss weight), L[S] (per-sample loss); then the gradient
// (kNP) and, in BF16 mode, the per-chunk partial sums [S / kChunk][kPart].
struct TrainWs {
  float *X, *A1, *A2, *G1, *G2, *G3, *SW, *SL;
  __host__ __device__ TrainWs(float* ws, int S)
      : X(ws), A1(X + kIn * S), A2(A1 + kH * S), G1(A2 + kH * S), G2(G1 + kH * S), G3(G2 + kH * S),
        SW(G3 + kC * S), SL(SW + S) {}
};
constexpr int kRowsPerSample = kIn + 4 * kH + kC + 2;

// ----------------------------------------------------------- FP32 mode
__global__ __launch_bounds__(256) void k_train_fwd_bwd(const float* __restrict__ params, const float* __restrict__ x,
                                                       const int32_t* __restrict__ labels,
                                                       const float* __restrict__ cw, int B, int S,
                                                       float* __restrict__ ws, int fp32) {
  __shared__ float P[kNP];
  for (int q = threadIdx.x; q < kNP; q += blockDim.x) {
    bool weight = q < oB1 || (q >= oW2 && q < oB2) || (q >= oW3 && q < oB3);
    P[q] = weight ? rnd(params[q], fp32) : params[q];
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const TrainWs t(ws, S);
  // z > 0 of the hidden pre-activations as bit masks (the backward needs
  // nothing else of them)
  float xi[kIn], a1[kH], a2[kH];
  uint64_t m1 = 0, m2 = 0;
  for (int m = 0; m < kIn; ++m) {
    xi[m] = rnd(x[static_cast<int64_t>(i) * kIn + m], fp32);
    t.X[m * S + i] = xi[m];
  }
  for (int o = 0; o < kH; ++o) {
    float s = 0.0f;
    for (int m = 0; m < kIn; ++m) s = fmaf(P[oW1 + o * kIn + m], xi[m], s);
    const float z = s + P[oB1 + o];
    if (z > 0.0f) m1 |= uint64_t{1} << o;
    a1[o] = rnd(fmaxf(z, 0.0f), fp32);
    t.A1[o * S + i] = a1[o];
  }
  for (int o = 0; o < kH; ++o) {
    float s = 0.0f;
    for (int m = 0; m < kH; ++m) s = fmaf(P[oW2 + o * kH + m], a1[m], s);
    const float z = s + P[oB2 + o];
    if (z > 0.0f) m2 |= uint64_t{1} << o;
    a2[o] = rnd(fmaxf(z, 0.0f), fp32);
    t.A2[o * S + i] = a2[o];
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
  t.SW[i] = w;
  t.SL[i] = w * (logf(se) + zm - z3[y]);
  // errors are scaled by the per-sample weight; the 1 / sum(w) factor is
  // applied in the reductions
  float g3[kC];
  for (int o = 0; o < kC; ++o) {
    g3[o] = w * (e[o] / se - (o == y ? 1.0f : 0.0f));
    t.G3[o * S + i] = g3[o];
  }
  float g2[kH];
  for (int m = 0; m < kH; ++m) {
    float s = 0.0f;
    for (int o = 0; o < kC; ++o) s = fmaf(g3[o], P[oW3 + o * kH + m], s);
    g2[m] = (m2 >> m) & 1 ? s : 0.0f;
    t.G2[m * S + i] = g2[m];
  }
  for (int m = 0; m < kH; ++m) {
    float s = 0.0f;
    for (int o = 0; o < kH; ++o) s = fmaf(g2[o], P[oW2 + o * kH + m], s);
    t.G1[m * S + i] = (m1 >> m) & 1 ? s : 0.0f;
  }
}

// One workgroup per output row of a weight matrix (plus one for the loss):
// grad[o][m] = sum_i G[o][i] A[m][i] / sum_i w_i, bias grad = sum_i G[o][i] / sum_i w_i.
__global__ __launch_bounds__(256) void k_train_reduce(int B, int S, const float* __restrict__ ws,
                                                      float* __restrict__ grads, float* __restrict__ loss) {
  __shared__ float red[256];
  const TrainWs t(const_cast<float*>(ws), S);
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
  for (int i = threadIdx.x; i < B; i += blockDim.x) wsum += t.SW[i];
  wsum = block_sum(wsum);
  const float inv = 1.0f / wsum;
  int row = blockIdx.x;
  if (row == kH + kH + kC) {
    float l = 0.0f;
    for (int i = threadIdx.x; i < B; i += blockDim.x) l += t.SL[i];
    l = block_sum(l);
    if (threadIdx.x == 0) *loss = l * inv;
    return;
  }
  const float* G;
  const float* A;
  int nin, wofs, bofs, o;
  if (row < kH) {
    o = row;
    G = t.G1 + o * S;
    A = t.X;
    nin = kIn;
    wofs = oW1;
    bofs = oB1;
  } else if (row < 2 * kH) {
    o = row - kH;
    G = t.G2 + o * S;
    A = t.A1;
    nin = kH;
    wofs = oW2;
    bofs = oB2;
  } else {
    o = row - 2 * kH;
    G = t.G3 + o * S;
    A = t.A2;
    nin = kH;
    wofs = oW3;
    bofs = oB3;
  }
  for (int m = -1; m < nin; ++m) {
    float s = 0.0f;
    for (int i = threadIdx.x; i < B; i += blockDim.x) s += G[i] * (m < 0 ? 1.0f : A[m * S + i]);
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

// ----------------------------------------------------------- BF16 mode
// Transposed layer-2 fragments for the error product G1^T = W2^T G2^T:
// lane (c, g) of output tile t (input units 16 t + c as MFMA rows) and
// block kb holds the bf16 weights W2[h][16 t + c] for the hidden units h of
// its k slots, in the slot order of the forward (sdnn_slot), so that the
// lane's own layer-2 errors form the B operand unchanged.  8 tiles x 4
// words per lane.
constexpr int kTransWords = 32;

__device__ __forceinline__ uint32_t w2t_word(const float* __restrict__ W2, int lane, int w) {
  const int g = lane >> 4, c = lane & 15;
  const int tb = w >> 2, t = tb >> 1, kb = tb & 1, j = 2 * (w & 3);
  return bf16_pair(W2[sdnn_slot(kb, g, j) * kH + 16 * t + c], W2[sdnn_slot(kb, g, j + 1) * kH + 16 * t + c]);
}

// bf16 bits of a value that is already bf16-exact.
__device__ __forceinline__ __bf16 bf16_exact(float f) {
  return __builtin_bit_cast(__bf16, static_cast<uint16_t>(__float_as_uint(f) >> 16));
}

// Forward and backward of the batch, 16 samples per wave (lane l: sample
// l % 16 of its group, features / hidden rows of lane group g = l / 16, as
// in sdnn_mfma).  Samples at or beyond B (row padding) store zero weight,
// loss and errors.
__global__ __launch_bounds__(256) void k_train_mfma(const float* __restrict__ params, const float* __restrict__ x,
                                                    const int32_t* __restrict__ labels, const float* __restrict__ cw,
                                                    int B, int S, float* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) uint32_t tab[64 * kSdnnFragWords];
  __shared__ __attribute__((aligned(16))) uint32_t tabt[64 * kTransWords];
  __shared__ float w3r[kC * kH];
  for (int q = threadIdx.x; q < 64 * kSdnnFragWords; q += blockDim.x)
    tab[q] = sdnn_frag_word(params, q / kSdnnFragWords, q % kSdnnFragWords);
  for (int q = threadIdx.x; q < 64 * kTransWords; q += blockDim.x)
    tabt[q] = w2t_word(params + oW2, q / kTransWords, q % kTransWords);
  for (int q = threadIdx.x; q < kC * kH; q += blockDim.x) w3r[q] = bf16_round(params[oW3 + q]);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int i = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + c;  // this lane's sample
  if (i - c >= S) return;  // whole group beyond the padded rows (wave-uniform)
  const TrainWs t(ws, S);
  const bool real = i < B;
  SdnnFrag F;
  load_sdnn_frag(tab, F);

  // forward
  float xr[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    xr[j] = real ? bf16_round(x[static_cast<int64_t>(i) * kIn + 4 * g + j]) : 0.0f;
    t.X[(4 * g + j) * S + i] = xr[j];
  }
  sdnn_s16x4 xb;
#pragma unroll
  for (int j = 0; j < 4; ++j) xb[j] = static_cast<short>(__float_as_uint(xr[j]) >> 16);
  const sdnn_f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  sdnn_f32x4 z1[4];
#pragma unroll
  for (int ht = 0; ht < 4; ++ht) {
    z1[ht] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F.w1[ht], xb, zero, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) z1[ht][r] += F.b1[ht][r];
  }
  sdnn_bf16x8 h1[2];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int ht = 2 * kb + (j >> 2), r = j & 3;
      const float a = bf16_round(fmaxf(z1[ht][r], 0.0f));
      t.A1[(16 * ht + 4 * g + r) * S + i] = a;
      h1[kb][j] = bf16_exact(a);
    }
  sdnn_f32x4 z2[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    z2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[mt][0], h1[0], zero, 0, 0, 0);
    z2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[mt][1], h1[1], z2[mt], 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) z2[mt][r] += F.b2[mt][r];
  }
  sdnn_bf16x8 h2[2];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mt = 2 * kb + (j >> 2), r = j & 3;
      const float a = bf16_round(fmaxf(z2[mt][r], 0.0f));
      t.A2[(16 * mt + 4 * g + r) * S + i] = a;
      h2[kb][j] = bf16_exact(a);
    }
  sdnn_f32x4 z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w3[0], h2[0], zero, 0, 0, 0);
  z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w3[1], h2[1], z3, 0, 0, 0);
  // logits: rows 0..2 of lane group 0; every lane of the sample takes them
  float lg[kC];
#pragma unroll
  for (int o = 0; o < kC; ++o) lg[o] = __shfl(z3[o] + F.b3[o], c);

  // loss and output errors (weighted; 1 / sum(w) in the finish)
  const int y = real ? labels[i] : 0;
  const float w = real ? cw[y] : 0.0f;
  const float zm = fmaxf(lg[0], fmaxf(lg[1], lg[2]));
  float e[kC], se = 0.0f;
#pragma unroll
  for (int o = 0; o < kC; ++o) {
    e[o] = expf(lg[o] - zm);
    se += e[o];
  }
  float g3[kC];
#pragma unroll
  for (int o = 0; o < kC; ++o) g3[o] = w * (e[o] / se - (o == y ? 1.0f : 0.0f));
  if (g == 0) {
    t.SW[i] = w;
    t.SL[i] = real ? w * (logf(se) + zm - lg[y]) : 0.0f;
#pragma unroll
    for (int o = 0; o < kC; ++o) t.G3[o * S + i] = g3[o];
  }

  // layer-2 errors of this lane's 16 hidden rows (a 3-term sum, as FP32
  // fmas), split into bf16 hi + lo B fragments in the forward's slot order
  sdnn_bf16x8 ehi[2], elo[2];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mt = 2 * kb + (j >> 2), r = j & 3, u = 16 * mt + 4 * g + r;
      float s = 0.0f;
#pragma unroll
      for (int o = 0; o < kC; ++o) s = fmaf(g3[o], w3r[o * kH + u], s);
      const float e2 = z2[mt][r] > 0.0f ? s : 0.0f;
      t.G2[u * S + i] = e2;
      const float hi = bf16_round(e2);
      ehi[kb][j] = bf16_exact(hi);
      elo[kb][j] = bf16_exact(bf16_round(e2 - hi));
    }
  // layer-1 errors: G1^T = W2^T G2^T on the matrix cores, masked by z1 > 0
  const uint4* tt = reinterpret_cast<const uint4*>(tabt + lane * kTransWords);
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const sdnn_bf16x8 wa = __builtin_bit_cast(sdnn_bf16x8, tt[2 * ot]);
    const sdnn_bf16x8 wb = __builtin_bit_cast(sdnn_bf16x8, tt[2 * ot + 1]);
    sdnn_f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, ehi[0], zero, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, ehi[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, elo[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, elo[1], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) t.G1[(16 * ot + 4 * g + r) * S + i] = z1[ot][r] > 0.0f ? acc[r] : 0.0f;
  }
}

// Eight consecutive floats of a workspace row as bf16 hi + lo parts, or (lo
// null) as exact bf16 values.
__device__ __forceinline__ void load8_split(const float* __restrict__ p, sdnn_bf16x8& hi, sdnn_bf16x8* lo) {
  const float4 u = reinterpret_cast<const float4*>(p)[0], v = reinterpret_cast<const float4*>(p)[1];
  const float f[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (lo) {
      const float h = bf16_round(f[j]);
      hi[j] = bf16_exact(h);
      (*lo)[j] = bf16_exact(bf16_round(f[j] - h));
    } else {
      hi[j] = bf16_exact(f[j]);
    }
  }
}

// Gradient tile `job` of chunk `blockIdx.x / kGradJobs` (one wave):
// sum over the chunk's samples of error row x activation column, errors as
// bf16 hi + lo (A operand, 16 rows x 32 samples per step), activations or
// ones as exact bf16 (B operand, 32 samples x 16 columns).
__global__ __launch_bounds__(64) void k_train_grad_mfma(int S, const float* __restrict__ ws,
                                                        float* __restrict__ part) {
  const int chunk = blockIdx.x / kGradJobs, job = blockIdx.x % kGradJobs;
  const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
  const TrainWs t(const_cast<float*>(ws), S);
  const int64_t i0 = static_cast<int64_t>(chunk) * kChunk;
  float* out = part + static_cast<int64_t>(chunk) * kPart;
  if (job == kGradJobs - 1) {
    // weight and loss sums of the chunk, in a fixed order
    float sw = 0.0f, sl = 0.0f;
#pragma unroll
    for (int q = 0; q < kChunk / 64; ++q) {
      sw += t.SW[i0 + q * 64 + lane];
      sl += t.SL[i0 + q * 64 + lane];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      sw += __shfl_xor(sw, d);
      sl += __shfl_xor(sl, d);
    }
    if (lane == 0) {
      out[kNP] = sw;
      out[kNP + 1] = sl;
    }
    return;
  }
  // error rows (A), activation columns (B; null: ones), number of error
  // rows, and where result (row, column) goes
  const float* Ar;
  const float* Bc = nullptr;
  int nrows = 16, dst, ldd;
  if (job < 16) {
    const int mt = job >> 2, nt = job & 3;
    Ar = t.G2 + 16 * mt * S;
    Bc = t.A1 + 16 * nt * S;
    dst = oW2 + 16 * mt * kH + 16 * nt;
    ldd = kH;
  } else if (job < 20) {
    const int mt = job - 16;
    Ar = t.G1 + 16 * mt * S;
    Bc = t.X;
    dst = oW1 + 16 * mt * kIn;
    ldd = kIn;
  } else if (job < 24) {
    const int nt = job - 20;
    Ar = t.G3;
    Bc = t.A2 + 16 * nt * S;
    nrows = kC;
    dst = oW3 + 16 * nt;
    ldd = kH;
  } else if (job < 28) {
    Ar = t.G1 + 16 * (job - 24) * S;
    dst = oB1 + 16 * (job - 24);
    ldd = 0;
  } else if (job < 32) {
    Ar = t.G2 + 16 * (job - 28) * S;
    dst = oB2 + 16 * (job - 28);
    ldd = 0;
  } else {
    Ar = t.G3;
    nrows = kC;
    dst = oB3;
    ldd = 0;
  }
  const sdnn_f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  sdnn_f32x4 acc = zero;
  sdnn_bf16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = bf16_exact(1.0f);
  const bool arow = c < nrows;  // rows beyond the error rows are zero
  for (int k0 = 0; k0 < kChunk; k0 += 32) {
    const int64_t s0 = i0 + k0 + 8 * g;
    sdnn_bf16x8 ah, al, b;
    if (arow) {
      load8_split(Ar + static_cast<int64_t>(c) * S + s0, ah, &al);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) ah[j] = al[j] = bf16_exact(0.0f);
    }
    if (Bc)
      load8_split(Bc + static_cast<int64_t>(c) * S + s0, b, nullptr);
    else
      b = ones;
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, acc, 0, 0, 0);
  }
  // result (row 4 g + r, column c) of the tile
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * g + r;
    if (row >= nrows) continue;
    if (ldd)
      out[dst + row * ldd + c] = acc[r];
    else if (c == 0)
      out[dst + row] = acc[r];
  }
}

// Chunk sums in chunk order, the 1 / sum(w) factor, the loss, and Adam.
__global__ void k_train_finish(int nchunk, const float* __restrict__ part, float* __restrict__ grads,
                               float* __restrict__ loss, float* __restrict__ p, float* __restrict__ m,
                               float* __restrict__ v, float lr, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kNP) return;
  float wsum = 0.0f, gsum = 0.0f;
  for (int k = 0; k < nchunk; ++k) {
    wsum += part[static_cast<int64_t>(k) * kPart + kNP];
    gsum += part[static_cast<int64_t>(k) * kPart + q];
  }
  const float inv = 1.0f / wsum;
  if (q == 0) {
    float l = 0.0f;
    for (int k = 0; k < nchunk; ++k) l += part[static_cast<int64_t>(k) * kPart + kNP + 1];
    *loss = l * inv;
  }
  const float gg = gsum * inv;
  grads[q] = gg;
  const float mm = 0.9f * m[q] + 0.1f * gg;
  const float vv = 0.999f * v[q] + 0.001f * gg * gg;
  m[q] = mm;
  v[q] = vv;
  p[q] = p[q] - lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

}  // namespace

// Padded row stride of a batch and the workspace floats it needs: the
// per-sample rows, one gradient vector and the per-chunk partial sums.
constexpr int padded_batch(int B) { return (B + kChunk - 1) / kChunk * kChunk; }
constexpr size_t train_floats(int B) {
  return static_cast<size_t>(padded_batch(B)) * kRowsPerSample + kNP +
         static_cast<size_t>(padded_batch(B) / kChunk) * kPart;
}

// Library-owned scratch of the allocation-free training step: the per-sample
// activations and errors of a batch of at most FCS_SDNN_TRAIN_MAX_BATCH
// samples, one gradient vector and the per-chunk partial sums (9.8 MB).  Each
// GPU the library runs on holds its own copy until the process ends.
constexpr size_t kScratchFloats = train_floats(FCS_SDNN_TRAIN_MAX_BATCH);
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

size_t sdnn_train_floats(int B) { return train_floats(B); }

hipError_t launch_sdnn_train(float* params, float* m, float* v, int t, float lr, const float* x,
                             const int32_t* labels, const float* cw, int B, float* loss, float* grads_out,
                             float* ws, int fp32, hipStream_t s) {
  const int S = padded_batch(B);
  float* grads = grads_out ? grads_out : ws + static_cast<size_t>(S) * kRowsPerSample;
  const double c1 = 1.0 - __builtin_pow(0.9, t), c2 = 1.0 - __builtin_pow(0.999, t);
  if (fp32) {
    hipLaunchKernelGGL(k_train_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, s, params, x, labels, cw, B, S, ws, 1);
    hipLaunchKernelGGL(k_train_reduce, dim3(2 * kH + kC + 1), dim3(256), 0, s, B, S, ws, grads, loss);
    hipLaunchKernelGGL(k_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, params, m, v, grads, kNP, lr,
                       static_cast<float>(c1), static_cast<float>(c2));
    return hipGetLastError();
  }
  float* part = ws + static_cast<size_t>(S) * kRowsPerSample + kNP;
  const int nchunk = S / kChunk;
  hipLaunchKernelGGL(k_train_mfma, dim3(S / 64), dim3(256), 0, s, params, x, labels, cw, B, S, ws);
  hipLaunchKernelGGL(k_train_grad_mfma, dim3(nchunk * kGradJobs), dim3(64), 0, s, S, ws, part);
  hipLaunchKernelGGL(k_train_finish, dim3((kNP + 255) / 256), dim3(256), 0, s, nchunk, part, grads, loss, params, m,
                     v, lr, static_cast<float>(c1), static_cast<float>(c2));
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
