// Grouped FC derivative contraction on gfx950 matrix cores.
//
// The FC derivative along a grid line of n points is a fixed linear map
// (continuation, spectral multiplier, restriction: Sec. 2 and the stage
// algorithm of Sec. 5), so all lines of all subpatches that share a length
// are one product  Y[line][t] = sum_s Op[t][s] X[line][s].  One launch
// covers every (subpatch, direction, operand set) through a tile list; a
// 256-thread workgroup computes 64 outputs t x 64 lines, staging operator and
// line chunks in LDS; each of the four waves owns a 32 x 32 block made of
// 2 x 2 16x16 MFMA tiles.
//
// Precision variants: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4)
// and split BF16 (v_mfma_f32_16x16x32_bf16): X - x0 and Op are split into
// bf16 hi + lo parts; hi*hi accumulates in one FP32 register set and
// hi*lo + lo*hi in another; the two are added in FP64 together with the
// exact offset term x0 * rowsum(Op).
#include "gemm.h"

namespace fcs {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kTM = 64;  // outputs t per tile
constexpr int kTL = 64;  // lines per tile

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// Address of element (line, s) of a task.
__device__ __forceinline__ int64_t elem(const GemmTask& T, int line, int s) {
  int c = line / T.nrow;
  int r = line - c * T.nrow;
  return c * T.comp_stride + static_cast<int64_t>(r) * T.row_stride + static_cast<int64_t>(s) * T.s_stride;
}

// Output rows held by a lane: the FP32/BF16 16x16 MFMAs give lane l rows
// 4 (l / 16) + r, the FP64 16x16x4 MFMA rows l / 16 + 4 r (r = 0..3);
// columns are l % 16 in both.
template <bool kF64Layout, typename Acc>
__device__ __forceinline__ void store_tile(const GemmTask& T, int nlines, int t0, int line0, int wt, int wl,
                                           int lane, const Acc (&acc)[2][2], const double* x0s,
                                           const double* rowsum) {
  for (int ti = 0; ti < 2; ++ti)
    for (int li = 0; li < 2; ++li) {
      int line = line0 + wl + 16 * li + (lane & 15);
      if (line >= nlines) continue;
      int64_t base = elem(T, line, 0);
      for (int r = 0; r < 4; ++r) {
        int t = t0 + wt + 16 * ti + (kF64Layout ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        if (t >= T.n) continue;
        double v = static_cast<double>(acc[ti][li][r]);
        if (rowsum) v += x0s[wl + 16 * li + (lane & 15)] * rowsum[t];
        T.dst[base + static_cast<int64_t>(t) * T.s_stride] = v;
      }
    }
}

template <int KC>
__global__ __launch_bounds__(256) void k_gemm_f64(const GemmTask* __restrict__ tasks,
                                                  const GemmTile* __restrict__ tiles, OpTables ops) {
  __shared__ double Xs[kTL][KC + 1];
  __shared__ double Ds[kTM][KC + 1];
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp;
  const double* __restrict__ D = ops.f64 + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wt = (wave >> 1) * 32, wl = (wave & 1) * 32;
  f64x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += KC) {
    if (T.s_stride == 1) {
      for (int e = tid; e < kTL * KC; e += 256) {
        int l = e / KC, kk = e % KC, line = tile.line0 + l, s = k0 + kk;
        Xs[l][kk] = (line < nlines && s < n) ? T.src[elem(T, line, s)] : 0.0;
      }
    } else {
      for (int e = tid; e < kTL * KC; e += 256) {
        int l = e % kTL, kk = e / kTL, line = tile.line0 + l, s = k0 + kk;
        Xs[l][kk] = (line < nlines && s < n) ? T.src[elem(T, line, s)] : 0.0;
      }
    }
    for (int e = tid; e < kTM * KC; e += 256) {
      int t = e / KC, kk = e % KC, tt = tile.t0 + t, s = k0 + kk;
      Ds[t][kk] = (tt < n && s < n) ? D[static_cast<int64_t>(tt) * n + s] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = ks + (lane >> 4), rr = lane & 15;
      double a0 = Ds[wt + rr][kr], a1 = Ds[wt + 16 + rr][kr];
      double b0 = Xs[wl + rr][kr], b1 = Xs[wl + 16 + rr][kr];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  store_tile<true>(T, nlines, tile.t0, tile.line0, wt, wl, lane, acc, nullptr, nullptr);
}

template <int KC>
__global__ __launch_bounds__(256) void k_gemm_f32(const GemmTask* __restrict__ tasks,
                                                  const GemmTile* __restrict__ tiles, OpTables ops) {
  __shared__ float Xs[kTL][KC + 1];
  __shared__ float Ds[kTM][KC + 1];
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp;
  const float* __restrict__ D = ops.f32 + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wt = (wave >> 1) * 32, wl = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += KC) {
    if (T.s_stride == 1) {
      for (int e = tid; e < kTL * KC; e += 256) {
        int l = e / KC, kk = e % KC, line = tile.line0 + l, s = k0 + kk;
        Xs[l][kk] = (line < nlines && s < n) ? static_cast<float>(T.src[elem(T, line, s)]) : 0.0f;
      }
    } else {
      for (int e = tid; e < kTL * KC; e += 256) {
        int l = e % kTL, kk = e / kTL, line = tile.line0 + l, s = k0 + kk;
        Xs[l][kk] = (line < nlines && s < n) ? static_cast<float>(T.src[elem(T, line, s)]) : 0.0f;
      }
    }
    for (int e = tid; e < kTM * KC; e += 256) {
      int t = e / KC, kk = e % KC, tt = tile.t0 + t, s = k0 + kk;
      Ds[t][kk] = (tt < n && s < n) ? D[static_cast<int64_t>(tt) * n + s] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = ks + (lane >> 4), rr = lane & 15;
      float a0 = Ds[wt + rr][kr], a1 = Ds[wt + 16 + rr][kr];
      float b0 = Xs[wl + rr][kr], b1 = Xs[wl + 16 + rr][kr];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  store_tile<false>(T, nlines, tile.t0, tile.line0, wt, wl, lane, acc, nullptr, nullptr);
}

// Split-BF16: K chunk of 32 (one MFMA depth); rows padded to 40 halves so
// each lane's 8-element operand is one aligned 16-byte LDS read.
__global__ __launch_bounds__(256) void k_gemm_bf16x3(const GemmTask* __restrict__ tasks,
                                                     const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr int KC = 32, PITCH = 40;
  __shared__ __attribute__((aligned(16))) uint16_t Xh[kTL][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Xl[kTL][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Dh[kTM][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Dl[kTM][PITCH];
  __shared__ double x0s[kTL];
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp;
  const uint16_t* __restrict__ Bh = ops.bhi + ops.off[T.op];
  const uint16_t* __restrict__ Bl = ops.blo + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wt = (wave >> 1) * 32, wl = (wave & 1) * 32;
  if (tid < kTL) {
    int line = tile.line0 + tid;
    x0s[tid] = line < nlines ? T.src[elem(T, line, 0)] : 0.0;
  }
  __syncthreads();
  f32x4 am[2][2], ac[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) am[a][b] = ac[a][b] = f32x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += KC) {
    for (int e = tid; e < kTL * KC; e += 256) {
      int l, kk;
      if (T.s_stride == 1) {
        l = e / KC;
        kk = e % KC;
      } else {
        l = e % kTL;
        kk = e / kTL;
      }
      int line = tile.line0 + l, s = k0 + kk;
      float f = (line < nlines && s < n) ? static_cast<float>(T.src[elem(T, line, s)] - x0s[l]) : 0.0f;
      uint16_t h = f2bf(f);
      Xh[l][kk] = h;
      Xl[l][kk] = f2bf(f - bf2f(h));
    }
    for (int e = tid; e < kTM * KC; e += 256) {
      int t = e / KC, kk = e % KC, tt = tile.t0 + t, s = k0 + kk;
      bool in = tt < n && s < n;
      Dh[t][kk] = in ? Bh[static_cast<int64_t>(tt) * n + s] : 0;
      Dl[t][kk] = in ? Bl[static_cast<int64_t>(tt) * n + s] : 0;
    }
    __syncthreads();
    const int rr = lane & 15, kb = 8 * (lane >> 4);
    bf16x8 ah0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dh[wt + rr][kb]));
    bf16x8 ah1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dh[wt + 16 + rr][kb]));
    bf16x8 al0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dl[wt + rr][kb]));
    bf16x8 al1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dl[wt + 16 + rr][kb]));
    bf16x8 bh0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xh[wl + rr][kb]));
    bf16x8 bh1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xh[wl + 16 + rr][kb]));
    bf16x8 bl0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xl[wl + rr][kb]));
    bf16x8 bl1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xl[wl + 16 + rr][kb]));
    am[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bh0, am[0][0], 0, 0, 0);
    am[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bh1, am[0][1], 0, 0, 0);
    am[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bh0, am[1][0], 0, 0, 0);
    am[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bh1, am[1][1], 0, 0, 0);
    ac[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bl0, ac[0][0], 0, 0, 0);
    ac[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bl1, ac[0][1], 0, 0, 0);
    ac[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bl0, ac[1][0], 0, 0, 0);
    ac[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bl1, ac[1][1], 0, 0, 0);
    ac[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al0, bh0, ac[0][0], 0, 0, 0);
    ac[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al0, bh1, ac[0][1], 0, 0, 0);
    ac[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al1, bh0, ac[1][0], 0, 0, 0);
    ac[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al1, bh1, ac[1][1], 0, 0, 0);
    __syncthreads();
  }
  const double* rowsum = ops.rowsum + ops.roff[T.op];
  for (int ti = 0; ti < 2; ++ti)
    for (int li = 0; li < 2; ++li) {
      int lloc = wl + 16 * li + (lane & 15), line = tile.line0 + lloc;
      if (line >= nlines) continue;
      int64_t base = elem(T, line, 0);
      for (int r = 0; r < 4; ++r) {
        int t = tile.t0 + wt + 16 * ti + 4 * (lane >> 4) + r;
        if (t >= n) continue;
        double v = static_cast<double>(am[ti][li][r]) + static_cast<double>(ac[ti][li][r]) + x0s[lloc] * rowsum[t];
        T.dst[base + static_cast<int64_t>(t) * T.s_stride] = v;
      }
    }
}

}  // namespace

hipError_t launch_gemm(int precision, const GemmTask* tasks, const GemmTile* tiles, int ntiles,
                       const OpTables& ops, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(256);
  if (precision == 0) {
    hipLaunchKernelGGL(k_gemm_f64<16>, grid, block, 0, stream, tasks, tiles, ops);
  } else if (precision == 1) {
    hipLaunchKernelGGL(k_gemm_f32<16>, grid, block, 0, stream, tasks, tiles, ops);
  } else {
    hipLaunchKernelGGL(k_gemm_bf16x3, grid, block, 0, stream, tasks, tiles, ops);
  }
  return hipGetLastError();
}

}  // namespace fcs
