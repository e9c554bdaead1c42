// Grouped FC derivative contraction on gfx950 matrix cores.
//
// The FC derivative along a grid line of n points is a fixed linear map
// (continuation, spectral multiplier, restriction: Sec. 2 and the stage
// algorithm of Sec. 5), so all lines of all subpatches that share a length
// form one product  Y[line][t] = sum_s Op[t][s] X[line][s].  One launch covers
// every (subpatch, direction, operand set) through a tile list.  A 256-thread
// workgroup owns 64 lines and up to 256 outputs t: each operand chunk is
// loaded once into LDS and reused for all outputs; wave w computes the
// 16-output blocks w, w + 4, ... for all 64 lines (4 x 4 MFMA tiles).
//
// The operand roles are chosen per direction so that the results leave the
// matrix cores as 16 consecutive values per row of lanes: along q^1 (output
// contiguous in t) the lines are the MFMA rows, along q^2 (lines contiguous
// in memory) the outputs are.
//
// Precisions: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4) and split
// BF16 (v_mfma_f32_16x16x32_bf16): X - x0 and Op are split into bf16 hi + lo;
// hi*hi accumulates in one FP32 register set, hi*lo + lo*hi in another, and
// the two are added in FP64 with the exact offset term x0 * rowsum(Op).
//
// Flux tasks compute their operand in the loader: component c of
// a f_x + b f_y from the conserved state (affine subpatches; Sec. 2 fluxes).
#include <algorithm>

#include "gemm.h"

namespace fcs {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kLB = 64;   // lines per workgroup

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// Per-workgroup line tables: source base, destination base, component.
struct LineTab {
  int64_t src[kLB];
  int64_t dst[kLB];
  int32_t comp[kLB];
};

__device__ __forceinline__ void build_lines(const GemmTask& T, int line0, int nlines, LineTab& L) {
  const int l = threadIdx.x;
  if (l < kLB) {
    int line = line0 + l;
    if (line < nlines) {
      int r = line / T.ncomp, c = line - r * T.ncomp;
      int64_t rb = static_cast<int64_t>(r) * T.row_stride;
      L.src[l] = T.flux ? rb : rb + c * T.comp_stride;
      L.dst[l] = rb + c * T.comp_stride;
      L.comp[l] = c;
    } else {
      L.src[l] = -1;
      L.dst[l] = -1;
      L.comp[l] = 0;
    }
  }
}

// Operand value (line l of the tile, position s) in FP64.
__device__ __forceinline__ double operand(const GemmTask& T, const LineTab& L, int l, int s) {
  const int64_t b = L.src[l] + static_cast<int64_t>(s) * T.s_stride;
  if (!T.flux) return T.src[b];
  const double* U = T.src;
  const int64_t P = T.comp_stride;
  double r = U[b], mx = U[b + P], my = U[b + 2 * P], E = U[b + 3 * P];
  double p = T.gm1 * (E - 0.5 * (mx * mx + my * my) / r);
  double u = mx / r, w = my / r, fx, fy;
  switch (L.comp[l]) {
    case 0: fx = mx; fy = my; break;
    case 1: fx = mx * u + p; fy = my * u; break;
    case 2: fx = mx * w; fy = my * w + p; break;
    default: fx = u * (E + p); fy = w * (E + p); break;
  }
  return T.fa * fx + T.fb * fy;
}

// Element (q, kk) of an operand chunk handled by a thread: along q^1 the
// chunk is read line by line (k contiguous), along q^2 position by position
// (lines contiguous).
template <int KC>
__device__ __forceinline__ void chunk_index(bool q1, int e, int& l, int& kk) {
  if (q1) {
    l = e / KC;
    kk = e % KC;
  } else {
    l = e % kLB;
    kk = e / kLB;
  }
}

template <bool kF64, int TB, typename Acc, typename Acc2>
__device__ __forceinline__ void store_acc(const GemmTask& T, const LineTab& L, int t0, int nt, bool swapped,
                                          int wave, int lane, Acc (&acc)[TB][4], Acc2 (*acc2)[4],
                                          const double* x0s, const double* rowsum) {
#pragma unroll
  for (int i = 0; i < TB; ++i) {
    const int tb = wave + 4 * i;
    if (16 * tb >= nt) continue;
#pragma unroll
    for (int lb = 0; lb < 4; ++lb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kF64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int col = lane & 15;
        int lloc, tloc;
        if (swapped) {
          lloc = 16 * lb + row;
          tloc = 16 * tb + col;
        } else {
          tloc = 16 * tb + row;
          lloc = 16 * lb + col;
        }
        if (tloc >= nt || L.dst[lloc] < 0) continue;
        double v = static_cast<double>(acc[i][lb][r]);
        if (acc2) v += static_cast<double>(acc2[i][lb][r]);
        if (rowsum) v += x0s[lloc] * rowsum[t0 + tloc];
        T.dst[L.dst[lloc] + static_cast<int64_t>(t0 + tloc) * T.s_stride] = v;
      }
    }
  }
}

// Register staging of one operand chunk: the global loads of chunk k + 1 are
// issued before the matrix-core loop of chunk k and written to LDS after it.
template <int KC>
struct XStage {  // NOLINT
  static constexpr int N = kLB * KC / 256;
  double raw[N][4];
  __device__ __forceinline__ void load(const GemmTask& T, const LineTab& L, bool q1, int k0, int n) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      int l, kk;
      chunk_index<KC>(q1, threadIdx.x + 256 * p, l, kk);
      const int s = k0 + kk;
      raw[p][0] = raw[p][1] = raw[p][2] = raw[p][3] = 0.0;
      if (L.src[l] < 0 || s >= n) continue;
      const int64_t b = L.src[l] + static_cast<int64_t>(s) * T.s_stride;
      raw[p][0] = T.src[b];
      if (T.flux) {
        raw[p][1] = T.src[b + T.comp_stride];
        raw[p][2] = T.src[b + 2 * T.comp_stride];
        raw[p][3] = T.src[b + 3 * T.comp_stride];
      }
    }
  }
  // operand value of staged element p (0 outside the task)
  __device__ __forceinline__ double value(const GemmTask& T, const LineTab& L, bool q1, int p, int k0, int n) const {
    int l, kk;
    chunk_index<KC>(q1, threadIdx.x + 256 * p, l, kk);
    if (L.src[l] < 0 || k0 + kk >= n) return 0.0;
    if (!T.flux) return raw[p][0];
    const double r = raw[p][0], mx = raw[p][1], my = raw[p][2], E = raw[p][3];
    const double pr = T.gm1 * (E - 0.5 * (mx * mx + my * my) / r);
    const double u = mx / r, w = my / r;
    double fx, fy;
    switch (L.comp[l]) {
      case 0: fx = mx; fy = my; break;
      case 1: fx = mx * u + pr; fy = my * u; break;
      case 2: fx = mx * w; fy = my * w + pr; break;
      default: fx = u * (E + pr); fy = w * (E + pr); break;
    }
    return T.fa * fx + T.fb * fy;
  }
  __device__ __forceinline__ int line(bool q1, int p) const {
    int l, kk;
    chunk_index<KC>(q1, threadIdx.x + 256 * p, l, kk);
    return l;
  }
  __device__ __forceinline__ int col(bool q1, int p) const {
    int l, kk;
    chunk_index<KC>(q1, threadIdx.x + 256 * p, l, kk);
    return kk;
  }
};

template <typename E, int KC, int TT>
struct DStage {
  static constexpr int N = TT * KC / 256;
  E v[N];
  __device__ __forceinline__ void load(const E* __restrict__ D, int t0, int nt, int k0, int n) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      const int e = threadIdx.x + 256 * p, t = e / KC, s = k0 + e % KC;
      v[p] = (t < nt && s < n) ? D[static_cast<int64_t>(t0 + t) * n + s] : E(0);
    }
  }
};

// FP64 or FP32 operands on the 16x16x4 MFMA of that type.  TB: 16-output
// blocks per wave (the workgroup covers 64 TB outputs); PF: register
// prefetch of the next chunk.
template <typename Elem, int KC, int TB, bool PF>
__global__ __launch_bounds__(256) void k_gemm_fp(const GemmTask* __restrict__ tasks,
                                                 const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr bool kF64 = sizeof(Elem) == 8;
  constexpr int kTT = 64 * TB;
  typedef Elem vec4 __attribute__((ext_vector_type(4)));
  __shared__ Elem Xs[kLB][KC + 1];
  __shared__ Elem Ds[kTT][KC + 1];
  __shared__ LineTab L;
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const Elem* __restrict__ D;
  if constexpr (kF64)
    D = ops.f64 + ops.off[T.op];
  else
    D = ops.f32 + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool q1 = T.s_stride == 1;
  build_lines(T, tile.line0, nlines, L);
  vec4 acc[TB][4];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[i][b] = vec4{0, 0, 0, 0};
  __syncthreads();
  XStage<KC> xs;
  DStage<Elem, KC, kTT> ds;
  xs.load(T, L, q1, 0, n);
  ds.load(D, t0, nt, 0, n);
  for (int k0 = 0; k0 < n; k0 += KC) {
    if (!PF && k0 > 0) {
      xs.load(T, L, q1, k0, n);
      ds.load(D, t0, nt, k0, n);
    }
#pragma unroll
    for (int p = 0; p < XStage<KC>::N; ++p) Xs[xs.line(q1, p)][xs.col(q1, p)] = static_cast<Elem>(xs.value(T, L, q1, p, k0, n));
#pragma unroll
    for (int p = 0; p < DStage<Elem, KC, kTT>::N; ++p) {
      const int e = tid + 256 * p;
      Ds[e / KC][e % KC] = ds.v[p];
    }
    __syncthreads();
    if (PF && k0 + KC < n) {
      xs.load(T, L, q1, k0 + KC, n);
      ds.load(D, t0, nt, k0 + KC, n);
    }
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = ks + (lane >> 4), rr = lane & 15;
      Elem xb[4];
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) xb[lb] = Xs[16 * lb + rr][kr];
#pragma unroll
      for (int i = 0; i < TB; ++i) {
        const int tb = wave + 4 * i;
        if (16 * tb >= nt) continue;
        const Elem da = Ds[16 * tb + rr][kr];
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
          if constexpr (kF64)
            acc[i][lb] = q1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(xb[lb], da, acc[i][lb], 0, 0, 0)
                            : __builtin_amdgcn_mfma_f64_16x16x4f64(da, xb[lb], acc[i][lb], 0, 0, 0);
          else
            acc[i][lb] = q1 ? __builtin_amdgcn_mfma_f32_16x16x4f32(xb[lb], da, acc[i][lb], 0, 0, 0)
                            : __builtin_amdgcn_mfma_f32_16x16x4f32(da, xb[lb], acc[i][lb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  store_acc<kF64, TB>(T, L, t0, nt, q1, wave, lane, acc, static_cast<vec4(*)[4]>(nullptr), nullptr, nullptr);
}

// Split BF16: chunk of 32 (one MFMA depth); rows padded to 40 halves so each
// lane's 8-element operand is one aligned 16-byte LDS read.
template <int TB, bool PF>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(const GemmTask* __restrict__ tasks,
                                                     const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr int KC = 32, PITCH = 40, kTT = 64 * TB;
  __shared__ __attribute__((aligned(16))) uint16_t Xh[kLB][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Xl[kLB][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Dh[kTT][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Dl[kTT][PITCH];
  __shared__ double x0s[kLB];
  __shared__ LineTab L;
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const uint16_t* __restrict__ Bh = ops.bhi + ops.off[T.op];
  const uint16_t* __restrict__ Bl = ops.blo + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool q1 = T.s_stride == 1;
  build_lines(T, tile.line0, nlines, L);
  __syncthreads();
  if (tid < kLB) x0s[tid] = L.src[tid] >= 0 ? operand(T, L, tid, 0) : 0.0;
  f32x4 am[TB][4], ac[TB][4];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) am[i][b] = ac[i][b] = f32x4{0, 0, 0, 0};
  __syncthreads();
  XStage<KC> xs;
  DStage<uint16_t, KC, kTT> dh, dl;
  xs.load(T, L, q1, 0, n);
  dh.load(Bh, t0, nt, 0, n);
  dl.load(Bl, t0, nt, 0, n);
  for (int k0 = 0; k0 < n; k0 += KC) {
    if (!PF && k0 > 0) {
      xs.load(T, L, q1, k0, n);
      dh.load(Bh, t0, nt, k0, n);
      dl.load(Bl, t0, nt, k0, n);
    }
#pragma unroll
    for (int p = 0; p < XStage<KC>::N; ++p) {
      const int l = xs.line(q1, p), kk = xs.col(q1, p);
      const bool in = L.src[l] >= 0 && k0 + kk < n;
      const float f = in ? static_cast<float>(xs.value(T, L, q1, p, k0, n) - x0s[l]) : 0.0f;
      const uint16_t h = f2bf(f);
      Xh[l][kk] = h;
      Xl[l][kk] = f2bf(f - bf2f(h));
    }
#pragma unroll
    for (int p = 0; p < DStage<uint16_t, KC, kTT>::N; ++p) {
      const int e = tid + 256 * p;
      Dh[e / KC][e % KC] = dh.v[p];
      Dl[e / KC][e % KC] = dl.v[p];
    }
    __syncthreads();
    if (PF && k0 + KC < n) {
      xs.load(T, L, q1, k0 + KC, n);
      dh.load(Bh, t0, nt, k0 + KC, n);
      dl.load(Bl, t0, nt, k0 + KC, n);
    }
    const int rr = lane & 15, kb = 8 * (lane >> 4);
    bf16x8 xh[4], xl[4];
#pragma unroll
    for (int lb = 0; lb < 4; ++lb) {
      xh[lb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xh[16 * lb + rr][kb]));
      xl[lb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xl[16 * lb + rr][kb]));
    }
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      const int tb = wave + 4 * i;
      if (16 * tb >= nt) continue;
      const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dh[16 * tb + rr][kb]));
      const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dl[16 * tb + rr][kb]));
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        if (q1) {
          am[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[lb], bh, am[i][lb], 0, 0, 0);
          ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[lb], bl, ac[i][lb], 0, 0, 0);
          ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[lb], bh, ac[i][lb], 0, 0, 0);
        } else {
          am[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, xh[lb], am[i][lb], 0, 0, 0);
          ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, xl[lb], ac[i][lb], 0, 0, 0);
          ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, xh[lb], ac[i][lb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // the two FP32 accumulations are added in FP64 at the store
  store_acc<false, TB>(T, L, t0, nt, q1, wave, lane, am, ac, x0s, ops.rowsum + ops.roff[T.op]);
}

}  // namespace

// ---------------------------------------------------------------------------
// Lines in registers.  Wave w owns the lines line0 + 16 w .. + 15; lane l
// holds line 16 w + (l & 15) and, in each chunk, the KL consecutive
// positions k0 + KL (l >> 4) + j (KL = 4 for the 16x16x4 MFMAs, 8 for the
// 16x16x32 BF16 MFMA).  Both operands use this permuted order of the chunk,
// so a lane reads contiguous elements of its own line straight from global
// memory; only the operator chunk, shared by the four waves, goes through
// LDS.  Output roles as in the staged kernels.
__device__ __forceinline__ void line_setup(const GemmTask& T, int line, int nlines, int64_t& sbase, int& comp) {
  sbase = -1;
  comp = 0;
  if (line < nlines) {
    int r = line / T.ncomp, c = line - r * T.ncomp;
    int64_t rb = static_cast<int64_t>(r) * T.row_stride;
    sbase = T.flux ? rb : rb + c * T.comp_stride;
    comp = c;
  }
}

template <int KL>
struct LineRegs {
  double raw[KL][4];
  __device__ __forceinline__ void load(const GemmTask& T, int64_t sbase, int kbeg, int n) {
#pragma unroll
    for (int j = 0; j < KL; ++j) {
      const int s = kbeg + j;
      raw[j][0] = raw[j][1] = raw[j][2] = raw[j][3] = 0.0;
      if (sbase < 0 || s >= n) continue;
      const int64_t b = sbase + static_cast<int64_t>(s) * T.s_stride;
      raw[j][0] = T.src[b];
      if (T.flux) {
        raw[j][1] = T.src[b + T.comp_stride];
        raw[j][2] = T.src[b + 2 * T.comp_stride];
        raw[j][3] = T.src[b + 3 * T.comp_stride];
      }
    }
  }
  __device__ __forceinline__ double value(const GemmTask& T, int comp, int j, bool in) const {
    if (!in) return 0.0;
    if (!T.flux) return raw[j][0];
    const double r = raw[j][0], mx = raw[j][1], my = raw[j][2], E = raw[j][3];
    const double pr = T.gm1 * (E - 0.5 * (mx * mx + my * my) / r);
    const double u = mx / r, w = my / r;
    double fx, fy;
    switch (comp) {
      case 0: fx = mx; fy = my; break;
      case 1: fx = mx * u + pr; fy = my * u; break;
      case 2: fx = mx * w; fy = my * w + pr; break;
      default: fx = u * (E + pr); fy = w * (E + pr); break;
    }
    return T.fa * fx + T.fb * fy;
  }
};

template <bool kF64, int NB, typename Acc, typename Acc2>
__device__ __forceinline__ void store_reg(const GemmTask& T, const LineTab& L, int t0, int nt, bool swapped,
                                          int wave, int lane, Acc (&acc)[NB], Acc2* acc2, const double* x0s,
                                          const double* rowsum) {
  const int rr = lane & 15, g = lane >> 4;
#pragma unroll
  for (int tb = 0; tb < NB; ++tb) {
    if (16 * tb >= nt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = kF64 ? g + 4 * r : 4 * g + r;
      int lloc, tloc;
      if (swapped) {
        lloc = 16 * wave + row;
        tloc = 16 * tb + rr;
      } else {
        tloc = 16 * tb + row;
        lloc = 16 * wave + rr;
      }
      if (tloc >= nt || L.dst[lloc] < 0) continue;
      double v = static_cast<double>(acc[tb][r]);
      if (acc2) v += static_cast<double>(acc2[tb][r]);
      if (rowsum) v += x0s[lloc] * rowsum[t0 + tloc];
      T.dst[L.dst[lloc] + static_cast<int64_t>(t0 + tloc) * T.s_stride] = v;
    }
  }
}

template <typename Elem, int NB>
__global__ __launch_bounds__(256) void k_gemm_reg(const GemmTask* __restrict__ tasks,
                                                  const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr bool kF64 = sizeof(Elem) == 8;
  constexpr int KC = 16, KL = 4, TT = 16 * NB, ND = TT * KC / 256;
  typedef Elem vec4 __attribute__((ext_vector_type(4)));
  __shared__ Elem Ds[TT][KC + 1];
  __shared__ LineTab L;
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(TT, n - t0);
  const Elem* __restrict__ D;
  if constexpr (kF64)
    D = ops.f64 + ops.off[T.op];
  else
    D = ops.f32 + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, rr = lane & 15, g = lane >> 4;
  const bool q1 = T.s_stride == 1;
  build_lines(T, tile.line0, nlines, L);
  int64_t sbase;
  int comp;
  line_setup(T, tile.line0 + 16 * wave + rr, nlines, sbase, comp);
  vec4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = vec4{0, 0, 0, 0};
  LineRegs<KL> xr;
  Elem dreg[ND];
  xr.load(T, sbase, KL * g, n);
#pragma unroll
  for (int p = 0; p < ND; ++p) {
    const int e = tid + 256 * p, t = e / KC, s = e % KC;
    dreg[p] = (t < nt && s < n) ? D[static_cast<int64_t>(t0 + t) * n + s] : Elem(0);
  }
  for (int k0 = 0; k0 < n; k0 += KC) {
    Elem xv[KL];
#pragma unroll
    for (int j = 0; j < KL; ++j) xv[j] = static_cast<Elem>(xr.value(T, comp, j, sbase >= 0 && k0 + KL * g + j < n));
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      const int e = tid + 256 * p;
      Ds[e / KC][e % KC] = dreg[p];
    }
    __syncthreads();
    if (k0 + KC < n) {
      xr.load(T, sbase, k0 + KC + KL * g, n);
#pragma unroll
      for (int p = 0; p < ND; ++p) {
        const int e = tid + 256 * p, t = e / KC, s = k0 + KC + e % KC;
        dreg[p] = (t < nt && s < n) ? D[static_cast<int64_t>(t0 + t) * n + s] : Elem(0);
      }
    }
#pragma unroll
    for (int j = 0; j < KL; ++j) {
#pragma unroll
      for (int tb = 0; tb < NB; ++tb) {
        if (16 * tb >= nt) continue;
        const Elem da = Ds[16 * tb + rr][KL * g + j];
        if constexpr (kF64)
          acc[tb] = q1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(xv[j], da, acc[tb], 0, 0, 0)
                       : __builtin_amdgcn_mfma_f64_16x16x4f64(da, xv[j], acc[tb], 0, 0, 0);
        else
          acc[tb] = q1 ? __builtin_amdgcn_mfma_f32_16x16x4f32(xv[j], da, acc[tb], 0, 0, 0)
                       : __builtin_amdgcn_mfma_f32_16x16x4f32(da, xv[j], acc[tb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  store_reg<kF64, NB>(T, L, t0, nt, q1, wave, lane, acc, static_cast<vec4*>(nullptr), nullptr, nullptr);
}

template <int NB>
__global__ __launch_bounds__(256) void k_gemm_reg_bf16x3(const GemmTask* __restrict__ tasks,
                                                         const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr int KC = 32, KL = 8, PITCH = 40, TT = 16 * NB, ND = TT * KC / 256;
  __shared__ __attribute__((aligned(16))) uint16_t Dh[TT][PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Dl[TT][PITCH];
  __shared__ LineTab L;
  __shared__ double x0s[kLB];
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(TT, n - t0);
  const uint16_t* __restrict__ Bh = ops.bhi + ops.off[T.op];
  const uint16_t* __restrict__ Bl = ops.blo + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, rr = lane & 15, g = lane >> 4;
  const bool q1 = T.s_stride == 1;
  build_lines(T, tile.line0, nlines, L);
  int64_t sbase;
  int comp;
  const int lloc = 16 * wave + rr;
  line_setup(T, tile.line0 + lloc, nlines, sbase, comp);
  double x0 = 0.0;
  {
    LineRegs<1> first;
    first.load(T, sbase, 0, n);
    x0 = first.value(T, comp, 0, sbase >= 0);
  }
  if (g == 0) x0s[lloc] = x0;
  f32x4 am[NB], ac[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) am[b] = ac[b] = f32x4{0, 0, 0, 0};
  LineRegs<KL> xr;
  uint16_t dh[ND], dl[ND];
  xr.load(T, sbase, KL * g, n);
#pragma unroll
  for (int p = 0; p < ND; ++p) {
    const int e = tid + 256 * p, t = e / KC, s = e % KC;
    const bool in = t < nt && s < n;
    dh[p] = in ? Bh[static_cast<int64_t>(t0 + t) * n + s] : 0;
    dl[p] = in ? Bl[static_cast<int64_t>(t0 + t) * n + s] : 0;
  }
  for (int k0 = 0; k0 < n; k0 += KC) {
    uint16_t xh[KL], xl[KL];
#pragma unroll
    for (int j = 0; j < KL; ++j) {
      const bool in = sbase >= 0 && k0 + KL * g + j < n;
      const float f = in ? static_cast<float>(xr.value(T, comp, j, true) - x0) : 0.0f;
      xh[j] = f2bf(f);
      xl[j] = f2bf(f - bf2f(xh[j]));
    }
    bf16x8 ah, al;
#pragma unroll
    for (int j = 0; j < KL; ++j) {
      ah[j] = __builtin_bit_cast(__bf16, xh[j]);
      al[j] = __builtin_bit_cast(__bf16, xl[j]);
    }
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      const int e = tid + 256 * p;
      Dh[e / KC][e % KC] = dh[p];
      Dl[e / KC][e % KC] = dl[p];
    }
    __syncthreads();
    if (k0 + KC < n) {
      xr.load(T, sbase, k0 + KC + KL * g, n);
#pragma unroll
      for (int p = 0; p < ND; ++p) {
        const int e = tid + 256 * p, t = e / KC, s = k0 + KC + e % KC;
        const bool in = t < nt && s < n;
        dh[p] = in ? Bh[static_cast<int64_t>(t0 + t) * n + s] : 0;
        dl[p] = in ? Bl[static_cast<int64_t>(t0 + t) * n + s] : 0;
      }
    }
#pragma unroll
    for (int tb = 0; tb < NB; ++tb) {
      if (16 * tb >= nt) continue;
      const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dh[16 * tb + rr][KL * g]));
      const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dl[16 * tb + rr][KL * g]));
      if (q1) {
        am[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, am[tb], 0, 0, 0);
        ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, ac[tb], 0, 0, 0);
        ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, ac[tb], 0, 0, 0);
      } else {
        am[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, ah, am[tb], 0, 0, 0);
        ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, al, ac[tb], 0, 0, 0);
        ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, ah, ac[tb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  store_reg<false, NB>(T, L, t0, nt, q1, wave, lane, am, ac, x0s, ops.rowsum + ops.roff[T.op]);
}

template <typename Elem, int KC>
void launch_fp(const GemmVariant& v, dim3 g, dim3 b, hipStream_t st, const GemmTask* tasks, const GemmTile* tiles,
               const OpTables& ops) {
  if (v.tb == 1) {
    if (v.prefetch) hipLaunchKernelGGL((k_gemm_fp<Elem, KC, 1, true>), g, b, 0, st, tasks, tiles, ops);
    else hipLaunchKernelGGL((k_gemm_fp<Elem, KC, 1, false>), g, b, 0, st, tasks, tiles, ops);
  } else if (v.tb == 2) {
    if (v.prefetch) hipLaunchKernelGGL((k_gemm_fp<Elem, KC, 2, true>), g, b, 0, st, tasks, tiles, ops);
    else hipLaunchKernelGGL((k_gemm_fp<Elem, KC, 2, false>), g, b, 0, st, tasks, tiles, ops);
  } else {
    if (v.prefetch) hipLaunchKernelGGL((k_gemm_fp<Elem, KC, 4, true>), g, b, 0, st, tasks, tiles, ops);
    else hipLaunchKernelGGL((k_gemm_fp<Elem, KC, 4, false>), g, b, 0, st, tasks, tiles, ops);
  }
}

hipError_t launch_gemm(int precision, const GemmVariant& v, const GemmTask* tasks, const GemmTile* tiles,
                       int ntiles, const OpTables& ops, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  if (v.kind == 2) return launch_gemm_os(precision, v, tasks, tiles, ntiles, ops, stream);
  dim3 grid(ntiles), block(256);
  if (v.kind == 1) {
#define FCS_REG(E, NB) hipLaunchKernelGGL((k_gemm_reg<E, NB>), grid, block, 0, stream, tasks, tiles, ops)
#define FCS_REGB(NB) hipLaunchKernelGGL((k_gemm_reg_bf16x3<NB>), grid, block, 0, stream, tasks, tiles, ops)
    if (precision == 0) {
      if (v.nb == 4) FCS_REG(double, 4);
      else if (v.nb == 8) FCS_REG(double, 8);
      else FCS_REG(double, 16);
    } else if (precision == 1) {
      if (v.nb == 4) FCS_REG(float, 4);
      else if (v.nb == 8) FCS_REG(float, 8);
      else FCS_REG(float, 16);
    } else {
      if (v.nb == 4) FCS_REGB(4);
      else if (v.nb == 8) FCS_REGB(8);
      else FCS_REGB(16);
    }
#undef FCS_REG
#undef FCS_REGB
    return hipGetLastError();
  }
  if (precision == 0) {
    launch_fp<double, 16>(v, grid, block, stream, tasks, tiles, ops);
  } else if (precision == 1) {
    launch_fp<float, 16>(v, grid, block, stream, tasks, tiles, ops);
  } else if (v.tb == 1) {
    if (v.prefetch) hipLaunchKernelGGL((k_gemm_bf16x3<1, true>), grid, block, 0, stream, tasks, tiles, ops);
    else hipLaunchKernelGGL((k_gemm_bf16x3<1, false>), grid, block, 0, stream, tasks, tiles, ops);
  } else {
    if (v.prefetch) hipLaunchKernelGGL((k_gemm_bf16x3<2, true>), grid, block, 0, stream, tasks, tiles, ops);
    else hipLaunchKernelGGL((k_gemm_bf16x3<2, false>), grid, block, 0, stream, tasks, tiles, ops);
  }
  return hipGetLastError();
}

int gemm_lines_per_tile() { return kLB; }
int gemm_outputs_per_tile(const GemmVariant& v) {
  if (v.kind == 1) return 16 * v.nb;
  return 64 * (v.tb < 1 ? 1 : v.tb);
}

const GemmVariant* gemm_variants(int precision, int* count) {
  // {tb, prefetch, kind, nb, lds_kb, group}
  static const GemmVariant fp[] = {{1, true, 0, 4, 64, 4},  {2, true, 0, 4, 64, 4},  {1, false, 1, 8, 64, 4},
                                   {1, false, 2, 16, 64, 2}, {1, false, 2, 16, 64, 4}, {1, false, 2, 16, 128, 4},
                                   {1, false, 2, 16, 128, 8}, {1, false, 2, 16, 64, 8}};
  static const GemmVariant bf[] = {{1, true, 0, 4, 64, 4},  {2, true, 0, 4, 64, 4},   {1, false, 1, 8, 64, 4},
                                   {1, false, 2, 16, 64, 2}, {1, false, 2, 16, 64, 4}, {1, false, 2, 16, 128, 4},
                                   {1, false, 2, 16, 128, 8}, {1, false, 2, 16, 64, 8}};
  *count = 8;
  return precision == 2 ? bf : fp;
}

void gemm_build_tiles(int precision, GemmVariant& v, const int32_t* n, const int32_t* nlines, size_t ntasks,
                      std::vector<GemmTile>& tiles) {
  tiles.clear();
  if (v.kind != 2) {
    const int step = gemm_outputs_per_tile(v);
    for (size_t q = 0; q < ntasks; ++q)
      for (int t0 = 0; t0 < n[q]; t0 += step)
        for (int l0 = 0; l0 < nlines[q]; l0 += kLB) tiles.push_back({static_cast<int32_t>(q), l0, t0, 0});
    v.dyn_lds = 0;
    return;
  }
  size_t lds = 0;
  int maxtt = 16;
  for (size_t q = 0; q < ntasks; ++q) {
    const int tt = gemm_os_rows(precision, v, n[q]);
    maxtt = std::max(maxtt, tt);
    size_t row_bytes;
    if (precision == 2)
      row_bytes = 4 * static_cast<size_t>((n[q] + 31) / 32 * 32 + 8);
    else
      row_bytes = (precision == 0 ? 8 : 4) * static_cast<size_t>((n[q] + 15) / 16 * 16 + 1);
    lds = std::max(lds, tt * row_bytes);
    const int nblk = (nlines[q] + kLB - 1) / kLB;
    for (int t0 = 0; t0 < n[q]; t0 += tt)
      for (int b0 = 0; b0 < nblk; b0 += v.group) {
        const int nb = std::min(v.group, nblk - b0);
        tiles.push_back({static_cast<int32_t>(q), b0 * kLB, t0, nb | (tt << 16)});
      }
  }
  v.nb = maxtt > 128 ? 16 : 8;
  v.dyn_lds = lds;
}

}  // namespace fcs
