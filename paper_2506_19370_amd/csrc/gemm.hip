// Grouped FC derivative contraction on gfx950 matrix cores.
//
// The FC derivative along a grid line of n points is a fixed linear map
// (continuation, spectral multiplier, restriction: Sec. 2 and the stage
// algorithm of Sec. 5), so all lines of all subpatches that share a length
// form one product  Y[line][t] = sum_s Op[t][s] X[line][s].  One launch covers
// every (subpatch, direction, operand set) through a tile list.  A 256-thread
// workgroup owns 64 lines and 64 tb outputs (tb = 1 or 2) and walks the
// operator depth in chunks of kc columns; wave w computes the 16 lines
// 16 w .. 16 w + 15 for all 4 tb 16-output blocks of the tile.  The blocks
// past the line length (the ragged last tile of a line, about a quarter of
// the products at line lengths near 100) are skipped by every wave alike.
//
// Staging is branch-free and double-buffered in LDS: the global loads of
// chunk k + 1 are in flight while the matrix cores work on chunk k, and one
// barrier per chunk separates the buffers.  Operators are zero-padded (rows
// to 256, columns to 32), so operator reads need no bounds tests; operand
// positions past the line end are clamped to the last point (their operator
// column is zero) and lines past the task end are clamped to its last line
// (their results are not stored).
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
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>

#include "fc_builder.h"
#include "gemm.h"

namespace fcs {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kLB = 64;  // lines per workgroup

// Operand and result pointers come from the task table in memory, so the
// compiler cannot tell their address space and would access them with FLAT
// instructions.  Those count in the LDS wait counter too: every wait for an
// LDS read would then also wait for the operand loads of the next chunk.
// All operands and results are device global memory.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ const gdouble* gsrc(const double* p) { return (const gdouble*)p; }
__device__ __forceinline__ gdouble* gdst64(void* p) { return (gdouble*)p; }
__device__ __forceinline__ gfloat* gdst32(void* p) { return (gfloat*)p; }

// Element offset of position 0 of a line (row fastest numbering).
// A tile with nothing to compute: padding of an XCD-ordered list, or a tile
// none of whose lines is needed in this step (the skip flags are uniform
// over the workgroup, so the whole workgroup leaves together).  A set bit w
// alone (lines 16 w .. 16 w + 15 not needed) lets the staged kernels' wave w
// take the path of a wave past the task's end: no products, no stores.
__device__ __forceinline__ bool tile_idle(const GemmTile& t) { return t.task < 0 || (t.skip & 15) == 15; }

__device__ __forceinline__ int64_t line_base(const GemmTask& T, int line) {
  const int c = line / T.nrow, r = line - c * T.nrow;
  return static_cast<int64_t>(c) * T.comp_stride + static_cast<int64_t>(r) * T.row_stride;
}

// Position (line l, column kk) of element e of an operand chunk: along q^1
// the chunk is read line by line (columns contiguous), along q^2 column by
// column (lines contiguous).
template <int KC>
__device__ __forceinline__ void chunk_pos(bool q1, int e, int& l, int& kk) {
  if (q1) {
    l = e / KC;
    kk = e % KC;
  } else {
    l = e % kLB;
    kk = e / kLB;
  }
}

// Operand loader of one thread: NX elements of every chunk, at fixed lines.
template <int KC>
struct XLoad {
  static constexpr int NX = kLB * KC / 256;
  const gdouble* base[NX];
  __device__ __forceinline__ void init(const GemmTask& T, int line0, int nlines, bool q1) {
#pragma unroll
    for (int p = 0; p < NX; ++p) {
      int l, kk;
      chunk_pos<KC>(q1, threadIdx.x + 256 * p, l, kk);
      base[p] = gsrc(T.src) + line_base(T, min(line0 + l, nlines - 1));
    }
  }
  __device__ __forceinline__ void load(double (&v)[NX], bool q1, int k0, int n, int sstride) const {
#pragma unroll
    for (int p = 0; p < NX; ++p) {
      int l, kk;
      chunk_pos<KC>(q1, threadIdx.x + 256 * p, l, kk);
      v[p] = base[p][static_cast<int64_t>(min(k0 + kk, n - 1)) * sstride];
    }
  }
};

// Stores the accumulators of one tile.  FP64 MFMA results sit at row
// (lane / 16) + 4 r, FP32 results at row 4 (lane / 16) + r; column lane % 16.
template <bool kF64, int TB, typename Acc>
__device__ __forceinline__ void store_tile(const GemmTask& T, const int64_t* dst, int nl, int t0, int nt, bool q1,
                                           int wave, int lane, const Acc (&acc)[TB][4], const Acc (*acc2)[4],
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
        const int lloc = q1 ? 16 * lb + row : 16 * lb + col;
        const int tloc = q1 ? 16 * tb + col : 16 * tb + row;
        if (tloc >= nt || lloc >= nl) continue;
        double v = static_cast<double>(acc[i][lb][r]);
        if (acc2) v += static_cast<double>(acc2[i][lb][r]);
        if (rowsum) v += x0s[lloc] * rowsum[t0 + tloc];
        const int64_t o = dst[lloc] + static_cast<int64_t>(t0 + tloc) * T.s_stride;
        if (T.out_f32)
          gdst32(T.dst)[o] = static_cast<float>(v);
        else
          gdst64(T.dst)[o] = v;
      }
    }
  }
}

// Stores the accumulators of a wave that owns the 16 lines 16 wave ..
// 16 wave + 15 and the NB output blocks of the tile (same register layout).
template <bool kF64, int NB, typename Acc>
__device__ __forceinline__ void store_lines(const GemmTask& T, const int64_t* dst, int nl, int t0, int nt, bool q1,
                                            int wave, int lane, const Acc (&acc)[NB]) {
#pragma unroll
  for (int ob = 0; ob < NB; ++ob) {
    if (16 * ob >= nt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = kF64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
      const int col = lane & 15;
      const int lloc = 16 * wave + (q1 ? row : col);
      const int tloc = 16 * ob + (q1 ? col : row);
      if (tloc >= nt || lloc >= nl) continue;
      const int64_t o = dst[lloc] + static_cast<int64_t>(t0 + tloc) * T.s_stride;
      if (T.out_f32)
        gdst32(T.dst)[o] = static_cast<float>(acc[ob][r]);
      else
        gdst64(T.dst)[o] = static_cast<double>(acc[ob][r]);
    }
  }
}

// Calls f(std::integral_constant<int, min(nb, K)>) for 0 <= nb.
template <int K, typename F>
__device__ __forceinline__ void with_live(int nb, F&& f) {
  if constexpr (K == 0) {
    f(std::integral_constant<int, 0>{});
  } else {
    if (nb >= K)
      f(std::integral_constant<int, K>{});
    else
      with_live<K - 1>(nb, f);
  }
}

// Calls f(std::integral_constant<int, u>{}) for u = 0 .. N - 1 in order.
template <int N, int U = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (U < N) {
    f(std::integral_constant<int, U>{});
    static_for<N, U + 1>(f);
  }
}

// FP64 or FP32 operands on the 16x16x4 MFMA of that type.
template <typename Elem, int KC, int TB>
struct SmemFp {
  Elem Xs[2][kLB][KC + 1];
  Elem Ds[2][64 * TB][KC + 1];
  int64_t dst[kLB];
};

template <typename Elem, int KC, int TB, bool Q1, int PF>
__device__ __forceinline__ void gemm_fp_dir(const GemmTask& T, const GemmTile tile, const OpTables& ops,
                                            SmemFp<Elem, KC, TB>& sm) {
  constexpr bool kF64 = sizeof(Elem) == 8;
  constexpr int kTT = 64 * TB;
  constexpr int kDV = 16 / sizeof(Elem);        // operator elements per 16-byte load
  constexpr int ND = kTT * KC / (256 * kDV);    // 16-byte operator loads per thread
  constexpr int NX = XLoad<KC>::NX;
  static_assert(ND >= 1, "tile too small for the operator loader");
  static_assert(PF == 1 || PF == 2, "prefetch depth 1 or 2");
  typedef Elem vec4 __attribute__((ext_vector_type(4)));
  auto& Xs = sm.Xs;
  auto& Ds = sm.Ds;
  int64_t* dst = sm.dst;
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const int nl = min(kLB, nlines - tile.line0);
  const int ld = ops.ld[T.op];
  const Elem* __restrict__ D;
  if constexpr (kF64)
    D = ops.f64 + ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  else
    D = ops.f32 + ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr bool q1 = Q1;
  if (tid < kLB) dst[tid] = line_base(T, min(tile.line0 + tid, nlines - 1));
  XLoad<KC> xl;
  xl.init(T, tile.line0, nlines, q1);
  // register sets of the chunks in flight: one (PF = 1) or two (PF = 2,
  // even chunks in set 0, odd chunks in set 1)
  double xr[PF][NX];
  uint4 dr[PF][ND];
  auto load = [&](int set, int c) {
    xl.load(xr[set], q1, c * KC, n, T.s_stride);
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      const int e = (tid + 256 * p) * kDV, t = e / KC, kk = e % KC;
      dr[set][p] = *reinterpret_cast<const uint4*>(D + static_cast<int64_t>(t) * ld + c * KC + kk);
    }
  };
  auto stage = [&](int b, int set) {
#pragma unroll
    for (int p = 0; p < NX; ++p) {
      int l, kk;
      chunk_pos<KC>(q1, tid + 256 * p, l, kk);
      Xs[b][l][kk] = static_cast<Elem>(xr[set][p]);
    }
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      const int e = (tid + 256 * p) * kDV, t = e / KC, kk = e % KC;
      const Elem* v = reinterpret_cast<const Elem*>(&dr[set][p]);
#pragma unroll
      for (int j = 0; j < kDV; ++j) Ds[b][t][kk + j] = v[j];
    }
  };
  // Output blocks that hold outputs (none if this wave's lines are past the
  // task's end); the same count on every wave of a full line tile.  The
  // chunk loop is instantiated per count, so the accumulators keep static
  // registers; every instantiation takes part in the same loads and barriers.
  const int nb = 16 * wave < nl && !((tile.skip >> wave) & 1) ? (nt + 15) >> 4 : 0;
  const int nk = (n + KC - 1) / KC;
  // With two chunks in flight every load is issued unconditionally (chunk
  // indices past the end clamped to the last chunk, inside the padded
  // operator rows), so that each wait covers only the older set.
  load(0, 0);
  if constexpr (PF == 2) load(1, min(1, nk - 1));
  stage(0, 0);
  __syncthreads();
  if constexpr (PF == 2) load(0, min(2, nk - 1));
  with_live<4 * TB>(nb, [&](auto live) {
    constexpr int NL = decltype(live)::value;
    vec4 acc[NL > 0 ? NL : 1];
#pragma unroll
    for (int ob = 0; ob < NL; ++ob) acc[ob] = vec4{0, 0, 0, 0};
    auto products = [&](int b) {
      if constexpr (NL > 0) {
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
          const int kr = ks + (lane >> 4), rr = lane & 15;
          const Elem xa = Xs[b][16 * wave + rr][kr];
#pragma unroll
          for (int ob = 0; ob < NL; ++ob) {
            const Elem da = Ds[b][16 * ob + rr][kr];
            if constexpr (kF64)
              acc[ob] = q1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(xa, da, acc[ob], 0, 0, 0)
                           : __builtin_amdgcn_mfma_f64_16x16x4f64(da, xa, acc[ob], 0, 0, 0);
            else
              acc[ob] = q1 ? __builtin_amdgcn_mfma_f32_16x16x4f32(xa, da, acc[ob], 0, 0, 0)
                           : __builtin_amdgcn_mfma_f32_16x16x4f32(da, xa, acc[ob], 0, 0, 0);
          }
        }
      }
    };
    if constexpr (PF == 1) {
      for (int c = 0; c < nk; ++c) {
        const int b = c & 1;
        if (c + 1 < nk) load(0, c + 1);
        products(b);
        if (c + 1 < nk) stage(b ^ 1, 0);
        __syncthreads();
      }
    } else {
      // chunk c in LDS buffer c & 1, chunks c + 1 and c + 2 in flight in the
      // register sets (c + 1) & 1 and c & 1; unrolled by two so that the
      // sets keep fixed registers
      for (int c = 0; c < nk; c += 2) {
        products(0);
        if (c + 1 < nk) stage(1, 1);
        __syncthreads();
        load(1, min(c + 3, nk - 1));
        if (c + 1 >= nk) break;
        products(1);
        if (c + 2 < nk) stage(0, 0);
        __syncthreads();
        load(0, min(c + 4, nk - 1));
      }
    }
    if constexpr (NL > 0) store_lines<kF64, NL>(T, dst, nl, t0, nt, q1, wave, lane, acc);
  });
}

// The direction decides the operand roles of every MFMA; it is resolved
// once per tile so that the inner loop holds no branch.
template <typename Elem, int KC, int TB, int PF = 1>
__device__ __forceinline__ void gemm_fp(const GemmTask* __restrict__ tasks, const GemmTile tile,
                                        const OpTables& ops) {
  __shared__ SmemFp<Elem, KC, TB> sm;
  const GemmTask T = tasks[tile.task];
  if (T.s_stride == 1)
    gemm_fp_dir<Elem, KC, TB, true, PF>(T, tile, ops, sm);
  else
    gemm_fp_dir<Elem, KC, TB, false, PF>(T, tile, ops, sm);
}

// Operator in registers: only the operand lines (shared by the four waves)
// are staged in LDS; each wave loads the operator rows of its own output
// blocks straight from L2 into MFMA operand registers.  Within a chunk of 16
// columns the reduction runs in the order k = 4 g + j (lane group g = lane /
// 16, step j), so a lane's operator values for the chunk are 4 consecutive
// columns of one row (16-byte loads) and its operand values 4 consecutive
// columns of one line (16-byte LDS reads).  The operator loads of chunk c+1
// are issued before the products of chunk c.  TB (2 or 4) 16-output blocks
// per wave: a workgroup covers 64 lines x 64 TB outputs; a wave skips the
// loads and products of its blocks past the line end.
template <typename Elem, int KC>
struct SmemXs {
  alignas(16) Elem Xs[2][kLB][KC + 16 / sizeof(Elem)];
  int64_t dst[kLB];
};

template <typename Elem, int KC, int TB, bool Q1>
__device__ __forceinline__ void gemm_xs_dir(const GemmTask& T, const GemmTile tile, const OpTables& ops,
                                            SmemXs<Elem, KC>& sm) {
  constexpr bool kF64 = sizeof(Elem) == 8;
  constexpr int kTT = 64 * TB;
  constexpr int PITCH = KC + 16 / sizeof(Elem);   // 16-byte aligned rows
  constexpr int NX = kLB * KC / 256;              // operand values per thread and chunk
  constexpr int NS = KC / 16;                     // 16-column sub-chunks
  constexpr int DQ = 4 * sizeof(Elem) / 16;       // 16-byte loads per 4 operator values
  typedef Elem vec4 __attribute__((ext_vector_type(4)));
  auto& Xs = sm.Xs;
  int64_t* dst = sm.dst;
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const int nl = min(kLB, nlines - tile.line0);
  const int ld = ops.ld[T.op];
  const Elem* __restrict__ D;
  if constexpr (kF64)
    D = ops.f64 + ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  else
    D = ops.f32 + ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4,
            rr = lane & 15;
  constexpr bool q1 = Q1;
  if (tid < kLB) dst[tid] = line_base(T, min(tile.line0 + tid, nlines - 1));
  // operand staging: one line and NX consecutive columns per thread
  const int xs_line = q1 ? tid / (256 / kLB) : tid % kLB;
  const int xs_col = NX * (q1 ? tid % (256 / kLB) : tid / kLB);
  const gdouble* __restrict__ xbase = gsrc(T.src) + line_base(T, min(tile.line0 + xs_line, nlines - 1));
  double xr[NX];
  auto load_x = [&](int k0) {
#pragma unroll
    for (int j = 0; j < NX; ++j) xr[j] = xbase[static_cast<int64_t>(min(k0 + xs_col + j, n - 1)) * T.s_stride];
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int j = 0; j < NX; ++j) Xs[b][xs_line][xs_col + j] = static_cast<Elem>(xr[j]);
  };
  // operator fragments: block i of this wave, sub-chunk s, 4 values (blocks
  // past the tile's outputs read zero-padded rows and are not stored)
  uint4 dr[TB][NS][DQ] = {};  // blocks past the line end stay zero
  auto load_d = [&](int k0) {
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      if (16 * (wave + 4 * i) >= nt) continue;  // block past the line end: no products
      const Elem* row = D + static_cast<int64_t>(16 * (wave + 4 * i) + rr) * ld + k0 + 4 * g;
#pragma unroll
      for (int sc = 0; sc < NS; ++sc)
#pragma unroll
        for (int q = 0; q < DQ; ++q)
          dr[i][sc][q] = *reinterpret_cast<const uint4*>(row + 16 * sc + q * (16 / sizeof(Elem)));
    }
  };
  vec4 acc[TB][4];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[i][b] = vec4{0, 0, 0, 0};
  const int nk = (n + KC - 1) / KC;
  load_x(0);
  load_d(0);
  stage(0);
  __syncthreads();
  for (int c = 0; c < nk; ++c) {
    const int b = c & 1;
    uint4 dn[TB][NS][DQ];
#pragma unroll
    for (int i = 0; i < TB; ++i)
#pragma unroll
      for (int sc = 0; sc < NS; ++sc)
#pragma unroll
        for (int q = 0; q < DQ; ++q) dn[i][sc][q] = dr[i][sc][q];
    if (c + 1 < nk) {
      load_x((c + 1) * KC);
      load_d((c + 1) * KC);
    }
#pragma unroll
    for (int sc = 0; sc < NS; ++sc) {
      Elem xv[4][4];  // [line block][step]
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        const Elem* xp = &Xs[b][16 * lb + rr][16 * sc + 4 * g];
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
          const uint4 v = *reinterpret_cast<const uint4*>(xp + q * (16 / sizeof(Elem)));
          const Elem* e = reinterpret_cast<const Elem*>(&v);
#pragma unroll
          for (int j = 0; j < 16 / static_cast<int>(sizeof(Elem)); ++j) xv[lb][q * (16 / sizeof(Elem)) + j] = e[j];
        }
      }
#pragma unroll
      for (int i = 0; i < TB; ++i) {
        if (16 * (wave + 4 * i) >= nt) continue;
        const Elem* dv = reinterpret_cast<const Elem*>(&dn[i][sc][0]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int lb = 0; lb < 4; ++lb) {
            if constexpr (kF64)
              acc[i][lb] = q1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(xv[lb][j], dv[j], acc[i][lb], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f64_16x16x4f64(dv[j], xv[lb][j], acc[i][lb], 0, 0, 0);
            else
              acc[i][lb] = q1 ? __builtin_amdgcn_mfma_f32_16x16x4f32(xv[lb][j], dv[j], acc[i][lb], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f32_16x16x4f32(dv[j], xv[lb][j], acc[i][lb], 0, 0, 0);
          }
      }
    }
    if (c + 1 < nk) stage(b ^ 1);
    __syncthreads();
  }
  store_tile<kF64, TB>(T, dst, nl, t0, nt, q1, wave, lane, acc, static_cast<const vec4(*)[4]>(nullptr), nullptr,
                       nullptr);
}

template <typename Elem, int KC, int TB>
__device__ __forceinline__ void gemm_xs(const GemmTask* __restrict__ tasks, const GemmTile tile, const OpTables& ops) {
  __shared__ SmemXs<Elem, KC> sm;
  const GemmTask T = tasks[tile.task];
  if (T.s_stride == 1)
    gemm_xs_dir<Elem, KC, TB, true>(T, tile, ops, sm);
  else
    gemm_xs_dir<Elem, KC, TB, false>(T, tile, ops, sm);
}

template <typename Elem, int KC, int TB>
__global__ __launch_bounds__(256, sizeof(Elem) == 8 ? 2 : 1) void k_gemm_xs(const GemmTask* __restrict__ tasks,
                                                 const GemmTile* __restrict__ tiles, OpTables ops) {
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  gemm_xs<Elem, KC, TB>(tasks, tile, ops);
}

// Wide staging ("xw"): a tile's operand lines are staged in LDS a slab of
// SLAB columns at a time, with all of the slab's global loads in flight at
// once (one memory latency per slab instead of one per 16 columns); the
// products of the slab then run from LDS, with each wave's operator rows
// loaded from L2 into registers one 16-column step ahead (reduction order
// k = 4 g + j within a step, as in the operator-in-registers kernel).  Other
// workgroups on the CU overlap one tile's slab loads with another's
// products.
template <typename Elem, int SLAB>
struct SmemXw {
  alignas(16) Elem Xs[kLB][SLAB + 16 / sizeof(Elem)];
  int64_t dst[kLB];
};

template <typename Elem, int SLAB, int TB, bool Q1>
__device__ __forceinline__ void gemm_xw_dir(const GemmTask& T, const GemmTile tile, const OpTables& ops,
                                            SmemXw<Elem, SLAB>& sm) {
  constexpr bool kF64 = sizeof(Elem) == 8;
  constexpr int kTT = 64 * TB;
  constexpr int NX = kLB * SLAB / 256;           // operand values per thread and slab
  constexpr int DQ = 4 * sizeof(Elem) / 16;      // 16-byte loads per 4 operator values
  constexpr int EV = 16 / sizeof(Elem);          // elements per 16 bytes
  constexpr bool q1 = Q1;
  typedef Elem vec4 __attribute__((ext_vector_type(4)));
  auto& Xs = sm.Xs;
  int64_t* dst = sm.dst;
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const int nl = min(kLB, nlines - tile.line0);
  const int ld = ops.ld[T.op];
  const Elem* __restrict__ D;
  if constexpr (kF64)
    D = ops.f64 + ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  else
    D = ops.f32 + ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4,
            rr = lane & 15;
  if (tid < kLB) dst[tid] = line_base(T, min(tile.line0 + tid, nlines - 1));
  const int xs_line = q1 ? tid / (256 / kLB) : tid % kLB;
  const int xs_col = NX * (q1 ? tid % (256 / kLB) : tid / kLB);
  const gdouble* __restrict__ xbase = gsrc(T.src) + line_base(T, min(tile.line0 + xs_line, nlines - 1));
  // operator rows of this wave's output blocks (zero-padded beyond n)
  const Elem* drow[TB];
#pragma unroll
  for (int i = 0; i < TB; ++i) drow[i] = D + static_cast<int64_t>(16 * (wave + 4 * i) + rr) * ld + 4 * g;
  const int nsteps = (n + 15) / 16;  // 16-column steps over the whole line (operator columns padded to 32)
  uint4 dcur[TB][DQ] = {}, dnext[TB][DQ] = {};  // blocks past the line end stay zero
  auto load_d = [&](uint4 (&d)[TB][DQ], int step) {
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      if (16 * (wave + 4 * i) >= nt) continue;  // block past the line end: no products
#pragma unroll
      for (int q = 0; q < DQ; ++q) d[i][q] = *reinterpret_cast<const uint4*>(drow[i] + 16 * step + q * EV);
    }
  };
  vec4 acc[TB][4];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[i][b] = vec4{0, 0, 0, 0};
  load_d(dcur, 0);
  for (int s0 = 0; s0 < n; s0 += SLAB) {
    // stage the slab: every load of the slab in flight before the first store
    double xr[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) xr[j] = xbase[static_cast<int64_t>(min(s0 + xs_col + j, n - 1)) * T.s_stride];
    __syncthreads();  // the previous slab's products have read Xs
#pragma unroll
    for (int j = 0; j < NX; ++j) Xs[xs_line][xs_col + j] = static_cast<Elem>(xr[j]);
    __syncthreads();
    const int step0 = s0 / 16, nsub = min(SLAB / 16, nsteps - step0);
    for (int sc = 0; sc < nsub; ++sc) {
      if (step0 + sc + 1 < nsteps) load_d(dnext, step0 + sc + 1);
      Elem xv[4][4];  // [line block][step j]
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        const Elem* xp = &Xs[16 * lb + rr][16 * sc + 4 * g];
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
          const uint4 v = *reinterpret_cast<const uint4*>(xp + q * EV);
          const Elem* e = reinterpret_cast<const Elem*>(&v);
#pragma unroll
          for (int j = 0; j < EV; ++j) xv[lb][q * EV + j] = e[j];
        }
      }
#pragma unroll
      for (int i = 0; i < TB; ++i) {
        if (16 * (wave + 4 * i) >= nt) continue;
        const Elem* dv = reinterpret_cast<const Elem*>(&dcur[i][0]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int lb = 0; lb < 4; ++lb) {
            if constexpr (kF64)
              acc[i][lb] = q1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(xv[lb][j], dv[j], acc[i][lb], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f64_16x16x4f64(dv[j], xv[lb][j], acc[i][lb], 0, 0, 0);
            else
              acc[i][lb] = q1 ? __builtin_amdgcn_mfma_f32_16x16x4f32(xv[lb][j], dv[j], acc[i][lb], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f32_16x16x4f32(dv[j], xv[lb][j], acc[i][lb], 0, 0, 0);
          }
      }
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int q = 0; q < DQ; ++q) dcur[i][q] = dnext[i][q];
    }
  }
  store_tile<kF64, TB>(T, dst, nl, t0, nt, q1, wave, lane, acc, static_cast<const vec4(*)[4]>(nullptr), nullptr,
                       nullptr);
}

template <typename Elem, int SLAB, int TB>
__global__ __launch_bounds__(256) void k_gemm_xw(const GemmTask* __restrict__ tasks, const GemmTile* __restrict__ tiles,
                                                 OpTables ops) {
  __shared__ SmemXw<Elem, SLAB> sm;
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  const GemmTask T = tasks[tile.task];
  if (T.s_stride == 1)
    gemm_xw_dir<Elem, SLAB, TB, true>(T, tile, ops, sm);
  else
    gemm_xw_dir<Elem, SLAB, TB, false>(T, tile, ops, sm);
}

// Wide staging for split BF16: the slab holds X - x0 as bf16 hi and lo; the
// 16x16x32 products take 8 consecutive columns per lane on both operands.
template <int SLAB>
struct SmemXwBf {
  alignas(16) uint16_t Xh[kLB][SLAB + 8];
  alignas(16) uint16_t Xl[kLB][SLAB + 8];
  double x0s[kLB];
  int64_t dst[kLB];
};

template <int SLAB, int TB, bool Q1>
__device__ __forceinline__ void gemm_xw_bf16x3_dir(const GemmTask& T, const GemmTile tile, const OpTables& ops,
                                                   SmemXwBf<SLAB>& sm) {
  constexpr int kTT = 64 * TB;
  constexpr int NX = kLB * SLAB / 256;  // operand values per thread and slab
  constexpr bool q1 = Q1;
  auto& Xh = sm.Xh;
  auto& Xl = sm.Xl;
  double* x0s = sm.x0s;
  int64_t* dst = sm.dst;
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const int nl = min(kLB, nlines - tile.line0);
  const int ld = ops.ld[T.op];
  const int64_t dbase = ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4,
            rr = lane & 15;
  if (tid < kLB) {
    dst[tid] = line_base(T, min(tile.line0 + tid, nlines - 1));
    x0s[tid] = gsrc(T.src)[dst[tid]];
  }
  const int xs_line = q1 ? tid / (256 / kLB) : tid % kLB;
  const int xs_col = NX * (q1 ? tid % (256 / kLB) : tid / kLB);
  const gdouble* __restrict__ xbase = gsrc(T.src) + line_base(T, min(tile.line0 + xs_line, nlines - 1));
  const double x0 = xbase[0];
  const uint16_t* bh[TB];
  const uint16_t* bl[TB];
#pragma unroll
  for (int i = 0; i < TB; ++i) {
    const int64_t o = dbase + static_cast<int64_t>(16 * (wave + 4 * i) + rr) * ld + 8 * g;
    bh[i] = ops.bhi + o;
    bl[i] = ops.blo + o;
  }
  const int nsteps = (n + 31) / 32;  // 32-column steps (operator columns padded to 32)
  uint4 hcur[TB] = {}, lcur[TB] = {}, hnext[TB] = {}, lnext[TB] = {};  // blocks past the line end stay zero
  auto load_d = [&](uint4 (&h)[TB], uint4 (&l)[TB], int step) {
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      if (16 * (wave + 4 * i) >= nt) continue;  // block past the line end: no products
      h[i] = *reinterpret_cast<const uint4*>(bh[i] + 32 * step);
      l[i] = *reinterpret_cast<const uint4*>(bl[i] + 32 * step);
    }
  };
  f32x4 am[TB][4], ac[TB][4];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) am[i][b] = ac[i][b] = f32x4{0, 0, 0, 0};
  load_d(hcur, lcur, 0);
  for (int s0 = 0; s0 < n; s0 += SLAB) {
    double xr[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) xr[j] = xbase[static_cast<int64_t>(min(s0 + xs_col + j, n - 1)) * T.s_stride];
    __syncthreads();
#pragma unroll
    for (int j0 = 0; j0 < NX; j0 += 8) {
      bf16x8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float f = static_cast<float>(xr[j0 + j] - x0);
        h[j] = static_cast<__bf16>(f);  // round to nearest even (v_cvt_pk_bf16_f32)
        l[j] = static_cast<__bf16>(f - static_cast<float>(h[j]));
      }
      *reinterpret_cast<bf16x8*>(&Xh[xs_line][xs_col + j0]) = h;
      *reinterpret_cast<bf16x8*>(&Xl[xs_line][xs_col + j0]) = l;
    }
    __syncthreads();
    const int step0 = s0 / 32, nsub = min(SLAB / 32, nsteps - step0);
    for (int sc = 0; sc < nsub; ++sc) {
      if (step0 + sc + 1 < nsteps) load_d(hnext, lnext, step0 + sc + 1);
      bf16x8 xh[4], xlo[4];
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        xh[lb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xh[16 * lb + rr][32 * sc + 8 * g]));
        xlo[lb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xl[16 * lb + rr][32 * sc + 8 * g]));
      }
#pragma unroll
      for (int i = 0; i < TB; ++i) {
        if (16 * (wave + 4 * i) >= nt) continue;
        const bf16x8 dh = __builtin_bit_cast(bf16x8, hcur[i]);
        const bf16x8 dl = __builtin_bit_cast(bf16x8, lcur[i]);
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
          if (q1) {
            am[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[lb], dh, am[i][lb], 0, 0, 0);
            ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[lb], dl, ac[i][lb], 0, 0, 0);
            ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xlo[lb], dh, ac[i][lb], 0, 0, 0);
          } else {
            am[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, xh[lb], am[i][lb], 0, 0, 0);
            ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, xlo[lb], ac[i][lb], 0, 0, 0);
            ac[i][lb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dl, xh[lb], ac[i][lb], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < TB; ++i) {
        hcur[i] = hnext[i];
        lcur[i] = lnext[i];
      }
    }
  }
  store_tile<false, TB>(T, dst, nl, t0, nt, q1, wave, lane, am, ac, x0s, ops.rowsum + ops.roff[T.op]);
}

template <int SLAB, int TB>
__global__ __launch_bounds__(256) void k_gemm_xw_bf16x3(const GemmTask* __restrict__ tasks,
                                                        const GemmTile* __restrict__ tiles, OpTables ops) {
  __shared__ SmemXwBf<SLAB> sm;
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  const GemmTask T = tasks[tile.task];
  if (T.s_stride == 1)
    gemm_xw_bf16x3_dir<SLAB, TB, true>(T, tile, ops, sm);
  else
    gemm_xw_bf16x3_dir<SLAB, TB, false>(T, tile, ops, sm);
}

// Persistent form over the XCD queues.  The tile list holds 8 interleaved
// queues (tile 8 r + x belongs to queue x, each queue longest tile first).
// The grid is a multiple of 8 workgroups; workgroup b serves queue b mod 8
// (the XCD it is dispatched to), takes tile r = b / 8 first and later ones
// from the queue's counter ctr[x], offset by the workgroups per queue.  The
// next index is requested before the current tile is computed, so the
// atomic's latency hides behind it.  ctr[8] counts finished workgroups; the
// last one resets all nine counters, so the next launch (graph replays
// included) starts from zero without a memset.
template <typename Body>
__device__ __forceinline__ void xcd_queue_tiles(int ntiles, int* ctr, Body body) {
  __shared__ int next_r;
  const int x = blockIdx.x & 7, per_q = gridDim.x >> 3, qlen = ntiles >> 3;
  int r = blockIdx.x >> 3;
  while (r < qlen) {
    int nr = 0;
    if (threadIdx.x == 0) nr = atomicAdd(&ctr[x], 1) + per_q;
    body(8 * r + x);
    if (threadIdx.x == 0) next_r = nr;
    __syncthreads();  // also: every wave is done with the tile's LDS
    r = next_r;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&ctr[8], 1) == static_cast<int>(gridDim.x) - 1)
      for (int q = 0; q < 9; ++q) atomicExch(&ctr[q], 0);
  }
}

// Stage contractions (every SSPRK stage) ...
// Launch bounds: the second argument asks for that many waves per SIMD, which
// bounds the registers per lane.
// MINB workgroups per CU (the launch bound caps the registers at 512 /
// MINB per lane): 8-column FP64 chunks (19 KB of LDS) let seven share a CU,
// enough for the whole step-channel stage task set in one round (that form
// spills 24 bytes per lane; the others do not); the two-chunk prefetch of
// 16-column FP64 chunks needs the registers of three.
// PF: chunks whose loads are in flight while a chunk is on the matrix cores.
template <typename Elem, int KC, int TB, int MINB, int PF>
__global__ __launch_bounds__(256, MINB) void k_gemm_fp(const GemmTask* __restrict__ tasks,
                                                    const GemmTile* __restrict__ tiles, OpTables ops) {
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  gemm_fp<Elem, KC, TB, PF>(tasks, tile, ops);
}

template <typename Elem, int KC, int TB>
__global__ __launch_bounds__(256, 4) void k_gemm_fp_persist(const GemmTask* __restrict__ tasks,
                                                         const GemmTile* __restrict__ tiles, int ntiles,
                                                         OpTables ops, int* ctr) {
  xcd_queue_tiles(ntiles, ctr, [&](int t) {
    const GemmTile tile = tiles[t];
    if (!tile_idle(tile)) gemm_fp<Elem, KC, TB>(tasks, tile, ops);
  });
}

// ... and the once-per-step FP64 contractions (viscosity gradient, filter),
// under their own name so that profiles tell the two apart.
__global__ __launch_bounds__(256, 4) void k_gemm_step(const GemmTask* __restrict__ tasks,
                                                   const GemmTile* __restrict__ tiles, OpTables ops) {
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  gemm_fp<double, 16, 1>(tasks, tile, ops);
}

// Split BF16: chunks of KC columns (one or two MFMA depths of 32); LDS rows
// padded by 8 halves so each lane's 8-element operand is one aligned 16-byte
// read.  NS parts per value: 2 (hi + lo; products hh, hl, lh) or 3 (hi +
// mid + lo; products hh, hm, mh, hl, mm, lh), one FP32 accumulator per
// order of magnitude, summed in FP64 at the store.
template <int TB, int NS = 2, int KC = 32>
struct SmemBf {
  static constexpr int PITCH = KC + 8;
  alignas(16) uint16_t Xh[2][kLB][PITCH];
  alignas(16) uint16_t Xl[2][kLB][PITCH];
  alignas(16) uint16_t Xm[NS == 3 ? 2 : 1][NS == 3 ? kLB : 1][PITCH];
  alignas(16) uint16_t Dh[2][64 * TB][PITCH];
  alignas(16) uint16_t Dl[2][64 * TB][PITCH];
  alignas(16) uint16_t Dm[NS == 3 ? 2 : 1][NS == 3 ? 64 * TB : 1][PITCH];
  double x0s[kLB];
  int64_t dst[kLB];
};

// Registers of one chunk's global loads (operand lines and operator rows).
template <int NXG, int ND, int NS>
struct BfChunk {
  double xr[8 * NXG];
  uint4 hr[ND], lr[ND], mr[NS == 3 ? ND : 1];
};

// One tile of the split-BF16 contraction.  The chunk loop keeps PF chunks'
// global loads in flight: A holds chunk c + 1 while the products of chunk c
// run, and is staged into the free LDS buffer after them; with PF = 2, B
// holds chunk c + 2, moves into A, and is refilled with chunk c + 3 (plain
// register moves: no slot is indexed at run time).
template <int TB, int NS, int KC, int PF, bool Q1>
__device__ __forceinline__ void gemm_bf16x3_dir(const GemmTask& T, const GemmTile tile, const OpTables& ops,
                                                SmemBf<TB, NS, KC>& sm, int maxl = kLB) {
  constexpr int kTT = 64 * TB;
  constexpr int ND = kTT * KC / (256 * 8);  // 16-byte loads per thread and table
  constexpr int NXG = KC / 32;              // groups of 8 columns per thread
  auto& Xh = sm.Xh;
  auto& Xl = sm.Xl;
  auto& Dh = sm.Dh;
  auto& Dl = sm.Dl;
  double* x0s = sm.x0s;
  int64_t* dst = sm.dst;
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0, nt = min(kTT, n - t0);
  const int nl = min(maxl, nlines - tile.line0);
  const int ld = ops.ld[T.op];
  const int64_t dbase = ops.off[T.op] + static_cast<int64_t>(t0) * ld;
  const uint16_t* __restrict__ Bh = ops.bhi + dbase;
  const uint16_t* __restrict__ Bl = ops.blo + dbase;
  const uint16_t* __restrict__ Bm = NS == 3 ? ops.bmid + dbase : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr bool q1 = Q1;
  // Operand staging.  Along q^2 (lines adjacent in memory) thread t owns
  // line t % 64 and NXG groups of 8 consecutive columns: each load reads 64
  // neighbouring lines at one column, and each group is split with packed
  // conversions and stored as 16 bytes per table.  Along q^1 (columns
  // contiguous) thread t owns column pair 2 (t % 16), +1 (and +32 per
  // further group) of the four lines t / 16 + 16 i: sixteen lanes read one
  // line's chunk, and each pair is stored as 4 bytes per table.
  const int pc = 2 * (tid & 15), qs = tid >> 4;              // q^1 mapping
  const int xl_line = tid & 63, xl_col = 8 * (tid >> 6);    // q^2 mapping
  const gdouble* xb[q1 ? 4 : 1];
  double x0v[q1 ? 4 : 1];
#pragma unroll
  for (int i = 0; i < (q1 ? 4 : 1); ++i) {
    xb[i] = gsrc(T.src) + line_base(T, min(tile.line0 + (q1 ? qs + 16 * i : xl_line), nlines - 1));
    x0v[i] = xb[i][0];  // line offset (first point of the line)
  }
  if (tid < kLB) {
    dst[tid] = line_base(T, min(tile.line0 + tid, nlines - 1));
    x0s[tid] = gsrc(T.src)[dst[tid]];
  }
  using Chunk = BfChunk<NXG, ND, NS>;
  Chunk A, B;
  auto load = [&](Chunk& r, int k0) __attribute__((always_inline)) {
    if constexpr (q1) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int g = 0; g < NXG; ++g)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            r.xr[8 * g + 2 * i + h] = xb[i][min(k0 + 32 * g + pc + h, n - 1)];
    } else {
#pragma unroll
      for (int g = 0; g < NXG; ++g)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          r.xr[8 * g + j] = xb[0][static_cast<int64_t>(min(k0 + 32 * g + xl_col + j, n - 1)) * T.s_stride];
    }
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      const int e = (tid + 256 * p) * 8, t = e / KC, kk = e % KC;
      const int64_t o = static_cast<int64_t>(t) * ld + k0 + kk;
      r.hr[p] = *reinterpret_cast<const uint4*>(Bh + o);
      r.lr[p] = *reinterpret_cast<const uint4*>(Bl + o);
      if constexpr (NS == 3) r.mr[p] = *reinterpret_cast<const uint4*>(Bm + o);
    }
  };
  // hi (+ mid) + lo parts of x - x0 (FP32 difference, parts rounded to
  // nearest even by v_cvt_pk_bf16_f32; each remainder is exact in FP32)
  struct Parts {
    __bf16 h, md, l;
  };
  auto split = [&](double v, double x0) __attribute__((always_inline)) {
    Parts o;
    const float f = static_cast<float>(v - x0);
    o.h = static_cast<__bf16>(f);
    const float r1 = f - static_cast<float>(o.h);
    if constexpr (NS == 3) {
      o.md = static_cast<__bf16>(r1);
      o.l = static_cast<__bf16>(r1 - static_cast<float>(o.md));
    } else {
      o.md = o.h;
      o.l = static_cast<__bf16>(r1);
    }
    return o;
  };
  auto stage = [&](const Chunk& r, int b) __attribute__((always_inline)) {
    if constexpr (q1) {
      typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int g = 0; g < NXG; ++g) {
          bf16x2 h, l, md;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const Parts o = split(r.xr[8 * g + 2 * i + q], x0v[i]);
            h[q] = o.h;
            md[q] = o.md;
            l[q] = o.l;
          }
          const int line = qs + 16 * i, col = 32 * g + pc;
          *reinterpret_cast<bf16x2*>(&Xh[b][line][col]) = h;
          *reinterpret_cast<bf16x2*>(&Xl[b][line][col]) = l;
          if constexpr (NS == 3) *reinterpret_cast<bf16x2*>(&sm.Xm[b][line][col]) = md;
        }
    } else {
#pragma unroll
      for (int g = 0; g < NXG; ++g) {
        bf16x8 h, l, md;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const Parts o = split(r.xr[8 * g + j], x0v[0]);
          h[j] = o.h;
          md[j] = o.md;
          l[j] = o.l;
        }
        *reinterpret_cast<bf16x8*>(&Xh[b][xl_line][xl_col + 32 * g]) = h;
        *reinterpret_cast<bf16x8*>(&Xl[b][xl_line][xl_col + 32 * g]) = l;
        if constexpr (NS == 3) *reinterpret_cast<bf16x8*>(&sm.Xm[b][xl_line][xl_col + 32 * g]) = md;
      }
    }
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      const int e = (tid + 256 * p) * 8, t = e / KC, kk = e % KC;
      *reinterpret_cast<uint4*>(&Dh[b][t][kk]) = r.hr[p];
      *reinterpret_cast<uint4*>(&Dl[b][t][kk]) = r.lr[p];
      if constexpr (NS == 3) *reinterpret_cast<uint4*>(&sm.Dm[b][t][kk]) = r.mr[p];
    }
  };
  const int nk = (n + KC - 1) / KC;
  load(A, 0);
  stage(A, 0);
  __syncthreads();
  if (1 < nk) load(A, KC);
  if (PF == 2 && 2 < nk) load(B, 2 * KC);
  const int rr = lane & 15, kb = 8 * (lane >> 4);
  // Wave w owns the 16 lines 16 w .. 16 w + 15 and every output block of the
  // tile; blocks past the line end are skipped by all waves alike (the chunk
  // loop is instantiated per count of live blocks, as in the FP64/FP32
  // kernel).
  const int nb = 16 * wave < nl && !((tile.skip >> wave) & 1) ? (nt + 15) >> 4 : 0;
  const double* rowsum = ops.rowsum + ops.roff[T.op];
  with_live<4 * TB>(nb, [&](auto live) __attribute__((always_inline)) {
    constexpr int NL = decltype(live)::value;
    f32x4 bm[NL > 0 ? NL : 1], bc[NL > 0 ? NL : 1], b3[NS == 3 && NL > 0 ? NL : 1];
#pragma unroll
    for (int ob = 0; ob < NL; ++ob) bm[ob] = bc[ob] = f32x4{0, 0, 0, 0};
    if constexpr (NS == 3) {
#pragma unroll
      for (int ob = 0; ob < NL; ++ob) b3[ob] = f32x4{0, 0, 0, 0};
    }
    // A x B with the operand roles of the direction (along q^1 the lines are
    // the rows, along q^2 the outputs are)
    auto mm = [&](const bf16x8& x, const bf16x8& d, f32x4 acc) __attribute__((always_inline)) {
      return q1 ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, d, acc, 0, 0, 0)
                : __builtin_amdgcn_mfma_f32_16x16x32_bf16(d, x, acc, 0, 0, 0);
    };
    auto products = [&](int b) __attribute__((always_inline)) {
      if constexpr (NL > 0) {
#pragma unroll
        for (int ks = 0; ks < NXG; ++ks) {
          const int kc = kb + 32 * ks;
          const bf16x8 xh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xh[b][16 * wave + rr][kc]));
          const bf16x8 xlo =
              __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Xl[b][16 * wave + rr][kc]));
          bf16x8 xmd{};
          if constexpr (NS == 3)
            xmd = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&sm.Xm[b][16 * wave + rr][kc]));
#pragma unroll
          for (int ob = 0; ob < NL; ++ob) {
            const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dh[b][16 * ob + rr][kc]));
            const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Dl[b][16 * ob + rr][kc]));
            if constexpr (NS == 3) {
              const bf16x8 bmd =
                  __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&sm.Dm[b][16 * ob + rr][kc]));
              bm[ob] = mm(xh, bh, bm[ob]);
              bc[ob] = mm(xh, bmd, bc[ob]);
              bc[ob] = mm(xmd, bh, bc[ob]);
              b3[ob] = mm(xh, bl, b3[ob]);
              b3[ob] = mm(xmd, bmd, b3[ob]);
              b3[ob] = mm(xlo, bh, b3[ob]);
            } else {
              bm[ob] = mm(xh, bh, bm[ob]);
              bc[ob] = mm(xh, bl, bc[ob]);
              bc[ob] = mm(xlo, bh, bc[ob]);
            }
          }
        }
      }
    };
#pragma unroll 1
    for (int c = 0; c < nk; ++c) {
      products(c & 1);
      if (c + 1 < nk) stage(A, (c + 1) & 1);
      __syncthreads();
      if constexpr (PF == 2) {
        A = B;
        if (c + 3 < nk) load(B, (c + 3) * KC);
      } else {
        if (c + 2 < nk) load(A, (c + 2) * KC);
      }
    }
    // the FP32 accumulations are added in FP64 at the store, with the exact
    // offset term x0 * rowsum
    if constexpr (NL > 0) {
#pragma unroll
      for (int ob = 0; ob < NL; ++ob) {
        if (16 * ob >= nt) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * (lane >> 4) + r, col = lane & 15;
          const int lloc = 16 * wave + (q1 ? row : col);
          const int tloc = 16 * ob + (q1 ? col : row);
          if (tloc >= nt || lloc >= nl) continue;
          double v = static_cast<double>(bm[ob][r]) + static_cast<double>(bc[ob][r]);
          if constexpr (NS == 3) v += static_cast<double>(b3[ob][r]);
          v += x0s[lloc] * rowsum[t0 + tloc];
          const int64_t o = dst[lloc] + static_cast<int64_t>(t0 + tloc) * T.s_stride;
          if (T.out_f32)
            gdst32(T.dst)[o] = static_cast<float>(v);
          else
            gdst64(T.dst)[o] = v;
        }
      }
    }
  });
}

template <int TB, int NS = 2, int KC = 32, int PF = 1>
__device__ __forceinline__ void gemm_bf16x3(const GemmTask* __restrict__ tasks, const GemmTile tile,
                                            const OpTables& ops) {
  __shared__ SmemBf<TB, NS, KC> sm;
  const GemmTask T = tasks[tile.task];
  if (T.s_stride == 1)
    gemm_bf16x3_dir<TB, NS, KC, PF, true>(T, tile, ops, sm);
  else
    gemm_bf16x3_dir<TB, NS, KC, PF, false>(T, tile, ops, sm);
}

// Line-stationary split BF16 (lines of at most line_max<LINES>() points): one
// workgroup stages the hi and lo parts of its 64 lines over their whole
// length into LDS once, and then forms every output of those lines: wave w
// takes the 16-output blocks w, w + 4, ... and, for each, runs the chunks of
// 32 columns with the operator rows read from L2 straight into MFMA
// operands (the next chunk's rows are loaded during the current chunk's
// products).  Operand lines are read from memory once per line tile instead
// of once per output tile, and the chunk loop needs no barrier.  Lines
// longer than the LDS rows take the staged shape (64-line tiles) or a
// register path (32-line tiles: operands read from memory per product).
// Longest line whose hi and lo parts fit the LDS rows (78 KB for 64 lines:
// two workgroups per CU; 39 KB for 32 lines: four).
template <int LINES>
constexpr int line_max() {
  return 304;
}
template <int LINES>
struct SmemLine {
  static constexpr int PITCH = line_max<LINES>() + 8;  // halves
  alignas(16) uint16_t Xh[LINES][PITCH];
  alignas(16) uint16_t Xl[LINES][PITCH];
  double x0s[LINES];
  int64_t dst[LINES];
};

// LINES lines per tile (64, or 32: half the LDS, more workgroups per CU).
template <int LINES, bool Q1>
__device__ __forceinline__ void gemm_bf16x3_line_dir(const GemmTask& T, const GemmTile tile, const OpTables& ops,
                                                     SmemLine<LINES>& sm) {
  constexpr int NLB = LINES / 16;      // 16-line blocks
  constexpr int GPP = 256 / LINES;     // q^2 staging: 8-column groups per pass
  const int n = T.n, nlines = T.nrow * T.ncomp;
  const int nl = min(LINES, nlines - tile.line0);
  const int ld = ops.ld[T.op];
  const int nk = (n + 31) / 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr bool q1 = Q1;
  if (tid < LINES) {
    sm.dst[tid] = line_base(T, min(tile.line0 + tid, nlines - 1));
    sm.x0s[tid] = gsrc(T.src)[sm.dst[tid]];
  }
  auto mm = [&](const bf16x8& x, const bf16x8& d, f32x4 acc) __attribute__((always_inline)) {
    return q1 ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, d, acc, 0, 0, 0)
              : __builtin_amdgcn_mfma_f32_16x16x32_bf16(d, x, acc, 0, 0, 0);
  };
  const int rr = lane & 15, kb = 8 * (lane >> 4);
  const double* rowsum = ops.rowsum + ops.roff[T.op];
  const int nob = (n + 15) / 16;
  // line blocks with work (16 lines each; the skip bits mark blocks of lines
  // on inactive grid lines)
  int lbmask = 0;
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb)
    if (16 * lb < nl && !((tile.skip >> lb) & 1)) lbmask |= 1 << lb;
  auto store = [&](int ob, int lb, const f32x4& am, const f32x4& ac) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * (lane >> 4) + r, col = lane & 15;
      const int lloc = 16 * lb + (q1 ? row : col);
      const int t = 16 * ob + (q1 ? col : row);
      if (t >= n || lloc >= nl) continue;
      const double v = static_cast<double>(am[r]) + static_cast<double>(ac[r]) + sm.x0s[lloc] * rowsum[t];
      const int64_t o = sm.dst[lloc] + static_cast<int64_t>(t) * T.s_stride;
      if (T.out_f32)
        gdst32(T.dst)[o] = static_cast<float>(v);
      else
        gdst64(T.dst)[o] = v;
    }
  };
  if (n > line_max<LINES>()) {
    // Lines longer than the LDS rows: each product reads its 8 operand
    // values straight from memory and splits them in registers (operand
    // lines re-read from L2 once per output block; such lines are rare).
    __syncthreads();
#pragma unroll 1
    for (int ob = wave; ob < nob; ob += 4) {
      const int64_t rbase = ops.off[T.op] + static_cast<int64_t>(16 * ob + rr) * ld + kb;
#pragma unroll 1
      for (int lb = 0; lb < NLB; ++lb) {
        if (!((lbmask >> lb) & 1)) continue;
        const int ll = 16 * lb + rr;
        const gdouble* __restrict__ xb = gsrc(T.src) + sm.dst[ll];
        const double x0 = sm.x0s[ll];
        f32x4 am = {0, 0, 0, 0}, ac = {0, 0, 0, 0};
#pragma unroll 1
        for (int c = 0; c < nk; ++c) {
          const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(ops.bhi + rbase + 32 * c));
          const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(ops.blo + rbase + 32 * c));
          bf16x8 xh, xl;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const double v = xb[static_cast<int64_t>(min(32 * c + kb + j, n - 1)) * T.s_stride];
            const float f = static_cast<float>(v - x0);
            xh[j] = static_cast<__bf16>(f);
            xl[j] = static_cast<__bf16>(f - static_cast<float>(xh[j]));
          }
          am = mm(xh, bh, am);
          ac = mm(xh, bl, ac);
          ac = mm(xl, bh, ac);
        }
        store(ob, lb, am, ac);
      }
    }
    return;
  }
  // Staging, as in the staged shape: along q^1 sixteen lanes per line (a
  // column pair each), along q^2 one line per lane (8 consecutive columns).
  // Only the 8-column groups that meet the line are stored (columns past its
  // end repeat its last value); a product's group past the line end reads
  // group 0 instead, whose values meet zero operator columns there.
  const int n8 = (n + 7) & ~7;
  auto split2 = [&](double v, double x0, __bf16& h, __bf16& l) __attribute__((always_inline)) {
    const float f = static_cast<float>(v - x0);
    const __bf16 hh = static_cast<__bf16>(f);
    h = hh;
    l = static_cast<__bf16>(f - static_cast<float>(hh));
  };
  // loads of kCG chunks (groups) are issued together (many loads in flight
  // per thread), then split and stored
  constexpr int kCG = 4;
  if constexpr (q1) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const int pc = 2 * (tid & 15), qs = tid >> 4;
    const gdouble* xb[NLB];
    double x0[NLB];
#pragma unroll
    for (int i = 0; i < NLB; ++i) {
      xb[i] = gsrc(T.src) + line_base(T, min(tile.line0 + qs + 16 * i, nlines - 1));
      x0[i] = xb[i][0];
    }
#pragma unroll 1
    for (int c0 = 0; c0 < nk; c0 += kCG) {
      double v[kCG][NLB][2];
#pragma unroll
      for (int cc = 0; cc < kCG; ++cc)
#pragma unroll
        for (int i = 0; i < NLB; ++i)
#pragma unroll
          for (int h = 0; h < 2; ++h) v[cc][i][h] = xb[i][min(32 * (c0 + cc) + pc + h, n - 1)];
#pragma unroll
      for (int cc = 0; cc < kCG; ++cc) {
        const int col = 32 * (c0 + cc) + pc;
        if (col >= n8) continue;
#pragma unroll
        for (int i = 0; i < NLB; ++i) {
          __bf16 h0, l0, h1, l1;
          split2(v[cc][i][0], x0[i], h0, l0);
          split2(v[cc][i][1], x0[i], h1, l1);
          bf16x2 h, l;
          h[0] = h0;
          h[1] = h1;
          l[0] = l0;
          l[1] = l1;
          *reinterpret_cast<bf16x2*>(&sm.Xh[qs + 16 * i][col]) = h;
          *reinterpret_cast<bf16x2*>(&sm.Xl[qs + 16 * i][col]) = l;
        }
      }
    }
  } else {
    const int line = tid % LINES, g0 = tid / LINES;
    const gdouble* __restrict__ xb = gsrc(T.src) + line_base(T, min(tile.line0 + line, nlines - 1));
    const double x0 = xb[0];
    const int ng = n8 / 8;
#pragma unroll 1
    for (int m0 = 0; m0 * GPP < ng; m0 += kCG) {
      double v[kCG][8];
#pragma unroll
      for (int mm = 0; mm < kCG; ++mm)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          v[mm][j] = xb[static_cast<int64_t>(min(8 * (g0 + GPP * (m0 + mm)) + j, n - 1)) * T.s_stride];
#pragma unroll
      for (int mm = 0; mm < kCG; ++mm) {
        const int col = 8 * (g0 + GPP * (m0 + mm));
        if (col >= n8) continue;
        bf16x8 h, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 hj, lj;
          split2(v[mm][j], x0, hj, lj);
          h[j] = hj;
          l[j] = lj;
        }
        *reinterpret_cast<bf16x8*>(&sm.Xh[line][col]) = h;
        *reinterpret_cast<bf16x8*>(&sm.Xl[line][col]) = l;
      }
    }
  }
  __syncthreads();
  // NB output blocks at a time (blocks ob, ob + 4, ...: the operand reads
  // from LDS serve NB x 3 products)
  auto blocks = [&](auto nb_c, int ob0) __attribute__((always_inline)) {
    constexpr int NB = decltype(nb_c)::value;
    const uint16_t* Bh[NB];
    const uint16_t* Bl[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      // operator row of this lane (zero-padded tables: rows past n are zero)
      const int64_t rbase = ops.off[T.op] + static_cast<int64_t>(16 * (ob0 + 4 * i) + rr) * ld + kb;
      Bh[i] = ops.bhi + rbase;
      Bl[i] = ops.blo + rbase;
    }
    f32x4 bm[NB][NLB], bc[NB][NLB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb) bm[i][lb] = bc[i][lb] = f32x4{0, 0, 0, 0};
    // operator rows of the next kPD chunks in flight (a register queue
    // shifted by one each chunk); every line block is multiplied (the
    // staged lines are valid data; skipped blocks are only not stored),
    // which keeps the chunk loop free of branches
    constexpr int kPD = 2;
    uint4 dh[kPD][NB], dl[kPD][NB];
#pragma unroll
    for (int q = 0; q < kPD; ++q)
      if (q < nk)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          dh[q][i] = *reinterpret_cast<const uint4*>(Bh[i] + 32 * q);
          dl[q][i] = *reinterpret_cast<const uint4*>(Bl[i] + 32 * q);
        }
#pragma unroll 1
    for (int c = 0; c < nk; ++c) {
      bf16x8 bh[NB], bl[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        bh[i] = __builtin_bit_cast(bf16x8, dh[0][i]);
        bl[i] = __builtin_bit_cast(bf16x8, dl[0][i]);
      }
#pragma unroll
      for (int q = 0; q + 1 < kPD; ++q)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          dh[q][i] = dh[q + 1][i];
          dl[q][i] = dl[q + 1][i];
        }
      if (c + kPD < nk)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          dh[kPD - 1][i] = *reinterpret_cast<const uint4*>(Bh[i] + 32 * (c + kPD));
          dl[kPD - 1][i] = *reinterpret_cast<const uint4*>(Bl[i] + 32 * (c + kPD));
        }
      const int kx = 32 * c + kb < n ? 32 * c + kb : 0;
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb) {
        const bf16x8 xh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&sm.Xh[16 * lb + rr][kx]));
        const bf16x8 xl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&sm.Xl[16 * lb + rr][kx]));
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          bm[i][lb] = mm(xh, bh[i], bm[i][lb]);
          bc[i][lb] = mm(xh, bl[i], bc[i][lb]);
          bc[i][lb] = mm(xl, bh[i], bc[i][lb]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb)
        if ((lbmask >> lb) & 1) store(ob0 + 4 * i, lb, bm[i][lb], bc[i][lb]);
  };
  int ob = wave;
#pragma unroll 1
  for (; ob + 4 < nob; ob += 8) blocks(std::integral_constant<int, 2>{}, ob);
  if (ob < nob) blocks(std::integral_constant<int, 1>{}, ob);
}

template <int LINES>
__global__ __launch_bounds__(256) void k_gemm_bf16x3_line(const GemmTask* __restrict__ tasks,
                                                          const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr size_t kBytes = LINES == 64 && sizeof(SmemBf<1, 2, 32>) > sizeof(SmemLine<LINES>)
                                ? sizeof(SmemBf<1, 2, 32>)
                                : sizeof(SmemLine<LINES>);
  __shared__ __attribute__((aligned(16))) char smem[kBytes];
  const GemmTile tile = tiles[blockIdx.x];
  constexpr int kAll = (1 << (LINES / 16)) - 1;  // skip bits of this tile's line blocks
  if (tile.task < 0 || (tile.skip & kAll) == kAll) return;
  const GemmTask T = tasks[tile.task];
  if constexpr (LINES == 64) {
    // with two workgroups per CU (set by the LDS) the staged shape's
    // registers cost no occupancy: longer lines run it, output tile by
    // output tile (faster than the register path on lines of 300-330)
    if (T.n > line_max<LINES>()) {
      SmemBf<1, 2, 32>& sb = *reinterpret_cast<SmemBf<1, 2, 32>*>(smem);
      for (int t0 = 0; t0 < T.n; t0 += 64) {
        GemmTile t = tile;
        t.t0 = t0;
        if (T.s_stride == 1)
          gemm_bf16x3_dir<1, 2, 32, 1, true>(T, t, ops, sb);
        else
          gemm_bf16x3_dir<1, 2, 32, 1, false>(T, t, ops, sb);
        __syncthreads();  // the next output tile restages the LDS buffers
      }
      return;
    }
  }
  SmemLine<LINES>& sm = *reinterpret_cast<SmemLine<LINES>*>(smem);
  if (T.s_stride == 1)
    gemm_bf16x3_line_dir<LINES, true>(T, tile, ops, sm);
  else
    gemm_bf16x3_line_dir<LINES, false>(T, tile, ops, sm);
}

// Split BF16 x6: three parts per value, six products (about FP32 accuracy
// from BF16 matrix cores); one output block of 64 per tile (LDS).
__global__ __launch_bounds__(256) void k_gemm_bf16x6(const GemmTask* __restrict__ tasks,
                                                     const GemmTile* __restrict__ tiles, OpTables ops) {
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  gemm_bf16x3<1, 3>(tasks, tile, ops);
}

template <int TB, int KC = 32, int PF = 1>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(const GemmTask* __restrict__ tasks,
                                                     const GemmTile* __restrict__ tiles, OpTables ops) {
  const GemmTile tile = tiles[blockIdx.x];
  if (tile_idle(tile)) return;
  gemm_bf16x3<TB, 2, KC, PF>(tasks, tile, ops);
}

template <int TB>
__global__ __launch_bounds__(256) void k_gemm_bf16x3_persist(const GemmTask* __restrict__ tasks,
                                                             const GemmTile* __restrict__ tiles, int ntiles,
                                                             OpTables ops, int* ctr) {
  xcd_queue_tiles(ntiles, ctr, [&](int t) {
    const GemmTile tile = tiles[t];
    if (!tile_idle(tile)) gemm_bf16x3<TB>(tasks, tile, ops);
  });
}

// Resident workgroups of a kernel on the current device (cached per kernel
// and device).
template <typename K>
int device_slots(K kernel) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess)
    return 0;
  const int slots = std::max(1, cus * per_cu);
  cache[key] = slots;
  return slots;
}

template <typename K, typename... Args>
hipError_t launch_persist(K kernel, int ntiles, hipStream_t stream, Args... args) {
  // a multiple of 8 workgroups (one set per XCD queue), at most one per
  // resident slot and per tile
  const int slots = device_slots(kernel) / 8 * 8;
  if (slots <= 0 || ntiles % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kernel, dim3(std::min(ntiles, slots)), dim3(256), 0, stream, args...);
  return hipGetLastError();
}

uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
float host_bf16_to_f(uint16_t h) {
  uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace

int OpPack::add(int len, int k) {
  for (size_t q = 0; q < n.size(); ++q)
    if (n[q] == len && kind[q] == k) return static_cast<int>(q);
  n.push_back(len);
  kind.push_back(k);
  ld.push_back(op_ld(len));
  off.push_back(elems);
  roff.push_back(rows);
  elems += static_cast<int64_t>(op_rows(len)) * op_ld(len);
  rows += op_rows(len);
  return static_cast<int>(n.size()) - 1;
}

bool OpPack::fill(int d, int C, std::vector<double>& f64, std::vector<double>& rowsum) const {
  f64.assign(elems, 0.0);
  rowsum.assign(rows, 0.0);
  for (size_t q = 0; q < n.size(); ++q) {
    const std::vector<double>* op = fc_operator(n[q], d, C, kind[q]);
    if (!op) return false;
    const int m = n[q];
    for (int t = 0; t < m; ++t) {
      double s = 0;
      for (int k = 0; k < m; ++k) {
        const double v = (*op)[static_cast<size_t>(t) * m + k];
        f64[off[q] + static_cast<int64_t>(t) * ld[q] + k] = v;
        s += v;
      }
      rowsum[roff[q] + t] = s;
    }
  }
  return true;
}

void split_bf16x3(const std::vector<double>& x, std::vector<uint16_t>& hi, std::vector<uint16_t>& mid,
                  std::vector<uint16_t>& lo) {
  hi.resize(x.size());
  mid.resize(x.size());
  lo.resize(x.size());
  for (size_t q = 0; q < x.size(); ++q) {
    const float f = static_cast<float>(x[q]);
    hi[q] = host_bf16(f);
    const float r = f - host_bf16_to_f(hi[q]);
    mid[q] = host_bf16(r);
    lo[q] = host_bf16(r - host_bf16_to_f(mid[q]));
  }
}

void split_bf16(const std::vector<double>& x, std::vector<uint16_t>& hi, std::vector<uint16_t>& lo) {
  hi.resize(x.size());
  lo.resize(x.size());
  for (size_t q = 0; q < x.size(); ++q) {
    const float f = static_cast<float>(x[q]);
    hi[q] = host_bf16(f);
    lo[q] = host_bf16(f - host_bf16_to_f(hi[q]));
  }
}

hipError_t launch_gemm_step(const GemmTask* tasks, const GemmTile* tiles, int ntiles, const OpTables& ops,
                            hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_step, dim3(ntiles), dim3(256), 0, stream, tasks, tiles, ops);
  return hipGetLastError();
}

hipError_t launch_gemm(int precision, const GemmVariant& v, const GemmTask* tasks, const GemmTile* tiles,
                       int ntiles, const OpTables& ops, int* counters, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  if (v.persist) {
    if (!counters) return hipErrorInvalidValue;
#define FCS_PFP(E, KC, TB) \
  return launch_persist(k_gemm_fp_persist<E, KC, TB>, ntiles, stream, tasks, tiles, ntiles, ops, counters)
    if (precision == 0) {
      if (v.tb == 2) FCS_PFP(double, 16, 2);
      FCS_PFP(double, 16, 1);
    }
    if (precision == 1) {
      if (v.kc == 32) {
        if (v.tb == 2) FCS_PFP(float, 32, 2);
        FCS_PFP(float, 32, 1);
      }
      if (v.tb == 2) FCS_PFP(float, 16, 2);
      FCS_PFP(float, 16, 1);
    }
#undef FCS_PFP
    if (v.tb == 2) return launch_persist(k_gemm_bf16x3_persist<2>, ntiles, stream, tasks, tiles, ntiles, ops, counters);
    return launch_persist(k_gemm_bf16x3_persist<1>, ntiles, stream, tasks, tiles, ntiles, ops, counters);
  }
  dim3 grid(ntiles), block(256);
  if (v.xw) {
    if (precision == 0) {
      if (v.tb == 4) hipLaunchKernelGGL((k_gemm_xw<double, 64, 4>), grid, block, 0, stream, tasks, tiles, ops);
      else hipLaunchKernelGGL((k_gemm_xw<double, 64, 2>), grid, block, 0, stream, tasks, tiles, ops);
    } else if (precision == 1) {
      if (v.tb == 4) hipLaunchKernelGGL((k_gemm_xw<float, 128, 4>), grid, block, 0, stream, tasks, tiles, ops);
      else hipLaunchKernelGGL((k_gemm_xw<float, 128, 2>), grid, block, 0, stream, tasks, tiles, ops);
    } else {
      if (v.tb == 4) hipLaunchKernelGGL((k_gemm_xw_bf16x3<128, 4>), grid, block, 0, stream, tasks, tiles, ops);
      else hipLaunchKernelGGL((k_gemm_xw_bf16x3<128, 2>), grid, block, 0, stream, tasks, tiles, ops);
    }
    return hipGetLastError();
  }
  if (v.xs) {
#define FCS_XS(E, KC, TB) hipLaunchKernelGGL((k_gemm_xs<E, KC, TB>), grid, block, 0, stream, tasks, tiles, ops)
    if (precision == 0) {
      if (v.tb == 4) FCS_XS(double, 16, 4);
      else FCS_XS(double, 16, 2);
    } else if (precision == 1) {
      if (v.kc == 32) {
        if (v.tb == 4) FCS_XS(float, 32, 4);
        else FCS_XS(float, 32, 2);
      } else {
        if (v.tb == 4) FCS_XS(float, 16, 4);
        else FCS_XS(float, 16, 2);
      }
    } else {
      return hipErrorInvalidValue;
    }
#undef FCS_XS
    return hipGetLastError();
  }
  // staged kernel instances (element, chunk, tb, workgroups per CU, prefetch)
#define FCS_FP(E, KC, TB, MB, PF)                                                               \
  if (v.kc == KC && v.tb == TB && v.minb == MB && v.pf == PF) {                                \
    hipLaunchKernelGGL((k_gemm_fp<E, KC, TB, MB, PF>), grid, block, 0, stream, tasks, tiles, ops); \
    return hipGetLastError();                                                                   \
  }
  if (precision == 0) {
    // FP64 chunks of 8 or 16 columns: 32 would exceed 64 KiB of static LDS
    FCS_FP(double, 16, 1, 4, 1)
    FCS_FP(double, 16, 2, 4, 1)
    FCS_FP(double, 8, 1, 7, 1)
    FCS_FP(double, 16, 1, 3, 2)
    FCS_FP(double, 8, 1, 4, 2)
    return hipErrorInvalidValue;
  }
  if (precision == 1) {
    FCS_FP(float, 16, 1, 4, 1)
    FCS_FP(float, 16, 2, 4, 1)
    FCS_FP(float, 32, 1, 4, 1)
    FCS_FP(float, 32, 2, 4, 1)
    FCS_FP(float, 16, 1, 4, 2)
    FCS_FP(float, 16, 1, 7, 1)
    return hipErrorInvalidValue;
  }
  if (precision == 3) {
    hipLaunchKernelGGL(k_gemm_bf16x6, grid, block, 0, stream, tasks, tiles, ops);
  } else if (v.line) {
    if (v.lines == 32)
      hipLaunchKernelGGL(k_gemm_bf16x3_line<32>, grid, block, 0, stream, tasks, tiles, ops);
    else
      hipLaunchKernelGGL(k_gemm_bf16x3_line<64>, grid, block, 0, stream, tasks, tiles, ops);
  } else if (v.kc == 64) {
    hipLaunchKernelGGL((k_gemm_bf16x3<1, 64, 1>), grid, block, 0, stream, tasks, tiles, ops);
  } else if (v.tb == 2) {
    if (v.pf == 2)
      hipLaunchKernelGGL((k_gemm_bf16x3<2, 32, 2>), grid, block, 0, stream, tasks, tiles, ops);
    else
      hipLaunchKernelGGL((k_gemm_bf16x3<2>), grid, block, 0, stream, tasks, tiles, ops);
  } else {
    if (v.pf == 2)
      hipLaunchKernelGGL((k_gemm_bf16x3<1, 32, 2>), grid, block, 0, stream, tasks, tiles, ops);
    else
      hipLaunchKernelGGL((k_gemm_bf16x3<1>), grid, block, 0, stream, tasks, tiles, ops);
  }
#undef FCS_FP
  return hipGetLastError();
}

int gemm_lines_per_tile() { return kLB; }
int gemm_outputs_per_tile(const GemmVariant& v) {
  // the line-stationary shape covers every output of its lines in one tile
  return v.line ? (1 << 24) : 64 * (v.tb == 4 ? 4 : (v.tb == 2 ? 2 : 1));
}

const GemmVariant* gemm_variants(int precision, int* count) {
  // {tb, kc, persist, xs, xw, pf, minb}
  static const GemmVariant f64[] = {{1, 16, false, false, false}, {2, 16, false, false, false},
                                    {1, 16, true, false, false},  {2, 16, true, false, false},
                                    {2, 16, false, true, false},  {4, 16, false, true, false},
                                    {2, 16, false, false, true},  {4, 16, false, false, true},
                                    {1, 8, false, false, false, 1, 7}, {1, 16, false, false, false, 2, 3},
                                    {1, 8, false, false, false, 2, 4}};
  static const GemmVariant f32[] = {{1, 16, false, false, false}, {2, 16, false, false, false},
                                    {1, 32, false, false, false}, {1, 16, true, false, false},
                                    {1, 32, true, false, false},  {2, 16, false, true, false},
                                    {4, 16, false, true, false},  {2, 32, false, true, false},
                                    {4, 32, false, true, false},  {2, 16, false, false, true},
                                    {4, 16, false, false, true},  {1, 16, false, false, false, 2, 4},
                                    {1, 16, false, false, false, 1, 7}};
  static const GemmVariant bf[] = {{1, 32, false, false, false}, {2, 32, false, false, false},
                                   {1, 32, true, false, false},  {2, 32, true, false, false},
                                   {2, 32, false, false, true},  {4, 32, false, false, true},
                                   {1, 32, false, false, false, 2}, {1, 64, false, false, false},
                                   {2, 32, false, false, false, 2}, {1, 32, false, false, false, 1, 4, true},
                                   {1, 32, false, false, false, 1, 4, true, 32}};
  static const GemmVariant bf6[] = {{1, 32, false, false, false}};
  *count = precision == 0 ? 11 : (precision == 1 ? 13 : (precision == 2 ? 11 : 1));
  return precision == 0 ? f64 : (precision == 1 ? f32 : (precision == 2 ? bf : bf6));
}

void gemm_build_tiles(const GemmVariant& v, const int32_t* n, const int32_t* nlines, size_t ntasks,
                      std::vector<GemmTile>& tiles, const uint8_t* late) {
  tiles.clear();
  const int step = gemm_outputs_per_tile(v);
  const int lpt = v.lines;  // lines per tile
  // Workgroups are dispatched round-robin over the 8 XCDs, each with its own
  // L2.  Every task (one operator) is given to one XCD, balancing the work,
  // and the per-XCD queues are interleaved so that tile i runs on XCD i mod 8:
  // a task's operator rows and operand lines are then fetched into one L2
  // only (the output tiles of a 64-line block re-read its lines from there).
  // Short queues are padded with empty tiles.
  // A queue that fits in about two rounds of the XCD's resident workgroups
  // (at most 8 per CU on its 32 CUs) runs longest tile first (cost ~
  // operator depth x outputs of the tile), in snake order over bands of 32:
  // the dispatcher hands consecutive workgroups of an XCD to different CUs,
  // so every CU receives a mix of long and short tiles and the short ones
  // fill the last round.  Longer queues keep each task's tiles together,
  // which keeps its operator rows and operand lines in L2 while they run.
  // Tasks marked late (tiles that a launch may skip) are balanced over the
  // queues on their own and follow all other tiles of their queue, so the
  // tiles that always run are dispatched first and spread evenly over the
  // CUs whatever the skipped set.
  constexpr int kXcd = 8;
  constexpr int kCusPerXcd = 32;
  std::vector<std::vector<GemmTile>> queue[2] = {std::vector<std::vector<GemmTile>>(kXcd),
                                                 std::vector<std::vector<GemmTile>>(kXcd)};
  std::vector<double> load[2] = {std::vector<double>(kXcd, 0.0), std::vector<double>(kXcd, 0.0)};
  // tasks go to the least-loaded queue of their class (heaviest first when
  // the queues will be sorted, in task order otherwise); each queue keeps
  // its tasks in task order
  constexpr size_t kSortedQueue = 2 * 8 * kCusPerXcd;
  auto task_load = [&](size_t q) { return static_cast<double>((nlines[q] + lpt - 1) / lpt) * n[q] * n[q]; };
  auto cls = [&](size_t q) { return late && late[q] ? 1 : 0; };
  size_t total = 0;
  for (size_t q = 0; q < ntasks; ++q)
    total += static_cast<size_t>((nlines[q] + lpt - 1) / lpt) * ((n[q] + step - 1) / step);
  std::vector<size_t> order(ntasks);
  for (size_t q = 0; q < ntasks; ++q) order[q] = q;
  if (total <= kXcd * kSortedQueue)
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return task_load(a) > task_load(b); });
  std::vector<int> task_queue(ntasks, 0);
  for (size_t q : order) {
    std::vector<double>& ld = load[cls(q)];
    const int x = static_cast<int>(std::min_element(ld.begin(), ld.end()) - ld.begin());
    task_queue[q] = x;
    ld[x] += task_load(q);
  }
  for (size_t q = 0; q < ntasks; ++q) {
    const int nblk = (nlines[q] + lpt - 1) / lpt;
    for (int b = 0; b < nblk; ++b)
      for (int t0 = 0; t0 < n[q]; t0 += step)
        queue[cls(q)][task_queue[q]].push_back({static_cast<int32_t>(q), b * lpt, t0, 0});
  }
  auto cost = [&](const GemmTile& t) { return n[t.task] * std::min(step, n[t.task] - t.t0); };
  size_t len = 0;
  std::vector<std::vector<GemmTile>> merged(kXcd);
  for (int x = 0; x < kXcd; ++x) {
    const size_t qlen = queue[0][x].size() + queue[1][x].size();
    for (auto& part : queue) {
      std::vector<GemmTile>& qx = part[x];
      // (the line-stationary shape has one tile per line block and shares
      // nothing but operator rows between a task's tiles: always sorted)
      if (v.persist || v.line || qlen <= kSortedQueue) {
        std::stable_sort(qx.begin(), qx.end(),
                         [&](const GemmTile& a, const GemmTile& b) { return cost(a) > cost(b); });
        // snake order: every other band of one tile per CU reversed, so that
        // the CU that receives a band's largest tile receives the next
        // band's smallest
        if (!v.persist)
          for (size_t b0 = kCusPerXcd; b0 < qx.size(); b0 += 2 * kCusPerXcd)
            std::reverse(qx.begin() + b0, qx.begin() + std::min(qx.size(), b0 + kCusPerXcd));
      }
      merged[x].insert(merged[x].end(), qx.begin(), qx.end());
    }
    len = std::max(len, merged[x].size());
  }
  for (size_t r = 0; r < len; ++r)
    for (int x = 0; x < kXcd; ++x) tiles.push_back(r < merged[x].size() ? merged[x][r] : GemmTile{-1, 0, 0, 0});
}

}  // namespace fcs
