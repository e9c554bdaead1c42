// Operator-stationary grouped FC contraction (same product as gemm.hip:
// Y[line][t] = sum_s Op[t][s] X[line][s] for all lines of all tasks).
//
// A workgroup copies the rows [t0, t0 + TT) of its task's operator into LDS
// once and then streams `group` blocks of 64 lines through it with no
// further barrier: wave w owns lines 16 w .. 16 w + 15 of each block; lane
// l holds line 16 w + (l & 15) and, in k-step q, the KL consecutive
// positions 16 q... (KL = 4: positions KS q + 4 (l >> 4) + j of a 16-wide
// step for the 16x16x4 MFMAs; KL = 8 of a 32-wide step for the BF16
// 16x16x32 MFMA).  The same permuted order is used for the operator, so a
// lane reads contiguous elements of its own line from global memory, one
// step ahead of the matrix-core work.  Output roles as in gemm.hip; the
// destination of another lane's line comes through a cross-lane shuffle.
#include <algorithm>

#include "gemm.h"

namespace fcs {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) {
  int lo = __shfl(static_cast<int>(v & 0xffffffff), src);
  int hi = __shfl(static_cast<int>(v >> 32), src);
  return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}

struct LineAddr {
  int64_t src = -1, dst = -1;
  int comp = 0;
};

__device__ __forceinline__ LineAddr line_addr(const GemmTask& T, int line, int nlines) {
  LineAddr a;
  if (line < nlines) {
    int r = line / T.ncomp, c = line - r * T.ncomp;
    int64_t rb = static_cast<int64_t>(r) * T.row_stride;
    a.src = T.flux ? rb : rb + c * T.comp_stride;
    a.dst = rb + c * T.comp_stride;
    a.comp = c;
  }
  return a;
}

// KL consecutive operand values of a line (plain operands only: tasks whose
// operand is computed from the state are not scheduled on these kernels).
template <int KL>
struct Raw {
  double v[KL];
  __device__ __forceinline__ void load(const GemmTask& T, const LineAddr& a, int s0, int n) {
#pragma unroll
    for (int j = 0; j < KL; ++j) {
      const int s = s0 + j;
      v[j] = (a.src >= 0 && s < n) ? T.src[a.src + static_cast<int64_t>(s) * T.s_stride] : 0.0;
    }
  }
  __device__ __forceinline__ double value(const GemmTask&, int, int j) const { return v[j]; }
};

// Tile fields: line0 = first line, t0 = first output; pad = nblocks | TT << 16.
template <typename Elem, int NB>
__global__ __launch_bounds__(256) void k_gemm_os(const GemmTask* __restrict__ tasks,
                                                 const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr bool kF64 = sizeof(Elem) == 8;
  constexpr int KS = 16, KL = 4;
  typedef Elem vec4 __attribute__((ext_vector_type(4)));
  extern __shared__ __align__(16) unsigned char smem[];
  Elem* Ds = reinterpret_cast<Elem*>(smem);
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0;
  const int nblk = tile.pad & 0xffff, TT = tile.pad >> 16, nt = min(TT, n - t0);
  const int kpad = (n + KS - 1) / KS * KS, pitch = kpad + 1;
  const Elem* __restrict__ D;
  if constexpr (kF64)
    D = ops.f64 + ops.off[T.op];
  else
    D = ops.f32 + ops.off[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, rr = lane & 15, g = lane >> 4;
  const bool q1 = T.s_stride == 1;
  // operator rows t0 .. t0 + nt, zero padded to kpad columns
  for (int e = tid; e < nt * kpad; e += 256) {
    const int t = e / kpad, s = e - t * kpad;
    Ds[t * pitch + s] = s < n ? D[static_cast<int64_t>(t0 + t) * n + s] : Elem(0);
  }
  __syncthreads();
  const int nsteps = kpad / KS;
  for (int blk = 0; blk < nblk; ++blk) {
    const int line = tile.line0 + 64 * blk + 16 * wave + rr;
    const LineAddr a = line_addr(T, line, nlines);
    vec4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = vec4{0, 0, 0, 0};
    // three-deep ring: the loads of step q + 2 are issued before the
    // matrix-core work of step q
    auto step = [&](const Raw<KL>& x, int q) {
      Elem xv[KL];
#pragma unroll
      for (int j = 0; j < KL; ++j) xv[j] = static_cast<Elem>(x.v[j]);
#pragma unroll
      for (int j = 0; j < KL; ++j) {
        const Elem* drow = Ds + rr * pitch + KS * q + KL * g + j;
#pragma unroll
        for (int tb = 0; tb < NB; ++tb) {
          if (16 * tb >= nt) break;
          const Elem da = drow[16 * tb * pitch];
          if constexpr (kF64)
            acc[tb] = q1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(xv[j], da, acc[tb], 0, 0, 0)
                         : __builtin_amdgcn_mfma_f64_16x16x4f64(da, xv[j], acc[tb], 0, 0, 0);
          else
            acc[tb] = q1 ? __builtin_amdgcn_mfma_f32_16x16x4f32(xv[j], da, acc[tb], 0, 0, 0)
                         : __builtin_amdgcn_mfma_f32_16x16x4f32(da, xv[j], acc[tb], 0, 0, 0);
        }
      }
    };
    Raw<KL> r0, r1, r2;
    r0.load(T, a, KL * g, n);
    if (nsteps > 1) r1.load(T, a, KS + KL * g, n);
    for (int q = 0; q < nsteps; q += 3) {
      if (q + 2 < nsteps) r2.load(T, a, KS * (q + 2) + KL * g, n);
      step(r0, q);
      if (q + 1 >= nsteps) break;
      if (q + 3 < nsteps) r0.load(T, a, KS * (q + 3) + KL * g, n);
      step(r1, q + 1);
      if (q + 2 >= nsteps) break;
      if (q + 4 < nsteps) r1.load(T, a, KS * (q + 4) + KL * g, n);
      step(r2, q + 2);
    }
    // store: along q^1 the MFMA rows are lines (other lanes' lines), along
    // q^2 they are outputs
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = kF64 ? g + 4 * r : 4 * g + r;
      const int64_t drow = shfl64(a.dst, 16 * (lane >> 6) + row);  // lane `row` of this wave
      for (int tb = 0; tb < NB; ++tb) {
        if (16 * tb >= nt) break;
        int tloc;
        int64_t base;
        if (q1) {
          tloc = 16 * tb + rr;
          base = drow;
        } else {
          tloc = 16 * tb + row;
          base = a.dst;
        }
        if (tloc >= nt || base < 0) continue;
        T.dst[base + static_cast<int64_t>(t0 + tloc) * T.s_stride] = static_cast<double>(acc[tb][r]);
      }
    }
  }
}

template <int NB>
__global__ __launch_bounds__(256) void k_gemm_os_bf16x3(const GemmTask* __restrict__ tasks,
                                                        const GemmTile* __restrict__ tiles, OpTables ops) {
  constexpr int KS = 32, KL = 8;
  extern __shared__ __align__(16) unsigned char smem[];
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask T = tasks[tile.task];
  const int n = T.n, nlines = T.nrow * T.ncomp, t0 = tile.t0;
  const int nblk = tile.pad & 0xffff, TT = tile.pad >> 16, nt = min(TT, n - t0);
  const int kpad = (n + KS - 1) / KS * KS, pitch = kpad + 8;  // halves; rows 16-byte aligned
  uint16_t* Dh = reinterpret_cast<uint16_t*>(smem);
  uint16_t* Dl = Dh + static_cast<size_t>(TT) * pitch;
  const uint16_t* __restrict__ Bh = ops.bhi + ops.off[T.op];
  const uint16_t* __restrict__ Bl = ops.blo + ops.off[T.op];
  const double* __restrict__ rowsum = ops.rowsum + ops.roff[T.op];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, rr = lane & 15, g = lane >> 4;
  const bool q1 = T.s_stride == 1;
  for (int e = tid; e < nt * kpad; e += 256) {
    const int t = e / kpad, s = e - t * kpad;
    const bool in = s < n;
    const int64_t o = static_cast<int64_t>(t0 + t) * n + s;
    Dh[t * pitch + s] = in ? Bh[o] : 0;
    Dl[t * pitch + s] = in ? Bl[o] : 0;
  }
  __syncthreads();
  const int nsteps = kpad / KS;
  for (int blk = 0; blk < nblk; ++blk) {
    const int line = tile.line0 + 64 * blk + 16 * wave + rr;
    const LineAddr a = line_addr(T, line, nlines);
    double x0 = 0.0;
    {
      Raw<1> f;
      f.load(T, a, 0, n);
      x0 = a.src >= 0 ? f.value(T, a.comp, 0) : 0.0;
    }
    f32x4 am[NB], ac[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) am[b] = ac[b] = f32x4{0, 0, 0, 0};
    auto step = [&](const Raw<KL>& x, int q) {
      bf16x8 xh, xl;
#pragma unroll
      for (int j = 0; j < KL; ++j) {
        const bool in = a.src >= 0 && KS * q + KL * g + j < n;
        const float f = in ? static_cast<float>(x.v[j] - x0) : 0.0f;
        const uint16_t h = f2bf(f);
        xh[j] = __builtin_bit_cast(__bf16, h);
        xl[j] = __builtin_bit_cast(__bf16, f2bf(f - bf2f(h)));
      }
      const int koff = KS * q + KL * g;
#pragma unroll
      for (int tb = 0; tb < NB; ++tb) {
        if (16 * tb >= nt) break;
        const int row = (16 * tb + rr) * pitch + koff;
        const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(Dh + row));
        const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(Dl + row));
        if (q1) {
          am[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bh, am[tb], 0, 0, 0);
          ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bl, ac[tb], 0, 0, 0);
          ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, bh, ac[tb], 0, 0, 0);
        } else {
          am[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, xh, am[tb], 0, 0, 0);
          ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, xl, ac[tb], 0, 0, 0);
          ac[tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, xh, ac[tb], 0, 0, 0);
        }
      }
    };
    Raw<KL> r0, r1, r2;
    r0.load(T, a, KL * g, n);
    if (nsteps > 1) r1.load(T, a, KS + KL * g, n);
    for (int q = 0; q < nsteps; q += 3) {
      if (q + 2 < nsteps) r2.load(T, a, KS * (q + 2) + KL * g, n);
      step(r0, q);
      if (q + 1 >= nsteps) break;
      if (q + 3 < nsteps) r0.load(T, a, KS * (q + 3) + KL * g, n);
      step(r1, q + 1);
      if (q + 2 >= nsteps) break;
      if (q + 4 < nsteps) r1.load(T, a, KS * (q + 4) + KL * g, n);
      step(r2, q + 2);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * g + r;
      const int64_t drow = shfl64(a.dst, row);
      const double x0row = __shfl(x0, row);
      for (int tb = 0; tb < NB; ++tb) {
        if (16 * tb >= nt) break;
        int tloc;
        int64_t base;
        double off;
        if (q1) {
          tloc = 16 * tb + rr;
          base = drow;
          off = x0row;
        } else {
          tloc = 16 * tb + row;
          base = a.dst;
          off = x0;
        }
        if (tloc >= nt || base < 0) continue;
        const double v = static_cast<double>(am[tb][r]) + static_cast<double>(ac[tb][r]) + off * rowsum[t0 + tloc];
        T.dst[base + static_cast<int64_t>(t0 + tloc) * T.s_stride] = v;
      }
    }
  }
}

}  // namespace

int gemm_os_rows(int precision, const GemmVariant& v, int n) {
  const size_t budget = static_cast<size_t>(v.lds_kb) * 1024;
  size_t row_bytes;
  if (precision == 2) {
    const int kpad = (n + 31) / 32 * 32;
    row_bytes = 2 * 2 * static_cast<size_t>(kpad + 8);
  } else {
    const int kpad = (n + 15) / 16 * 16;
    row_bytes = (precision == 0 ? 8 : 4) * static_cast<size_t>(kpad + 1);
  }
  int tt = static_cast<int>(budget / row_bytes) / 16 * 16;
  tt = std::max(16, std::min(tt, 256));
  return std::min(tt, (n + 15) / 16 * 16);
}

hipError_t launch_gemm_os(int precision, const GemmVariant& v, const GemmTask* tasks, const GemmTile* tiles,
                          int ntiles, const OpTables& ops, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(256);
  const size_t lds = v.dyn_lds;
  // kernels that may use more than the default 64 KiB of dynamic LDS
  static bool attr_set = false;
  if (!attr_set) {
    const int maxlds = 160 * 1024;
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_os_bf16x3<8>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_os_bf16x3<16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_os<float, 8>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_os<float, 16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_os<double, 8>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_os<double, 16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    attr_set = true;
  }
  if (precision == 2) {
    if (v.nb <= 8)
      hipLaunchKernelGGL((k_gemm_os_bf16x3<8>), grid, block, lds, stream, tasks, tiles, ops);
    else
      hipLaunchKernelGGL((k_gemm_os_bf16x3<16>), grid, block, lds, stream, tasks, tiles, ops);
  } else if (precision == 1) {
    if (v.nb <= 8)
      hipLaunchKernelGGL((k_gemm_os<float, 8>), grid, block, lds, stream, tasks, tiles, ops);
    else
      hipLaunchKernelGGL((k_gemm_os<float, 16>), grid, block, lds, stream, tasks, tiles, ops);
  } else {
    if (v.nb <= 8)
      hipLaunchKernelGGL((k_gemm_os<double, 8>), grid, block, lds, stream, tasks, tiles, ops);
    else
      hipLaunchKernelGGL((k_gemm_os<double, 16>), grid, block, lds, stream, tasks, tiles, ops);
  }
  return hipGetLastError();
}

}  // namespace fcs
