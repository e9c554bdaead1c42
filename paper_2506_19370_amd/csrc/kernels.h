// Device-side data structures shared by the HIP kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fcs {

// One set of lines that share a line length, run position and operator:
// out[line][t] = sum_s Op[t][s] in[line][s].  Lines are numbered with the
// row fastest: line = c * nrow + r addresses element
// base + c * comp_stride + r * row_stride + s * s_stride, so that along q^2
// (row_stride 1) neighbouring lines are neighbouring doubles.
struct GemmTask {
  const double* src;
  void* dst;        // double, or float when out_f32
  int64_t comp_stride;
  int32_t row_stride, s_stride;
  int32_t nrow, ncomp;
  int32_t n;        // line length = operator size
  int32_t op;       // operator index (into the operator tables)
  int32_t out_f32;  // results stored as FP32 (mixed-precision stage derivatives)
  // Viscous derivatives on a lattice subpatch: entry of row 0 in the
  // per-line activity flags (row r at act + r); -1 for tasks always computed.
  int32_t act;
};

// skip: bit w set when none of the tile's lines 16 w .. 16 w + 15 is needed
// in the current step; all four bits: the tile is not needed at all
// (written on the device from the line activity flags; 0 from the host).
struct GemmTile {
  int32_t task, line0, t0, skip;
};


// Operator tables: FP64, FP32 and split BF16 copies of every dense operator
// (zero-padded, row-major with leading dimension ld[k]), and FP64 row sums
// (used to take the line offset out of the split-BF16 products exactly).
struct OpTables {
  const int64_t* off;       // element offset of operator k
  const int32_t* ld;        // leading dimension of operator k
  const double* f64;
  const float* f32;
  const uint16_t* bhi;
  const uint16_t* blo;      // split BF16: the second part (x3) or the third (x6)
  const uint16_t* bmid;     // split BF16 x6: the second part (else null)
  const double* rowsum;     // row sums of operator k at roff[k]
  const int64_t* roff;
};

struct PatchDev {
  int64_t offset;
  int32_t n1, n2;
  int32_t row_run;  // index of row 0 in the run tables
  int32_t col_run;  // index of column 0
  int32_t affine;
  // lattice subpatch with skippable viscous lines: activity flag of row j at
  // act_row + j and of column i at act_col + i; -1 otherwise
  int32_t act_row, act_col;
  int32_t pad;
  // affine subpatches: the metric terms, the same at every active point
  // (q^k_x, q^k_y and g^{kl}; the Laplacian terms of the index coordinates
  // vanish)
  double t1x, t1y, t2x, t2y, g11, g12, g22;
};

// Per-point flags.
enum : uint8_t { kActive = 1, kFringe = 2, kXFringe = 4, kAffine = 8, kBoundary = 16 };

// Boundary conditions of one point (Sec. 5 item 4): slip (zero normal
// momentum, pressure kept; both momentum components zero at a corner of two
// slip sides), then Dirichlet data (inflow state or exact vortex).
struct BcEntry {
  int64_t k;
  double nx, ny;
  int32_t slip;      // 0 none, 1 projection, 2 corner
  int32_t dirichlet; // 0 none, 1 fixed state e[], 2 exact vortex at (x, y)
  double e[4];
  double x, y;
};

// Viscosity blend rows in factored form (see BlendTerm on the host): row q
// is wself * u(dst) + sum over its terms [t0, t1) of
// scale * sum_b wj[b] sum_a wi[a] u(base + b * stride + a).
struct BlendRowDev {
  int64_t dst;
  double wself;
  int32_t t0, t1;
};
struct BlendTermDev {
  int64_t base;
  int32_t stride, ni, nj, pad;
  double scale;
  double wi[6], wj[6];
};

// A grid line that ends at one or two no-slip adiabatic wall nodes: the
// wall values of theta make the FC first derivative along it vanish there
// (both ends together when both are walls).
struct WallLine {
  int64_t first;   // global index of the line's first point
  int64_t stride;  // index step along the line (1 or n1)
  int32_t n;       // points on the line
  int32_t op;      // its first-derivative operator
  int32_t pos[2];  // positions of the wall nodes on the line (pos[1] < 0: one)
  int32_t keep[2]; // 1: the node keeps its Dirichlet data (solved, not written)
  int32_t pad;
};

}  // namespace fcs
