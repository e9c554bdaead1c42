// Device-side data structures shared by the HIP kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fcs {

// One set of lines that share a line length, run position and operator:
// out[line][t] = sum_s Op[t][s] in[line][s].  line = c * nrow + r addresses
// element base + c * comp_stride + r * row_stride + s * s_stride.
struct GemmTask {
  const double* src;
  double* dst;
  int64_t comp_stride;
  int32_t row_stride, s_stride;
  int32_t nrow, ncomp;
  int32_t n;       // line length = operator size
  int32_t op;      // operator index (into the operator tables)
};

struct GemmTile {
  int32_t task, line0, t0, pad;
};

// Operator tables: FP64, FP32 and split BF16 copies of every dense operator,
// and FP64 row sums (used to take the line offset out of the split-BF16
// products exactly).
struct OpTables {
  const int64_t* off;       // element offset of operator k (n*n elements)
  const double* f64;
  const float* f32;
  const uint16_t* bhi;
  const uint16_t* blo;
  const double* rowsum;     // offset off[k] / n ... (n entries at roff[k])
  const int64_t* roff;
};

struct PatchDev {
  int64_t offset;
  int32_t n1, n2;
  int32_t row_run;  // index of row 0 in the run tables
  int32_t col_run;  // index of column 0
  int32_t affine;
  int32_t pad;
};

// Per-point flags.
enum : uint8_t { kActive = 1, kFringe = 2, kXFringe = 4, kAffine = 8 };

struct SlipEntry {
  int64_t k;
  double nx, ny;
  int32_t corner;
  int32_t pad;
};

struct DirichletEntry {
  int64_t k;
  double e[4];
};

struct ExactEntry {
  int64_t k;
  double x, y;
};

}  // namespace fcs
