// Launch interface of the grouped FC contraction kernels and the host-side
// packing of their operator tables.
#pragma once
#include <cstddef>
#include <vector>

#include "kernels.h"

namespace fcs {

// Operator tables are stored zero-padded: operator k occupies
// op_rows(n) x op_ld(n) elements (row-major, leading dimension op_ld), so a
// contraction tile never tests operator bounds.  The padding is sized for the
// largest tile (256 outputs) and the deepest chunk (64 columns, split BF16).
constexpr int kOpRowPad = 256;
// Device counters (ints) that one persistent contraction launch uses.
constexpr int kGemmCounters = 16;
constexpr int kOpColPad = 64;
inline int op_ld(int n) { return (n + kOpColPad - 1) / kOpColPad * kOpColPad; }
inline int op_rows(int n) { return (n + kOpRowPad - 1) / kOpRowPad * kOpRowPad; }

// A set of distinct (length, kind) operators and their packed layout.
struct OpPack {
  std::vector<int32_t> n, kind, ld;
  std::vector<int64_t> off, roff;  // element offset of each operator, of its row sums
  int64_t elems = 0, rows = 0;
  int add(int len, int k);  // index of (len, k), appended if new
  // FP64 tables (padded operators and row sums) for FC parameters (d, C);
  // false if an operator cannot be built.
  bool fill(int d, int C, std::vector<double>& f64, std::vector<double>& rowsum) const;
};
// Round-to-nearest-even split of x (as FP32) into bf16 hi + lo.
void split_bf16(const std::vector<double>& x, std::vector<uint16_t>& hi, std::vector<uint16_t>& lo);
// Three-part split of the FP32 value: hi + mid + lo (split BF16 x6).
void split_bf16x3(const std::vector<double>& x, std::vector<uint16_t>& hi, std::vector<uint16_t>& mid,
                  std::vector<uint16_t>& lo);

// Tile shape of a contraction launch: a workgroup covers 64 lines and 64 tb
// outputs (tb = 1 or 2) and walks the operator depth in chunks of kc
// (16 or 32; the split-BF16 kernel always uses 32).
// persist: one workgroup per resident slot (a multiple of 8), each taking
// tiles of its XCD's queue from a device counter (kGemmCounters ints, zero
// before the first launch; each launch leaves them zero), every queue sorted
// longest tile first.
// xs: operand lines staged in LDS, operator rows loaded straight into MFMA
// registers (tb 2 or 4; FP64 and FP32).
// xw: operand lines staged in LDS a wide slab at a time (128 columns, 64 in
// FP64), operator rows in registers (tb 2 or 4; all precisions).
// pf: the staged kernel keeps the loads of one or two chunks in flight.
struct GemmVariant {
  int tb = 1;
  int kc = 16;
  bool persist = false;
  bool xs = false;
  bool xw = false;
  int pf = 1;    // staged kernel: chunks whose loads are in flight (1 or 2)
  int minb = 4;  // staged kernel: workgroups per CU of its launch bound
  bool line = false;  // split BF16: line-stationary (all outputs of a line tile)
  int lines = 64;     // lines per tile (the line-stationary shape: 64 or 32)
};
hipError_t launch_gemm(int precision, const GemmVariant& v, const GemmTask* tasks, const GemmTile* tiles,
                       int ntiles, const OpTables& ops, int* counters, hipStream_t stream);
// FP64 contraction with the default tile (64 lines x 64 outputs), launched
// under its own kernel name for the once-per-step phases.
hipError_t launch_gemm_step(const GemmTask* tasks, const GemmTile* tiles, int ntiles, const OpTables& ops,
                            hipStream_t stream);
int gemm_lines_per_tile();
int gemm_outputs_per_tile(const GemmVariant& v);
// Tiles of one task set (operator sizes n, lines nrow * ncomp per task).
// late (or null): tasks whose tiles a launch may skip; they are placed after
// the other tiles of each XCD queue.
void gemm_build_tiles(const GemmVariant& v, const int32_t* n, const int32_t* nlines, size_t ntasks,
                      std::vector<GemmTile>& tiles, const uint8_t* late = nullptr);
// Candidate variants for the autotuner.
const GemmVariant* gemm_variants(int precision, int* count);
}  // namespace fcs
