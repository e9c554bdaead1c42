// Launch interface of the grouped FC contraction kernels.
#pragma once
#include <cstddef>
#include <vector>

#include "kernels.h"

namespace fcs {
// precision: 0 FP64, 1 FP32, 2 split BF16 (see gemm.hip).
// Tile shape of a contraction launch: tb 16-output blocks per wave (a
// workgroup covers 64 lines x 64 tb outputs), register prefetch on or off.
// kind 1: lines in registers (each wave owns 16 lines and nb 16-output
// blocks; the workgroup covers 64 lines x 16 nb outputs).
// kind 2: operator-stationary (the workgroup keeps an operator tile of up to
// lds_kb KiB in LDS and streams `group` 64-line blocks through it).
struct GemmVariant {
  int tb = 1;
  bool prefetch = false;
  int kind = 0;
  int nb = 4;
  int lds_kb = 64;
  int group = 4;
  size_t dyn_lds = 0;  // set by gemm_build_tiles
};
// Tiles of one task set (operator sizes n, lines nrow * ncomp per task) for
// a variant; kind 2 encodes the output range and the line-block count in
// the tile and sets v.dyn_lds.
void gemm_build_tiles(int precision, GemmVariant& v, const int32_t* n, const int32_t* nlines, size_t ntasks,
                      std::vector<GemmTile>& tiles);
hipError_t launch_gemm_os(int precision, const GemmVariant& v, const GemmTask* tasks, const GemmTile* tiles,
                          int ntiles, const OpTables& ops, hipStream_t stream);
// Output rows of an operator-stationary tile for a line length n.
int gemm_os_rows(int precision, const GemmVariant& v, int n);
hipError_t launch_gemm(int precision, const GemmVariant& v, const GemmTask* tasks, const GemmTile* tiles,
                       int ntiles, const OpTables& ops, hipStream_t stream);
int gemm_lines_per_tile();
int gemm_outputs_per_tile(const GemmVariant& v);
// Candidate variants for the autotuner.
const GemmVariant* gemm_variants(int precision, int* count);
}  // namespace fcs
