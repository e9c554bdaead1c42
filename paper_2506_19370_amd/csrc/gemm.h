// Launch interface of the grouped FC contraction kernels.
#pragma once
#include "kernels.h"

namespace fcs {
// precision: 0 FP64, 1 FP32, 2 split BF16 (see gemm.hip).
hipError_t launch_gemm(int precision, const GemmTask* tasks, const GemmTile* tiles, int ntiles,
                       const OpTables& ops, hipStream_t stream);
}  // namespace fcs
