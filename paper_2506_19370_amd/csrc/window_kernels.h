// Launch interface of the standalone window-classification kernels.
#pragma once
#include "kernels.h"

namespace fcs {

struct ModalBasis {
  double v[256];
};

// mode 1: modal fallback (basis), 2: SDNN (params, FCS_SDNN_NPARAM floats).
hipError_t launch_classify_windows(int mode, const float* params, const ModalBasis& basis, const double* windows,
                                   int64_t nwin, uint8_t* tau, float* logits, hipStream_t s);

void modal_basis16(double* out);

}  // namespace fcs
