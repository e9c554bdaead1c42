// Launch interface of the classifier training kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fcs {
// Floats of device workspace for a batch of B samples.
size_t sdnn_train_floats(int B);
hipError_t launch_sdnn_train(float* params, float* m, float* v, int t, float lr, const float* x,
                             const int32_t* labels, const float* cw, int B, float* loss, float* grads_out,
                             float* ws, int fp32, hipStream_t s);
}  // namespace fcs
