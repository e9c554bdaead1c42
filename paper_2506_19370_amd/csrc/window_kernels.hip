// Smoothness classification of arbitrary batches of 16-point windows
// (Sec. 4, Alg. 3): the SDNN and the modal-decay fallback, one window per
// thread, network parameters staged in LDS.
#include "window_kernels.h"

#include "classify.h"
#include "stage_kernels.h"

namespace fcs {

namespace {

__global__ __launch_bounds__(256) void k_classify_windows(int mode, const float* __restrict__ params, ModalBasis basis,
                                                          const double* __restrict__ windows, int64_t nwin,
                                                          uint8_t* __restrict__ tau, float* __restrict__ logits) {
  __shared__ float W[FCS_SDNN_NPARAM_DEV];
  __shared__ double B[256];
  if (mode == 2) {
    load_sdnn_params(params, W, FCS_SDNN_NPARAM_DEV);
  } else {
    for (int q = threadIdx.x; q < 256; q += blockDim.x) B[q] = basis.v[q];
  }
  __syncthreads();
  int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  double v[16];
  for (int m = 0; m < 16; ++m) v[m] = windows[w * 16 + m];
  int t;
  if (mode == 2) {
    float z[3];
    t = classify_sdnn(v, W, z);
    if (logits)
      for (int o = 0; o < 3; ++o) logits[w * 3 + o] = z[o];
  } else {
    t = classify_modal(v, B);
  }
  tau[w] = static_cast<uint8_t>(t);
}

}  // namespace

hipError_t launch_classify_windows(int mode, const float* params, const ModalBasis& basis, const double* windows,
                                   int64_t nwin, uint8_t* tau, float* logits, hipStream_t s) {
  if (nwin <= 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>((nwin + 255) / 256));
  hipLaunchKernelGGL(k_classify_windows, grid, dim3(256), 0, s, mode, params, basis, windows, nwin, tau, logits);
  return hipGetLastError();
}

}  // namespace fcs
