// Smoothness classification of arbitrary batches of 16-point windows
// (Sec. 4, Alg. 3): the SDNN on the matrix cores (16 windows per wave and
// round) and the modal-decay fallback (one window per thread).
#include "window_kernels.h"

#include "classify.h"
#include "stage_kernels.h"

namespace fcs {

namespace {

__global__ __launch_bounds__(256) void k_classify_modal(ModalBasis basis, const double* __restrict__ windows,
                                                        int64_t nwin, uint8_t* __restrict__ tau) {
  __shared__ double B[256];
  for (int q = threadIdx.x; q < 256; q += blockDim.x) B[q] = basis.v[q];
  __syncthreads();
  int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  double v[16];
  for (int m = 0; m < 16; ++m) v[m] = windows[w * 16 + m];
  tau[w] = static_cast<uint8_t>(classify_modal(v, B));
}

// 256 windows per workgroup, 64 per wave in 4 rounds of 16.
__global__ __launch_bounds__(256) void k_classify_sdnn_windows(const float* __restrict__ params,
                                                               const double* __restrict__ windows, int64_t nwin,
                                                               uint8_t* __restrict__ tau, float* __restrict__ logits) {
  __shared__ __attribute__((aligned(16))) uint32_t table[64 * kSdnnFragWords];
  build_sdnn_table(params, table);
  SdnnFrag F;
  load_sdnn_frag(table, F);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t w0 = static_cast<int64_t>(blockIdx.x) * 256 + (threadIdx.x >> 6) * 64;
#pragma unroll 1
  for (int r = 0; r < 4; ++r) {
    const int64_t w = w0 + 16 * r + c;
    const bool in = w < nwin;
    double v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = in ? windows[w * 16 + 4 * g + j] : 0.0;
    float x[4], z[3];
    const bool live = sdnn_features(v, x);
    sdnn_mfma(F, x, z);
    if (g == 0 && in) {
      tau[w] = static_cast<uint8_t>(live ? sdnn_argmax(z) : 0);
      if (logits)
        for (int o = 0; o < 3; ++o) logits[w * 3 + o] = live ? z[o] : 0.0f;
    }
  }
}

}  // namespace

hipError_t launch_classify_windows(int mode, const float* params, const ModalBasis& basis, const double* windows,
                                   int64_t nwin, uint8_t* tau, float* logits, hipStream_t s) {
  if (nwin <= 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>((nwin + 255) / 256));
  if (mode == 2)
    hipLaunchKernelGGL(k_classify_sdnn_windows, grid, dim3(256), 0, s, params, windows, nwin, tau, logits);
  else
    hipLaunchKernelGGL(k_classify_modal, grid, dim3(256), 0, s, basis, windows, nwin, tau);
  return hipGetLastError();
}

}  // namespace fcs
