// Smoothness classification of arbitrary batches of 16-point windows
// (Sec. 4, Alg. 3): the SDNN on the matrix cores (16 windows per wave and
// round) and the modal-decay fallback (one window per thread).
#include "window_kernels.h"

#include <algorithm>

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

// Grid-stride form: every workgroup packs the fragment table into LDS once
// and its waves walk rounds of 16 windows (round r covers windows 16 r ..
// 16 r + 15), fetching the next round's values while the current one is on
// the matrix cores.
constexpr int kWindowBlocks = 2048;

__global__ __launch_bounds__(256) void k_classify_sdnn_windows(const float* __restrict__ params,
                                                               const double* __restrict__ windows, int64_t nwin,
                                                               uint8_t* __restrict__ tau, float* __restrict__ logits) {
  __shared__ __attribute__((aligned(16))) uint32_t table[64 * kSdnnFragWords];
  build_sdnn_table(params, table);
  SdnnFrag F;
  load_sdnn_frag(table, F);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t nround = (nwin + 15) / 16;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * 4;
  auto fetch = [&](int64_t r, double (&v)[4]) {
    const int64_t w = 16 * r + c;
    const bool in = r < nround && w < nwin;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = in ? windows[w * 16 + 4 * g + j] : 0.0;
  };
  int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);  // the same for all lanes of a wave
  double vc[4];
  fetch(r, vc);
#pragma unroll 1
  for (; r < nround; r += nwaves) {
    double vn[4];
    fetch(r + nwaves, vn);
    const int64_t w = 16 * r + c;
    float x[4], z[3];
    const bool live = sdnn_features(vc, x);
    sdnn_mfma(F, x, z);  // all 64 lanes take part
    if (g == 0 && w < nwin) {
      tau[w] = static_cast<uint8_t>(live ? sdnn_argmax(z) : 0);
      if (logits)
        for (int o = 0; o < 3; ++o) logits[w * 3 + o] = live ? z[o] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) vc[j] = vn[j];
  }
}

}  // namespace

hipError_t launch_classify_windows(int mode, const float* params, const ModalBasis& basis, const double* windows,
                                   int64_t nwin, uint8_t* tau, float* logits, hipStream_t s) {
  if (nwin <= 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>((nwin + 255) / 256));
  if (mode == 2) {
    const int64_t nround = (nwin + 15) / 16;
    const dim3 sgrid(static_cast<unsigned>(std::min<int64_t>((nround + 3) / 4, kWindowBlocks)));
    hipLaunchKernelGGL(k_classify_sdnn_windows, sgrid, dim3(256), 0, s, params, windows, nwin, tau, logits);
  } else
    hipLaunchKernelGGL(k_classify_modal, grid, dim3(256), 0, s, basis, windows, nwin, tau);
  return hipGetLastError();
}

}  // namespace fcs
