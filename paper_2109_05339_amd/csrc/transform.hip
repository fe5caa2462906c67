// Separable transforms between the N^3 model modes and the 2N-per-axis fine
// grid.  The zero-padded 3D FFT plus kernel deconvolution of an ES-kernel
// NUFFT is applied one axis at a time as a contraction with a small table
// W[l][k] = exp(+-2 pi i k l / nf) / psi_hat(k): padding and truncation fold
// into the table's shape, and the deconvolution into its rows.
#include "internal.h"

namespace spfel {

// Y[a][k][b] = sum_l X[a][l][b] W[l][k]; one thread per output element with
// b fastest, so reads of X are contiguous in b (or broadcast when B = 1) and
// reads of W are contiguous in k (or broadcast).
template <bool XC, int OUT>
__global__ __launch_bounds__(256) void contract_kernel(const void *__restrict__ X_,
                                                       const float2 *__restrict__ W,
                                                       void *__restrict__ Y_, int A, int L,
                                                       int K, int B) {
  const int64_t total = (int64_t)A * K * B;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int b = (int)(t % B);
  const int64_t r = t / B;
  const int k = (int)(r % K);
  const int a = (int)(r / K);
  float re = 0.f, im = 0.f;
  const int64_t xbase = (int64_t)a * L * B + b;
  if (XC) {
    const float2 *X = static_cast<const float2 *>(X_);
    for (int l = 0; l < L; ++l) {
      const float2 x = X[xbase + (int64_t)l * B];
      const float2 w = W[(int64_t)l * K + k];
      re = fmaf(x.x, w.x, re);
      re = fmaf(-x.y, w.y, re);
      im = fmaf(x.x, w.y, im);
      im = fmaf(x.y, w.x, im);
    }
  } else {
    const float *X = static_cast<const float *>(X_);
    for (int l = 0; l < L; ++l) {
      const float x = X[xbase + (int64_t)l * B];
      const float2 w = W[(int64_t)l * K + k];
      re = fmaf(x, w.x, re);
      im = fmaf(x, w.y, im);
    }
  }
  if (OUT == 0) {
    static_cast<float2 *>(Y_)[t] = make_float2(re, im);
  } else if (OUT == 1) {
    static_cast<float *>(Y_)[t] = re;
  } else if (OUT == 2) {
    static_cast<float *>(Y_)[t] += re;
  } else {
    float2 *Y = static_cast<float2 *>(Y_);
    const float2 y = Y[t];
    Y[t] = make_float2(y.x + re, y.y + im);
  }
}

hipError_t launch_contract(const void *X, bool x_complex, const float2 *W, void *Y,
                           int out_mode, int A, int L, int K, int B, hipStream_t s) {
  const int64_t total = (int64_t)A * K * B;
  if (total == 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
#define SPFEL_CONTRACT(XC, O) \
  hipLaunchKernelGGL((contract_kernel<XC, O>), grid, block, 0, s, X, W, Y, A, L, K, B)
  if (x_complex) {
    switch (out_mode) {
      case 0: SPFEL_CONTRACT(true, 0); break;
      case 1: SPFEL_CONTRACT(true, 1); break;
      case 2: SPFEL_CONTRACT(true, 2); break;
      default: SPFEL_CONTRACT(true, 3); break;
    }
  } else {
    switch (out_mode) {
      case 0: SPFEL_CONTRACT(false, 0); break;
      case 1: SPFEL_CONTRACT(false, 1); break;
      case 2: SPFEL_CONTRACT(false, 2); break;
      default: SPFEL_CONTRACT(false, 3); break;
    }
  }
#undef SPFEL_CONTRACT
  return hipGetLastError();
}

// Zero fill with a kernel (kept out of memset nodes so callers may capture
// the stream in a graph).
__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t *__restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<uint32_t *>(p), n);
  return hipGetLastError();
}

}  // namespace spfel
