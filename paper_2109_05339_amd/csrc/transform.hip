// Separable transforms between the N^3 model modes and the 2N-per-axis fine
// grid.  The zero-padded 3D FFT plus kernel deconvolution of an ES-kernel
// NUFFT is applied one axis at a time as a contraction with a small table
// W[l][k] = exp(+-2 pi i k l / nf) / psi_hat(k): padding and truncation fold
// into the table's shape, and the deconvolution into its rows.
#include "internal.h"

namespace spfel {

// Y[a][k][b] = sum_l X[a][l][b] W[l][k]; one thread per KB consecutive
// outputs along k (same a and b; the last group of an odd K is partial),
// b fastest across threads, so reads of X are contiguous in b (or broadcast
// when B = 1), each X value serves KB outputs, and reads of W are
// contiguous in k (or broadcast).  Every output is summed over l in order,
// whatever KB.
template <bool XC, int OUT, int KB, bool PART>
__global__ __launch_bounds__(256) void contract_kernel(const void *__restrict__ X_,
                                                       const float2 *__restrict__ W,
                                                       void *__restrict__ Y_, int A, int L,
                                                       int K, int B) {
  const int KG = (K + KB - 1) / KB;
  const int64_t total = (int64_t)A * KG * B;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int b = (int)(t % B);
  const int64_t r = t / B;
  const int k0 = (int)(r % KG) * KB;
  const int a = (int)(r / KG);
  float re[KB], im[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q) re[q] = im[q] = 0.f;
  const int64_t xbase = (int64_t)a * L * B + b;
  for (int l = 0; l < L; ++l) {
    float xr, xi = 0.f;
    if (XC) {
      const float2 x = static_cast<const float2 *>(X_)[xbase + (int64_t)l * B];
      xr = x.x;
      xi = x.y;
    } else {
      xr = static_cast<const float *>(X_)[xbase + (int64_t)l * B];
    }
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      // PART (K % KB != 0): past the end of k, read the last column; the sum
      // is dropped
      const float2 w = W[(int64_t)l * K + (PART ? min(k0 + q, K - 1) : k0 + q)];
      re[q] = fmaf(xr, w.x, re[q]);
      if (XC) re[q] = fmaf(-xi, w.y, re[q]);
      im[q] = fmaf(xr, w.y, im[q]);
      if (XC) im[q] = fmaf(xi, w.x, im[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < KB; ++q) {
    if (PART && k0 + q >= K) break;
    const int64_t o = ((int64_t)a * K + k0 + q) * B + b;
    if (OUT == 0) {
      static_cast<float2 *>(Y_)[o] = make_float2(re[q], im[q]);
    } else if (OUT == 1) {
      static_cast<float *>(Y_)[o] = re[q];
    } else if (OUT == 2) {
      static_cast<float *>(Y_)[o] += re[q];
    } else {
      float2 *Y = static_cast<float2 *>(Y_);
      const float2 y = Y[o];
      Y[o] = make_float2(y.x + re[q], y.y + im[q]);
    }
  }
}

template <int KB, bool PART>
static hipError_t contract_kb(const void *X, bool x_complex, const float2 *W, void *Y,
                              int out_mode, int A, int L, int K, int B, hipStream_t s) {
  const int64_t total = (int64_t)A * ((K + KB - 1) / KB) * B;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
#define SPFEL_CONTRACT(XC, O) \
  hipLaunchKernelGGL((contract_kernel<XC, O, KB, PART>), grid, block, 0, s, X, W, Y, A, L, K, B)
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

hipError_t launch_contract(const void *X, bool x_complex, const float2 *W, void *Y,
                           int out_mode, int A, int L, int K, int B, hipStream_t s) {
  if ((int64_t)A * K * B == 0) return hipSuccess;
  return K % 2 == 0 ? contract_kb<2, false>(X, x_complex, W, Y, out_mode, A, L, K, B, s)
                    : contract_kb<2, true>(X, x_complex, W, Y, out_mode, A, L, K, B, s);
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
