// Weighted residual r = scale (*scale_dev) w (s - d) and loss sum w |s - d|^2
// of slices against images: the data term of the D-weighted least squares
// behind merging (section II-C, Eq. (1)-(2)); its spread is the loss
// gradient.  The loss accumulates in float64: the scalar is differenced in
// finite-difference checks far below float32 resolution of a sum of 10^7 -
// 10^8 terms (one float64 add per element; the kernel is bound by HBM).
#include "internal.h"

namespace spfel {

constexpr int kResThreads = 256;

template <bool CPLX>
__global__ __launch_bounds__(kResThreads) void residual_kernel(
    const void *__restrict__ s_, const void *__restrict__ d_, const float *__restrict__ w,
    int64_t count, float scale, const float *__restrict__ scale_dev, void *__restrict__ r_,
    double *__restrict__ partials) {
  __shared__ double sh[kResThreads];
  if (scale_dev) scale *= *scale_dev;
  const int64_t per = (count + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(count, lo + per);
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kResThreads) {
    const float wt = w ? w[i] : 1.0f;
    if (CPLX) {
      const float2 s = static_cast<const float2 *>(s_)[i];
      const float2 d = static_cast<const float2 *>(d_)[i];
      const float er = s.x - d.x, ei = s.y - d.y;
      acc += (double)wt * ((double)er * er + (double)ei * ei);
      if (r_) static_cast<float2 *>(r_)[i] = make_float2(scale * wt * er, scale * wt * ei);
    } else {
      const float e = static_cast<const float *>(s_)[i] - static_cast<const float *>(d_)[i];
      acc += (double)wt * ((double)e * e);
      if (r_) static_cast<float *>(r_)[i] = scale * wt * e;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kResThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// Sums the per-block partials in block order into *loss.
__global__ void loss_finish_kernel(const double *__restrict__ partials, int n,
                                   double *__restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += partials[i];
    *loss += t;
  }
}

hipError_t launch_residual(bool cplx, const void *s, const void *d, const float *w, int64_t count,
                           float scale, const float *scale_dev, void *r, double *partials,
                           double *loss, hipStream_t st) {
  int64_t blocks = (count + 4 * kResThreads - 1) / (4 * kResThreads);
  if (blocks > kMaxPartials) blocks = kMaxPartials;
  if (blocks < 1) blocks = 1;
  if (cplx)
    hipLaunchKernelGGL((residual_kernel<true>), dim3((unsigned)blocks), dim3(kResThreads), 0, st, s,
                       d, w, count, scale, scale_dev, r, partials);
  else
    hipLaunchKernelGGL((residual_kernel<false>), dim3((unsigned)blocks), dim3(kResThreads), 0, st,
                       s, d, w, count, scale, scale_dev, r, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !loss) return e;
  hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(64), 0, st, partials, (int)blocks, loss);
  return hipGetLastError();
}

}  // namespace spfel
