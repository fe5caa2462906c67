// Type-1 spreading (merging A*, section II-C Eq. (2)): every value y at a
// rotated Ewald-sphere point adds y psi psi psi to the w^3 fine-grid cells
// of its support; this is the transpose of the slicing interpolation.
// Points given by the caller's own detector array spread with one global
// atomic per support cell; the registered detector takes the binned
// matrix-core path of spread_binned.hip.
#include "device_common.h"
#include "internal.h"

namespace spfel {

template <int W, bool CPLX>
__global__ __launch_bounds__(256) void spread_atomic_kernel(
    void *__restrict__ acc_, int nf, float beta, const float *__restrict__ quats, int64_t n_img,
    const float *__restrict__ detq, int64_t P, const void *__restrict__ values_,
    const float *__restrict__ weights) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_img * P) return;
  const int64_t n = idx / P;
  const int64_t p = idx - n * P;
  double R[9];
  bool ok = quat_rot(quats + 4 * n, R);
  const double q0 = detq[3 * p], q1 = detq[3 * p + 1], q2 = detq[3 * p + 2];
  const double scale = (double)nf / (2.0 * M_PI);
  int base[3];
  float frac[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = R[3 * d] * q0 + R[3 * d + 1] * q1 + R[3 * d + 2] * q2;
    ok = ok && support_split<W>(x * scale, nf, base[d], frac[d]);
  }
  if (!ok) return;
  float yr, yi = 0.f;
  if (CPLX) {
    const float2 v = static_cast<const float2 *>(values_)[idx];
    yr = v.x;
    yi = v.y;
  } else {
    yr = static_cast<const float *>(values_)[idx];
  }
  if (weights) {
    const float wt = weights[idx];
    yr *= wt;
    yi *= wt;
  }
  float w0[W], w1[W], w2[W];
  es_weights<W>(frac[0], beta, w0);
  es_weights<W>(frac[1], beta, w1);
  es_weights<W>(frac[2], beta, w2);
  int o1[W], o2[W];
#pragma unroll
  for (int a = 0; a < W; ++a) {
    int i1 = base[1] + a;
    i1 -= (i1 >= nf) ? nf : 0;
    int i2 = base[2] + a;
    i2 -= (i2 >= nf) ? nf : 0;
    o1[a] = i1 * nf;
    o2[a] = i2;
  }
  const int nf2 = nf * nf;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    int i0 = base[0] + a;
    i0 -= (i0 >= nf) ? nf : 0;
    const float ra = w0[a] * yr, ia = w0[a] * yi;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const float rb = w1[b] * ra, ib = w1[b] * ia;
      const int64_t rowoff = (int64_t)i0 * nf2 + o1[b];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        if (CPLX) {
          float *cell = static_cast<float *>(acc_) + 2 * (rowoff + o2[c]);
          unsafeAtomicAdd(cell, w2[c] * rb);
          unsafeAtomicAdd(cell + 1, w2[c] * ib);
        } else {
          unsafeAtomicAdd(static_cast<float *>(acc_) + rowoff + o2[c], w2[c] * rb);
        }
      }
    }
  }
}


template <int W>
static hipError_t spread_w(const Plan &pl, const float *quats, int64_t n_img, const float *detq,
                           int64_t P, const void *values, const float *weights, hipStream_t s) {
  const bool cplx = pl.domain == SPFEL_COMPLEX;
  const int64_t total = n_img * P;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (cplx)
    hipLaunchKernelGGL((spread_atomic_kernel<W, true>), grid, block, 0, s, pl.acc, pl.nf,
                       (float)pl.beta, quats, n_img, detq, P, values, weights);
  else
    hipLaunchKernelGGL((spread_atomic_kernel<W, false>), grid, block, 0, s, pl.acc, pl.nf,
                       (float)pl.beta, quats, n_img, detq, P, values, weights);
  return hipGetLastError();
}

hipError_t launch_spread(const Plan &pl, const float *quats, int64_t n_img, const float *detq,
                         int64_t P, const void *values, const float *weights, hipStream_t s) {
  if (detq == nullptr) return launch_spread_binned(pl, quats, n_img, P, values, weights, s);
  switch (pl.w) {
    case 4: return spread_w<4>(pl, quats, n_img, detq, P, values, weights, s);
    case 5: return spread_w<5>(pl, quats, n_img, detq, P, values, weights, s);
    case 6: return spread_w<6>(pl, quats, n_img, detq, P, values, weights, s);
    case 7: return spread_w<7>(pl, quats, n_img, detq, P, values, weights, s);
    default: return spread_w<8>(pl, quats, n_img, detq, P, values, weights, s);
  }
}

}  // namespace spfel
