// Type-2 interpolation (slicing, section II-A): each model image pixel is
// the ES-kernel-weighted sum of the w^3 fine-grid cells around its rotated
// Ewald-sphere point, s(x) = sum_{a,b,c} u[l0 + (a,b,c)] psi psi psi.
#include "device_common.h"
#include "internal.h"

namespace spfel {

template <int W, bool CPLX>
__global__ __launch_bounds__(256) void interp_gather_kernel(
    const void *__restrict__ u_, int nf, float beta, const float *__restrict__ quats, int64_t M,
    const float *__restrict__ detq, int64_t P, void *__restrict__ out_,
    uint16_t *__restrict__ out_bf16) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * P) return;
  const int64_t m = idx / P;
  const int64_t p = idx - m * P;
  double R[9];
  bool ok = quat_rot(quats + 4 * m, R);
  const double q0 = detq[3 * p], q1 = detq[3 * p + 1], q2 = detq[3 * p + 2];
  const double scale = (double)nf / (2.0 * M_PI);
  int base[3];
  float frac[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = R[3 * d] * q0 + R[3 * d + 1] * q1 + R[3 * d + 2] * q2;
    ok = ok && support_split<W>(x * scale, nf, base[d], frac[d]);
  }
  if (!ok) {
    const float nan = __uint_as_float(0x7fc00000u);
    if (CPLX) {
      if (out_) static_cast<float2 *>(out_)[idx] = make_float2(nan, nan);
    } else {
      if (out_) static_cast<float *>(out_)[idx] = nan;
      if (out_bf16) out_bf16[idx] = 0x7fc0u;
    }
    return;
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
  if (CPLX) {
    const float2 *u = static_cast<const float2 *>(u_);
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      int i0 = base[0] + a;
      i0 -= (i0 >= nf) ? nf : 0;
      const float2 *plane = u + (int64_t)i0 * nf2;
      float pr = 0.f, pi = 0.f;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const float2 *row = plane + o1[b];
        float rr = 0.f, ri = 0.f;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const float2 v = row[o2[c]];
          rr = fmaf(w2[c], v.x, rr);
          ri = fmaf(w2[c], v.y, ri);
        }
        pr = fmaf(w1[b], rr, pr);
        pi = fmaf(w1[b], ri, pi);
      }
      sr = fmaf(w0[a], pr, sr);
      si = fmaf(w0[a], pi, si);
    }
    if (out_) static_cast<float2 *>(out_)[idx] = make_float2(sr, si);
  } else {
    const float *u = static_cast<const float *>(u_);
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      int i0 = base[0] + a;
      i0 -= (i0 >= nf) ? nf : 0;
      const float *plane = u + (int64_t)i0 * nf2;
      float pr = 0.f;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const float *row = plane + o1[b];
        float rr = 0.f;
#pragma unroll
        for (int c = 0; c < W; ++c) rr = fmaf(w2[c], row[o2[c]], rr);
        pr = fmaf(w1[b], rr, pr);
      }
      s = fmaf(w0[a], pr, s);
    }
    if (out_) static_cast<float *>(out_)[idx] = s;
    if (out_bf16) out_bf16[idx] = f32_to_bf16(s);
  }
}

template <int W>
static hipError_t interp_w(const Plan &pl, const float *quats, int64_t M, const float *detq,
                           int64_t P, void *out, uint16_t *out_bf16, hipStream_t s) {
  const int64_t total = M * P;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (pl.domain == SPFEL_COMPLEX)
    hipLaunchKernelGGL((interp_gather_kernel<W, true>), grid, block, 0, s, pl.u, pl.nf,
                       (float)pl.beta, quats, M, detq, P, out, out_bf16);
  else
    hipLaunchKernelGGL((interp_gather_kernel<W, false>), grid, block, 0, s, pl.u, pl.nf,
                       (float)pl.beta, quats, M, detq, P, out, out_bf16);
  return hipGetLastError();
}

hipError_t launch_interp(const Plan &pl, const float *quats, int64_t M, const float *detq,
                         int64_t P, void *out, uint16_t *out_bf16, hipStream_t s) {
  switch (pl.w) {
    case 4: return interp_w<4>(pl, quats, M, detq, P, out, out_bf16, s);
    case 5: return interp_w<5>(pl, quats, M, detq, P, out, out_bf16, s);
    case 6: return interp_w<6>(pl, quats, M, detq, P, out, out_bf16, s);
    case 7: return interp_w<7>(pl, quats, M, detq, P, out, out_bf16, s);
    default: return interp_w<8>(pl, quats, M, detq, P, out, out_bf16, s);
  }
}

// Squared norm of each row: 256 threads take strided partial sums (one
// fused multiply-add per element), then a pairwise tree in LDS; the order
// is fixed, so the result is deterministic.
template <bool BF>
__global__ __launch_bounds__(256) void row_norm2_kernel(const void *__restrict__ x_, int64_t cols,
                                                        float *__restrict__ out) {
  __shared__ float sh[256];
  const int64_t row = blockIdx.x;
  float acc = 0.f;
  if (BF) {
    const uint16_t *x = static_cast<const uint16_t *>(x_) + row * cols;
    for (int64_t c = threadIdx.x; c < cols; c += 256) {
      const float v = bf16_to_f32(x[c]);
      acc = fmaf(v, v, acc);
    }
  } else {
    const float *x = static_cast<const float *>(x_) + row * cols;
    for (int64_t c = threadIdx.x; c < cols; c += 256) {
      const float v = x[c];
      acc = fmaf(v, v, acc);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[row] = sh[0];
}

hipError_t launch_row_norm2(const void *x, bool bf16, int64_t rows, int64_t cols, float *out,
                            hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL((row_norm2_kernel<true>), dim3((unsigned)rows), dim3(256), 0, s, x, cols, out);
  else
    hipLaunchKernelGGL((row_norm2_kernel<false>), dim3((unsigned)rows), dim3(256), 0, s, x, cols, out);
  return hipGetLastError();
}

}  // namespace spfel
