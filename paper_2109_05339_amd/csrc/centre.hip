// Operands of the BF16 distance GEMM (section II-B, precision form).
//
// Every distance is unchanged when one vector c is subtracted from all model
// images and all images: |(s - c) - (d - c)| = |s - d|.  The bright low-q
// intensity common to every slice and image is removed that way, so the
// BF16 rounding acts on small centred values.  The matcher's proxy is the
// exact squared distance of the rounded rows, and the per-row rounding
// error norms computed here bound how far it can sit from the true one
// (|sqrt(D) - sqrt(b)| <= e_m + f_n).
#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace spfel {

// Column mean: one thread per column, rows summed in runs of 32 whose
// partial sums are added in order (a fixed order, so the result is
// deterministic; two-level sums keep the rounding chain near rows/32 + 32).
__global__ __launch_bounds__(256) void column_mean_kernel(const float *__restrict__ x, int64_t rows,
                                                          int64_t cols, int round_int,
                                                          float *__restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const float *p = x + c;
  float total = 0.f;
  int64_t r = 0;
  for (; r + 32 <= rows; r += 32) {
    float run = 0.f;
#pragma unroll 16
    for (int i = 0; i < 32; ++i) run += __builtin_nontemporal_load(p + (r + i) * cols);
    total += run;
  }
  float run = 0.f;
  for (; r < rows; ++r) run += __builtin_nontemporal_load(p + r * cols);
  total += run;
  const float mean = total / (float)rows;
  out[c] = round_int ? rintf(mean) : mean;
}

hipError_t launch_column_mean(const float *x, int64_t rows, int64_t cols, int round_int,
                              float *out, hipStream_t s) {
  hipLaunchKernelGGL(column_mean_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, x,
                     rows, cols, round_int, out);
  return hipGetLastError();
}

// One block per row: v = bf16(x - c) (one float32 subtraction, then round to
// nearest even), norm2 = sum v^2 and the rounding-error norm |v - (x - c)|,
// each from 256 strided partial sums and a pairwise tree (fixed order).
// The stored error is an upper bound on the exact one: the float32 sum is
// scaled by `infl` (1 + gamma of its rounding chain) and the float32
// subtraction's own rounding (at most 2^-24 |x - c| per element) is added
// as 2^-23 |v|.
// f32_to_bf16 written as a select instead of an early return (same
// values, NaN stays NaN), so the streaming loop below carries no branch per
// value and its loads stay grouped.
__device__ inline uint16_t bf16_round(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const uint32_t quiet = (u >> 16) | 0x40u;
  return (uint16_t)((u & 0x7fffffffu) > 0x7f800000u ? quiet : rounded);
}

__global__ __launch_bounds__(256) void bf16_centred_kernel(
    const float *__restrict__ x, const float *__restrict__ c, int64_t cols,
    uint16_t *__restrict__ out, float *__restrict__ norm2, float *__restrict__ err, int vec,
    float infl) {
  __shared__ float sh[2][256];
  const int64_t row = blockIdx.x;
  const float *xr = x + row * cols;
  uint16_t *orow = out + row * cols;
  float a = 0.f, b = 0.f;
  auto one = [&](float v, float cc) -> uint16_t {
    const float d = v - cc;
    const uint16_t h = bf16_round(d);
    const float r = bf16_to_f32(h);
    const float q = r - d;   // exact: r is d rounded to fewer bits
    a = fmaf(r, r, a);
    b = fmaf(q, q, b);
    return h;
  };
  if (vec) {
    const int64_t groups = cols / 4;
    const float4 *x4 = reinterpret_cast<const float4 *>(xr);
    const float4 *c4 = reinterpret_cast<const float4 *>(c);
    uint2 *o2 = reinterpret_cast<uint2 *>(orow);
    auto group = [&](int64_t g, float4 v, float4 cc) {
      const uint32_t h0 = one(v.x, cc.x), h1 = one(v.y, cc.y);
      const uint32_t h2 = one(v.z, cc.z), h3 = one(v.w, cc.w);
      o2[g] = make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
    };
    // four groups' loads in flight per thread; the sums still run over g
    // in increasing order
    auto walk = [&](auto has_c) {
      constexpr bool C = decltype(has_c)::value;
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      int64_t g = threadIdx.x;
      for (; g + 3 * 256 < groups; g += 4 * 256) {
        float4 v[4], cc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v[u] = x4[g + u * 256];
          cc[u] = C ? c4[g + u * 256] : z;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) group(g + u * 256, v[u], cc[u]);
      }
      for (; g < groups; g += 256) group(g, x4[g], C ? c4[g] : z);
    };
    if (c)
      walk(std::true_type{});
    else
      walk(std::false_type{});
  } else {
    for (int64_t k = threadIdx.x; k < cols; k += 256) orow[k] = one(xr[k], c ? c[k] : 0.f);
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float n2 = sh[0][0];
    if (norm2) norm2[row] = n2;
    if (err) err[row] = fmaf(sqrtf(sh[1][0]), infl, 0x1p-23f * sqrtf(n2));
  }
}

hipError_t launch_bf16_centred(const float *x, int64_t rows, int64_t cols, const float *c,
                               uint16_t *out, float *norm2, float *err, hipStream_t s) {
  auto al = [](const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
  const int vec = cols % 4 == 0 && al(x, 16) && (c == nullptr || al(c, 16)) && al(out, 8);
  // rounding chain of the error sum: cols/256 strided terms, 8 tree levels
  const double L = (double)((cols + 255) / 256) + 16.0, u = 0x1p-24;
  const float infl = (float)(1.0 + 2.0 * L * u / (1.0 - L * u));
  hipLaunchKernelGGL(bf16_centred_kernel, dim3((unsigned)rows), dim3(256), 0, s, x, c, cols, out,
                     norm2, err, vec, infl);
  return hipGetLastError();
}

// out[r][p] = x[r][p] g[p] (in place allowed).
__global__ __launch_bounds__(256) void scale_columns_kernel(const float *x, int64_t rows,
                                                            int64_t cols,
                                                            const float *__restrict__ g, float *out,
                                                            int vec) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    const int64_t q4 = cols / 4, n4 = rows * q4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
      const int64_t c4 = i % q4;
      float4 v = reinterpret_cast<const float4 *>(x)[i];
      const float4 s = reinterpret_cast<const float4 *>(g)[c4];
      v.x *= s.x;
      v.y *= s.y;
      v.z *= s.z;
      v.w *= s.w;
      reinterpret_cast<float4 *>(out)[i] = v;
    }
  } else {
    const int64_t n = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      out[i] = x[i] * g[i % cols];
  }
}

hipError_t launch_scale_columns(const float *x, int64_t rows, int64_t cols, const float *g,
                                float *out, hipStream_t s) {
  auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const int vec = cols % 4 == 0 && al(x) && al(g) && al(out);
  int64_t blocks = (rows * cols / (vec ? 4 : 1) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scale_columns_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, rows, cols,
                     g, out, vec);
  return hipGetLastError();
}

}  // namespace spfel
