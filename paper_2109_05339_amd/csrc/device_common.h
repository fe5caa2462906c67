// Device helpers shared by the slicing, spreading and matching kernels:
// orientation matrices, the kernel-support split of a fine-grid coordinate,
// the ES kernel weights, bfloat16 rounding and order-preserving keys.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spfel {

// Rotation matrix (row-major) of quaternion (w, x, y, z), Hamilton
// convention, normalised by dividing by |q|^2; false for a zero or
// non-finite quaternion.
__device__ inline bool quat_rot(const float *__restrict__ q4, double R[9]) {
  const double w = q4[0], x = q4[1], y = q4[2], z = q4[3];
  const double n2 = w * w + x * x + y * y + z * z;
  if (!(n2 > 0.0) || !(n2 < 1e300)) return false;
  const double s = 2.0 / n2;
  R[0] = 1.0 - s * (y * y + z * z);
  R[1] = s * (x * y - w * z);
  R[2] = s * (x * z + w * y);
  R[3] = s * (x * y + w * z);
  R[4] = 1.0 - s * (x * x + z * z);
  R[5] = s * (y * z - w * x);
  R[6] = s * (x * z - w * y);
  R[7] = s * (y * z + w * x);
  R[8] = 1.0 - s * (x * x + y * y);
  return true;
}

// Fine-grid coordinate t (cells) -> first support cell l0 = ceil(t - W/2)
// reduced modulo nf into [0, nf), and the offset frac = t - l0 in
// (W/2 - 1, W/2].  False if t is not finite or absurdly large.
template <int W>
__device__ inline bool support_split(double t, int nf, int &base, float &frac) {
  if (!(fabs(t) < 1e9)) return false;
  const double l0 = ceil(t - 0.5 * W);
  frac = (float)(t - l0);
  double b = l0 - (double)nf * floor(l0 / (double)nf);
  int bi = (int)b;
  if (bi >= nf) bi -= nf;
  if (bi < 0) bi += nf;
  base = bi;
  return true;
}

// ES kernel weights psi(frac - a), a = 0..W-1, with
// psi(tau) = exp(beta (sqrt(1 - (2 tau / W)^2) - 1)) = 2^(c sqrt(r) - c),
// c = beta log2(e).  The hardware square root and base-2 exponential
// (about 1 ulp each) are used directly.  The exponent lies in [-c, 0]; its
// rounding error, |c| 2^-24 ln 2, is below 1e-6 relative for the usual
// beta = 2.30 w (w <= 8) and below 5e-6 at the largest accepted beta (80),
// and psi >= 2^-c > 2^-126 stays a normal number, so no denormal handling
// is needed.
template <int W>
__device__ inline void es_weights(float frac, float beta, float (&wt)[W]) {
  const float c = beta * 1.44269504088896341f;
  const float k = 2.0f / (float)W;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const float z = fmaf(frac, k, -(float)a * k);
    const float r = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
    wt[a] = __builtin_amdgcn_exp2f(fmaf(c, __builtin_amdgcn_sqrtf(r), -c));
  }
}

// float -> bfloat16 bits, round to nearest, ties to even (NaN stays NaN).
__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Order-preserving map float -> uint32 (a < b  <=>  key(a) < key(b)).
__device__ inline uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Minimum over the 64 lanes of a wavefront (all lanes active), returned to
// every lane.  DPP row operations fused into the minimum (two quad-permute
// butterflies, then the half and full row mirrors) give each row of 16
// lanes its minimum; the four rows' results are then read out as scalars.
__device__ inline int wave_min(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));  // row_mirror
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Block-wide minimum and maximum of three ints over a block of four
// wavefronts; sh is 4 x 6 ints of shared memory.  Ends with a barrier.
__device__ inline void block_minmax3(int (&mn)[3], int (&mx)[3], int (*sh)[6]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mn[d] = wave_min(mn[d]);
    mx[d] = -wave_min(-mx[d]);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sh[wave][d] = mn[d];
      sh[wave][3 + d] = mx[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mn[d] = min(min(sh[0][d], sh[1][d]), min(sh[2][d], sh[3][d]));
    mx[d] = max(max(sh[0][3 + d], sh[1][3 + d]), max(sh[2][3 + d], sh[3][3 + d]));
  }
}

// Blocks are dealt round-robin to the 8 XCDs; this remaps the block id so
// each XCD works through a contiguous range of the logical block order (and
// neighbouring logical blocks share that XCD's L2).
__device__ inline int64_t xcd_contiguous_block() {
  const int64_t G = gridDim.x, bid = blockIdx.x;
  const int64_t xcd = bid & 7, slot = bid >> 3, per = G >> 3, rem = G & 7;
  return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + slot;
}

}  // namespace spfel
