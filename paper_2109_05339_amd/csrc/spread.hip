// Type-1 spreading (merging A*, section II-C Eq. (2)): every value y at a
// rotated Ewald-sphere point adds y psi psi psi to the w^3 fine-grid cells
// of its support; this is the transpose of the slicing interpolation.
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


__device__ inline int wrap_mod_s(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------------------
// Matrix-core spreading over the registered detector.  For one image and one
// compact tile, the brick of support cells is a sum of the points' separable
// stencils:
//   brick[i0][(i1, i2)] = sum_p (y_p psi(t0_p - i0)) (psi(t1_p - i1) psi(t2_p - i2)),
// a (e0 x npts) . (npts x e1 e2) product whose operands are generated on the
// fly from per-point data in LDS and fed to v_mfma_f32_32x32x2_f32 (most
// operand entries are zero; the matrix cores still beat LDS float atomics by
// an order of magnitude).  Points are counting-sorted by their axis-1 cell so
// each 32-column block of the product visits only the points that can touch
// its rows.  The product sits in registers and is added to the fine grid
// with one global atomic per nonzero cell.  Tiles whose brick exceeds
// 64 x 64 x 64 fall back to per-point global atomics.
typedef float floatx16_s __attribute__((ext_vector_type(16)));

template <int W, bool CPLX>
__global__ __launch_bounds__(kTile) void spread_mfma_kernel(
    float *__restrict__ acc, int nf, float beta, const float *__restrict__ quats, int64_t n_img,
    const float *__restrict__ dets, const int32_t *__restrict__ perm, int64_t P, int tiles,
    const void *__restrict__ values_, const float *__restrict__ weights) {
  // sorted points (slot kTile: a point of zero weights that pads the last
  // product step): support origin relative to the brick, one byte per axis,
  // and a row of weights: axis-0 weights times the value (re; im), axis-1
  // and axis-2 weights, each list followed by a zero so that an offset
  // outside the support, clamped to W, reads 0
  constexpr int kOA = 0, kOAI = W + 1, kOB = (CPLX ? 2 : 1) * (W + 1), kOC = kOB + W + 1;
  constexpr int kRow = kOC + W + 1;
  __shared__ int pk[kTile + 1];
  __shared__ float pw[kTile + 1][kRow];
  __shared__ int red[4][6];
  __shared__ int wrap[3][64];
  __shared__ int cnt[66];                 // points per axis-1 cell, then exclusive offsets

  const int64_t vb = xcd_contiguous_block();
  const int64_t n = vb / tiles;
  const int tile = (int)(vb - n * tiles);
  const int64_t i = (int64_t)tile * kTile + threadIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool inb = i < P;
  double R[9];
  const bool qok = quat_rot(quats + 4 * n, R);
  const double scale = (double)nf / (2.0 * M_PI);
  int l0[3] = {0, 0, 0};
  float frac[3] = {0.f, 0.f, 0.f};
  bool valid = inb && qok;
  float yr = 0.f, yi = 0.f;
  if (valid) {
    const double q0 = dets[3 * i], q1 = dets[3 * i + 1], q2 = dets[3 * i + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = (R[3 * d] * q0 + R[3 * d + 1] * q1 + R[3 * d + 2] * q2) * scale;
      if (!(fabs(t) < 1e8)) {
        valid = false;
      } else {
        const double c = ceil(t - 0.5 * W);
        l0[d] = (int)c;
        frac[d] = (float)(t - c);
      }
    }
    const int64_t o = n * P + perm[i];
    if (CPLX) {
      const float2 v = static_cast<const float2 *>(values_)[o];
      yr = v.x;
      yi = v.y;
    } else {
      yr = static_cast<const float *>(values_)[o];
    }
    if (weights) {
      const float wt = weights[o];
      yr *= wt;
      yi *= wt;
    }
  }
  int mn[3], mx[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mn[d] = valid ? l0[d] : 0x7fffffff;
    mx[d] = valid ? l0[d] : -0x7fffffff;
  }
  if (tid < 66) cnt[tid] = 0;
  block_minmax3(mn, mx, red);
  if (!(mn[0] <= mx[0])) return;  // no valid point in the block (uniform)
  const int e0 = mx[0] - mn[0] + W, e1 = mx[1] - mn[1] + W, e2 = mx[2] - mn[2] + W;
  float w0[W], w1[W], w2[W];
  if (valid) {
    es_weights<W>(frac[0], beta, w0);
    es_weights<W>(frac[1], beta, w1);
    es_weights<W>(frac[2], beta, w2);
  }
  if (e0 > 64 || e1 > 64 || e2 > 64) {
    // fallback: per-point global atomics
    if (!valid) return;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const int g0 = wrap_mod_s(l0[0] + a, nf);
      const float ra = w0[a] * yr, ia = w0[a] * yi;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const int g1 = wrap_mod_s(l0[1] + b, nf);
        const float rb = w1[b] * ra, ib = w1[b] * ia;
        const int64_t row = ((int64_t)g0 * nf + g1) * nf;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const int64_t cell = row + wrap_mod_s(l0[2] + c, nf);
          if (CPLX) {
            unsafeAtomicAdd(acc + 2 * cell, w2[c] * rb);
            unsafeAtomicAdd(acc + 2 * cell + 1, w2[c] * ib);
          } else {
            unsafeAtomicAdd(acc + cell, w2[c] * rb);
          }
        }
      }
    }
    return;
  }
  // counting sort of the valid points by their axis-1 cell
  const int k1 = l0[1] - mn[1];
  if (valid) atomicAdd(&cnt[k1 + 1], 1);
  if (tid < 64) {
    const int t = tid;
    if (t < e0) wrap[0][t] = wrap_mod_s(mn[0] + t, nf);
    if (t < e1) wrap[1][t] = wrap_mod_s(mn[1] + t, nf);
    if (t < e2) wrap[2][t] = wrap_mod_s(mn[2] + t, nf);
  }
  __syncthreads();
  if (tid == 0) {
    for (int c = 1; c <= e1; ++c) cnt[c] += cnt[c - 1];   // cnt[c] = points with cell < c
  }
  __syncthreads();
  if (valid) {
    const int slot = atomicAdd(&cnt[k1], 1);   // cnt[k1] runs up to the old cnt[k1 + 1]
    pk[slot] = (l0[0] - mn[0]) | (k1 << 8) | ((l0[2] - mn[2]) << 16);
    float *row = pw[slot];
#pragma unroll
    for (int a = 0; a < W; ++a) {
      row[kOA + a] = w0[a] * yr;
      if (CPLX) row[kOAI + a] = w0[a] * yi;
      row[kOB + a] = w1[a];
      row[kOC + a] = w2[a];
    }
    row[kOA + W] = 0.f;
    if (CPLX) row[kOAI + W] = 0.f;
    row[kOB + W] = 0.f;
    row[kOC + W] = 0.f;
  }
  if (tid == 0) {
    pk[kTile] = 0;
#pragma unroll
    for (int e = 0; e < kRow; ++e) pw[kTile][e] = 0.f;
  }
  __syncthreads();
  // after the scatter, cnt[c] = points with cell <= c; the first point of
  // cell c is at cnt[c - 1] (0 for c = 0)
  const int nvalid = cnt[e1 - 1];
  const int lr = lane & 31, lh = lane >> 5;
  const int ncol = e1 * e2;
  const int mblocks = (e0 + 31) >> 5, nblocks = (ncol + 31) >> 5;
  const float inv_e2 = 1.0f / (float)e2;
  for (int job = wave; job < mblocks * nblocks; job += 4) {
    const int mb = job / nblocks, nb = job - mb * nblocks;
    const int ncell = nb * 32 + lr;
    const int j1c = (int)(((float)ncell + 0.5f) * inv_e2);
    const int j2 = ncell - j1c * e2;
    // columns past the brick take an axis-1 cell no point reaches
    const int j1 = ncell < ncol ? j1c : 1024;
    const int i0 = mb * 32 + lr;
    // points whose axis-1 support meets rows [r_lo, r_hi] of this block
    const int r_lo = (nb * 32) / e2, r_hi = min(e1 - 1, (nb * 32 + 31) / e2);
    const int c_lo = max(0, r_lo - W + 1);
    const int k_beg = c_lo > 0 ? cnt[c_lo - 1] : 0;
    const int k_end = cnt[r_hi];
    floatx16_s accr, acci;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accr[r] = 0.f;
      acci[r] = 0.f;
    }
    // one product step: lane half lh supplies point p (offsets outside the
    // support clamp to the zero entry W)
    auto step = [&](int p) {
      const int o = pk[p];
      const unsigned da = min((unsigned)(i0 - (o & 255)), (unsigned)W);
      const unsigned db = min((unsigned)(j1 - ((o >> 8) & 255)), (unsigned)W);
      const unsigned dc = min((unsigned)(j2 - (o >> 16)), (unsigned)W);
      const float *row = pw[p];
      const float b = row[kOB + db] * row[kOC + dc];
      accr = __builtin_amdgcn_mfma_f32_32x32x2f32(row[kOA + da], b, accr, 0, 0, 0);
      if (CPLX) acci = __builtin_amdgcn_mfma_f32_32x32x2f32(row[kOAI + da], b, acci, 0, 0, 0);
    };
    // the range is the same for the whole wavefront
    const int kb = __builtin_amdgcn_readfirstlane(k_beg), ke = __builtin_amdgcn_readfirstlane(k_end);
    int k0 = kb;
    for (; k0 + 2 <= ke; k0 += 2) step(k0 + lh);
    if (k0 < ke) step(k0 + lh < ke ? k0 + lh : kTile);
    if (ncell < ncol) {
      const int64_t colg = (int64_t)wrap[1][j1] * nf + wrap[2][j2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = mb * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
        if (row < e0) {
          const int64_t cell = (int64_t)wrap[0][row] * nf * nf + colg;
          if (CPLX) {
            if (accr[r] != 0.f) unsafeAtomicAdd(acc + 2 * cell, accr[r]);
            if (acci[r] != 0.f) unsafeAtomicAdd(acc + 2 * cell + 1, acci[r]);
          } else {
            if (accr[r] != 0.f) unsafeAtomicAdd(acc + cell, accr[r]);
          }
        }
      }
    }
  }
  (void)nvalid;
}

template <int W>
static hipError_t spread_w(const Plan &pl, const float *quats, int64_t n_img, const float *detq,
                           int64_t P, const void *values, const float *weights, hipStream_t s) {
  const bool cplx = pl.domain == SPFEL_COMPLEX;
  if (detq == nullptr) {
    const int tiles = (int)((P + kTile - 1) / kTile);
    const int64_t blocks = n_img * tiles;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    float *acc = static_cast<float *>(pl.acc);
    if (cplx)
      hipLaunchKernelGGL((spread_mfma_kernel<W, true>), dim3((unsigned)blocks), dim3(kTile), 0, s,
                         acc, pl.nf, (float)pl.beta, quats, n_img, pl.det_sorted, pl.det_perm, P,
                         tiles, values, weights);
    else
      hipLaunchKernelGGL((spread_mfma_kernel<W, false>), dim3((unsigned)blocks), dim3(kTile), 0,
                         s, acc, pl.nf, (float)pl.beta, quats, n_img, pl.det_sorted, pl.det_perm,
                         P, tiles, values, weights);
    return hipGetLastError();
  }
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
  switch (pl.w) {
    case 4: return spread_w<4>(pl, quats, n_img, detq, P, values, weights, s);
    case 5: return spread_w<5>(pl, quats, n_img, detq, P, values, weights, s);
    case 6: return spread_w<6>(pl, quats, n_img, detq, P, values, weights, s);
    case 7: return spread_w<7>(pl, quats, n_img, detq, P, values, weights, s);
    default: return spread_w<8>(pl, quats, n_img, detq, P, values, weights, s);
  }
}

}  // namespace spfel
