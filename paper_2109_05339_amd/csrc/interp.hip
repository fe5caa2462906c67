// Type-2 interpolation (slicing, section II-A): each model image pixel is
// the ES-kernel-weighted sum of the w^3 fine-grid cells around its rotated
// Ewald-sphere point, s(x) = sum_{a,b,c} u[l0 + (a,b,c)] psi psi psi.
//
// The fine grid is stored centred: cell l (periodic in n_f) sits at index
// (l + n_f / 2) mod n_f along each axis, so the cells around the origin,
// where every orientation's points cluster, are contiguous and a support
// brick wraps only when it reaches |l| ~ n_f / 2, which Ewald-sphere points
// inside the Nyquist ball never do.
#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace spfel {

// Scaled rotation of each orientation, rot[9 m + 3 d + e] =
// R(q_m)[d][e] n_f / (2 pi) in float64, computed once per orientation for
// all of its points; a zero or non-finite quaternion stores NaN.
__global__ __launch_bounds__(256) void rotation_kernel(const float *__restrict__ quats, int64_t M,
                                                       double scale, double *__restrict__ rot) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double R[9];
  const bool ok = quat_rot(quats + 4 * m, R);
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
#pragma unroll
  for (int k = 0; k < 9; ++k) rot[9 * m + k] = ok ? R[k] * scale : nan;
}

hipError_t launch_rotations(const float *quats, int64_t M, double scale, double *rot,
                            hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(rotation_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, quats, M,
                     scale, rot);
  return hipGetLastError();
}

template <int W, bool CPLX>
__global__ __launch_bounds__(256) void interp_gather_kernel(
    const void *__restrict__ u_, int nf, float beta, const double *__restrict__ rot, int64_t M,
    const float *__restrict__ detq, int64_t P, void *__restrict__ out_) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * P) return;
  const int64_t m = idx / P;
  const int64_t p = idx - m * P;
  const double *R = rot + 9 * m;
  bool ok = R[0] == R[0];
  const double q0 = detq[3 * p], q1 = detq[3 * p + 1], q2 = detq[3 * p + 2];
  int base[3];
  float frac[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = R[3 * d] * q0 + R[3 * d + 1] * q1 + R[3 * d + 2] * q2;
    ok = ok && support_split<W>(t, nf, base[d], frac[d]);
    base[d] += nf >> 1;   // centred storage
    base[d] -= base[d] >= nf ? nf : 0;
  }
  if (!ok) {
    const float nan = __uint_as_float(0x7fc00000u);
    if (CPLX) {
      if (out_) static_cast<float2 *>(out_)[idx] = make_float2(nan, nan);
    } else {
      if (out_) static_cast<float *>(out_)[idx] = nan;
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
  }
}


// ---------------------------------------------------------------------------
// Tiled interpolation over the registered detector.  One block of kTile
// threads takes one orientation and one detector tile (kTile consecutive
// points of the Hilbert-ordered template, hence a compact patch): the rotated points' support
// cells span a small axis-aligned brick of the fine grid, which the block
// stages in LDS with coalesced row reads; the w^3 gather then reads LDS
// instead of L1/L2.  A brick larger than the LDS budget (possible only for
// unusually spread tiles) makes the block gather from global memory.
// LDS budget of a brick: 29 KB of float (5 blocks per CU, the kernel then
// fits in 81 registers) or 64 KB of float2 cells.
template <bool CPLX>
constexpr int brick_bytes() { return CPLX ? 65536 : 29696; }

// The LDS serves 128 bytes per cycle: a wavefront's reads of T cells go
// through in passes of 128 / sizeof(T) lanes, and bank conflicts arise
// among the lanes of one pass.  kLayouts candidate brick layouts are scored
// per block.
constexpr int kLayouts = 8;

// v mod n in [0, n); the common case (v within one period of the range)
// takes one conditional add, the integer division only the rest.
__device__ inline int wrap_mod(int v, int n) {
  v += v < 0 ? n : 0;
  if ((unsigned)v >= (unsigned)n) {
    v %= n;
    v += v < 0 ? n : 0;
  }
  return v;
}

template <int W, bool CPLX>
__global__ __launch_bounds__(kTile, CPLX ? 4 : 5) void interp_tiled_kernel(
    const void *__restrict__ u_, int nf, float beta, const double *__restrict__ rot, int64_t M,
    const float *__restrict__ dets, const int32_t *__restrict__ perm, int64_t P, int tiles,
    void *__restrict__ out_) {
  typedef typename std::conditional<CPLX, float2, float>::type T;
  constexpr int kCap = brick_bytes<CPLX>() / (int)sizeof(T);
  __shared__ __attribute__((aligned(16))) T brick[kCap];
  __shared__ int red[4][6];
  __shared__ int wrap[3][64];
  __shared__ int layout[1];

  const int vb = (int)xcd_contiguous_block();   // the grid has < 2^31 blocks
  const int64_t m = vb / tiles;
  const int tile = vb - (int)m * tiles;
  const int64_t i = (int64_t)tile * kTile + threadIdx.x;
  const bool inb = i < P;
  const double *R = rot + 9 * m;   // block-uniform: scalar loads
  const bool qok = R[0] == R[0];
  int l0[3] = {0, 0, 0};
  float frac[3] = {0.f, 0.f, 0.f};
  bool valid = inb && qok;
  if (valid) {
    const double q0 = dets[3 * i], q1 = dets[3 * i + 1], q2 = dets[3 * i + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = R[3 * d] * q0 + R[3 * d + 1] * q1 + R[3 * d + 2] * q2;
      if (!(fabs(t) < 1e8)) {
        valid = false;
      } else {
        const double c = ceil(t - 0.5 * W);
        l0[d] = (int)c;
        frac[d] = (float)(t - c);
      }
    }
  }
  int mn[3], mx[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mn[d] = valid ? l0[d] : 0x7fffffff;
    mx[d] = valid ? l0[d] : -0x7fffffff;
  }
  block_minmax3(mn, mx, red);
  const bool any = mn[0] <= mx[0];
  const int e0 = mx[0] - mn[0] + W, e1 = mx[1] - mn[1] + W, e2 = mx[2] - mn[2] + W;
  // Brick layout: cell (x0, x1, x2) at x0 * s0 + x1 * p2 + x2, with the row
  // pitch p2 >= p4 (e2 rounded up to whole 16-byte segments, so a segment
  // store never spills into the next row) and the plane stride
  // s0 >= e1 * p2.  The small paddings are chosen per block: a wavefront's
  // 64 lanes read 64 cells at a common offset from their support origins,
  // so the LDS bank conflicts of every gather read are those of the lanes'
  // origin addresses.  The first wavefront scores each candidate layout by
  // letting every lane write its origin address into a table slot named by
  // the address's bank group (one table per LDS pass of lanes) and read the
  // slot back: a lane that finds another address there shares its banks
  // with a different cell in its pass.  The candidate with the fewest such
  // lanes wins (ties: the first); the other wavefronts' patches lie next to
  // the first's, under the same rotation, and share its choice.  Eight
  // candidates (row paddings 0-3, plane offsets 0 and 2) choose as well as
  // sixteen (offsets 0-3) at half the probe's cost.
  constexpr int kVec = 16 / (int)sizeof(T);
  const int nseg = (e2 + kVec - 1) / kVec;
  const int p4 = nseg * kVec;
  const bool use_lds = any && e0 <= 64 && e1 <= 64 && e2 <= 64 && e0 * e1 * p4 <= kCap;
  const bool choose = use_lds && e0 * (e1 * (p4 + 3) + 2) <= kCap;
  if (use_lds && threadIdx.x < 64) {
    // fine-grid offsets of every brick plane, row and column, wrapped once
    // per block (n_f <= 1022, so n_f^3 cells index in 32 bits)
    const int t = threadIdx.x, half = nf >> 1;
    if (t < e0) wrap[0][t] = wrap_mod(mn[0] + t + half, nf) * nf * nf;
    if (t < e1) wrap[1][t] = wrap_mod(mn[1] + t + half, nf) * nf;
    if (t < e2) wrap[2][t] = wrap_mod(mn[2] + t + half, nf);
    if (choose) {
      // candidate c = 2 pe + d / 2: p2 = p4 + pe, s0 = e1 p2 + d (d = 0, 2),
      // so the origin address is row * (p4 + pe) + d * x0 + x2 with
      // row = x0 e1 + x1
      const int x0 = l0[0] - mn[0], row = x0 * e1 + (l0[1] - mn[1]);
      // a table per candidate and pass of kPass lanes, one slot per bank
      // group (cell address mod kPass) plus one for invalid lanes
      constexpr int kPass = 128 / (int)sizeof(T), kPasses = 64 / kPass;
      int *tab = reinterpret_cast<int *>(brick) + (t / kPass) * (kPass + 1);
      int addr[kLayouts], slot[kLayouts];
      int a_pe = row * p4 + (l0[2] - mn[2]);
#pragma unroll
      for (int pe = 0; pe < 4; ++pe) {
        int a = a_pe;
#pragma unroll
        for (int dd = 0; dd < 2; ++dd) {
          const int c = 2 * pe + dd;
          addr[c] = a;
          slot[c] = kPasses * c * (kPass + 1) + (valid ? (a & (kPass - 1)) : kPass);
          tab[slot[c]] = a;
          a += 2 * x0;
        }
        a_pe += row;
      }
      // The read-back must see the other lanes' writes, not this lane's own
      // store forwarded by the compiler: a compiler memory barrier keeps the
      // loads after the stores, and a wavefront's LDS accesses complete in
      // order, so every write has landed before the reads.
      __asm__ __volatile__("" ::: "memory");
      int got[kLayouts];
#pragma unroll
      for (int c = 0; c < kLayouts; ++c) got[c] = tab[slot[c]];
      int best_key = 0x7fffffff;
#pragma unroll
      for (int c = 0; c < kLayouts; ++c) {
        const int n = __popcll(__ballot(valid && got[c] != addr[c]));
        best_key = min(best_key, (n << 4) | c);
      }
      if (t == 0) layout[0] = best_key & 15;   // c < 8
    }
  }
  if (use_lds) __syncthreads();
  int p2 = p4, s0 = e1 * p4;
  if (choose) {
    const int best = layout[0];
    p2 = p4 + (best >> 1);
    s0 = e1 * p2 + 2 * (best & 1);
  }
  const T *u = static_cast<const T *>(u_);
  if (use_lds) {
    // The brick holds e0 x e1 rows of e2 cells.  When a row neither wraps
    // nor reaches the end of a fine-grid row, it is moved in 16-byte
    // segments (kVec cells; the last segment may read up to kVec - 1 cells
    // past the brick row, still inside the same fine-grid row, into the
    // row's padding); otherwise one cell at a time.  Several loads per
    // thread are in flight before their stores.  Quotients by small extents
    // e <= 64 use a float reciprocal: the exact quotient (n + 1/2) / e lies
    // at least 1 / (2 e) >= 1/128 from an integer, far above the product's
    // error (quotients below 2^13, the reciprocal within 1 ulp).
    const int g2 = wrap[2][0];
    const bool rows_contiguous = g2 + p4 <= nf;
    const float inv_e1 = __builtin_amdgcn_rcpf((float)e1);
    if (rows_contiguous) {
      const int items = e0 * e1 * nseg;
      const float inv_ns = __builtin_amdgcn_rcpf((float)nseg);
      for (int c0 = threadIdx.x; c0 < items; c0 += 4 * kTile) {
        T v[4][kVec];
        int dst[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = c0 + k * kTile;
          if (c < items) {
            const int r = (int)(((float)c + 0.5f) * inv_ns);
            const int q = c - r * nseg;
            const int a = (int)(((float)r + 0.5f) * inv_e1);
            const int b = r - a * e1;
            const T *src = u + (wrap[0][a] + wrap[1][b] + g2 + q * kVec);
            __builtin_memcpy(&v[k][0], src, 16);
            dst[k] = a * s0 + b * p2 + q * kVec;
          }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (c0 + k * kTile < items) {
#pragma unroll
            for (int e = 0; e < kVec; ++e) brick[dst[k] + e] = v[k][e];
          }
        }
      }
    } else {
      const int cells = e0 * e1 * e2;
      const float inv_e2 = __builtin_amdgcn_rcpf((float)e2);
      for (int c0 = threadIdx.x; c0 < cells; c0 += 8 * kTile) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + k * kTile;
          if (c < cells) {
            const int r = (int)(((float)c + 0.5f) * inv_e2);
            const int cc = c - r * e2;
            const int a = (int)(((float)r + 0.5f) * inv_e1);
            const int b = r - a * e1;
            v[k] = u[wrap[0][a] + wrap[1][b] + wrap[2][cc]];
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + k * kTile;
          if (c < cells) {
            const int r = (int)(((float)c + 0.5f) * inv_e2);
            const int a = (int)(((float)r + 0.5f) * inv_e1);
            brick[a * s0 + (r - a * e1) * p2 + (c - r * e2)] = v[k];
          }
        }
      }
    }
  }
  float w0[W], w1[W], w2[W];
  if (valid) {
    es_weights<W>(frac[0], beta, w0);
    es_weights<W>(frac[1], beta, w1);
    es_weights<W>(frac[2], beta, w2);
  }
  if (use_lds) __syncthreads();
  if (!inb) return;
  const int64_t o = m * P + perm[i];
  if (!valid) {
    const float nan = __uint_as_float(0x7fc00000u);
    if (CPLX) {
      if (out_) static_cast<float2 *>(out_)[o] = make_float2(nan, nan);
    } else {
      if (out_) static_cast<float *>(out_)[o] = nan;
    }
    return;
  }
  float sr = 0.f, si = 0.f;
  if (use_lds) {
    const int base = (l0[0] - mn[0]) * s0 + (l0[1] - mn[1]) * p2 + (l0[2] - mn[2]);
#pragma unroll
    for (int a = 0; a < W; ++a) {
      float pr = 0.f, pi = 0.f;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const T *row = brick + base + a * s0 + b * p2;
        float rr = 0.f, ri = 0.f;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          if constexpr (CPLX) {
            const float2 v = row[c];
            rr = fmaf(w2[c], v.x, rr);
            ri = fmaf(w2[c], v.y, ri);
          } else {
            rr = fmaf(w2[c], row[c], rr);
          }
        }
        pr = fmaf(w1[b], rr, pr);
        if (CPLX) pi = fmaf(w1[b], ri, pi);
      }
      sr = fmaf(w0[a], pr, sr);
      if (CPLX) si = fmaf(w0[a], pi, si);
    }
  } else {
    int g0[W], g1[W], g2[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
      g0[a] = wrap_mod(l0[0] + a + (nf >> 1), nf);
      g1[a] = wrap_mod(l0[1] + a + (nf >> 1), nf);
      g2[a] = wrap_mod(l0[2] + a + (nf >> 1), nf);
    }
#pragma unroll
    for (int a = 0; a < W; ++a) {
      float pr = 0.f, pi = 0.f;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const T *row = u + ((int64_t)g0[a] * nf + g1[b]) * nf;
        float rr = 0.f, ri = 0.f;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          if constexpr (CPLX) {
            const float2 v = row[g2[c]];
            rr = fmaf(w2[c], v.x, rr);
            ri = fmaf(w2[c], v.y, ri);
          } else {
            rr = fmaf(w2[c], row[g2[c]], rr);
          }
        }
        pr = fmaf(w1[b], rr, pr);
        if (CPLX) pi = fmaf(w1[b], ri, pi);
      }
      sr = fmaf(w0[a], pr, sr);
      if (CPLX) si = fmaf(w0[a], pi, si);
    }
  }
  if (CPLX) {
    if (out_) static_cast<float2 *>(out_)[o] = make_float2(sr, si);
  } else {
    if (out_) static_cast<float *>(out_)[o] = sr;
  }
}

template <int W>
static hipError_t interp_w(const Plan &pl, const double *rot, int64_t M, const float *detq,
                           int64_t P, void *out, hipStream_t s) {
  const bool cplx = pl.domain == SPFEL_COMPLEX;
  if (detq == nullptr) {
    const int tiles = (int)((P + kTile - 1) / kTile);
    const int64_t blocks = M * tiles;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (cplx)
      hipLaunchKernelGGL((interp_tiled_kernel<W, true>), dim3((unsigned)blocks), dim3(kTile), 0, s,
                         pl.u, pl.nf, (float)pl.beta, rot, M, pl.det_sorted, pl.det_perm, P,
                         tiles, out);
    else
      hipLaunchKernelGGL((interp_tiled_kernel<W, false>), dim3((unsigned)blocks), dim3(kTile), 0,
                         s, pl.u, pl.nf, (float)pl.beta, rot, M, pl.det_sorted, pl.det_perm, P,
                         tiles, out);
    return hipGetLastError();
  }
  const int64_t total = M * P;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (cplx)
    hipLaunchKernelGGL((interp_gather_kernel<W, true>), grid, block, 0, s, pl.u, pl.nf,
                       (float)pl.beta, rot, M, detq, P, out);
  else
    hipLaunchKernelGGL((interp_gather_kernel<W, false>), grid, block, 0, s, pl.u, pl.nf,
                       (float)pl.beta, rot, M, detq, P, out);
  return hipGetLastError();
}

// Orientations go in batches of kRotCap: each batch's scaled rotations are
// computed into the plan's table, then its points are interpolated.
hipError_t launch_interp(const Plan &pl, const float *quats, int64_t M, const float *detq,
                         int64_t P, void *out, hipStream_t s) {
  const size_t el = pl.domain == SPFEL_COMPLEX ? 8 : 4;
  const double scale = (double)pl.nf / (2.0 * M_PI);
  for (int64_t m0 = 0; m0 < M; m0 += kRotCap) {
    const int64_t mc = M - m0 < kRotCap ? M - m0 : kRotCap;
    hipLaunchKernelGGL(rotation_kernel, dim3((unsigned)((mc + 255) / 256)), dim3(256), 0, s,
                       quats + 4 * m0, mc, scale, pl.rot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void *o = out ? static_cast<char *>(out) + (size_t)m0 * P * el : nullptr;
    switch (pl.w) {
      case 4: e = interp_w<4>(pl, pl.rot, mc, detq, P, o, s); break;
      case 5: e = interp_w<5>(pl, pl.rot, mc, detq, P, o, s); break;
      case 6: e = interp_w<6>(pl, pl.rot, mc, detq, P, o, s); break;
      case 7: e = interp_w<7>(pl, pl.rot, mc, detq, P, o, s); break;
      default: e = interp_w<8>(pl, pl.rot, mc, detq, P, o, s); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Squared norm of each row: 256 threads take strided partial sums (one
// fused multiply-add per element), then a pairwise tree in LDS; the order
// is fixed, so the result is deterministic.
template <bool BF>
__global__ __launch_bounds__(256) void row_norm2_kernel(const void *__restrict__ x_, int64_t cols,
                                                        float *__restrict__ out, int vec) {
  __shared__ float sh[256];
  const int64_t row = blockIdx.x;
  float acc = 0.f;
  if (vec) {
    // 16-byte aligned rows of a whole number of 16-byte groups: each thread
    // takes whole groups (8 bf16 or 4 float), in order
    const uint4 *x = reinterpret_cast<const uint4 *>(static_cast<const char *>(x_) +
                                                     row * cols * (BF ? 2 : 4));
    const int64_t groups = cols / (BF ? 8 : 4);
    for (int64_t g = threadIdx.x; g < groups; g += 256) {
      const uint4 v = x[g];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (BF) {
          const float lo = __uint_as_float(w[e] << 16), hi = __uint_as_float(w[e] & 0xffff0000u);
          acc = fmaf(lo, lo, acc);
          acc = fmaf(hi, hi, acc);
        } else {
          const float f = __uint_as_float(w[e]);
          acc = fmaf(f, f, acc);
        }
      }
    }
  } else if (BF) {
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
  const int vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0 && cols % (bf16 ? 8 : 4) == 0;
  if (bf16)
    hipLaunchKernelGGL((row_norm2_kernel<true>), dim3((unsigned)rows), dim3(256), 0, s, x, cols, out, vec);
  else
    hipLaunchKernelGGL((row_norm2_kernel<false>), dim3((unsigned)rows), dim3(256), 0, s, x, cols, out, vec);
  return hipGetLastError();
}

}  // namespace spfel
