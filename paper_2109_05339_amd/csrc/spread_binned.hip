// Binned type-1 spreading over the registered detector (merging A*, section
// II-C Eq. (2)): every value y at a rotated Ewald-sphere point adds
// y psi psi psi to the w^3 fine-grid cells of its support.
//
// Points of many images are grouped by the fine-grid bin of their support
// origin, so that one block accumulates the stencils of thousands of
// points (from any image) into one brick before a single flush:
//   * bins: cubes of Bo = 17 - w support origins per axis, each with a
//     16 x 16 x 16 brick that holds every support cell of its points;
//   * pass 1 counts the points per (bin, axis-1 origin) key, a scan turns
//     the counts into offsets, and pass 2 scatters each point's value,
//     kernel offsets and origin to its key's slot (points of a bin thus
//     sorted by axis-1 origin);
//   * each bin's points are cut into subproblems of at most kSubMax;
//   * one block per subproblem: the brick lives in registers as 16 planes
//     (axis 1) of 16 x 16 (axis 0 x axis 2) v_mfma_f32_16x16x4f32
//     accumulators; four points per matrix step, each contributing
//     (y psi0 psi1[plane]) (row) times psi2 (column); only the planes a
//     group of four consecutive points reaches are stepped;
//   * the four wavefronts' bricks are summed in LDS in a fixed order and
//     added to the fine grid with one global atomic per nonzero cell.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace spfel {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int W>
constexpr int bin_origins() { return kBrick - W + 1; }

// Support origin (wrapped into [0, nf)) and kernel offsets of point i of
// the registered template under the scaled rotation Rs = R n_f / (2 pi)
// (the slicing kernels' coordinates, so both directions take the same
// support decisions).
template <int W>
__device__ inline bool point_support(const double *__restrict__ Rs, const float *__restrict__ dets,
                                     int64_t i, int nf, int (&L)[3], float (&frac)[3]) {
  const double q0 = dets[3 * i], q1 = dets[3 * i + 1], q2 = dets[3 * i + 2];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = Rs[3 * d] * q0 + Rs[3 * d + 1] * q1 + Rs[3 * d + 2] * q2;
    if (!(fabs(t) < 1e8)) return false;
    const double c = ceil(t - 0.5 * W);
    frac[d] = (float)(t - c);
    // c mod nf (|c| < 1e8 + W fits an int); points within one period of
    // the grid take the conditional add only
    int ci = (int)c;
    ci += ci < 0 ? nf : 0;
    if ((unsigned)ci >= (unsigned)nf) {
      ci %= nf;
      ci += ci < 0 ? nf : 0;
    }
    L[d] = ci;
  }
  return true;
}

// Block of kTile points (one image, one tile of the registered template):
// each valid point's key in an LDS table (one slot per distinct key; the
// table has as many slots as the block has points, so it never fills).
// Returns the point's slot (or -1) and its rank among the block's points
// of that key.
constexpr int kHash = kTile;

__device__ inline int table_insert(int *tkey, int *tcnt, int key, int &rank) {
  int h = (int)(((unsigned)key * 2654435761u) >> 24) & (kHash - 1);
  for (int probe = 0; probe < kHash; ++probe) {
    const int prev = atomicCAS(&tkey[h], -1, key);
    if (prev == -1 || prev == key) {
      rank = atomicAdd(&tcnt[h], 1);
      return h;
    }
    h = (h + 1) & (kHash - 1);
  }
  return -1;   // unreachable: at most kHash distinct keys per block
}

struct BinPoint {
  bool ok;
  int key, o0, o1, o2;
  float frac[3];
  float yr, yi;
};

template <int W, bool CPLX>
__device__ inline BinPoint bin_point(const double *__restrict__ rot, int64_t n0, int64_t n,
                                     int64_t i, bool inb,
                                     const float *__restrict__ dets, const int32_t *__restrict__ perm,
                                     int64_t P, int nf, int nb, const void *__restrict__ values,
                                     const float *__restrict__ weights, bool want_value) {
  constexpr int Bo = bin_origins<W>();
  BinPoint b;
  b.ok = false;
  b.key = 0;
  b.o0 = b.o1 = b.o2 = 0;
  b.yr = b.yi = 0.f;
  const double *Rs = rot + 9 * (n - n0);   // block-uniform
  if (!inb || !(Rs[0] == Rs[0])) return b;
  int L[3];
  if (!point_support<W>(Rs, dets, i, nf, L, b.frac)) return b;
  const int b0 = L[0] / Bo, b1 = L[1] / Bo, b2 = L[2] / Bo;
  b.o0 = L[0] - b0 * Bo;
  b.o1 = L[1] - b1 * Bo;
  b.o2 = L[2] - b2 * Bo;
  b.key = ((b0 * nb + b1) * nb + b2) * Bo + b.o1;
  b.ok = true;
  if (want_value) {
    const int64_t o = n * P + perm[i];
    if (CPLX) {
      const float2 v = static_cast<const float2 *>(values)[o];
      b.yr = v.x;
      b.yi = v.y;
    } else {
      b.yr = static_cast<const float *>(values)[o];
    }
    if (weights) {
      const float wt = weights[o];
      b.yr *= wt;
      b.yi *= wt;
    }
  }
  return b;
}

// Pass 1: points per key.
template <int W, bool CPLX>
__global__ __launch_bounds__(kTile) void bin_count_kernel(
    const double *__restrict__ rot, int64_t n0, const float *__restrict__ dets,
    const int32_t *__restrict__ perm, int64_t P, int tiles, int nf, int nb,
    int32_t *__restrict__ counts) {
  __shared__ int tkey[kHash], tcnt[kHash];
  const int64_t vb = xcd_contiguous_block();
  const int64_t n = n0 + vb / tiles;
  const int tile = (int)(vb % tiles);
  const int64_t i = (int64_t)tile * kTile + threadIdx.x;
  tkey[threadIdx.x] = -1;
  tcnt[threadIdx.x] = 0;
  __syncthreads();
  const BinPoint b = bin_point<W, CPLX>(rot, n0, n, i, i < P, dets, perm, P, nf, nb, nullptr,
                                        nullptr, false);
  if (b.ok) {
    int rank;
    table_insert(tkey, tcnt, b.key, rank);
  }
  __syncthreads();
  if (tkey[threadIdx.x] >= 0) atomicAdd(&counts[tkey[threadIdx.x]], tcnt[threadIdx.x]);
}

// Pass 2: each point to its key's next slot.  aux = (packed origin,
// imaginary value bits); REAL stores the packed origin alone, as an array
// of 32-bit words.
template <int W, bool CPLX>
__global__ __launch_bounds__(kTile) void bin_scatter_kernel(
    const double *__restrict__ rot, int64_t n0, const float *__restrict__ dets,
    const int32_t *__restrict__ perm, int64_t P, int tiles, int nf, int nb,
    const void *__restrict__ values, const float *__restrict__ weights,
    int32_t *__restrict__ cursor, float4 *__restrict__ pts, uint2 *__restrict__ aux) {
  __shared__ int tkey[kHash], tcnt[kHash], tbase[kHash];
  const int64_t vb = xcd_contiguous_block();
  const int64_t n = n0 + vb / tiles;
  const int tile = (int)(vb % tiles);
  const int64_t i = (int64_t)tile * kTile + threadIdx.x;
  tkey[threadIdx.x] = -1;
  tcnt[threadIdx.x] = 0;
  __syncthreads();
  const BinPoint b = bin_point<W, CPLX>(rot, n0, n, i, i < P, dets, perm, P, nf, nb, values,
                                        weights, true);
  int slot = -1, rank = 0;
  if (b.ok) slot = table_insert(tkey, tcnt, b.key, rank);
  __syncthreads();
  if (tkey[threadIdx.x] >= 0)
    tbase[threadIdx.x] = atomicAdd(&cursor[tkey[threadIdx.x]], tcnt[threadIdx.x]);
  __syncthreads();
  if (slot >= 0) {
    const int pos = tbase[slot] + rank;
    pts[pos] = make_float4(b.yr, b.frac[0], b.frac[1], b.frac[2]);
    const uint32_t packed = (uint32_t)(b.o0 | (b.o1 << 4) | (b.o2 << 8));
    if (CPLX)
      aux[pos] = make_uint2(packed, __float_as_uint(b.yi));
    else
      reinterpret_cast<uint32_t *>(aux)[pos] = packed;   // REAL: one word per point
  }
}

// Exclusive scan of n counts into off[0..n] (off[n] = total), in three
// launches: per-1024-element block scans, a scan of the block totals, and
// the block offsets added back (also copied to the scatter cursors).
constexpr int kScanBlock = 1024;

// (in and out may be the same array: every thread reads its four counts
// before any thread writes)
__global__ __launch_bounds__(256) void scan_local_kernel(const int32_t *in, int64_t n, int32_t *out,
                                                         int32_t *__restrict__ part) {
  __shared__ int32_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int32_t v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele over thread sums
    const int32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - s;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) part[blockIdx.x] = sh[255];
}

__global__ __launch_bounds__(256) void scan_part_kernel(int32_t *__restrict__ part, int nparts,
                                                        int32_t *__restrict__ total) {
  __shared__ int32_t sh[256];
  int32_t carry = 0;
  for (int c0 = 0; c0 < nparts; c0 += 256) {
    const int i = c0 + (int)threadIdx.x;
    const int32_t v = i < nparts ? part[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nparts) part[i] = carry + sh[threadIdx.x] - v;
    const int32_t blk = sh[255];
    __syncthreads();
    carry += blk;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void scan_add_kernel(int32_t *__restrict__ off, int64_t n,
                                                       const int32_t *__restrict__ part,
                                                       int32_t *__restrict__ cursor) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t v = off[i] + part[i / kScanBlock];
    off[i] = v;
    cursor[i] = v;
  }
}

// Subproblems: each bin's points (contiguous, keys bin * Bo .. bin * Bo +
// Bo - 1) cut into runs of at most kSubMax.
__global__ __launch_bounds__(256) void subproblem_kernel(const int32_t *__restrict__ off, int nbins,
                                                         int Bo, int32_t *__restrict__ nsub,
                                                         int4 *__restrict__ sub) {
  const int bin = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (bin >= nbins) return;
  const int start = off[(int64_t)bin * Bo], end = off[(int64_t)(bin + 1) * Bo];
  if (end <= start) return;
  const int ns = (end - start + kSubMax - 1) / kSubMax;
  const int base = atomicAdd(nsub, ns);
  for (int j = 0; j < ns; ++j)
    sub[base + j] = make_int4(bin, start + j * kSubMax, min(end, start + (j + 1) * kSubMax), 0);
}

// One block per subproblem (blocks past the device-side count exit).  The
// subproblem's points are sorted by axis-1 origin v; the key offsets give
// the run of each v.  For each v in turn (unrolled at compile time), the
// four wavefronts split the run into batches of 64 points (batch k of wave
// w: points 256 k + 64 w .. + 63 of the run), with no block barrier: a
// wavefront's lanes turn their points into brick-shifted weight rows in the
// wavefront's own LDS rows, then the wavefront steps its accumulators of
// planes v .. v + w - 1 over them, four points per matrix step.  One
// wavefront's transcendental weights thus overlap another's matrix steps.
template <int W, bool CPLX>
__global__ __launch_bounds__(256) void spread_binned_kernel(
    float *__restrict__ grid, int nf, float beta, int nb, const float4 *__restrict__ pts,
    const uint2 *__restrict__ aux, const int32_t *__restrict__ off, const int4 *__restrict__ sub,
    const int32_t *__restrict__ nsub) {
  constexpr int Bo = bin_origins<W>();
  constexpr int kPer = 64;                 // points per wavefront batch
  constexpr int kA = CPLX ? 2 : 1;
  // per wavefront and batch point: the brick-shifted rows y psi0 (re[, im])
  // and psi2 over the 16 brick cells of axes 0 and 2, and psi1 (its w
  // values).  Rows past the batch's points are zero: the lanes past the
  // batch write zero rows, and rows kPer .. kRows - 1 stay zero, so the
  // matrix steps (which read up to seven rows past the last point) need no
  // bound on their row index.  The psi1 rows have an odd pitch (9), so the
  // lanes writing their points' rows fall in distinct banks.
  constexpr int kRows = kPer + 7;
  __shared__ __attribute__((aligned(16))) float rowA[4][kA][kRows][kBrick];
  __shared__ __attribute__((aligned(16))) float rowB[4][kRows][kBrick];
  __shared__ __attribute__((aligned(16))) float rowC[4][kRows][9];
  if ((int)blockIdx.x >= *nsub) return;   // block-uniform
  const int4 sp = sub[blockIdx.x];
  const int bin = sp.x, start = sp.y, end = sp.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;

  floatx4 accr[kBrick], acci[CPLX ? kBrick : 1];
#pragma unroll
  for (int p = 0; p < kBrick; ++p) {
    accr[p] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (CPLX) acci[CPLX ? p : 0] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  for (int e = lane; e < (kRows - kPer) * kBrick; e += 64) {
    const int row = kPer + e / kBrick, col = e % kBrick;
    rowA[wave][0][row][col] = 0.f;
    if (CPLX) rowA[wave][kA - 1][row][col] = 0.f;
    rowB[wave][row][col] = 0.f;
    if (col < 9) rowC[wave][row][col] = 0.f;
  }
  const int64_t key0 = (int64_t)bin * Bo;
  // matrix-step reads: lane (r, kq) takes column r of row p0 + kq, a
  // per-lane base plus a wavefront-uniform row offset
  const float *const rdA = &rowA[wave][0][0][0] + kq * kBrick + r;
  const float *const rdAi = &rowA[wave][kA - 1][0][0] + kq * kBrick + r;
  const float *const rdB = &rowB[wave][0][0] + kq * kBrick + r;
  const float *const rdC = &rowC[wave][0][0] + kq * 9;

  auto run = [&](auto vc) {
    constexpr int V = decltype(vc)::value;
    const int lo = max(start, off[key0 + V]), hi = min(end, off[key0 + V + 1]);
    for (int b0 = lo + wave * kPer; b0 < hi; b0 += 4 * kPer) {
      const int cnt = min(kPer, hi - b0);
      // this batch's rows (the previous batch's reads were issued before
      // these writes, and a wavefront's LDS accesses complete in order)
      __builtin_amdgcn_wave_barrier();
      {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          reinterpret_cast<float4 *>(rowA[wave][0][lane])[q] = z;
          reinterpret_cast<float4 *>(rowB[wave][lane])[q] = z;
          if (CPLX) reinterpret_cast<float4 *>(rowA[wave][kA - 1][lane])[q] = z;
        }
      }
      if (lane >= cnt) {
#pragma unroll
        for (int a = 0; a < W; ++a) rowC[wave][lane][a] = 0.f;
      } else {
        const float4 pv = pts[b0 + lane];
        const uint2 ax = CPLX ? aux[b0 + lane]
                              : make_uint2(reinterpret_cast<const uint32_t *>(aux)[b0 + lane], 0u);
        const int o0 = ax.x & 15, o2 = (ax.x >> 8) & 15;
        float w0[W], w1[W], w2[W];
        es_weights<W>(pv.y, beta, w0);
        es_weights<W>(pv.z, beta, w1);
        es_weights<W>(pv.w, beta, w2);
        const float yi = __uint_as_float(ax.y);
#pragma unroll
        for (int a = 0; a < W; ++a) {
          rowA[wave][0][lane][o0 + a] = pv.x * w0[a];
          if (CPLX) rowA[wave][kA - 1][lane][o0 + a] = yi * w0[a];
          rowB[wave][lane][o2 + a] = w2[a];
          rowC[wave][lane][a] = w1[a];
        }
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wavefront's rows are written
      __builtin_amdgcn_wave_barrier();
      // Matrix steps of four points, software-pipelined over two register
      // sets: the next step's rows are read from LDS before this step's
      // matrix instructions issue (the scheduling barriers keep them there).
      const int ucnt = __builtin_amdgcn_readfirstlane(cnt);
      auto fetch = [&](int p0, float &fa, float &fai, float &fb, float (&fc)[W]) {
        fa = rdA[p0 * kBrick];
        fai = CPLX ? rdAi[p0 * kBrick] : 0.f;
        fb = rdB[p0 * kBrick];
#pragma unroll
        for (int d = 0; d < W; ++d) fc[d] = rdC[p0 * 9 + d];
      };
      auto step = [&](float a, float ai, float bv, const float (&c)[W]) {
#pragma unroll
        for (int d = 0; d < W; ++d) {
          accr[V + d] = __builtin_amdgcn_mfma_f32_16x16x4f32(a * c[d], bv, accr[V + d], 0, 0, 0);
          if (CPLX)
            acci[CPLX ? V + d : 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                ai * c[d], bv, acci[CPLX ? V + d : 0], 0, 0, 0);
        }
      };
      float xa0, xi0, xb0, xc0[W], xa1, xi1, xb1, xc1[W];
      fetch(0, xa0, xi0, xb0, xc0);
      // The first step's values pass through an empty asm statement: with
      // only loads flowing into the loop-carried set the compiler would fold
      // them into one load at the use, undoing the pipelining.
      __asm__ __volatile__("" : "+v"(xa0), "+v"(xi0), "+v"(xb0));
#pragma unroll
      for (int d = 0; d < W; ++d) __asm__ __volatile__("" : "+v"(xc0[d]));
      for (int p0 = 0; p0 < ucnt; p0 += 8) {
        fetch(p0 + 4, xa1, xi1, xb1, xc1);
        __builtin_amdgcn_sched_barrier(0);
        step(xa0, xi0, xb0, xc0);
        __builtin_amdgcn_sched_barrier(0);
        if (p0 + 4 >= ucnt) break;   // wavefront-uniform
        fetch(p0 + 8, xa0, xi0, xb0, xc0);
        __builtin_amdgcn_sched_barrier(0);
        step(xa1, xi1, xb1, xc1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  run(std::integral_constant<int, 0>{});
  run(std::integral_constant<int, 1>{});
  run(std::integral_constant<int, 2>{});
  run(std::integral_constant<int, 3>{});
  run(std::integral_constant<int, 4>{});
  run(std::integral_constant<int, 5>{});
  run(std::integral_constant<int, 6>{});
  run(std::integral_constant<int, 7>{});
  run(std::integral_constant<int, 8>{});
  if constexpr (Bo > 9) run(std::integral_constant<int, (Bo > 9 ? 9 : 0)>{});
  if constexpr (Bo > 10) run(std::integral_constant<int, (Bo > 10 ? 10 : 0)>{});
  if constexpr (Bo > 11) run(std::integral_constant<int, (Bo > 11 ? 11 : 0)>{});
  if constexpr (Bo > 12) run(std::integral_constant<int, (Bo > 12 ? 12 : 0)>{});
  // Sum the four wavefronts' bricks in LDS (wave 0 stores, then waves 1-3
  // add in order), then flush.  Result lane layout: lane l holds
  // accumulator plane pl, rows 4 (l / 16) + j (axis 0), column l % 16 (axis
  // 2).  Each axis-0 slab of 256 cells is padded by 4 floats, so the four
  // 16-lane groups of a wavefront (slabs 4 apart) fall in distinct banks.
  __syncthreads();
  float *red = &rowA[0][0][0][0];   // kA x 16 x 260 floats fill rowA exactly
  static_assert(sizeof(rowA) >= sizeof(float) * kA * kBrick * (kBrick * kBrick + 4),
                "reduction buffer");
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int pl = 0; pl < kBrick; ++pl)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i0 = 4 * kq + j;
          const int c = (i0 * kBrick + pl) * kBrick + r + 4 * i0;
          if (wv == 0) {
            red[kA * c] = accr[pl][j];
            if (CPLX) red[kA * c + 1] = acci[CPLX ? pl : 0][j];
          } else {
            red[kA * c] += accr[pl][j];
            if (CPLX) red[kA * c + 1] += acci[CPLX ? pl : 0][j];
          }
        }
    }
    __syncthreads();
  }
  const int bb2 = bin % nb, bb1 = (bin / nb) % nb, bb0 = bin / (nb * nb);
  const int lo0 = bb0 * Bo, lo1 = bb1 * Bo, lo2 = bb2 * Bo;
  for (int c = tid; c < kBrick * kBrick * kBrick; c += 256) {
    const int i2 = c & 15, i1 = (c >> 4) & 15, i0 = c >> 8;
    // lo < nf and i < 16: one subtraction wraps unless the grid is
    // smaller than a brick
    int g0 = lo0 + i0, g1 = lo1 + i1, g2 = lo2 + i2;
    if (g0 >= nf) g0 = nf >= kBrick ? g0 - nf : g0 % nf;
    if (g1 >= nf) g1 = nf >= kBrick ? g1 - nf : g1 % nf;
    if (g2 >= nf) g2 = nf >= kBrick ? g2 - nf : g2 % nf;
    const int64_t cell = ((int64_t)g0 * nf + g1) * nf + g2;
    const float vr = red[kA * (c + 4 * i0)];
    if (CPLX) {
      const float vi = red[kA * (c + 4 * i0) + 1];
      if (vr != 0.f) unsafeAtomicAdd(grid + 2 * cell, vr);
      if (vi != 0.f) unsafeAtomicAdd(grid + 2 * cell + 1, vi);
    } else {
      if (vr != 0.f) unsafeAtomicAdd(grid + cell, vr);
    }
  }
}

size_t bin_keys(int nf, int w) {
  const int Bo = kBrick - w + 1;
  const int nb = (nf + Bo - 1) / Bo;
  return (size_t)nb * nb * nb * Bo;
}

size_t bin_max_subproblems(int nf, int w, int64_t cap) {
  const int Bo = kBrick - w + 1;
  const int64_t nb = (nf + Bo - 1) / Bo;
  return (size_t)(cap / kSubMax + nb * nb * nb + 1);
}

template <int W, bool CPLX>
static hipError_t spread_binned_wc(const Plan &pl, const float *quats, int64_t n_img, int64_t P,
                                   const void *values, const float *weights, hipStream_t s) {
  constexpr int Bo = bin_origins<W>();
  const int nf = pl.nf;
  const int nb = (nf + Bo - 1) / Bo;
  const int64_t nbins = (int64_t)nb * nb * nb;
  const int64_t nkeys = nbins * Bo;
  const int tiles = (int)((P + kTile - 1) / kTile);
  const int64_t nparts = (nkeys + kScanBlock - 1) / kScanBlock;
  // Batch b is binned on the plan's stream into buffer set b % 2 and
  // spread on the caller's stream from it, so the binning of batch b + 1
  // (memory and atomics) runs beside the spread of batch b (matrix cores).
  // The plan's stream starts after the caller's work so far; every spread
  // waits for its batch's binning, and the binning of batch b + 2 for the
  // spread of batch b, which also orders all of it before the caller's
  // later work.
  hipStream_t bs = pl.bin_stream;
  hipError_t e = hipEventRecord(pl.ev_bin_start, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(bs, pl.ev_bin_start, 0);
  if (e != hipSuccess) return e;
  int64_t b = 0;
  for (int64_t n0 = 0; n0 < n_img; n0 += pl.bin_batch, ++b) {
    const int k = (int)(b & 1);
    const int64_t nbat = std::min<int64_t>(pl.bin_batch, n_img - n0);
    const int64_t blocks = nbat * tiles;
    if (b >= 2) {
      e = hipStreamWaitEvent(bs, pl.ev_spread[k], 0);
      if (e != hipSuccess) return e;
    }
    e = launch_rotations(quats + 4 * n0, nbat, (double)nf / (2.0 * M_PI), pl.rot, bs);
    if (e == hipSuccess) e = launch_fill_zero(pl.bin_off[k], (size_t)nkeys * 4, bs);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bin_count_kernel<W, CPLX>), dim3((unsigned)blocks), dim3(kTile), 0, bs,
                       pl.rot, n0, pl.det_sorted, pl.det_perm, P, tiles, nf, nb, pl.bin_off[k]);
    hipLaunchKernelGGL(scan_local_kernel, dim3((unsigned)nparts), dim3(256), 0, bs,
                       pl.bin_off[k], nkeys, pl.bin_off[k], pl.bin_part);
    hipLaunchKernelGGL(scan_part_kernel, dim3(1), dim3(256), 0, bs, pl.bin_part, (int)nparts,
                       pl.bin_off[k] + nkeys);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((nkeys + 255) / 256)), dim3(256), 0, bs,
                       pl.bin_off[k], nkeys, pl.bin_part, pl.bin_cur);
    e = launch_fill_zero(pl.bin_nsub[k], 4, bs);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(subproblem_kernel, dim3((unsigned)((nbins + 255) / 256)), dim3(256), 0, bs,
                       pl.bin_off[k], (int)nbins, Bo, pl.bin_nsub[k], pl.bin_sub[k]);
    hipLaunchKernelGGL((bin_scatter_kernel<W, CPLX>), dim3((unsigned)blocks), dim3(kTile), 0, bs,
                       pl.rot, n0, pl.det_sorted, pl.det_perm, P, tiles, nf, nb, values, weights,
                       pl.bin_cur, pl.bin_pts[k], pl.bin_aux[k]);
    e = hipEventRecord(pl.ev_binned[k], bs);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, pl.ev_binned[k], 0);
    if (e != hipSuccess) return e;
    const int64_t maxsub = (int64_t)bin_max_subproblems(nf, W, nbat * P);
    hipLaunchKernelGGL((spread_binned_kernel<W, CPLX>), dim3((unsigned)maxsub), dim3(256), 0, s,
                       static_cast<float *>(pl.acc), nf, (float)pl.beta, nb, pl.bin_pts[k],
                       pl.bin_aux[k], pl.bin_off[k], pl.bin_sub[k], pl.bin_nsub[k]);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(pl.ev_spread[k], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int W>
static hipError_t spread_binned_w(const Plan &pl, const float *quats, int64_t n_img, int64_t P,
                                  const void *values, const float *weights, hipStream_t s) {
  return pl.domain == SPFEL_COMPLEX
             ? spread_binned_wc<W, true>(pl, quats, n_img, P, values, weights, s)
             : spread_binned_wc<W, false>(pl, quats, n_img, P, values, weights, s);
}

hipError_t launch_spread_binned(const Plan &pl, const float *quats, int64_t n_img, int64_t P,
                                const void *values, const float *weights, hipStream_t s) {
  switch (pl.w) {
    case 4: return spread_binned_w<4>(pl, quats, n_img, P, values, weights, s);
    case 5: return spread_binned_w<5>(pl, quats, n_img, P, values, weights, s);
    case 6: return spread_binned_w<6>(pl, quats, n_img, P, values, weights, s);
    case 7: return spread_binned_w<7>(pl, quats, n_img, P, values, weights, s);
    default: return spread_binned_w<8>(pl, quats, n_img, P, values, weights, s);
  }
}

}  // namespace spfel
