// Orientation matching (section II-B): every image against every model
// image, D[m, n] = |s_m|^2 + |d_n|^2 - 2 s_m . d_n, nearest model wins.
//
// The cross term is a GEMM S (M x P) . D^T (P x n_img) on the matrix cores;
// the M x n_img distance matrix is never stored: each 128 x 128 tile reduces
// its columns in registers/LDS and publishes one result per image.
//   FP32: v_mfma_f32_32x32x2_f32, per-tile column argmin, then a 64-bit
//         atomicMin of (order-preserving distance key << 32 | model index),
//         so the lowest index wins ties across tiles and across calls.
//   BF16: v_mfma_f32_32x32x16_bf16 with float32 accumulation on centred,
//         rounded operands, per-tile column top-8 of the proxy distance; a
//         second kernel merges the tiles' candidates per image, rescores in
//         float32 those whose lower bound can beat the running best, and
//         certifies that no other model image can; images it cannot
//         certify are matched again against every model image in float32.
#include "device_common.h"
#include "internal.h"

namespace spfel {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBM = 128;   // model images per tile
constexpr int kBN = 128;   // images per tile
constexpr int kGroup = 8;  // m-tiles per launch-order group

// Tile of a block: blocks are dealt round-robin to the 8 XCDs, so the block
// id is first remapped to make each XCD's blocks a contiguous range, and
// that range is walked m-fastest in groups of `group` m-tiles, so the blocks
// resident on one XCD share slabs of S and D in that XCD's L2.
template <int group = kGroup>
__device__ inline void tile_of_block(int tiles_m, int tiles_n, int splits, int &tm, int &tn,
                                     int &split) {
  const int G = gridDim.x, bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3, per = G >> 3, rem = G & 7;
  int v = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + slot;
  const int tiles = tiles_m * tiles_n;
  split = v / tiles;
  v -= split * tiles;
  const int gsize = group * tiles_n;
  const int g = v / gsize;
  const int first = g * group;
  const int gm = min(tiles_m - first, group);
  const int w = v - g * gsize;
  tm = first + w % gm;
  tn = w / gm;
}

// ---------------------------------------------------------------- FP32 ----
constexpr int kBK = 32;         // floats of P per K step
constexpr int kLdF = kBK + 4;   // LDS row stride (floats)

// Four consecutive values X[r][k..k+3] of a row of length ld, zero beyond
// row `rows` or column `kend` (kend <= ld).  vec: 16-byte aligned rows and
// kend % 4 == 0, so a quad is either wholly inside or wholly outside.
__device__ inline float4 load_row4(const float *__restrict__ X, int64_t rows, int64_t r,
                                   int64_t kend, int64_t k, bool vec, int64_t ld) {
  if (r >= rows) return make_float4(0.f, 0.f, 0.f, 0.f);
  const float *p = X + r * ld + k;
  if (vec) return k < kend ? *reinterpret_cast<const float4 *>(p) : make_float4(0.f, 0.f, 0.f, 0.f);
  float4 v;
  v.x = k < kend ? p[0] : 0.f;
  v.y = k + 1 < kend ? p[1] : 0.f;
  v.z = k + 2 < kend ? p[2] : 0.f;
  v.w = k + 3 < kend ? p[3] : 0.f;
  return v;
}

// Split-K: block (split, tile) covers K range [split kchunk, (split+1)
// kchunk).  Every split stores its partial tile; the last split of a tile
// to arrive (per-tile counter) adds the partials in split order (a fixed
// order, so results do not depend on arrival order) and runs the epilogue.
//
// 512 threads = 8 wavefronts as 2 (M) x 4 (N); each wavefront owns a 64 x 32
// quarter-column of the 128 x 128 tile (two 32x32 MFMA accumulators plus two
// per-K-step partials), which keeps the register count low enough for four
// wavefronts per SIMD.
constexpr int kF32Threads = 512;

__global__ __launch_bounds__(kF32Threads) __attribute__((amdgpu_waves_per_eu(4, 4))) void match_f32_kernel(
    const float *__restrict__ S, const float *__restrict__ D, const float *__restrict__ sn,
    const float *__restrict__ dn, int64_t M, int64_t N, int64_t P, uint32_t m_offset,
    unsigned long long *__restrict__ keys, int tiles_m, int tiles_n, int vec, int splits,
    int64_t kchunk, float *__restrict__ partials, unsigned *__restrict__ counters) {
  // double-buffered A/B stages: one barrier per K step
  __shared__ __attribute__((aligned(16))) float As[2][kBM * kLdF];
  __shared__ __attribute__((aligned(16))) float Bs[2][kBN * kLdF];
  __shared__ float sns[kBM], dns[kBN];
  __shared__ unsigned long long red[2][kBN];
  __shared__ unsigned arrived;

  int tm, tn, split;
  tile_of_block(tiles_m, tiles_n, splits, tm, tn, split);
  const int64_t row0 = (int64_t)tm * kBM, col0 = (int64_t)tn * kBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3, lr = lane & 31, lh = lane >> 5;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(P, kbeg + kchunk);

  float4 ra[2], rb[2];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int id = tid + kF32Threads * i, r = id >> 3, c = (id & 7) * 4;
      ra[i] = load_row4(S, M, row0 + r, kend, k0 + c, vec, P);
      rb[i] = load_row4(D, N, col0 + r, kend, k0 + c, vec, P);
    }
  };

  floatx16 acc[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int id = tid + kF32Threads * i, r = id >> 3, c = (id & 7) * 4;
      *reinterpret_cast<float4 *>(&As[buf][r * kLdF + c]) = ra[i];
      *reinterpret_cast<float4 *>(&Bs[buf][r * kLdF + c]) = rb[i];
    }
  };
  gload(kbeg);
  lstore(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
    const bool more = k0 + kBK < kend;
    if (more) gload(k0 + kBK);
    // Fresh partial sums per K step keep every accumulation chain short:
    // at most 2 kBK roundings inside the step plus one per step.
    floatx16 part[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) part[i][r] = 0.f;
    const float *A = As[buf], *B = Bs[buf];
    // raised priority for the MFMA section (the other wavefronts' loads and
    // stores are served between its MFMAs, not ahead of them)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kk = 0; kk < kBK / 8; ++kk) {
      float4 a[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const float4 *>(&A[(wm * 64 + i * 32 + lr) * kLdF + kk * 8 + lh * 4]);
      const float4 b = *reinterpret_cast<const float4 *>(&B[(wn * 32 + lr) * kLdF + kk * 8 + lh * 4]);
      // Lane half lh supplies k = 4 lh + e for MFMA e: A and B use the same
      // permutation of the 8 k values, so the sum is unchanged.
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          part[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][e], b[e], part[i], 0, 0, 0);
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[i] += part[i];
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  if (splits > 1) {
    // publish this split's partial tile, then let the last arrival finish
    const int tile = tm * tiles_n + tn;
    float *mine = partials + ((int64_t)tile * splits + split) * (kBM * kBN);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) mine[(i * 16 + r) * kF32Threads + tid] = acc[i][r];
    __threadfence();
    __syncthreads();
    if (tid == 0) arrived = atomicAdd(counters + tile, 1u);
    __syncthreads();
    if (arrived != (unsigned)(splits - 1)) return;
    __threadfence();
    floatx16 sum[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) sum[i][r] = 0.f;
    for (int sp = 0; sp < splits; ++sp) {
      const float *part = partials + ((int64_t)tile * splits + sp) * (kBM * kBN);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          sum[i][r] += sp == split ? acc[i][r]
                                   : __builtin_nontemporal_load(&part[(i * 16 + r) * kF32Threads + tid]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[i] = sum[i];
    if (tid == 0) counters[tile] = 0u;  // ready for the next launch
  }
  if (tid < kBM) {
    sns[tid] = row0 + tid < M ? sn[row0 + tid] : 0.f;
  } else if (tid < kBM + kBN) {
    const int c = tid - kBM;
    dns[c] = col0 + c < N ? dn[col0 + c] : 0.f;
  }
  __syncthreads();
  {
    const int cl = wn * 32 + lr;
    unsigned long long best = ~0ull;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        // 32x32 MFMA output layout: lane holds column lane % 32 and rows
        // 8 (r / 4) + 4 (lane / 32) + r % 4.
        const int rl = wm * 64 + i * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
        if (row0 + rl < M) {
          const float d = fmaf(-2.0f, acc[i][r], sns[rl] + dns[cl]);
          const unsigned long long key =
              ((unsigned long long)float_key(d) << 32) | (uint32_t)(m_offset + (uint32_t)(row0 + rl));
          best = key < best ? key : best;
        }
      }
    const unsigned long long o = __shfl_xor(best, 32);
    best = o < best ? o : best;
    if (lh == 0) red[wm][cl] = best;
  }
  __syncthreads();
  if (tid < kBN) {
    const unsigned long long a = red[0][tid], b = red[1][tid];
    const unsigned long long k = a < b ? a : b;
    if (col0 + tid < N && k != ~0ull) atomicMin(keys + col0 + tid, k);
  }
}

__global__ void pack_keys_kernel(const int32_t *__restrict__ idx, const float *__restrict__ dist,
                                 unsigned long long *__restrict__ keys, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = ((unsigned long long)float_key(dist[i]) << 32) | (uint32_t)idx[i];
}

__global__ void unpack_keys_kernel(const unsigned long long *__restrict__ keys,
                                   int32_t *__restrict__ idx, float *__restrict__ dist, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const unsigned long long k = keys[i];
    idx[i] = (int32_t)(uint32_t)(k & 0xffffffffu);
    dist[i] = key_float((uint32_t)(k >> 32));
  }
}

hipError_t launch_pack_keys(const int32_t *idx, const float *dist, unsigned long long *keys,
                            int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(pack_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx,
                     dist, keys, n);
  return hipGetLastError();
}

hipError_t launch_unpack_keys(const unsigned long long *keys, int32_t *idx, float *dist, int64_t n,
                              hipStream_t s) {
  hipLaunchKernelGGL(unpack_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys,
                     idx, dist, n);
  return hipGetLastError();
}

static bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Resident blocks of match_f32_kernel on the whole chip (256 CUs x 2).
constexpr int kF32Slots = 512;

// Number of K splits that best fills the chip's resident blocks, with each
// split at least 1024 values of P long.  Only launches of under half a
// round of tiles are split: blocks are dispatched dynamically, so a partial
// last round costs less than the partial tiles' extra traffic (measured on
// 1,264 tiles of K = 16,384: unsplit 5.8 ms, two splits 6.7 ms).
int match_f32_splits(int64_t M, int64_t N, int64_t P) {
  const int64_t tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  if (2 * tiles >= kF32Slots) return 1;
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= 4; ++s) {
    if (s > 1 && P / s < 1024) break;
    const int64_t units = tiles * s;
    const int64_t rounds = (units + kF32Slots - 1) / kF32Slots;
    const double eff = (double)units / (double)(rounds * kF32Slots);
    if (eff > best_eff + 0.02) {
      best_eff = eff;
      best = s;
    }
  }
  return best;
}

size_t match_f32_workspace_bytes(int64_t M, int64_t N, int64_t P) {
  const int64_t tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  const int s = match_f32_splits(M, N, P);
  size_t b = (size_t)N * sizeof(unsigned long long);
  b = (b + 255) & ~(size_t)255;
  if (s > 1) {
    b += (size_t)tiles * sizeof(unsigned);
    b = (b + 255) & ~(size_t)255;
    b += (size_t)tiles * s * kBM * kBN * sizeof(float);
  }
  return b;
}

hipError_t launch_match_f32(const float *S, const float *D, const float *sn, const float *dn,
                            int64_t M, int64_t N, int64_t P, int64_t m_offset, void *workspace,
                            hipStream_t s) {
  const int tiles_m = (int)((M + kBM - 1) / kBM), tiles_n = (int)((N + kBN - 1) / kBN);
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  const int splits = match_f32_splits(M, N, P);
  const int64_t blocks = tiles * splits;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  // K chunk: a multiple of the K step (and of 4 for the vector loads)
  int64_t kchunk = (P + splits - 1) / splits;
  kchunk = (kchunk + kBK - 1) / kBK * kBK;
  const int vec = (P % 4 == 0) && al16(S) && al16(D);
  char *ws = static_cast<char *>(workspace);
  auto *keys = reinterpret_cast<unsigned long long *>(ws);
  size_t off = ((size_t)N * sizeof(unsigned long long) + 255) & ~(size_t)255;
  unsigned *counters = nullptr;
  float *partials = nullptr;
  if (splits > 1) {
    counters = reinterpret_cast<unsigned *>(ws + off);
    off = (off + (size_t)tiles * sizeof(unsigned) + 255) & ~(size_t)255;
    partials = reinterpret_cast<float *>(ws + off);
    hipError_t e = launch_fill_zero(counters, (size_t)tiles * sizeof(unsigned), s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(match_f32_kernel, dim3((unsigned)blocks), dim3(kF32Threads), 0, s, S, D, sn, dn, M, N,
                     P, (uint32_t)m_offset, keys, tiles_m, tiles_n, vec, splits, kchunk, partials,
                     counters);
  return hipGetLastError();
}

// ---------------------------------------------------------------- BF16 ----
constexpr int kBKH = 64;          // bf16 values of P per K step
constexpr int kLdH = kBKH + 8;    // LDS row stride (bf16 values)

__device__ inline uint4 load_row8h(const uint16_t *__restrict__ X, int64_t rows, int64_t r,
                                   int64_t P, int64_t k, bool vec) {
  if (r >= rows) return make_uint4(0u, 0u, 0u, 0u);
  const uint16_t *p = X + r * P + k;
  if (vec) return k < P ? *reinterpret_cast<const uint4 *>(p) : make_uint4(0u, 0u, 0u, 0u);
  uint32_t h[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = k + e < P ? p[e] : 0u;
  return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// Sorted (ascending) insertion into a register top-8; branch free.
__device__ inline void insert8(uint32_t (&top)[8], uint32_t x) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t lo = min(top[s], x);
    x = max(top[s], x);
    top[s] = lo;
  }
}
__device__ inline void insert8(unsigned long long (&top)[8], unsigned long long x) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const unsigned long long lo = top[s] < x ? top[s] : x;
    x = top[s] < x ? x : top[s];
    top[s] = lo;
  }
}

// The large-tile kernel is used when its 256 x 256 tiles fill at least four
// rounds of the chip's 256 resident blocks, P is a whole number of its
// 64-wide K steps and both operands are 16-byte aligned; otherwise
// 128 x 128 tiles.
int match_bf16_tile_rows(int64_t M, int64_t N, int64_t P, const void *S, const void *D) {
  if (P % 64 != 0 || !al16(S) || !al16(D)) return 128;
  const int64_t big = ((M + 255) / 256) * ((N + 255) / 256);
  return big >= 4 * 256 ? 256 : 128;
}

// Candidate buffer for the 128-row tiling, the larger of the two.
size_t match_bf16_candidate_bytes(int64_t M, int64_t N) {
  const int64_t tiles_m = (M + 127) / 128;
  return (size_t)tiles_m * (size_t)N * 8 * sizeof(uint32_t);
}

// Candidate word: proxy-distance key with its 7 low bits replaced by the
// row within the tile (a relative perturbation below 2^-15 of the proxy;
// clearing or setting those bits bounds the proxy from below or above).
__global__ __launch_bounds__(256, 2) void match_bf16_kernel(
    const uint16_t *__restrict__ S, const uint16_t *__restrict__ D, const float *__restrict__ sn,
    const float *__restrict__ dn, int64_t M, int64_t N, int64_t P, uint32_t *__restrict__ cand,
    int tiles_m, int tiles_n, int vec) {
  constexpr int kSeg = kBKH / 8;           // 16-byte segments per row and step
  constexpr int kLoads = kBM * kSeg / 256; // segments per thread and operand
  __shared__ __attribute__((aligned(16))) uint16_t As[kBM * kLdH];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN * kLdH];
  __shared__ float sns[kBM], dns[kBN];
  __shared__ uint32_t red[2][kBN][8];

  int tm, tn, split;
  tile_of_block(tiles_m, tiles_n, 1, tm, tn, split);
  const int64_t row0 = (int64_t)tm * kBM, col0 = (int64_t)tn * kBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 31, lh = lane >> 5;

  uint4 ra[kLoads], rb[kLoads];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
      const int id = tid + 256 * i, r = id / kSeg, c = (id % kSeg) * 8;
      ra[i] = load_row8h(S, M, row0 + r, P, k0 + c, vec);
      rb[i] = load_row8h(D, N, col0 + r, P, k0 + c, vec);
    }
  };

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  gload(0);
  for (int64_t k0 = 0; k0 < P; k0 += kBKH) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
      const int id = tid + 256 * i, r = id / kSeg, c = (id % kSeg) * 8;
      *reinterpret_cast<uint4 *>(&As[r * kLdH + c]) = ra[i];
      *reinterpret_cast<uint4 *>(&Bs[r * kLdH + c]) = rb[i];
    }
    __syncthreads();
    if (k0 + kBKH < P) gload(k0 + kBKH);
#pragma unroll
    for (int kk = 0; kk < kBKH / 16; ++kk) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm * 64 + i * 32 + lr) * kLdH + kk * 16 + lh * 8]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn * 64 + j * 32 + lr) * kLdH + kk * 16 + lh * 8]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }

  if (tid < kBM) {
    sns[tid] = row0 + tid < M ? sn[row0 + tid] : 0.f;
  } else {
    const int c = tid - kBM;
    dns[c] = col0 + c < N ? dn[col0 + c] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int cl = wn * 64 + j * 32 + lr;
    uint32_t top[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) top[s] = ~0u;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rl = wm * 64 + i * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
        if (row0 + rl < M) {
          const float b = fmaf(-2.0f, acc[i][j][r], sns[rl] + dns[cl]);
          insert8(top, (float_key(b) & ~127u) | (uint32_t)rl);
        }
      }
    uint32_t other[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) other[s] = __shfl_xor(top[s], 32);
#pragma unroll
    for (int s = 0; s < 8; ++s) insert8(top, other[s]);
    if (lh == 0) {
#pragma unroll
      for (int s = 0; s < 8; ++s) red[wm][cl][s] = top[s];
    }
  }
  __syncthreads();
  if (tid < kBN && col0 + tid < N) {
    uint32_t top[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) top[s] = red[0][tid][s];
#pragma unroll
    for (int s = 0; s < 8; ++s) insert8(top, red[1][tid][s]);
    uint4 *dst = reinterpret_cast<uint4 *>(cand + ((int64_t)tm * N + col0 + tid) * 8);
    dst[0] = make_uint4(top[0], top[1], top[2], top[3]);
    dst[1] = make_uint4(top[4], top[5], top[6], top[7]);
  }
}

// Large-tile form for launches with many tiles: 256 x 256 tiles, each of
// 8 wavefronts (two per SIMD) owning a 128 x 64 block (8 MFMA accumulators:
// 6 fragment reads per 8 MFMAs).  A and B stream from global memory straight
// into a double-buffered LDS ring (global_load_lds_dwordx4: each lane's 16
// bytes land at the instruction's LDS base + 16 x lane), one barrier per K
// step.  Rows are 128 bytes (64 bf16) without padding; the 16-byte chunk c
// of row r is stored at chunk c ^ f(r), f(r) = (r & 7) ^ ((r >> 3) & 1), so
// the 16 consecutive rows one fragment read touches fall in distinct bank
// groups.  Fragments are double-buffered in registers: the reads for the
// next 16-wide K slice are issued before the current slice's MFMAs.
// Requires P % 64 == 0 and 16-byte aligned rows; rows and columns past the
// matrix edge read the last row (their results are discarded).
constexpr int kBM2 = 256, kBN2 = 256, kBK2 = 64;
constexpr int kStage2 = (kBM2 + kBN2) * kBK2;   // bf16 values per LDS stage

__device__ inline int chunk_swizzle(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// Tile of a block of the large-tile kernel.  When the tile grid is a whole
// number of 16 x 16 squares, each round of 256 resident blocks (one per CU)
// covers one square: XCD x takes an 8 x 4 part of it (x % 2 selects the 8
// m-tiles, x / 2 the 4 n-tiles), so a round reads 32 distinct tiles of S and
// D instead of 40, each m-tile shared by four XCDs and each n-tile by two.
// Other grids use the grouped order.
__device__ inline void big_tile_of_block(int tiles_m, int tiles_n, int &tm, int &tn) {
  if ((tiles_m & 15) == 0 && (tiles_n & 15) == 0) {
    const int bid = blockIdx.x, x = bid & 7, s = bid >> 3;
    const int r = s >> 5, w = s & 31;
    const int sq_m = tiles_m >> 4;
    const int rm = r % sq_m, rn = r / sq_m;
    tm = rm * 16 + (x & 1) * 8 + (w & 7);
    tn = rn * 16 + (x >> 1) * 4 + (w >> 3);
  } else {
    int split;
    tile_of_block(tiles_m, tiles_n, 1, tm, tn, split);
  }
}

__global__ __launch_bounds__(512, 1) void match_bf16_big_kernel(
    const uint16_t *__restrict__ S, const uint16_t *__restrict__ D, const float *__restrict__ sn,
    const float *__restrict__ dn, int64_t M, int64_t N, int64_t P, uint32_t *__restrict__ cand,
    int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(16))) uint16_t smem[2 * kStage2];

  int tm, tn;
  big_tile_of_block(tiles_m, tiles_n, tm, tn);
  const int64_t row0 = (int64_t)tm * kBM2, col0 = (int64_t)tn * kBN2;
  // 8 wavefronts as 2 (M) x 4 (N), each owning a 128 x 64 block of the tile
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3, lr = lane & 31, lh = lane >> 5;

  // Loader: each wavefront moves 4 blocks of 8 rows of A and of B per K
  // step; block q's lane l carries row 8 q + l / 8, stored chunk l % 8,
  // which holds logical chunk (l % 8) ^ f(row).
  const uint16_t *srcA[4], *srcB[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = wave * 4 + i, r = q * 8 + (lane >> 3);
    const int lc = (lane & 7) ^ chunk_swizzle(r);
    const int64_t ga = min(row0 + r, M - 1), gb = min(col0 + r, N - 1);
    srcA[i] = S + ga * P + lc * 8;
    srcB[i] = D + gb * P + lc * 8;
  }
  auto issue = [&](int64_t k0, int buf) {
    uint16_t *As = smem + buf * kStage2;
    uint16_t *Bs = As + kBM2 * kBK2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = wave * 4 + i;
      __builtin_amdgcn_global_load_lds(srcA[i] + k0, (__attribute__((address_space(3))) void *)(As + q * 512), 16, 0, 0);
      __builtin_amdgcn_global_load_lds(srcB[i] + k0, (__attribute__((address_space(3))) void *)(Bs + q * 512), 16, 0, 0);
    }
  };

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // fragment rows share lr's swizzle: logical chunk 2 kk + lh sits at
  // 2 (kk ^ (f >> 1)) + ((lh ^ f) & 1)
  const int fl = chunk_swizzle(lr), fhi = fl >> 1, flo = (lh ^ fl) & 1;
  const int arow = (wm * 128 + lr) * kBK2, brow = (wn * 64 + lr) * kBK2;
  bf16x8 fa[2][4], fb[2][2];
  auto frags = [&](const uint16_t *As, const uint16_t *Bs, int kk, int slot) {
    const int c = (2 * (kk ^ fhi) + flo) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      fa[slot][i] = *reinterpret_cast<const bf16x8 *>(&As[arow + i * 32 * kBK2 + c]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      fb[slot][j] = *reinterpret_cast<const bf16x8 *>(&Bs[brow + j * 32 * kBK2 + c]);
  };

  const int64_t steps = P / kBK2;
  issue(0, 0);
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wavefront's loads are in LDS
  __syncthreads();
  for (int64_t st = 0; st < steps; ++st) {
    const int buf = (int)(st & 1);
    if (st + 1 < steps) issue((st + 1) * kBK2, buf ^ 1);
    const uint16_t *As = smem + buf * kStage2;
    const uint16_t *Bs = As + kBM2 * kBK2;
    frags(As, Bs, 0, 0);
#pragma unroll
    for (int kk = 0; kk < kBK2 / 16; ++kk) {
      // the scheduling barriers keep the next slice's reads ahead of this
      // slice's MFMAs (the compiler would otherwise sink them to save
      // registers and stall every MFMA group on a fresh LDS read)
      if (kk + 1 < kBK2 / 16) {
        frags(As, Bs, kk + 1, (kk + 1) & 1);
        // LDS reads complete in order: this slice's 6 are in once at most
        // the next slice's 6 are outstanding
        __builtin_amdgcn_s_waitcnt(0xC67F);   // lgkmcnt(6), vmcnt/expcnt not waited
      }
      __builtin_amdgcn_sched_barrier(0);
      // raised priority while issuing the MFMAs: the SIMD's other wavefront
      // is then served between them, not ahead of them
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[kk & 1][i], fb[kk & 1][j],
                                                              acc[i][j], 0, 0, 0);
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
  }

  // Epilogue (LDS reused): norms of the tile's rows and columns, then each
  // column's 8 smallest proxies; candidate words carry the row in 8 bits.
  float *sns = reinterpret_cast<float *>(smem);
  float *dns = sns + kBM2;
  uint32_t *red = reinterpret_cast<uint32_t *>(dns + kBN2);   // [2][kBN2][8]
  if (tid < kBM2) sns[tid] = row0 + tid < M ? sn[row0 + tid] : 0.f;
  else dns[tid - kBM2] = col0 + tid - kBM2 < N ? dn[col0 + tid - kBM2] : 0.f;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int cl = wn * 64 + j * 32 + lr;
    uint32_t top[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) top[q] = ~0u;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rl = wm * 128 + i * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
        if (row0 + rl < M) {
          const float b = fmaf(-2.0f, acc[i][j][r], sns[rl] + dns[cl]);
          insert8(top, (float_key(b) & ~255u) | (uint32_t)rl);
        }
      }
    uint32_t other[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) other[q] = __shfl_xor(top[q], 32);
#pragma unroll
    for (int q = 0; q < 8; ++q) insert8(top, other[q]);
    if (lh == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) red[(wm * kBN2 + cl) * 8 + q] = top[q];
    }
  }
  __syncthreads();
  if (tid < kBN2 && col0 + tid < N) {
    uint32_t top[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) top[q] = red[tid * 8 + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) insert8(top, red[(kBN2 + tid) * 8 + q]);
    uint4 *dst = reinterpret_cast<uint4 *>(cand + ((int64_t)tm * N + col0 + tid) * 8);
    dst[0] = make_uint4(top[0], top[1], top[2], top[3]);
    dst[1] = make_uint4(top[4], top[5], top[6], top[7]);
  }
}

hipError_t launch_match_bf16(const uint16_t *S, const uint16_t *D, const float *sn,
                             const float *dn, int64_t M, int64_t N, int64_t P, uint32_t *cand,
                             hipStream_t s) {
  const int vec = (P % 8 == 0) && al16(S) && al16(D);
  if (match_bf16_tile_rows(M, N, P, S, D) == 256) {
    const int tiles_m = (int)((M + kBM2 - 1) / kBM2), tiles_n = (int)((N + kBN2 - 1) / kBN2);
    const int64_t blocks = (int64_t)tiles_m * tiles_n;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(match_bf16_big_kernel, dim3((unsigned)blocks), dim3(512), 0, s, S, D, sn,
                       dn, M, N, P, cand, tiles_m, tiles_n);
    return hipGetLastError();
  }
  const int tiles_m = (int)((M + kBM - 1) / kBM), tiles_n = (int)((N + kBN - 1) / kBN);
  const int64_t blocks = (int64_t)tiles_m * tiles_n;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(match_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, S, D, sn, dn, M,
                     N, P, cand, tiles_m, tiles_n, vec);
  return hipGetLastError();
}

// Bounds of the certified rescore (float32 arithmetic; every bound carries
// a relative margin of 2^-16, far above the few roundings in its formula).
//   proxy b~ = |s^|^2 + |d^|^2 - 2 s^.d^ with the dot product accumulated
//     on the matrix cores: each v_mfma_f32_32x32x16_bf16 is taken as a tree
//     of its 16 exact products plus the add to the accumulator, every
//     rounding at most 2^-23 relative (truncation allowed), so a product
//     meets at most P/16 + 8 roundings:
//       |s^.d^ computed - s^.d^| <= g_acc sum_p |s^_p d^_p| <= g_acc |s^| |d^|,
//     g_acc = gamma_{P/16+8} at u = 2^-23 (a probe of the instruction on
//     random, wide-exponent and cancelling inputs measured at most
//     3.2 x 2^-24 (|C| + sum |p|) per instruction).  The norms (float32
//     sums of P/256 + 8 roundings) and the epilogue's two roundings add at
//     most g_n (|s^| + |d^|)^2, g_n = gamma_{P/256+24} at u = 2^-24:
//       A = 2 g_acc |s^| |d^| + g_n (|s^| + |d^|)^2 >= |b~ - |s^ - d^|^2|;
//   true distance D = |s - d|^2:  |sqrt(D) - |s^ - d^|| <= e_m + f_n;
//   float32 rescore D~ of D (direct sum of (s - d)^2, chains of at most
//     P/64 + 16 roundings):  |D~ - D| <= g_run D.
struct CertBounds {
  float g_acc, g_n, g_run;
};
__device__ inline float proxy_slack(const CertBounds &cb, float ns, float nd) {
  return 2.0f * cb.g_acc * ns * nd + cb.g_n * (ns + nd) * (ns + nd);
}
constexpr float kLo = 1.0f - 0x1p-16f, kHi = 1.0f + 0x1p-16f;

__device__ inline float lower_sqrt_dist(float b_lo, float A, float ef) {
  return sqrtf(fmaxf(b_lo - A, 0.f)) * kLo - ef * kHi;
}
__device__ inline float upper_sqrt_dist(float b_hi, float A, float ef) {
  return sqrtf(fmaxf(b_hi, 0.f) + A) * kHi + ef * kHi;
}
// sqrt of the largest exact distance a float32 rescored value d can stand for
__device__ inline float upper_sqrt_rescored(float d, float g_run) {
  return sqrtf(d * (1.0f + 2.0f * g_run)) * kHi;
}

// Sum over p of (s_p - d_p)^2 for one lane's share of a row (float32).
__device__ inline float direct_part(const float *__restrict__ srow, const float *__restrict__ drow,
                                    int64_t P, int lane, int vec) {
  float acc = 0.f;
  if (vec) {
    const float4 *s4 = reinterpret_cast<const float4 *>(srow);
    const float4 *d4 = reinterpret_cast<const float4 *>(drow);
    for (int64_t q = lane; q < P / 4; q += 64) {
      const float4 a = s4[q], b = d4[q];
      float t;
      t = a.x - b.x; acc = fmaf(t, t, acc);
      t = a.y - b.y; acc = fmaf(t, t, acc);
      t = a.z - b.z; acc = fmaf(t, t, acc);
      t = a.w - b.w; acc = fmaf(t, t, acc);
    }
  } else {
    for (int64_t p = lane; p < P; p += 64) {
      const float t = srow[p] - drow[p];
      acc = fmaf(t, t, acc);
    }
  }
  return acc;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Chunk maxima the certificate needs: max_m |s^_m| and max_m e_m.
__global__ __launch_bounds__(1024) void chunk_stats_kernel(const float *__restrict__ sn,
                                                           const float *__restrict__ se, int64_t M,
                                                           float *__restrict__ stats) {
  __shared__ float sh[2][1024];
  float a = 0.f, b = 0.f;
  for (int64_t m = threadIdx.x; m < M; m += 1024) {
    a = fmaxf(a, sqrtf(fmaxf(sn[m], 0.f)));
    b = fmaxf(b, se[m]);
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sh[0][threadIdx.x] = fmaxf(sh[0][threadIdx.x], sh[0][threadIdx.x + st]);
      sh[1][threadIdx.x] = fmaxf(sh[1][threadIdx.x], sh[1][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = sh[0][0];
    stats[1] = sh[1][0];
  }
}

// One wavefront per image:
//  1. merge every tile's 8 candidates into the image's 8 smallest proxies
//     (ties: lowest model index);
//  2. bound each candidate's true distance from below and above;
//  3. rescore in float32 (direct sum of squared differences) exactly the
//     candidates whose lower bound does not exceed both the running best
//     and the smallest upper bound among the 8 (no other candidate can be
//     the minimiser), and fold the best into (best_dist, best_idx);
//  4. certify the image: every model image outside the 8 has a true
//     distance at least the 8th proxy's lower bound (with the chunk's
//     largest norm and rounding error); if that bound does not exceed the
//     running best, the image goes on the fallback list (and flags[n] |= 1)
//     with its running best as the fallback's starting key.
__global__ __launch_bounds__(256) void rescore_kernel(
    const uint32_t *__restrict__ cand, int tiles_m, int tile_rows, int64_t M, int64_t N, int64_t P,
    uint32_t m_offset, const float *__restrict__ S32, const float *__restrict__ D32,
    const float *__restrict__ sn, const float *__restrict__ dn, const float *__restrict__ se,
    const float *__restrict__ de, const float *__restrict__ stats, CertBounds cb,
    int32_t *__restrict__ best_idx, float *__restrict__ best_dist, int32_t *__restrict__ flags,
    unsigned *__restrict__ fb_count, int32_t *__restrict__ fb_list,
    unsigned long long *__restrict__ fb_keys, int vec) {
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  const uint32_t low = (uint32_t)tile_rows - 1u;
  unsigned long long top[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) top[s] = ~0ull;
  const int total = tiles_m * 8;
  for (int c = lane; c < total; c += 64) {
    const int t = c >> 3, s = c & 7;
    const uint32_t k = cand[((int64_t)t * N + n) * 8 + s];
    if (k != ~0u) {
      const uint32_t m = (uint32_t)t * (uint32_t)tile_rows + (k & low);
      insert8(top, ((unsigned long long)(k & ~low) << 32) | m);
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    unsigned long long other[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) other[s] = __shfl_xor(top[s], off);
#pragma unroll
    for (int s = 0; s < 8; ++s) insert8(top, other[s]);
  }
  const float nd = sqrtf(fmaxf(dn[n], 0.f)), fd = de[n];
  int mi[8];
  bool valid[8];
  float lb[8];
  float ub_min = __builtin_inff();
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    valid[s] = top[s] != ~0ull;
    mi[s] = valid[s] ? (int)(uint32_t)(top[s] & 0xffffffffu) : 0;
    const uint32_t key = (uint32_t)(top[s] >> 32);
    const float ns = sqrtf(fmaxf(sn[mi[s]], 0.f));
    const float A = proxy_slack(cb, ns, nd);
    const float ef = se[mi[s]] + fd;
    lb[s] = lower_sqrt_dist(key_float(key), A, ef);
    if (valid[s]) ub_min = fminf(ub_min, upper_sqrt_dist(key_float(key | low), A, ef));
  }
  const float run = best_dist[n];
  const int32_t run_i = best_idx[n];
  const float thr = fminf(ub_min, upper_sqrt_rescored(run, cb.g_run));
  bool take[8];
  bool any = false;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    take[s] = valid[s] && lb[s] <= thr;
    any = any || take[s];
  }
  unsigned long long best = ~0ull;
  if (any) {
    const float *drow = D32 + n * P;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (take[s]) {   // wavefront-uniform
        const float d = wave_sum(direct_part(S32 + (int64_t)mi[s] * P, drow, P, lane, vec));
        const unsigned long long key =
            ((unsigned long long)float_key(d) << 32) | (uint32_t)(m_offset + (uint32_t)mi[s]);
        best = key < best ? key : best;
      }
    }
  }
  const unsigned long long run_key = ((unsigned long long)float_key(run) << 32) | (uint32_t)run_i;
  const unsigned long long now = best < run_key ? best : run_key;
  // certificate: only needed when model images lie outside the 8
  bool cert = true;
  if (M > 8) {
    const float A8 = proxy_slack(cb, stats[0], nd);
    const float lb8 = lower_sqrt_dist(key_float((uint32_t)(top[7] >> 32)), A8, stats[1] + fd);
    cert = lb8 > upper_sqrt_rescored(key_float((uint32_t)(now >> 32)), cb.g_run);
  }
  if (lane == 0) {
    if (now != run_key) {
      best_idx[n] = (int32_t)(uint32_t)(now & 0xffffffffu);
      best_dist[n] = key_float((uint32_t)(now >> 32));
    }
    if (!cert) {
      if (flags) flags[n] |= 1;
      const unsigned pos = atomicAdd(fb_count, 1u);
      fb_list[pos] = (int32_t)n;
      fb_keys[pos] = now;
    }
  }
}

// Fallback for uncertified images: each work item is (listed image, slab of
// 64 model images); the block's four wavefronts rescore 16 rows each in
// float32 (direct sums, as in the rescore) and fold their minimum into the
// image's key with a 64-bit atomicMin (lowest index on ties).  The number
// of listed images is read on the device; every block leaves the loop when
// the work items run out (none when every image was certified).
__global__ __launch_bounds__(256) void fallback_kernel(
    const float *__restrict__ S32, const float *__restrict__ D32, int64_t M, int64_t P,
    uint32_t m_offset, const unsigned *__restrict__ fb_count, const int32_t *__restrict__ fb_list,
    unsigned long long *__restrict__ fb_keys, int vec) {
  __shared__ unsigned long long red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t slabs = (M + 63) / 64;
  const int64_t items = (int64_t)(*fb_count) * slabs;
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    const int64_t pos = w / slabs, slab = w - pos * slabs;
    const int64_t n = fb_list[pos];
    const float *drow = D32 + n * P;
    unsigned long long best = ~0ull;
    for (int r = 0; r < 16; ++r) {
      const int64_t m = slab * 64 + wave * 16 + r;
      if (m >= M) break;   // wavefront-uniform
      const float d = wave_sum(direct_part(S32 + m * P, drow, P, lane, vec));
      const unsigned long long key =
          ((unsigned long long)float_key(d) << 32) | (uint32_t)(m_offset + (uint32_t)m);
      best = key < best ? key : best;
    }
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long k = red[0];
#pragma unroll
      for (int i = 1; i < 4; ++i) k = red[i] < k ? red[i] : k;
      if (k != ~0ull) atomicMin(fb_keys + pos, k);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void fallback_unpack_kernel(
    const unsigned *__restrict__ fb_count, const int32_t *__restrict__ fb_list,
    const unsigned long long *__restrict__ fb_keys, int32_t *__restrict__ best_idx,
    float *__restrict__ best_dist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)(*fb_count)) return;
  const int32_t n = fb_list[i];
  const unsigned long long k = fb_keys[i];
  best_idx[n] = (int32_t)(uint32_t)(k & 0xffffffffu);
  best_dist[n] = key_float((uint32_t)(k >> 32));
}

static double gamma_of(double L, double u) { return L * u / (1.0 - L * u); }

size_t match_rescore_bytes(int64_t N) {
  // stats (2 floats) and the fallback count, then the list and the keys
  return 256 + (((size_t)N * 4 + 255) & ~(size_t)255) + (size_t)N * 8;
}

hipError_t launch_rescore(const uint32_t *cand, int tile_rows, int64_t M, int64_t N, int64_t P,
                          int64_t m_offset, const float *S32, const float *D32, const float *sn,
                          const float *dn, const float *se, const float *de, int32_t *best_idx,
                          float *best_dist, int32_t *flags, void *scratch, hipStream_t s) {
  const int tr = tile_rows;
  const int tiles_m = (int)((M + tr - 1) / tr);
  const int vec = (P % 4 == 0) && al16(S32) && al16(D32);
  char *w = static_cast<char *>(scratch);
  float *stats = reinterpret_cast<float *>(w);
  unsigned *count = reinterpret_cast<unsigned *>(w + 16);
  int32_t *list = reinterpret_cast<int32_t *>(w + 256);
  auto *keys = reinterpret_cast<unsigned long long *>(w + 256 + (((size_t)N * 4 + 255) & ~(size_t)255));
  CertBounds cb;
  cb.g_acc = (float)gamma_of((double)(P / 16) + 8.0, 0x1p-23);
  cb.g_n = (float)gamma_of((double)(P / 256) + 24.0, 0x1p-24);
  cb.g_run = (float)gamma_of((double)(P / 64) + 16.0, 0x1p-24);
  hipError_t e = launch_fill_zero(count, 4, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chunk_stats_kernel, dim3(1), dim3(1024), 0, s, sn, se, M, stats);
  hipLaunchKernelGGL(rescore_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, cand, tiles_m,
                     tr, M, N, P, (uint32_t)m_offset, S32, D32, sn, dn, se, de, stats, cb, best_idx,
                     best_dist, flags, count, list, keys, vec);
  hipLaunchKernelGGL(fallback_kernel, dim3(1024), dim3(256), 0, s, S32, D32, M, P,
                     (uint32_t)m_offset, count, list, keys, vec);
  hipLaunchKernelGGL(fallback_unpack_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                     count, list, keys, best_idx, best_dist);
  return hipGetLastError();
}

}  // namespace spfel
