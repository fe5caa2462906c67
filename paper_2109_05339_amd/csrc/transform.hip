// Separable transforms between the N^3 model modes and the 2N-per-axis fine
// grid.  The zero-padded 3D FFT plus kernel deconvolution of an ES-kernel
// NUFFT is applied one axis at a time as a contraction with a small table
// W[l][k] = exp(+-2 pi i k l / nf) / psi_hat(k): padding and truncation fold
// into the table's shape, and the deconvolution into its rows.
#include "internal.h"

namespace spfel {

// Y[a][k][b] = sum_l X[a][l][b] W[l][k] on the matrix cores, as a complex
// GEMM per batch z:
// C[m][n] = sum_l P[m][l] Q[l][n] with element strides (a real operand has
// zero imaginary parts).  B = 1: P = X (rows a), Q = W, C = Y.  B > 1:
// P = W^T, Q = X[a] (one batch per a), C = Y[a].  Block tiles of 64 x 64
// complex outputs (four wavefronts of 32 x 32, 2 x 2 v_mfma_f32_16x16x4f32
// tiles each, real and imaginary accumulators), K steps of 8 complex l
// staged in LDS.  One instruction takes K = 4 real terms, i.e. 2 complex l
// with the real and imaginary parts interleaved: for the real accumulator
// the A operand is (Re P, -Im P) against (Re Q, Im Q), for the imaginary one
// (Im P, Re P) against the same B operand.  Lane layout of the instruction:
// lane t supplies A[t % 16][t / 16] and B[t / 16][t % 16] and receives
// D[4 (t / 16) + j][t % 16], j = 0..3.
constexpr int kCM = 64, kCN = 64, kCK = 8;
typedef float cfx4 __attribute__((ext_vector_type(4)));

template <bool PR, bool QR, int OUT, bool PUNIT_M>
__global__ __launch_bounds__(256) void contract_mfma_kernel(
    const void *__restrict__ P_, int64_t psm, int64_t psl, int64_t psz,
    const void *__restrict__ Q_, int64_t qsl, int64_t qsz, void *__restrict__ C_, int64_t csm,
    int64_t csz, int M, int N, int L, int tiles_m, int tiles_n) {
  __shared__ float2 Ps[kCK][kCM];
  __shared__ float2 Qs[kCK][kCN];
  const int64_t bid = blockIdx.x;
  const int64_t per = (int64_t)tiles_m * tiles_n;
  const int64_t z = bid / per;
  const int rem = (int)(bid - z * per);
  const int tm = rem / tiles_n, tn = rem - (rem / tiles_n) * tiles_n;
  const int m0 = tm * kCM, n0 = tn * kCN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int i = lane & 15, g = lane >> 4, part = g & 1, eh = g >> 1;

  auto loadP = [&](int m, int l) -> float2 {
    if (m >= M || l >= L) return make_float2(0.f, 0.f);
    const int64_t o = z * psz + (int64_t)m * psm + (int64_t)l * psl;
    if (PR) return make_float2(static_cast<const float *>(P_)[o], 0.f);
    return static_cast<const float2 *>(P_)[o];
  };
  auto loadQ = [&](int l, int n) -> float2 {
    if (n >= N || l >= L) return make_float2(0.f, 0.f);
    const int64_t o = z * qsz + (int64_t)l * qsl + n;
    if (QR) return make_float2(static_cast<const float *>(Q_)[o], 0.f);
    return static_cast<const float2 *>(Q_)[o];
  };

  cfx4 accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = cfx4{0.f, 0.f, 0.f, 0.f};
      acci[a][b] = cfx4{0.f, 0.f, 0.f, 0.f};
    }
  for (int l0 = 0; l0 < L; l0 += kCK) {
    // stage the P (64 x 8) and Q (8 x 64) tiles, unit-stride index fastest
    float2 pv[2], qv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      const int pm = PUNIT_M ? (e & (kCM - 1)) : (e >> 3);
      const int pl = PUNIT_M ? (e >> 6) : (e & (kCK - 1));
      pv[j] = loadP(m0 + pm, l0 + pl);
      qv[j] = loadQ(l0 + (e >> 6), n0 + (e & (kCN - 1)));
    }
    __syncthreads();   // the previous step's reads are done
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      const int pm = PUNIT_M ? (e & (kCM - 1)) : (e >> 3);
      const int pl = PUNIT_M ? (e >> 6) : (e & (kCK - 1));
      Ps[pl][pm] = pv[j];
      Qs[e >> 6][e & (kCN - 1)] = qv[j];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kCK / 2; ++kk) {
      const int e = 2 * kk + eh;
      float ar[2], ai[2], bq[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float2 p = Ps[e][wm * 32 + a * 16 + i];
        ar[a] = part ? -p.y : p.x;
        ai[a] = part ? p.x : p.y;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float2 q = Qs[e][wn * 32 + b * 16 + i];
        bq[b] = part ? q.y : q.x;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], bq[b], accr[a][b], 0, 0, 0);
          acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[a], bq[b], acci[a][b], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + wm * 32 + a * 16 + 4 * g + j, n = n0 + wn * 32 + b * 16 + i;
        if (m >= M || n >= N) continue;
        const int64_t o = z * csz + (int64_t)m * csm + n;
        const float re = accr[a][b][j], im = acci[a][b][j];
        if (OUT == 0) {
          static_cast<float2 *>(C_)[o] = make_float2(re, im);
        } else if (OUT == 1) {
          static_cast<float *>(C_)[o] = re;
        } else if (OUT == 2) {
          static_cast<float *>(C_)[o] += re;
        } else {
          float2 *C = static_cast<float2 *>(C_);
          const float2 y = C[o];
          C[o] = make_float2(y.x + re, y.y + im);
        }
      }
}

template <bool PR, bool QR, bool PUNIT_M>
static hipError_t contract_mfma(const void *P, int64_t psm, int64_t psl, int64_t psz,
                                const void *Q, int64_t qsl, int64_t qsz, void *C, int64_t csm,
                                int64_t csz, int M, int N, int L, int64_t batch, int out_mode,
                                hipStream_t s) {
  const int tiles_m = (M + kCM - 1) / kCM, tiles_n = (N + kCN - 1) / kCN;
  const int64_t blocks = batch * tiles_m * tiles_n;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(256);
#define SPFEL_CMFMA(O)                                                                      \
  hipLaunchKernelGGL((contract_mfma_kernel<PR, QR, O, PUNIT_M>), grid, block, 0, s, P, psm, \
                     psl, psz, Q, qsl, qsz, C, csm, csz, M, N, L, tiles_m, tiles_n)
  switch (out_mode) {
    case 0: SPFEL_CMFMA(0); break;
    case 1: SPFEL_CMFMA(1); break;
    case 2: SPFEL_CMFMA(2); break;
    default: SPFEL_CMFMA(3); break;
  }
#undef SPFEL_CMFMA
  return hipGetLastError();
}

hipError_t launch_contract(const void *X, bool x_complex, const float2 *W, void *Y,
                           int out_mode, int A, int L, int K, int B, hipStream_t s) {
  if ((int64_t)A * K * B == 0) return hipSuccess;
  if (B == 1) {
    // rows a of X against W: P = X (A x L), Q = W (L x K)
    return x_complex
               ? contract_mfma<false, false, false>(X, L, 1, 0, W, K, 0, Y, K, 0, A, K, L, 1,
                                                    out_mode, s)
               : contract_mfma<true, false, false>(X, L, 1, 0, W, K, 0, Y, K, 0, A, K, L, 1,
                                                   out_mode, s);
  }
  // per a: W^T (K x L) against X[a] (L x B)
  return x_complex
             ? contract_mfma<false, false, true>(W, 1, K, 0, X, B, (int64_t)L * B, Y, B,
                                                 (int64_t)K * B, K, B, L, A, out_mode, s)
             : contract_mfma<false, true, true>(W, 1, K, 0, X, B, (int64_t)L * B, Y, B,
                                                (int64_t)K * B, K, B, L, A, out_mode, s);
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
