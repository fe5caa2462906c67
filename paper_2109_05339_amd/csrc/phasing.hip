// Phasing (section II-D): the density rho on an N^3 grid and its Fourier
// coefficients are driven back and forth between the real-space constraints
// (support, positivity) and the measured amplitudes, by error reduction (ER)
// and hybrid input-output (HIO) steps, with shrinkwrap support updates.
// The 3D transforms are three separable DFT contractions with N x N tables
// (numpy's convention: forward e^{-2 pi i k.r / N}, inverse with 1 / N per
// axis); the shrinkwrap blur is three separable circular convolutions with
// the periodic Gaussian, as contractions with its circulant table.
#include <cmath>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace spfel {

constexpr int kPhBlocks = 256;

struct Phase {
  int device = 0, N = 0;
  float2 *Wf = nullptr;   // [N][N] exp(-2 pi i k l / N)
  float2 *Wi = nullptr;   // [N][N] exp(+2 pi i k l / N) / N
  float2 *Wg = nullptr;   // [N][N] circulant Gaussian g[(k - l) mod N]
  float2 *F = nullptr, *T1 = nullptr, *T2 = nullptr;   // N^3 each
  float *rp = nullptr;    // N^3: rho' (or the blurred |rho|)
  float *part = nullptr;  // 2 x kPhBlocks partial sums
  float *sums = nullptr;  // 2 floats
  size_t bytes = 0;
};

static std::mutex g_pmu;
static std::set<Phase *> g_plive;

static bool plive(Phase *p) {
  std::lock_guard<std::mutex> lk(g_pmu);
  return p && g_plive.count(p) > 0;
}

static void free_phase(Phase *p) {
  void *bufs[] = {p->Wf, p->Wi, p->Wg, p->F, p->T1, p->T2, p->rp, p->part, p->sums};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
}

// ---------------------------------------------------------------- kernels --

// Reciprocal-space projection, in place on F: where measured, F <- A F / |F|
// (A where F = 0); elsewhere F is kept.  Partial sums of (|F| - A)^2 and A^2
// over measured coefficients, fixed order (block b takes a contiguous range,
// 256 strided partials, a pairwise tree).
__global__ __launch_bounds__(256) void amplitude_projection_kernel(
    float2 *__restrict__ F, const float *__restrict__ amp, const uint8_t *__restrict__ measured,
    int64_t n, float *__restrict__ part) {
  __shared__ float sh[2][256];
  const int64_t per = (n + kPhBlocks - 1) / kPhBlocks;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  float e = 0.f, a2 = 0.f;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    if (measured && !measured[i]) continue;
    const float2 f = F[i];
    const float A = amp[i];
    const float mag = sqrtf(fmaf(f.x, f.x, f.y * f.y));
    const float d = mag - A;
    e = fmaf(d, d, e);
    a2 = fmaf(A, A, a2);
    F[i] = mag > 0.f ? make_float2(A * (f.x / mag), A * (f.y / mag)) : make_float2(A, 0.f);
  }
  sh[0][threadIdx.x] = e;
  sh[1][threadIdx.x] = a2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sh[0][0];
    part[kPhBlocks + blockIdx.x] = sh[1][0];
  }
}

// err[it] = (sum of the error partials) / (sum of the A^2 partials).
__global__ void phase_error_kernel(const float *__restrict__ part, float *__restrict__ err,
                                   int it) {
  if (threadIdx.x != 0) return;
  float e = 0.f, a = 0.f;
  for (int b = 0; b < kPhBlocks; ++b) {
    e += part[b];
    a += part[kPhBlocks + b];
  }
  if (err) err[it] = a > 0.f ? e / a : 0.f;
}

// Real-space step: where the constraint holds (support, and rho' >= 0 with
// positivity) rho <- rho'; elsewhere rho <- 0 (ER) or rho - beta rho' (HIO).
__global__ __launch_bounds__(256) void real_space_kernel(float *__restrict__ rho,
                                                         const float *__restrict__ rp,
                                                         const uint8_t *__restrict__ support,
                                                         int64_t n, int hio, float beta,
                                                         int positivity) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = rp[i];
  const bool holds = support[i] && (!positivity || v >= 0.f);
  rho[i] = holds ? v : (hio ? fmaf(-beta, v, rho[i]) : 0.f);
}

// |rho| into the real parts of a complex buffer's first half (the blur's
// first contraction reads float input).
__global__ __launch_bounds__(256) void abs_kernel(const float *__restrict__ rho, int64_t n,
                                                  float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fabsf(rho[i]);
}

// Circulant table of the periodic Gaussian: W[l][k] = g[(k - l) mod N],
// g[d] ~ exp(-d^2 / (2 sigma^2)) with d the signed periodic offset, unit sum
// (float64, rounded once).  One block.
__global__ __launch_bounds__(256) void gaussian_table_kernel(int N, double sigma,
                                                             float2 *__restrict__ W) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < N; j += 256) {
    const double d = j <= N / 2 ? j : j - N;
    s += exp(-d * d / (2.0 * sigma * sigma));
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double total = sh[0];
  for (int64_t t = threadIdx.x; t < (int64_t)N * N; t += 256) {
    const int l = (int)(t / N), k = (int)(t - (int64_t)l * N);
    int j = k - l;
    j += j < 0 ? N : 0;
    const double d = j <= N / 2 ? j : j - N;
    W[t] = make_float2((float)(exp(-d * d / (2.0 * sigma * sigma)) / total), 0.f);
  }
}

// Partial maxima of b (fixed order), then support = b >= tau max.
__global__ __launch_bounds__(256) void max_partial_kernel(const float *__restrict__ b, int64_t n,
                                                          float *__restrict__ part) {
  __shared__ float sh[256];
  const int64_t per = (n + kPhBlocks - 1) / kPhBlocks;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  float m = 0.f;   // b >= 0
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) m = fmaxf(m, b[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void threshold_kernel(const float *__restrict__ b, int64_t n,
                                                        const float *__restrict__ part, float tau,
                                                        uint8_t *__restrict__ support) {
  __shared__ float thr;
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int j = 0; j < kPhBlocks; ++j) m = fmaxf(m, part[j]);
    thr = tau * m;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) support[i] = b[i] >= thr ? 1 : 0;
}

static dim3 pgrid(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// 3D transform of rho (real) into F.
static hipError_t forward3(const Phase &p, const float *rho, hipStream_t st) {
  const int N = p.N;
  hipError_t e = launch_contract(rho, false, p.Wf, p.T1, 0, N * N, N, N, 1, st);
  if (e == hipSuccess) e = launch_contract(p.T1, true, p.Wf, p.T2, 0, N, N, N, N, st);
  if (e == hipSuccess) e = launch_contract(p.T2, true, p.Wf, p.F, 0, 1, N, N, N * N, st);
  return e;
}

// Real part of the inverse transform of F into out.
static hipError_t inverse3(const Phase &p, float *out, hipStream_t st) {
  const int N = p.N;
  hipError_t e = launch_contract(p.F, true, p.Wi, p.T1, 0, N * N, N, N, 1, st);
  if (e == hipSuccess) e = launch_contract(p.T1, true, p.Wi, p.T2, 0, N, N, N, N, st);
  if (e == hipSuccess) e = launch_contract(p.T2, true, p.Wi, out, 1, 1, N, N, N * N, st);
  return e;
}

}  // namespace spfel

using namespace spfel;

extern "C" {

int spfel_phase_create(spfel_phase *out, int n, int device) {
  clear_error();
  if (!out) return fail(SPFEL_EINVAL, "phase_create: out is NULL");
  *out = nullptr;
  if (n < 2) return fail(SPFEL_EINVAL, "phase_create: n must be >= 2");
  if (n > 1024) return fail(SPFEL_ERANGE, "phase_create: n > 1024");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "phase_create: hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(SPFEL_EINVAL, "phase_create: no such device");
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != device) (void)hipSetDevice(device);
  Phase *p = new (std::nothrow) Phase();
  if (!p) return fail(SPFEL_ENOMEM, "phase_create: host allocation");
  p->device = device;
  p->N = n;
  const size_t N = n, N3 = N * N * N;
  struct Req {
    void **ptr;
    size_t bytes;
  } reqs[] = {{reinterpret_cast<void **>(&p->Wf), N * N * 8},
              {reinterpret_cast<void **>(&p->Wi), N * N * 8},
              {reinterpret_cast<void **>(&p->Wg), N * N * 8},
              {reinterpret_cast<void **>(&p->F), N3 * 8},
              {reinterpret_cast<void **>(&p->T1), N3 * 8},
              {reinterpret_cast<void **>(&p->T2), N3 * 8},
              {reinterpret_cast<void **>(&p->rp), N3 * 4},
              {reinterpret_cast<void **>(&p->part), 2 * kPhBlocks * 4},
              {reinterpret_cast<void **>(&p->sums), 2 * 4}};
  for (auto &r : reqs) {
    e = hipMalloc(r.ptr, r.bytes);
    if (e != hipSuccess) {
      *r.ptr = nullptr;
      (void)hipGetLastError();
      free_phase(p);
      delete p;
      if (prev != device) (void)hipSetDevice(prev);
      return fail(SPFEL_ENOMEM, std::string("phase_create: hipMalloc: ") + hipGetErrorString(e));
    }
    p->bytes += r.bytes;
  }
  // DFT tables in float64 with the phase index reduced modulo N exactly
  std::vector<float2> Wf(N * N), Wi(N * N);
  for (size_t l = 0; l < N; ++l)
    for (size_t k = 0; k < N; ++k) {
      const double a = 2.0 * M_PI * (double)((l * k) % N) / (double)N;
      Wf[l * N + k] = make_float2((float)std::cos(a), (float)-std::sin(a));
      Wi[l * N + k] = make_float2((float)(std::cos(a) / (double)N), (float)(std::sin(a) / (double)N));
    }
  e = hipMemcpy(p->Wf, Wf.data(), N * N * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->Wi, Wi.data(), N * N * 8, hipMemcpyHostToDevice);
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    free_phase(p);
    delete p;
    return hip_fail(e, "phase_create: table upload");
  }
  {
    std::lock_guard<std::mutex> lk(g_pmu);
    g_plive.insert(p);
  }
  *out = reinterpret_cast<spfel_phase>(p);
  return SPFEL_OK;
}

int spfel_phase_destroy(spfel_phase h) {
  clear_error();
  Phase *p = reinterpret_cast<Phase *>(h);
  {
    std::lock_guard<std::mutex> lk(g_pmu);
    if (!p || g_plive.erase(p) == 0) return fail(SPFEL_ESTATE, "phase_destroy: not a live object");
  }
  free_phase(p);
  delete p;
  return SPFEL_OK;
}

int spfel_phase_iterate(spfel_phase h, float *rho, const float *amp, const uint8_t *measured,
                        const uint8_t *support, int n_iter, int mode, float beta,
                        int positivity, float *err, void *stream) {
  clear_error();
  Phase *p = reinterpret_cast<Phase *>(h);
  if (!plive(p)) return fail(SPFEL_ESTATE, "phase_iterate: not a live object");
  if (!rho || !amp || !support) return fail(SPFEL_EINVAL, "phase_iterate: NULL pointer");
  if (mode != SPFEL_PHASE_ER && mode != SPFEL_PHASE_HIO)
    return fail(SPFEL_EINVAL, "phase_iterate: mode must be ER or HIO");
  if (n_iter < 0) return fail(SPFEL_EINVAL, "phase_iterate: negative n_iter");
  if (!std::isfinite(beta)) return fail(SPFEL_EINVAL, "phase_iterate: beta not finite");
  if ((reinterpret_cast<uintptr_t>(rho) & 3) || (reinterpret_cast<uintptr_t>(amp) & 3) ||
      (err && (reinterpret_cast<uintptr_t>(err) & 3)))
    return fail(SPFEL_EINVAL, "phase_iterate: misaligned float array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n3 = (int64_t)p->N * p->N * p->N;
  for (int it = 0; it < n_iter; ++it) {
    hipError_t e = forward3(*p, rho, st);
    if (e != hipSuccess) return hip_fail(e, "phase_iterate: launch");
    hipLaunchKernelGGL(amplitude_projection_kernel, dim3(kPhBlocks), dim3(256), 0, st, p->F, amp,
                       measured, n3, p->part);
    hipLaunchKernelGGL(phase_error_kernel, dim3(1), dim3(64), 0, st, p->part, err, it);
    e = inverse3(*p, p->rp, st);
    if (e != hipSuccess) return hip_fail(e, "phase_iterate: launch");
    hipLaunchKernelGGL(real_space_kernel, pgrid(n3), dim3(256), 0, st, rho, p->rp, support, n3,
                       mode == SPFEL_PHASE_HIO ? 1 : 0, beta, positivity ? 1 : 0);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "phase_iterate: launch");
}

int spfel_phase_shrinkwrap(spfel_phase h, const float *rho, float sigma, float tau,
                           uint8_t *support, float *blurred, void *stream) {
  clear_error();
  Phase *p = reinterpret_cast<Phase *>(h);
  if (!plive(p)) return fail(SPFEL_ESTATE, "phase_shrinkwrap: not a live object");
  if (!rho || !support) return fail(SPFEL_EINVAL, "phase_shrinkwrap: NULL pointer");
  if (!(sigma > 0.f) || !std::isfinite(sigma)) return fail(SPFEL_EINVAL, "phase_shrinkwrap: sigma must be > 0");
  if (!(tau >= 0.f && tau <= 1.f)) return fail(SPFEL_EINVAL, "phase_shrinkwrap: tau must be in [0, 1]");
  if ((reinterpret_cast<uintptr_t>(rho) & 3) || (blurred && (reinterpret_cast<uintptr_t>(blurred) & 3)))
    return fail(SPFEL_EINVAL, "phase_shrinkwrap: misaligned float array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = p->N;
  const int64_t n3 = (int64_t)N * N * N;
  float *b = blurred ? blurred : p->rp;
  hipLaunchKernelGGL(gaussian_table_kernel, dim3(1), dim3(256), 0, st, N, (double)sigma, p->Wg);
  float *absr = reinterpret_cast<float *>(p->F);   // N^3 floats fit in F
  hipLaunchKernelGGL(abs_kernel, pgrid(n3), dim3(256), 0, st, rho, n3, absr);
  hipError_t e = launch_contract(absr, false, p->Wg, p->T1, 0, N * N, N, N, 1, st);
  if (e == hipSuccess) e = launch_contract(p->T1, true, p->Wg, p->T2, 0, N, N, N, N, st);
  if (e == hipSuccess) e = launch_contract(p->T2, true, p->Wg, b, 1, 1, N, N, N * N, st);
  if (e != hipSuccess) return hip_fail(e, "phase_shrinkwrap: launch");
  hipLaunchKernelGGL(max_partial_kernel, dim3(kPhBlocks), dim3(256), 0, st, b, n3, p->part);
  hipLaunchKernelGGL(threshold_kernel, pgrid(n3), dim3(256), 0, st, b, n3, p->part, tau, support);
  e = hipGetLastError();
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "phase_shrinkwrap: launch");
}

}  // extern "C"
