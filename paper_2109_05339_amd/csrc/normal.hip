// Regularised merging (section II-C, Eq. (2)):
//   (A* D A + lambda I) x = A* D b + lambda x0,
// with A* D A applied as a convolution on the Cartesian grid (the Toeplitz
// method): (A* D A)_{k k'} = T[k - k'], T the type-1 transform of the
// weights D on (2N - 1)^3 modes (REAL domain: A^T D A x = C * even(x), C the
// cosine transform of D).  On a grid of L = 2N cells per axis the circular
// convolution equals the linear one for |k - k'| <= N - 1 < L / 2, so one
// application is three separable DFT contractions N -> L, a pointwise
// product with the transformed kernel, and three contractions L -> N.
// Conjugate gradients solve up to kMaxSystems systems (one per lambda) at
// once, sharing every transform launch; the step sizes stay on the device.
#include <cmath>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace spfel {

constexpr int kMaxSystems = 16;
constexpr int kDotBlocks = 256;

struct Lambdas {
  float v[kMaxSystems];
};

struct Normal {
  int device = 0, N = 0, L = 0, domain = SPFEL_REAL, max_sys = 0;
  float2 *F = nullptr;     // [N][L]  exp(-2 pi i k l / L)
  float2 *G = nullptr;     // [L][N]  exp(+2 pi i k l / L) / L
  float2 *Hm = nullptr;    // [2N-1][L] exp(-2 pi i m l / L)
  float2 *That = nullptr;  // L^3: transform of the Toeplitz kernel
  float2 *X1 = nullptr, *X2 = nullptr, *X3 = nullptr;   // transform intermediates
  void *ve = nullptr;      // symmetrised input (REAL)
  void *x = nullptr, *r = nullptr, *p = nullptr, *Ap = nullptr;
  float *scal = nullptr;   // per system: rr, pAp, rr_new, spare
  float *part = nullptr;   // dot partial sums
  bool psf_set = false;
  size_t bytes = 0;
};

static std::mutex g_nmu;
static std::set<Normal *> g_nlive;

static bool nlive(Normal *p) {
  std::lock_guard<std::mutex> lk(g_nmu);
  return p && g_nlive.count(p) > 0;
}

static void free_normal(Normal *p) {
  void *bufs[] = {p->F, p->G, p->Hm, p->That, p->X1, p->X2, p->X3, p->ve,
                  p->x, p->r, p->p, p->Ap, p->scal, p->part};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
}

// ---------------------------------------------------------------- kernels --

// ve[s][k] = (v[s][k] + v[s][-k]) / 2 (REAL domain).
__global__ __launch_bounds__(256) void symmetrise_kernel(const float *__restrict__ v, int N,
                                                         int n, float *__restrict__ ve) {
  const int64_t N3 = (int64_t)N * N * N;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * N3) return;
  const int64_t s = t / N3, k = t - s * N3;
  const int64_t a = k / ((int64_t)N * N), b = (k / N) % N, c = k % N;
  const int64_t kr = ((N - 1 - a) * N + (N - 1 - b)) * N + (N - 1 - c);
  ve[t] = 0.5f * (v[s * N3 + k] + v[s * N3 + kr]);
}

// X[s][j] *= That[j] (complex), j < L^3.
__global__ __launch_bounds__(256) void kernel_product(float2 *__restrict__ X,
                                                      const float2 *__restrict__ T, int64_t L3,
                                                      int n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * L3) return;
  const float2 a = X[t], b = T[t % L3];
  X[t] = make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// y[s] += lambda_s v[s] (float32 values; complex vectors count twice).
__global__ __launch_bounds__(256) void add_lambda_kernel(float *__restrict__ y,
                                                         const float *__restrict__ v, int64_t len,
                                                         int n, Lambdas lam) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * len) return;
  y[t] = fmaf(lam.v[t / len], v[t], y[t]);
}

// Partial sums of sum_k u[s][k] v[k'] (real parts of conj(u) v for complex
// vectors stored as float pairs: the float-pair dot is exactly that), fixed
// order: block b of system s takes a contiguous range, 256 strided partials,
// a pairwise tree.  v_stride 0 broadcasts one vector to every system.
__global__ __launch_bounds__(256) void dot_partial_kernel(const float *__restrict__ u,
                                                          const float *__restrict__ v,
                                                          int64_t len, int64_t v_stride,
                                                          float *__restrict__ part) {
  __shared__ float sh[256];
  const int s = blockIdx.y;
  const int64_t per = (len + kDotBlocks - 1) / kDotBlocks;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(len, lo + per);
  const float *us = u + s * len, *vs = v + s * v_stride;
  float acc = 0.f;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc = fmaf(us[i], vs[i], acc);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[s * kDotBlocks + blockIdx.x] = sh[0];
}

// out[s * stride] = sum of the system's partials in block order.
__global__ void dot_final_kernel(const float *__restrict__ part, int n, float *__restrict__ out,
                                 int stride) {
  const int s = threadIdx.x;
  if (s >= n) return;
  float t = 0.f;
  for (int b = 0; b < kDotBlocks; ++b) t += part[s * kDotBlocks + b];
  out[s * stride] = t;
}

// CG start: x = x0, r = rhs + lambda x0 - Ap (Ap = A* D A x0 + lambda x0
// already), p = r.
__global__ __launch_bounds__(256) void cg_init_kernel(const float *__restrict__ rhs,
                                                      const float *__restrict__ x0,
                                                      const float *__restrict__ Ap, int64_t len,
                                                      int n, Lambdas lam, float *__restrict__ x,
                                                      float *__restrict__ r,
                                                      float *__restrict__ p) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * len) return;
  const int64_t k = t % len;
  const float v = fmaf(lam.v[t / len], x0[k], rhs[k]) - Ap[t];
  x[t] = x0[k];
  r[t] = v;
  p[t] = v;
}

// alpha = rr / pAp (0 once converged), x += alpha p, r -= alpha Ap.
__global__ __launch_bounds__(256) void cg_update_kernel(const float *__restrict__ scal,
                                                        const float *__restrict__ p,
                                                        const float *__restrict__ Ap,
                                                        int64_t len, int n,
                                                        float *__restrict__ x,
                                                        float *__restrict__ r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * len) return;
  const float *sc = scal + 4 * (t / len);
  const float alpha = sc[1] > 0.f && sc[0] > 0.f ? sc[0] / sc[1] : 0.f;
  x[t] = fmaf(alpha, p[t], x[t]);
  r[t] = fmaf(-alpha, Ap[t], r[t]);
}

// beta = rr_new / rr, p = r + beta p.
__global__ __launch_bounds__(256) void cg_direction_kernel(const float *__restrict__ scal,
                                                           const float *__restrict__ r,
                                                           int64_t len, int n,
                                                           float *__restrict__ p) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * len) return;
  const float *sc = scal + 4 * (t / len);
  const float beta = sc[0] > 0.f ? sc[2] / sc[0] : 0.f;
  p[t] = fmaf(beta, p[t], r[t]);
}

// rr = rr_new; residual history hist[s][it] = sqrt(rr).
__global__ void cg_advance_kernel(float *__restrict__ scal, int n, float *__restrict__ hist,
                                  int it, int stride, int use_new) {
  const int s = threadIdx.x;
  if (s >= n) return;
  if (use_new) scal[4 * s] = scal[4 * s + 2];
  if (hist) hist[s * stride + it] = sqrtf(fmaxf(scal[4 * s], 0.f));
}

// x[s] = x0 for every system.
__global__ __launch_bounds__(256) void broadcast_kernel(const float *__restrict__ x0, int64_t len,
                                                        int n, float *__restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * len) return;
  x[t] = x0[t % len];
}

// d = x - x0 (x0 shared).
__global__ __launch_bounds__(256) void diff_kernel(const float *__restrict__ x,
                                                   const float *__restrict__ x0, int64_t len,
                                                   int n, float *__restrict__ d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * len) return;
  d[t] = x[t] - x0[t % len];
}

// rho = x.Hx - 2 x.rhs + bdb, eta = |x - x0|^2 from the dots (scal[s][0..2]
// = x.Hx, x.rhs, eta); corner of the L-curve by the largest curvature of
// (log rho, log eta) over log lambda (central differences, end points
// excluded; uniform spacing in log lambda assumed).
__global__ void lcurve_kernel(const float *__restrict__ scal, int n, double bdb, Lambdas lam,
                              float *__restrict__ rho_eta, int32_t *__restrict__ corner) {
  if (threadIdx.x != 0) return;
  double u[kMaxSystems], v[kMaxSystems];
  for (int s = 0; s < n; ++s) {
    const double rho = (double)scal[4 * s] - 2.0 * (double)scal[4 * s + 1] + bdb;
    const double eta = (double)scal[4 * s + 2];
    rho_eta[2 * s] = (float)rho;
    rho_eta[2 * s + 1] = (float)eta;
    u[s] = log(fmax(rho, 1e-300));
    v[s] = log(fmax(eta, 1e-300));
  }
  if (!corner) return;
  int arg = n > 2 ? 1 : 0;
  if (n > 2) {
    const double dt = log((double)lam.v[1]) - log((double)lam.v[0]);
    double best = -1e300;
    for (int i = 1; i < n - 1; ++i) {
      const double du = (u[i + 1] - u[i - 1]) / (2 * dt), dv = (v[i + 1] - v[i - 1]) / (2 * dt);
      const double ddu = (u[i + 1] - 2 * u[i] + u[i - 1]) / (dt * dt);
      const double ddv = (v[i + 1] - 2 * v[i] + v[i - 1]) / (dt * dt);
      const double kappa = (du * ddv - ddu * dv) / pow(du * du + dv * dv, 1.5);
      if (kappa > best) {
        best = kappa;
        arg = i;
      }
    }
  }
  *corner = arg;
}

static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// y[s] = A* D A v[s] (+ lambda_s v[s]) for s < n.
static hipError_t normal_apply(const Normal &nm, const void *v, int n, const Lambdas *lam,
                               void *y, hipStream_t st) {
  const int N = nm.N, L = nm.L;
  const int64_t N3 = (int64_t)N * N * N, L3 = (int64_t)L * L * L;
  const bool cplx = nm.domain == SPFEL_COMPLEX;
  const void *in = v;
  if (!cplx) {
    hipLaunchKernelGGL(symmetrise_kernel, grid_of(n * N3), dim3(256), 0, st,
                       static_cast<const float *>(v), N, n, static_cast<float *>(nm.ve));
    in = nm.ve;
  }
  hipError_t e = launch_contract(in, cplx, nm.F, nm.X1, 0, n * N * N, N, L, 1, st);
  if (e == hipSuccess) e = launch_contract(nm.X1, true, nm.F, nm.X2, 0, n * N, N, L, L, st);
  if (e == hipSuccess) e = launch_contract(nm.X2, true, nm.F, nm.X3, 0, n, N, L, L * L, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel_product, grid_of(n * L3), dim3(256), 0, st, nm.X3, nm.That, L3, n);
  e = launch_contract(nm.X3, true, nm.G, nm.X2, 0, n * L * L, L, N, 1, st);
  if (e == hipSuccess) e = launch_contract(nm.X2, true, nm.G, nm.X1, 0, n * L, L, N, N, st);
  if (e == hipSuccess) e = launch_contract(nm.X1, true, nm.G, y, cplx ? 0 : 1, n, L, N, N * N, st);
  if (e != hipSuccess) return e;
  if (lam) {
    const int64_t len = N3 * (cplx ? 2 : 1);
    hipLaunchKernelGGL(add_lambda_kernel, grid_of(n * len), dim3(256), 0, st,
                       static_cast<float *>(y), static_cast<const float *>(v), len, n, *lam);
  }
  return hipGetLastError();
}

// out[s * stride] = u[s] . v[s or shared], over len floats.
static hipError_t dots(const Normal &nm, const void *u, const void *v, int64_t len,
                       int64_t v_stride, int n, float *out, int stride, hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks, n), dim3(256), 0, st,
                     static_cast<const float *>(u), static_cast<const float *>(v), len, v_stride,
                     nm.part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(64), 0, st, nm.part, n, out, stride);
  return hipGetLastError();
}

}  // namespace spfel

using namespace spfel;

extern "C" {

int spfel_normal_create(spfel_normal *out, int n_model, int domain, int max_systems,
                        int device) {
  clear_error();
  if (!out) return fail(SPFEL_EINVAL, "normal_create: out is NULL");
  *out = nullptr;
  if (n_model < 3 || n_model % 2 == 0) return fail(SPFEL_EINVAL, "normal_create: n_model must be odd and >= 3");
  if (n_model > 511) return fail(SPFEL_ERANGE, "normal_create: n_model > 511");
  if (domain != SPFEL_REAL && domain != SPFEL_COMPLEX)
    return fail(SPFEL_EINVAL, "normal_create: domain must be REAL or COMPLEX");
  if (max_systems < 1 || max_systems > kMaxSystems)
    return fail(SPFEL_EINVAL, "normal_create: max_systems must be 1..16");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "normal_create: hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(SPFEL_EINVAL, "normal_create: no such device");
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != device) (void)hipSetDevice(device);
  Normal *p = new (std::nothrow) Normal();
  if (!p) return fail(SPFEL_ENOMEM, "normal_create: host allocation");
  p->device = device;
  p->N = n_model;
  p->L = 2 * n_model;
  p->domain = domain;
  p->max_sys = max_systems;
  const int64_t N = n_model, L = p->L, M = 2 * N - 1, n = max_systems;
  const int64_t N3 = N * N * N, L3 = L * L * L;
  const size_t vec = (size_t)N3 * (domain == SPFEL_COMPLEX ? 8 : 4);
  struct Req {
    void **ptr;
    size_t bytes;
  } reqs[] = {{reinterpret_cast<void **>(&p->F), (size_t)N * L * 8},
              {reinterpret_cast<void **>(&p->G), (size_t)L * N * 8},
              {reinterpret_cast<void **>(&p->Hm), (size_t)M * L * 8},
              {reinterpret_cast<void **>(&p->That), (size_t)L3 * 8},
              {reinterpret_cast<void **>(&p->X1), (size_t)n * std::max(N * N * L, M * M * L) * 8},
              {reinterpret_cast<void **>(&p->X2), (size_t)n * std::max(N * L * L, M * L * L) * 8},
              {reinterpret_cast<void **>(&p->X3), (size_t)n * L3 * 8},
              {&p->ve, (size_t)n * N3 * 4},
              {&p->x, n * vec},
              {&p->r, n * vec},
              {&p->p, n * vec},
              {&p->Ap, n * vec},
              {reinterpret_cast<void **>(&p->scal), (size_t)kMaxSystems * 4 * 4},
              {reinterpret_cast<void **>(&p->part), (size_t)kMaxSystems * kDotBlocks * 4}};
  for (auto &r : reqs) {
    e = hipMalloc(r.ptr, r.bytes);
    if (e != hipSuccess) {
      *r.ptr = nullptr;
      (void)hipGetLastError();
      free_normal(p);
      delete p;
      if (prev != device) (void)hipSetDevice(prev);
      return fail(SPFEL_ENOMEM, std::string("normal_create: hipMalloc: ") + hipGetErrorString(e));
    }
    p->bytes += r.bytes;
  }
  // DFT tables in float64, rounded once; phases reduced modulo L exactly
  std::vector<float2> F(N * L), G(L * N), H(M * L);
  auto cis = [&](long k, long l, double sign, double scale) {
    long q = (k * l) % L;
    if (q < 0) q += L;
    const double a = 2.0 * M_PI * (double)q / (double)L;
    return make_float2((float)(std::cos(a) * scale), (float)(sign * std::sin(a) * scale));
  };
  const long h = (n_model - 1) / 2;
  for (long ki = 0; ki < N; ++ki)
    for (long l = 0; l < L; ++l) {
      F[ki * L + l] = cis(ki - h, l, -1.0, 1.0);
      G[l * N + ki] = cis(ki - h, l, +1.0, 1.0 / (double)L);
    }
  for (long mi = 0; mi < M; ++mi)
    for (long l = 0; l < L; ++l) H[mi * L + l] = cis(mi - (N - 1), l, -1.0, 1.0);
  e = hipMemcpy(p->F, F.data(), F.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->G, G.data(), G.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->Hm, H.data(), H.size() * 8, hipMemcpyHostToDevice);
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    free_normal(p);
    delete p;
    return hip_fail(e, "normal_create: table upload");
  }
  {
    std::lock_guard<std::mutex> lk(g_nmu);
    g_nlive.insert(p);
  }
  *out = reinterpret_cast<spfel_normal>(p);
  return SPFEL_OK;
}

int spfel_normal_destroy(spfel_normal h) {
  clear_error();
  Normal *p = reinterpret_cast<Normal *>(h);
  {
    std::lock_guard<std::mutex> lk(g_nmu);
    if (!p || g_nlive.erase(p) == 0) return fail(SPFEL_ESTATE, "normal_destroy: not a live object");
  }
  free_normal(p);
  delete p;
  return SPFEL_OK;
}

int spfel_normal_set_psf(spfel_normal h, const void *psf, void *stream) {
  clear_error();
  Normal *p = reinterpret_cast<Normal *>(h);
  if (!nlive(p)) return fail(SPFEL_ESTATE, "normal_set_psf: not a live object");
  if (!psf) return fail(SPFEL_EINVAL, "normal_set_psf: psf is NULL");
  const bool cplx = p->domain == SPFEL_COMPLEX;
  if ((reinterpret_cast<uintptr_t>(psf) & (cplx ? 7 : 3)) != 0)
    return fail(SPFEL_EINVAL, "normal_set_psf: psf misaligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int M = 2 * p->N - 1, L = p->L;
  // That = DFT_L of the kernel placed at m mod L: three contractions M -> L
  hipError_t e = launch_contract(psf, cplx, p->Hm, p->X1, 0, M * M, M, L, 1, st);
  if (e == hipSuccess) e = launch_contract(p->X1, true, p->Hm, p->X2, 0, M, M, L, L, st);
  if (e == hipSuccess) e = launch_contract(p->X2, true, p->Hm, p->That, 0, 1, M, L, L * L, st);
  if (e != hipSuccess) return hip_fail(e, "normal_set_psf: launch");
  p->psf_set = true;
  return SPFEL_OK;
}

// Vectors are float32 (REAL) or complex64 (COMPLEX) arrays.
static bool vec_aligned(const Normal *p, const void *v) {
  return (reinterpret_cast<uintptr_t>(v) & (p->domain == SPFEL_COMPLEX ? 7 : 3)) == 0;
}

static int check_lambdas(const Normal *p, int n, const float *lambdas, Lambdas &lam,
                         const char *who) {
  if (n < 1 || n > p->max_sys) return fail(SPFEL_EINVAL, std::string(who) + ": n out of 1..max_systems");
  if (!lambdas) return fail(SPFEL_EINVAL, std::string(who) + ": lambdas is NULL");
  for (int s = 0; s < kMaxSystems; ++s) lam.v[s] = 0.f;
  for (int s = 0; s < n; ++s) {
    if (!(lambdas[s] >= 0.f) || !std::isfinite(lambdas[s]))
      return fail(SPFEL_EINVAL, std::string(who) + ": lambdas must be finite and >= 0");
    lam.v[s] = lambdas[s];
  }
  return SPFEL_OK;
}

int spfel_normal_apply(spfel_normal h, const void *x, int n, const float *lambdas, void *y,
                       void *stream) {
  clear_error();
  Normal *p = reinterpret_cast<Normal *>(h);
  if (!nlive(p)) return fail(SPFEL_ESTATE, "normal_apply: not a live object");
  if (!p->psf_set) return fail(SPFEL_ESTATE, "normal_apply: set_psf has not been called");
  Lambdas lam;
  int rc = check_lambdas(p, n, lambdas, lam, "normal_apply");
  if (rc != SPFEL_OK) return rc;
  if (!x || !y) return fail(SPFEL_EINVAL, "normal_apply: NULL pointer");
  if (!vec_aligned(p, x) || !vec_aligned(p, y)) return fail(SPFEL_EINVAL, "normal_apply: misaligned vector");
  hipError_t e = normal_apply(*p, x, n, &lam, y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "normal_apply: launch");
}

int spfel_normal_solve(spfel_normal h, const void *rhs, const void *x0, int n,
                       const float *lambdas, int iters, void *x_out, float *residuals,
                       void *stream) {
  clear_error();
  Normal *p = reinterpret_cast<Normal *>(h);
  if (!nlive(p)) return fail(SPFEL_ESTATE, "normal_solve: not a live object");
  if (!p->psf_set) return fail(SPFEL_ESTATE, "normal_solve: set_psf has not been called");
  Lambdas lam;
  int rc = check_lambdas(p, n, lambdas, lam, "normal_solve");
  if (rc != SPFEL_OK) return rc;
  if (!rhs || !x0 || !x_out) return fail(SPFEL_EINVAL, "normal_solve: NULL pointer");
  if (!vec_aligned(p, rhs) || !vec_aligned(p, x0) || !vec_aligned(p, x_out) ||
      (reinterpret_cast<uintptr_t>(residuals) & 3))
    return fail(SPFEL_EINVAL, "normal_solve: misaligned vector");
  if (iters < 0 || iters > 100000) return fail(SPFEL_EINVAL, "normal_solve: iters out of 0..100000");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool cplx = p->domain == SPFEL_COMPLEX;
  const int64_t N3 = (int64_t)p->N * p->N * p->N, len = N3 * (cplx ? 2 : 1);
  const float *rf = static_cast<const float *>(rhs), *x0f = static_cast<const float *>(x0);
  float *xf = static_cast<float *>(x_out), *r = static_cast<float *>(p->r);
  float *pp = static_cast<float *>(p->p), *Ap = static_cast<float *>(p->Ap);
  const int stride = iters + 1;
  // x = x0 for every system, Ap = (A* D A + lambda) x0 on the batch of copies
  hipLaunchKernelGGL(broadcast_kernel, grid_of(n * len), dim3(256), 0, st, x0f, len, n, xf);
  hipError_t e = normal_apply(*p, xf, n, &lam, Ap, st);
  if (e != hipSuccess) return hip_fail(e, "normal_solve: launch");
  hipLaunchKernelGGL(cg_init_kernel, grid_of(n * len), dim3(256), 0, st, rf, x0f, Ap, len, n, lam,
                     xf, r, pp);
  e = dots(*p, r, r, len, len, n, p->scal, 4, st);
  if (e != hipSuccess) return hip_fail(e, "normal_solve: launch");
  hipLaunchKernelGGL(cg_advance_kernel, dim3(1), dim3(64), 0, st, p->scal, n, residuals, 0,
                     stride, 0);
  for (int it = 1; it <= iters; ++it) {
    e = normal_apply(*p, pp, n, &lam, Ap, st);
    if (e == hipSuccess) e = dots(*p, pp, Ap, len, len, n, p->scal + 1, 4, st);
    if (e != hipSuccess) return hip_fail(e, "normal_solve: launch");
    hipLaunchKernelGGL(cg_update_kernel, grid_of(n * len), dim3(256), 0, st, p->scal, pp, Ap, len,
                       n, xf, r);
    e = dots(*p, r, r, len, len, n, p->scal + 2, 4, st);
    if (e != hipSuccess) return hip_fail(e, "normal_solve: launch");
    hipLaunchKernelGGL(cg_direction_kernel, grid_of(n * len), dim3(256), 0, st, p->scal, r, len,
                       n, pp);
    hipLaunchKernelGGL(cg_advance_kernel, dim3(1), dim3(64), 0, st, p->scal, n, residuals, it,
                       stride, 1);
  }
  e = hipGetLastError();
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "normal_solve: launch");
}

int spfel_normal_lcurve(spfel_normal h, const void *x, const void *rhs, const void *x0, int n,
                        const float *lambdas, double bdb, float *rho_eta, int32_t *corner,
                        void *stream) {
  clear_error();
  Normal *p = reinterpret_cast<Normal *>(h);
  if (!nlive(p)) return fail(SPFEL_ESTATE, "normal_lcurve: not a live object");
  if (!p->psf_set) return fail(SPFEL_ESTATE, "normal_lcurve: set_psf has not been called");
  Lambdas lam;
  int rc = check_lambdas(p, n, lambdas, lam, "normal_lcurve");
  if (rc != SPFEL_OK) return rc;
  if (!x || !rhs || !x0 || !rho_eta) return fail(SPFEL_EINVAL, "normal_lcurve: NULL pointer");
  if (!vec_aligned(p, x) || !vec_aligned(p, rhs) || !vec_aligned(p, x0) ||
      (reinterpret_cast<uintptr_t>(rho_eta) & 3) || (reinterpret_cast<uintptr_t>(corner) & 3))
    return fail(SPFEL_EINVAL, "normal_lcurve: misaligned array");
  if (n >= 3)
    for (int s = 0; s < n; ++s)
      if (!(lambdas[s] > 0.f))
        return fail(SPFEL_EINVAL, "normal_lcurve: the corner needs lambdas > 0 (log spacing)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool cplx = p->domain == SPFEL_COMPLEX;
  const int64_t N3 = (int64_t)p->N * p->N * p->N, len = N3 * (cplx ? 2 : 1);
  // Ap = A* D A x (no lambda); scal[s] = (x.Ap, x.rhs, |x - x0|^2)
  hipError_t e = normal_apply(*p, x, n, nullptr, p->Ap, st);
  if (e == hipSuccess) e = dots(*p, x, p->Ap, len, len, n, p->scal, 4, st);
  if (e == hipSuccess) e = dots(*p, x, rhs, len, 0, n, p->scal + 1, 4, st);
  if (e != hipSuccess) return hip_fail(e, "normal_lcurve: launch");
  hipLaunchKernelGGL(diff_kernel, grid_of(n * len), dim3(256), 0, st,
                     static_cast<const float *>(x), static_cast<const float *>(x0), len, n,
                     static_cast<float *>(p->r));
  e = dots(*p, p->r, p->r, len, len, n, p->scal + 2, 4, st);
  if (e != hipSuccess) return hip_fail(e, "normal_lcurve: launch");
  hipLaunchKernelGGL(lcurve_kernel, dim3(1), dim3(64), 0, st, p->scal, n, bdb, lam, rho_eta,
                     corner);
  e = hipGetLastError();
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "normal_lcurve: launch");
}

}  // extern "C"
