// libspfel C ABI: argument validation, plan lifecycle and dispatch to the
// kernel launchers.  No exception crosses this file's extern "C" functions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <numeric>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace spfel {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return SPFEL_EHIP;
}
void clear_error() { g_err.clear(); }

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on the
// three-term recurrence of the Legendre polynomials.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &wt) {
  x.resize(n);
  wt.resize(n);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    wt[i] = wt[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// psi_hat(k) = int_{-w/2}^{w/2} psi(tau) cos(2 pi k tau / nf) dtau.  With
// tau = (w/2) sin(theta) the integrand exp(beta (cos theta - 1))
// cos(pi k w sin(theta) / nf) (w/2) cos(theta) is smooth on [-pi/2, pi/2],
// so Gauss-Legendre in theta converges geometrically.
void kernel_transform(int N, int nf, int w, double beta, double *out) {
  std::vector<double> z, wt;
  const int n = 160;
  gauss_legendre(n, z, wt);
  const int h = (N - 1) / 2;
  for (int k = -h; k <= h; ++k) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      double th = 0.5 * M_PI * z[i];
      double tau = 0.5 * w * std::sin(th);
      double g = std::exp(beta * (std::cos(th) - 1.0)) *
                 std::cos(2.0 * M_PI * k * tau / nf) * 0.5 * w * std::cos(th);
      s += wt[i] * g;
    }
    out[k + h] = 0.5 * M_PI * s;
  }
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi
// rotations: columns of V are the eigenvectors, ev the eigenvalues.
static void sym3_eigen(const double A_in[3][3], double V[3][3], double ev[3]) {
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[i][j] = A_in[i][j];
      V[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (off < 1e-30 * (A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2]) || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; ++i) ev[i] = A[i][i];
}

// Position of lattice cell (x, y) along the Hilbert curve filling an n x n
// lattice (n a power of two): descend the quadrants from the largest,
// adding each quadrant's offset and reflecting/transposing the coordinates
// into the sub-curve's frame.
static uint64_t hilbert_index(uint32_t n, uint32_t x, uint32_t y) {
  uint64_t d = 0;
  for (uint32_t s = n >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - (x & (s - 1));
        y = s - 1 - (y & (s - 1));
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

static std::mutex g_mu;
static std::set<Plan *> g_live;

static bool live(Plan *p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return p != nullptr && g_live.count(p) != 0;
}

// Switches to a device for the scope of a call and back.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

static bool aligned(const void *p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

static void free_bins(Plan *p) {
  void *bufs[] = {p->bin_pts[0], p->bin_pts[1], p->bin_aux[0], p->bin_aux[1], p->bin_off[0],
                  p->bin_off[1], p->bin_cur, p->bin_part, p->bin_sub[0], p->bin_sub[1],
                  p->bin_nsub[0], p->bin_nsub[1]};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  for (int k = 0; k < 2; ++k) {
    p->bin_pts[k] = nullptr;
    p->bin_aux[k] = nullptr;
    p->bin_off[k] = p->bin_nsub[k] = nullptr;
    p->bin_sub[k] = nullptr;
  }
  p->bin_cur = p->bin_part = nullptr;
  p->bin_cap = p->bin_batch = 0;
}

// Scratch of the binned spread for detectors of P points: batches of up to
// 2^27 points (and at most 65,536 images), key counts and offsets,
// subproblem list, the spread's inputs twice (binning and spreading of
// consecutive batches overlap).  Returns the bytes allocated, or 0 on
// failure (nothing kept).
static size_t alloc_bins(Plan *p, int64_t P) {
  const int64_t per = std::max<int64_t>(1, std::min<int64_t>(kBinBatchPoints / P, 65536));
  const int64_t cap = per * P;
  const size_t keys = bin_keys(p->nf, p->w);
  const size_t parts = (keys + 1023) / 1024;
  const size_t subs = bin_max_subproblems(p->nf, p->w, cap);
  struct Req {
    void **ptr;
    size_t bytes;
  } reqs[] = {{reinterpret_cast<void **>(&p->bin_pts[0]), (size_t)cap * sizeof(float4)},
              {reinterpret_cast<void **>(&p->bin_pts[1]), (size_t)cap * sizeof(float4)},
              {reinterpret_cast<void **>(&p->bin_aux[0]), (size_t)cap * sizeof(uint2)},
              {reinterpret_cast<void **>(&p->bin_aux[1]), (size_t)cap * sizeof(uint2)},
              {reinterpret_cast<void **>(&p->bin_off[0]), (keys + 1) * sizeof(int32_t)},
              {reinterpret_cast<void **>(&p->bin_off[1]), (keys + 1) * sizeof(int32_t)},
              {reinterpret_cast<void **>(&p->bin_cur), keys * sizeof(int32_t)},
              {reinterpret_cast<void **>(&p->bin_part), parts * sizeof(int32_t)},
              {reinterpret_cast<void **>(&p->bin_sub[0]), subs * sizeof(int4)},
              {reinterpret_cast<void **>(&p->bin_sub[1]), subs * sizeof(int4)},
              {reinterpret_cast<void **>(&p->bin_nsub[0]), 256},
              {reinterpret_cast<void **>(&p->bin_nsub[1]), 256}};
  size_t total = 0;
  for (auto &r : reqs) {
    if (hipMalloc(r.ptr, r.bytes) != hipSuccess) {
      *r.ptr = nullptr;
      (void)hipGetLastError();
      free_bins(p);
      return 0;
    }
    total += r.bytes;
  }
  p->bin_cap = cap;
  p->bin_batch = per;
  return total;
}

static void free_plan(Plan *p) {
  free_bins(p);
  void *bufs[] = {p->u, p->wpos, p->wneg, p->t1, p->t2, p->acc, p->partials, p->rot,
                  p->det_sorted, p->det_perm};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  hipEvent_t evs[] = {p->ev_start,     p->ev_sliced[0], p->ev_sliced[1], p->ev_matched[0],
                      p->ev_matched[1], p->ev_bin_start, p->ev_binned[0], p->ev_binned[1],
                      p->ev_spread[0],  p->ev_spread[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (p->bin_stream) (void)hipStreamDestroy(p->bin_stream);
}

static bool m_offset_overflow(int64_t M) { return M > 0x7fffffffLL; }

static bool test_fail_alloc() {
  const char *e = std::getenv("SPFEL_TEST_FAIL_ALLOC");
  return e != nullptr && e[0] == '1';
}

}  // namespace spfel

using namespace spfel;

extern "C" {

int spfel_version(void) { return 100; }

const char *spfel_last_error(void) { return g_err.c_str(); }

int spfel_plan_create(spfel_plan *out, int n_model, int kernel_width,
                      double upsampfac, double beta_over_w, int domain,
                      int device) {
  clear_error();
  if (!out) return fail(SPFEL_EINVAL, "plan_create: out is NULL");
  *out = nullptr;
  if (n_model < 3 || n_model % 2 == 0)
    return fail(SPFEL_EINVAL, "plan_create: n_model must be odd and >= 3");
  if (n_model > 511) return fail(SPFEL_ERANGE, "plan_create: n_model > 511");
  if (kernel_width < 2 || kernel_width > 16)
    return fail(SPFEL_EINVAL, "plan_create: kernel_width out of [2, 16]");
  if (kernel_width > n_model)
    return fail(SPFEL_EINVAL, "plan_create: kernel_width > n_model");
  if (kernel_width < 4 || kernel_width > 8)
    return fail(SPFEL_EUNSUPPORTED, "plan_create: kernel_width must be 4..8");
  if (!(upsampfac == 2.0))
    return fail(SPFEL_EUNSUPPORTED, "plan_create: only upsampfac 2.0 (n_f = 2N)");
  if (!(beta_over_w > 0.0 && beta_over_w <= 10.0))
    return fail(SPFEL_EINVAL, "plan_create: beta_over_w out of (0, 10]");
  if (domain != SPFEL_REAL && domain != SPFEL_COMPLEX)
    return fail(SPFEL_EINVAL, "plan_create: domain must be REAL or COMPLEX");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "plan_create: hipGetDeviceCount");
  if (device < 0 || device >= ndev)
    return fail(SPFEL_EINVAL, "plan_create: no such device");
  DeviceGuard g(device);
  if (g.err != hipSuccess) return hip_fail(g.err, "plan_create: hipSetDevice");

  Plan *p = new (std::nothrow) Plan();
  if (!p) return fail(SPFEL_ENOMEM, "plan_create: host allocation");
  p->device = device;
  p->N = n_model;
  p->nf = 2 * n_model;
  p->w = kernel_width;
  p->domain = domain;
  p->beta = beta_over_w * kernel_width;
  const size_t N = n_model, nf = p->nf;
  const size_t el = domain == SPFEL_COMPLEX ? sizeof(float2) : sizeof(float);
  const size_t grid_b = nf * nf * nf * el;
  const size_t tab_b = N * nf * sizeof(float2);
  const size_t tmp_b = 4 * N * N * N * sizeof(float2);
  struct Req {
    void **ptr;
    size_t bytes;
  } reqs[] = {{&p->u, grid_b},
              {reinterpret_cast<void **>(&p->wpos), tab_b},
              {reinterpret_cast<void **>(&p->wneg), tab_b},
              {reinterpret_cast<void **>(&p->t1), tmp_b},
              {reinterpret_cast<void **>(&p->t2), tmp_b},
              {&p->acc, grid_b},
              {reinterpret_cast<void **>(&p->partials), kMaxPartials * sizeof(double)},
              {reinterpret_cast<void **>(&p->rot), kRotCap * 9 * sizeof(double)}};
  for (auto &r : reqs) {
    if (test_fail_alloc()) {
      free_plan(p);
      delete p;
      return fail(SPFEL_ENOMEM, "plan_create: device allocation failed (forced by SPFEL_TEST_FAIL_ALLOC)");
    }
    e = hipMalloc(r.ptr, r.bytes);
    if (e != hipSuccess) {
      *r.ptr = nullptr;
      (void)hipGetLastError();
      free_plan(p);
      delete p;
      return fail(SPFEL_ENOMEM, std::string("plan_create: hipMalloc: ") + hipGetErrorString(e));
    }
    p->bytes += r.bytes;
  }
  for (hipEvent_t *ev : {&p->ev_start, &p->ev_sliced[0], &p->ev_sliced[1], &p->ev_matched[0],
                         &p->ev_matched[1], &p->ev_bin_start, &p->ev_binned[0], &p->ev_binned[1],
                         &p->ev_spread[0], &p->ev_spread[1]}) {
    e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      *ev = nullptr;
      free_plan(p);
      delete p;
      return hip_fail(e, "plan_create: hipEventCreate");
    }
  }
  e = hipStreamCreateWithFlags(&p->bin_stream, hipStreamNonBlocking);   // default priority
  if (e != hipSuccess) {
    p->bin_stream = nullptr;
    free_plan(p);
    delete p;
    return hip_fail(e, "plan_create: hipStreamCreate");
  }
  // Transform tables in float64, rounded once to float32.  The phase index
  // k l is reduced modulo nf exactly before the trigonometric evaluation.
  std::vector<double> ph(N);
  kernel_transform(n_model, p->nf, kernel_width, p->beta, ph.data());
  const int h = (n_model - 1) / 2;
  std::vector<float2> wp(N * nf), wn(nf * N);
  // wpos writes the interpolation grid in centred storage (cell l at index
  // (l + nf/2) mod nf): its phase is that of cell l = index - nf/2.
  for (int ki = 0; ki < n_model; ++ki) {
    const long k = ki - h;
    for (int l = 0; l < p->nf; ++l) {
      const long nl = (long)nf;
      long r = (k * l) % nl, rc = (k * ((long)l - nl / 2)) % nl;
      if (r < 0) r += nf;
      if (rc < 0) rc += nf;
      const double a = 2.0 * M_PI * (double)r / (double)nf;
      const double ac = 2.0 * M_PI * (double)rc / (double)nf;
      wp[(size_t)ki * nf + l] =
          make_float2((float)(std::cos(ac) / ph[ki]), (float)(std::sin(ac) / ph[ki]));
      wn[(size_t)l * N + ki] =
          make_float2((float)(std::cos(a) / ph[ki]), (float)(-std::sin(a) / ph[ki]));
    }
  }
  e = hipMemcpy(p->wpos, wp.data(), tab_b, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->wneg, wn.data(), tab_b, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    delete p;
    return hip_fail(e, "plan_create: table upload");
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.insert(p);
  }
  *out = reinterpret_cast<spfel_plan>(p);
  return SPFEL_OK;
}

int spfel_plan_destroy(spfel_plan plan) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!p || g_live.erase(p) == 0) return fail(SPFEL_ESTATE, "plan_destroy: not a live plan");
  }
  DeviceGuard g(p->device);
  free_plan(p);
  delete p;
  return SPFEL_OK;
}

int spfel_plan_info(spfel_plan plan, int *n_fine, size_t *device_bytes) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "plan_info: not a live plan");
  if (n_fine) *n_fine = p->nf;
  if (device_bytes) *device_bytes = p->bytes;
  return SPFEL_OK;
}

int spfel_set_detector(spfel_plan plan, const float *det_q, int64_t P, void *stream) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "set_detector: not a live plan");
  if (P <= 0) return fail(SPFEL_EINVAL, "set_detector: P must be positive");
  if (P > (int64_t)1 << 30) return fail(SPFEL_ERANGE, "set_detector: P too large");
  if (!det_q || !aligned(det_q, 4)) return fail(SPFEL_EINVAL, "set_detector: det_q NULL or misaligned");
  DeviceGuard g(p->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "set_detector: hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> h((size_t)P * 3);
  hipError_t e = hipMemcpyAsync(h.data(), det_q, h.size() * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "set_detector: copy to host");
  // Order the points along a Hilbert curve on their principal plane (the
  // detector template is a 2D surface): consecutive points are neighbours,
  // so each run of kTile points is a compact patch.  Non-finite points last.
  double mean[3] = {0, 0, 0};
  int64_t nfin = 0;
  std::vector<char> fin((size_t)P);
  for (int64_t i = 0; i < P; ++i) {
    fin[i] = std::isfinite(h[3 * i]) && std::isfinite(h[3 * i + 1]) && std::isfinite(h[3 * i + 2]);
    if (!fin[i]) continue;
    for (int d = 0; d < 3; ++d) mean[d] += h[3 * i + d];
    ++nfin;
  }
  for (int d = 0; d < 3; ++d) mean[d] /= (nfin > 0 ? (double)nfin : 1.0);
  double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int64_t i = 0; i < P; ++i) {
    if (!fin[i]) continue;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) C[a][b] += (h[3 * i + a] - mean[a]) * (h[3 * i + b] - mean[b]);
  }
  double V[3][3], ev[3];
  sym3_eigen(C, V, ev);
  int order[3] = {0, 1, 2};
  std::sort(order, order + 3, [&](int a, int b) { return ev[a] > ev[b]; });
  std::vector<double> uv((size_t)P * 2, 0.0);
  double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
  for (int64_t i = 0; i < P; ++i) {
    if (!fin[i]) continue;
    for (int k = 0; k < 2; ++k) {
      double v = 0.0;
      for (int d = 0; d < 3; ++d) v += (h[3 * i + d] - mean[d]) * V[d][order[k]];
      uv[2 * i + k] = v;
      lo[k] = std::min(lo[k], v);
      hi[k] = std::max(hi[k], v);
    }
  }
  // lattice of about twice the point spacing's resolution, a power of two
  int res = 1;
  while ((double)res * (double)res < 4.0 * (double)P && res < (1 << 15)) res <<= 1;
  const double span = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), 1e-300);
  std::vector<uint64_t> key((size_t)P);
  for (int64_t i = 0; i < P; ++i) {
    if (!fin[i]) {
      key[i] = ~0ull;
      continue;
    }
    uint32_t gx = (uint32_t)std::min(std::max((uv[2 * i] - lo[0]) / span * (res - 1) + 0.5, 0.0), (double)(res - 1));
    uint32_t gy = (uint32_t)std::min(std::max((uv[2 * i + 1] - lo[1]) / span * (res - 1) + 0.5, 0.0), (double)(res - 1));
    key[i] = hilbert_index((uint32_t)res, gx, gy);
  }
  std::vector<int32_t> perm((size_t)P);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  std::vector<float> sorted((size_t)P * 3);
  for (int64_t i = 0; i < P; ++i)
    for (int d = 0; d < 3; ++d) sorted[3 * i + d] = h[3 * (size_t)perm[i] + d];
  float *ds = nullptr;
  int32_t *dp = nullptr;
  e = hipMalloc(reinterpret_cast<void **>(&ds), sorted.size() * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&dp), perm.size() * sizeof(int32_t));
  if (e != hipSuccess) {
    if (ds) (void)hipFree(ds);
    (void)hipGetLastError();
    return fail(SPFEL_ENOMEM, "set_detector: hipMalloc");
  }
  e = hipMemcpy(ds, sorted.data(), sorted.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dp, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(ds);
    (void)hipFree(dp);
    return hip_fail(e, "set_detector: upload");
  }
  if (p->det_sorted) {
    p->bytes -= (size_t)p->det_P * 3 * sizeof(float) + (size_t)p->det_P * sizeof(int32_t);
    (void)hipFree(p->det_sorted);
    (void)hipFree(p->det_perm);
    p->det_sorted = nullptr;
    p->det_perm = nullptr;
    p->det_P = 0;
  }
  if (p->bin_cap) {
    p->bytes -= p->bin_bytes;
    free_bins(p);
    p->bin_bytes = 0;
  }
  const size_t bb = alloc_bins(p, P);
  if (bb == 0) {
    (void)hipFree(ds);
    (void)hipFree(dp);
    return fail(SPFEL_ENOMEM, "set_detector: hipMalloc of the spreading scratch");
  }
  p->bin_bytes = bb;
  p->bytes += bb;
  p->det_sorted = ds;
  p->det_perm = dp;
  p->det_P = P;
  p->bytes += sorted.size() * sizeof(float) + perm.size() * sizeof(int32_t);
  return SPFEL_OK;
}

int spfel_set_model(spfel_plan plan, const void *model, void *stream) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "set_model: not a live plan");
  if (!model) return fail(SPFEL_EINVAL, "set_model: model is NULL");
  const bool cplx = p->domain == SPFEL_COMPLEX;
  if (!aligned(model, cplx ? 8 : 4)) return fail(SPFEL_EINVAL, "set_model: model misaligned");
  DeviceGuard g(p->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "set_model: hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int N = p->N, nf = p->nf;
  // u[l] = sum_k m_k exp(+2 pi i k.l / nf) / (psi_hat psi_hat psi_hat), one
  // axis at a time: axis 2 (N^2 lines), axis 1, axis 0.
  hipError_t e = launch_contract(model, cplx, p->wpos, p->t1, 0, N * N, N, nf, 1, s);
  if (e == hipSuccess) e = launch_contract(p->t1, true, p->wpos, p->t2, 0, N, N, nf, nf, s);
  if (e == hipSuccess) e = launch_contract(p->t2, true, p->wpos, p->u, cplx ? 0 : 1, 1, N, nf, nf * nf, s);
  if (e != hipSuccess) return hip_fail(e, "set_model: launch");
  p->model_set = true;
  return SPFEL_OK;
}

int spfel_slice(spfel_plan plan, const float *quats, int64_t M,
                const float *det_q, int64_t P, void *out, float *out_norm2, void *stream) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "slice: not a live plan");
  if (!p->model_set) return fail(SPFEL_ESTATE, "slice: set_model has not been called");
  if (M < 0 || P < 0) return fail(SPFEL_EINVAL, "slice: negative size");
  const bool cplx = p->domain == SPFEL_COMPLEX;
  if (M == 0) return SPFEL_OK;
  if (P == 0) {
    if (out_norm2 && !aligned(out_norm2, 4)) return fail(SPFEL_EINVAL, "slice: out_norm2 misaligned");
    DeviceGuard g0(p->device);
    if (g0.err != hipSuccess) return hip_fail(g0.err, "slice: hipSetDevice");
    hipError_t e0 = out_norm2 ? launch_fill_zero(out_norm2, (size_t)M * sizeof(float),
                                                 static_cast<hipStream_t>(stream))
                              : hipSuccess;
    return e0 == hipSuccess ? SPFEL_OK : hip_fail(e0, "slice: launch");
  }
  if (!out && !out_norm2) return fail(SPFEL_EINVAL, "slice: no output requested");
  if (out_norm2 && !out) return fail(SPFEL_EINVAL, "slice: norms need out");
  if (!quats) return fail(SPFEL_EINVAL, "slice: quats is NULL");
  if (!det_q && P != p->det_P)
    return fail(SPFEL_EINVAL, "slice: det_q is NULL and P differs from the registered detector");
  if (!aligned(quats, 4) || (det_q && !aligned(det_q, 4))) return fail(SPFEL_EINVAL, "slice: input misaligned");
  if (!aligned(out, cplx ? 8 : 4)) return fail(SPFEL_EINVAL, "slice: out misaligned");
  if (out_norm2 && !aligned(out_norm2, 4)) return fail(SPFEL_EINVAL, "slice: out_norm2 misaligned");
  if (M > (int64_t)1 << 31 || P > (int64_t)1 << 30) return fail(SPFEL_ERANGE, "slice: M or P too large");
  DeviceGuard g(p->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "slice: hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_interp(*p, quats, M, det_q, P, out, s);
  if (e == hipSuccess && out_norm2) e = launch_row_norm2(out, false, M, cplx ? 2 * P : P, out_norm2, s);
  if (e != hipSuccess) return hip_fail(e, "slice: launch");
  return SPFEL_OK;
}

int spfel_row_norm2(const void *x, int dtype, int64_t rows, int64_t cols,
                    float *out, void *stream) {
  clear_error();
  if (rows < 0 || cols < 0) return fail(SPFEL_EINVAL, "row_norm2: negative size");
  if (dtype != SPFEL_F32 && dtype != SPFEL_BF16) return fail(SPFEL_EINVAL, "row_norm2: dtype");
  if (rows == 0) return SPFEL_OK;
  if (!out || (!x && cols > 0)) return fail(SPFEL_EINVAL, "row_norm2: NULL pointer");
  if (!aligned(out, 4) || (x && !aligned(x, dtype == SPFEL_F32 ? 4 : 2)))
    return fail(SPFEL_EINVAL, "row_norm2: misaligned");
  if (rows > (int64_t)1 << 31) return fail(SPFEL_ERANGE, "row_norm2: too many rows");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = cols == 0 ? launch_fill_zero(out, (size_t)rows * 4, s)
                           : launch_row_norm2(x, dtype == SPFEL_BF16, rows, cols, out, s);
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "row_norm2: launch");
}

int spfel_column_mean(const float *x, int64_t rows, int64_t cols, int round_to_integer,
                      float *out, void *stream) {
  clear_error();
  if (rows < 1 || cols < 0) return fail(SPFEL_EINVAL, "column_mean: rows must be >= 1, cols >= 0");
  if (cols == 0) return SPFEL_OK;
  if (!x || !out) return fail(SPFEL_EINVAL, "column_mean: NULL pointer");
  if (!aligned(x, 4) || !aligned(out, 4)) return fail(SPFEL_EINVAL, "column_mean: misaligned");
  if (cols > (int64_t)1 << 31) return fail(SPFEL_ERANGE, "column_mean: too many columns");
  hipError_t e = launch_column_mean(x, rows, cols, round_to_integer, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "column_mean: launch");
}

int spfel_bf16_centred(const float *x, int64_t rows, int64_t cols, const float *centre,
                       uint16_t *out, float *norm2, float *err, void *stream) {
  clear_error();
  if (rows < 0 || cols < 0) return fail(SPFEL_EINVAL, "bf16_centred: negative size");
  if (rows == 0) return SPFEL_OK;
  if (!norm2 && !err && !out) return fail(SPFEL_EINVAL, "bf16_centred: no output requested");
  if (!out) return fail(SPFEL_EINVAL, "bf16_centred: out is NULL");
  if (!x && cols > 0) return fail(SPFEL_EINVAL, "bf16_centred: x is NULL");
  if ((x && !aligned(x, 4)) || (centre && !aligned(centre, 4)) || !aligned(out, 2) ||
      (norm2 && !aligned(norm2, 4)) || (err && !aligned(err, 4)))
    return fail(SPFEL_EINVAL, "bf16_centred: misaligned pointer");
  if (rows > (int64_t)1 << 31 || cols > (int64_t)1 << 30) return fail(SPFEL_ERANGE, "bf16_centred: size too large");
  hipError_t e = launch_bf16_centred(x, rows, cols, centre, out, norm2, err, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "bf16_centred: launch");
}

int spfel_scale_columns(const float *x, int64_t rows, int64_t cols, const float *g, float *out,
                        void *stream) {
  clear_error();
  if (rows < 0 || cols < 0) return fail(SPFEL_EINVAL, "scale_columns: negative size");
  if (rows == 0 || cols == 0) return SPFEL_OK;
  if (!x || !g || !out) return fail(SPFEL_EINVAL, "scale_columns: NULL pointer");
  if (!aligned(x, 4) || !aligned(g, 4) || !aligned(out, 4))
    return fail(SPFEL_EINVAL, "scale_columns: misaligned pointer");
  hipError_t e = launch_scale_columns(x, rows, cols, g, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "scale_columns: launch");
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t spfel_match_workspace_bytes(int64_t M, int64_t n_img, int64_t P, int mode) {
  if (M < 0 || n_img < 0 || P < 0) return 0;
  size_t b = match_f32_workspace_bytes(M, n_img, P);
  if (mode == SPFEL_MATCH_BF16_RESCORE8)
    b = align256(match_bf16_candidate_bytes(M, n_img)) + match_rescore_bytes(n_img);
  return b < 256 ? 256 : b;
}

int spfel_match(const void *slices, const float *slice_norm2,
                const void *images, const float *image_norm2, int64_t M,
                int64_t n_img, int64_t P, int64_t m_offset, int mode,
                const float *slices_f32, const float *images_f32,
                const float *slice_err, const float *image_err,
                int32_t *best_idx, float *best_dist, int32_t *flags, void *workspace,
                size_t workspace_bytes, void *stream) {
  clear_error();
  if (M < 0 || n_img < 0 || P < 0 || m_offset < 0) return fail(SPFEL_EINVAL, "match: negative size");
  if (mode != SPFEL_MATCH_FP32 && mode != SPFEL_MATCH_BF16_RESCORE8)
    return fail(SPFEL_EINVAL, "match: unknown mode");
  if (m_offset + M > 0x7fffffffLL) return fail(SPFEL_ERANGE, "match: model index exceeds int32");
  if (P > (int64_t)1 << 30 || n_img > (int64_t)1 << 30) return fail(SPFEL_ERANGE, "match: size too large");
  if (M == 0 || n_img == 0) return SPFEL_OK;
  if (!slices || !images || !slice_norm2 || !image_norm2 || !best_idx || !best_dist)
    return fail(SPFEL_EINVAL, "match: NULL pointer");
  const bool bf = mode != SPFEL_MATCH_FP32;
  if (bf && (!slices_f32 || !images_f32 || !slice_err || !image_err))
    return fail(SPFEL_EINVAL, "match: BF16 mode needs slices_f32, images_f32, slice_err and image_err");
  if (!aligned(slices, bf ? 2 : 4) || !aligned(images, bf ? 2 : 4) || !aligned(slice_norm2, 4) ||
      !aligned(image_norm2, 4) || !aligned(best_idx, 4) || !aligned(best_dist, 4) ||
      (bf && (!aligned(slices_f32, 4) || !aligned(images_f32, 4) || !aligned(slice_err, 4) ||
              !aligned(image_err, 4) || (flags && !aligned(flags, 4)))))
    return fail(SPFEL_EINVAL, "match: misaligned pointer");
  const size_t need = spfel_match_workspace_bytes(M, n_img, P, mode);
  if (!workspace || workspace_bytes < need)
    return fail(SPFEL_EINVAL, "match: workspace smaller than spfel_match_workspace_bytes");
  if (!aligned(workspace, 256)) return fail(SPFEL_EINVAL, "match: workspace not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (!bf) {
    auto *keys = static_cast<unsigned long long *>(workspace);
    e = launch_pack_keys(best_idx, best_dist, keys, n_img, s);
    if (e == hipSuccess)
      e = launch_match_f32(static_cast<const float *>(slices), static_cast<const float *>(images),
                           slice_norm2, image_norm2, M, n_img, P, m_offset, workspace, s);
    if (e == hipSuccess) e = launch_unpack_keys(keys, best_idx, best_dist, n_img, s);
  } else {
    auto *cand = static_cast<uint32_t *>(workspace);
    char *scratch = static_cast<char *>(workspace) + align256(match_bf16_candidate_bytes(M, n_img));
    e = launch_match_bf16(static_cast<const uint16_t *>(slices), static_cast<const uint16_t *>(images),
                          slice_norm2, image_norm2, M, n_img, P, cand, s);
    if (e == hipSuccess)
      e = launch_rescore(cand, match_bf16_tile_rows(M, n_img, P, slices, images), M, n_img, P,
                         m_offset, slices_f32, images_f32, slice_norm2, image_norm2, slice_err,
                         image_err, best_idx, best_dist, flags, scratch, s);
  }
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "match: launch");
}

// Slice buffers of one pipeline stage, carved from the caller's workspace.
struct OrientStage {
  float *f32 = nullptr;      // chunk x P
  uint16_t *b16 = nullptr;   // chunk x P centred BF16 (BF16 mode)
  float *norm = nullptr;     // chunk: float32 norms (FP32 mode) or BF16 norms
  float *err = nullptr;      // chunk: rounding-error norms (BF16 mode)
};

static size_t orient_stage_bytes(int64_t chunk, int64_t P, int mode) {
  size_t b = align256((size_t)chunk * P * sizeof(float));
  if (mode == SPFEL_MATCH_BF16_RESCORE8) b += align256((size_t)chunk * P * 2) + align256((size_t)chunk * sizeof(float));
  b += align256((size_t)chunk * sizeof(float));
  return b;
}

// Largest matcher workspace over every chunk length up to `chunk` (the last
// chunk may be shorter, and split-K choices depend on the tile count).
static size_t match_ws_upto(int64_t chunk, int64_t n_img, int64_t P, int mode) {
  size_t b = 0;
  for (int64_t m = chunk; m > 0; m -= 128) b = std::max(b, spfel_match_workspace_bytes(m, n_img, P, mode));
  return b;
}

size_t spfel_orient_workspace_bytes(int64_t chunk, int64_t n_img, int64_t P, int mode) {
  if (chunk <= 0 || n_img < 0 || P < 0) return 0;
  return 2 * orient_stage_bytes(chunk, P, mode) + align256(match_ws_upto(chunk, n_img, P, mode));
}

int spfel_orient(spfel_plan plan, const float *quats, int64_t M, const float *det_q, int64_t P,
                 const float *pixel_scale, const void *images, const float *image_norm2,
                 const float *images_f32,
                 const float *image_err, const float *centre, int64_t n_img, int mode,
                 int64_t chunk, int32_t *best_idx, float *best_dist, int32_t *flags,
                 void *workspace, size_t workspace_bytes, void *stream, void *aux_stream) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "orient: not a live plan");
  if (!p->model_set) return fail(SPFEL_ESTATE, "orient: set_model has not been called");
  if (p->domain != SPFEL_REAL) return fail(SPFEL_EUNSUPPORTED, "orient: REAL plans only");
  if (M < 0 || P < 0 || n_img < 0) return fail(SPFEL_EINVAL, "orient: negative size");
  if (chunk <= 0) return fail(SPFEL_EINVAL, "orient: chunk must be positive");
  if (mode != SPFEL_MATCH_FP32 && mode != SPFEL_MATCH_BF16_RESCORE8)
    return fail(SPFEL_EINVAL, "orient: unknown mode");
  if (M == 0 || n_img == 0) return SPFEL_OK;
  if (P == 0) return fail(SPFEL_EINVAL, "orient: P must be positive");
  if (!det_q && P != p->det_P)
    return fail(SPFEL_EINVAL, "orient: det_q is NULL and P differs from the registered detector");
  if (!quats || !images || !image_norm2 || !best_idx || !best_dist)
    return fail(SPFEL_EINVAL, "orient: NULL pointer");
  const bool bf = mode == SPFEL_MATCH_BF16_RESCORE8;
  if (bf && (!images_f32 || !image_err))
    return fail(SPFEL_EINVAL, "orient: BF16 mode needs images_f32 and image_err");
  if (bf && centre && !aligned(centre, 4)) return fail(SPFEL_EINVAL, "orient: centre misaligned");
  if (pixel_scale && !aligned(pixel_scale, 4)) return fail(SPFEL_EINVAL, "orient: pixel_scale misaligned");
  if (m_offset_overflow(M)) return fail(SPFEL_ERANGE, "orient: model index exceeds int32");
  if (chunk > M) chunk = M;
  const size_t need = spfel_orient_workspace_bytes(chunk, n_img, P, mode);
  if (!workspace || workspace_bytes < need || !aligned(workspace, 256))
    return fail(SPFEL_EINVAL, "orient: workspace smaller than spfel_orient_workspace_bytes or not 256-byte aligned");
  DeviceGuard g(p->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "orient: hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStream_t a = static_cast<hipStream_t>(aux_stream);
  char *ws = static_cast<char *>(workspace);
  OrientStage st[2];
  const size_t sb = orient_stage_bytes(chunk, P, mode);
  for (int k = 0; k < 2; ++k) {
    char *b = ws + k * sb;
    st[k].f32 = reinterpret_cast<float *>(b);
    b += align256((size_t)chunk * P * sizeof(float));
    if (bf) {
      st[k].b16 = reinterpret_cast<uint16_t *>(b);
      b += align256((size_t)chunk * P * 2);
      st[k].err = reinterpret_cast<float *>(b);
      b += align256((size_t)chunk * sizeof(float));
    }
    st[k].norm = reinterpret_cast<float *>(b);
  }
  void *mws = ws + 2 * sb;
  const size_t mws_bytes = workspace_bytes - 2 * sb;
  hipError_t e = hipEventRecord(p->ev_start, s);
  if (e == hipSuccess && a != s) e = hipStreamWaitEvent(a, p->ev_start, 0);
  if (e != hipSuccess) return hip_fail(e, "orient: event");
  const int64_t nchunks = (M + chunk - 1) / chunk;
  int rc = SPFEL_OK;
  for (int64_t c = 0; c < nchunks && rc == SPFEL_OK; ++c) {
    const int k = (int)(c & 1);
    const int64_t m0 = c * chunk, mc = std::min(chunk, M - m0);
    // slice stage on the auxiliary stream (after this buffer's last match)
    if (c >= 2 && a != s) {
      e = hipStreamWaitEvent(a, p->ev_matched[k], 0);
      if (e != hipSuccess) return hip_fail(e, "orient: event");
    }
    rc = spfel_slice(plan, quats + 4 * m0, mc, det_q, P, st[k].f32,
                     bf || pixel_scale ? nullptr : st[k].norm, a);
    if (rc != SPFEL_OK) return rc;
    if (pixel_scale) {
      rc = spfel_scale_columns(st[k].f32, mc, P, pixel_scale, st[k].f32, a);
      if (rc == SPFEL_OK && !bf) rc = spfel_row_norm2(st[k].f32, SPFEL_F32, mc, P, st[k].norm, a);
      if (rc != SPFEL_OK) return rc;
    }
    if (bf) {
      rc = spfel_bf16_centred(st[k].f32, mc, P, centre, st[k].b16, st[k].norm, st[k].err, a);
      if (rc != SPFEL_OK) return rc;
    }
    e = hipEventRecord(p->ev_sliced[k], a);
    if (e == hipSuccess && a != s) e = hipStreamWaitEvent(s, p->ev_sliced[k], 0);
    if (e != hipSuccess) return hip_fail(e, "orient: event");
    // match stage on the caller's stream
    const void *sl = bf ? static_cast<const void *>(st[k].b16) : static_cast<const void *>(st[k].f32);
    rc = spfel_match(sl, st[k].norm, images, image_norm2, mc, n_img, P, m0, mode,
                     bf ? st[k].f32 : nullptr, images_f32, bf ? st[k].err : nullptr, image_err,
                     best_idx, best_dist, flags, mws, mws_bytes, s);
    if (rc != SPFEL_OK) return rc;
    e = hipEventRecord(p->ev_matched[k], s);
    if (e != hipSuccess) return hip_fail(e, "orient: event");
  }
  return rc;
}

int spfel_merge_adjoint(spfel_plan plan, const float *quats, int64_t n_img,
                        const float *det_q, int64_t P, const void *values,
                        const float *weights, void *out, int flags,
                        void *stream) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "merge_adjoint: not a live plan");
  if (n_img < 0 || P < 0) return fail(SPFEL_EINVAL, "merge_adjoint: negative size");
  if (flags & ~(SPFEL_MERGE_ACCUMULATE | SPFEL_MERGE_DEFER))
    return fail(SPFEL_EINVAL, "merge_adjoint: unknown flag");
  const bool defer = (flags & SPFEL_MERGE_DEFER) != 0;
  const bool cplx = p->domain == SPFEL_COMPLEX;
  if (!defer && !out) return fail(SPFEL_EINVAL, "merge_adjoint: out is NULL");
  if (out && !aligned(out, cplx ? 8 : 4)) return fail(SPFEL_EINVAL, "merge_adjoint: out misaligned");
  const bool any = n_img > 0 && P > 0;
  if (any) {
    if (!quats || !values) return fail(SPFEL_EINVAL, "merge_adjoint: NULL input");
    if (!det_q && P != p->det_P)
      return fail(SPFEL_EINVAL, "merge_adjoint: det_q is NULL and P differs from the registered detector");
    if (!aligned(quats, 4) || (det_q && !aligned(det_q, 4)) || !aligned(values, cplx ? 8 : 4) ||
        (weights && !aligned(weights, 4)))
      return fail(SPFEL_EINVAL, "merge_adjoint: input misaligned");
    if (n_img > (int64_t)1 << 31 || P > (int64_t)1 << 30)
      return fail(SPFEL_ERANGE, "merge_adjoint: size too large");
  }
  DeviceGuard g(p->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "merge_adjoint: hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nf = p->nf;
  const size_t grid_b = nf * nf * nf * (cplx ? sizeof(float2) : sizeof(float));
  hipError_t e = hipSuccess;
  if (!p->pending) e = launch_fill_zero(p->acc, grid_b, s);
  if (e == hipSuccess && any) e = launch_spread(*p, quats, n_img, det_q, P, values, weights, s);
  if (e != hipSuccess) return hip_fail(e, "merge_adjoint: launch");
  p->pending = true;
  if (defer) return SPFEL_OK;
  p->pending = false;
  const int N = p->N, nfi = p->nf;
  const bool acc = (flags & SPFEL_MERGE_ACCUMULATE) != 0;
  // f_k = sum_l v_l exp(-2 pi i k.l / nf) / (psi_hat psi_hat psi_hat),
  // truncated to the N^3 modes: axis 2, axis 1, axis 0.
  e = launch_contract(p->acc, cplx, p->wneg, p->t1, 0, nfi * nfi, nfi, N, 1, s);
  if (e == hipSuccess) e = launch_contract(p->t1, true, p->wneg, p->t2, 0, nfi, nfi, N, N, s);
  if (e == hipSuccess)
    e = launch_contract(p->t2, true, p->wneg, out, cplx ? (acc ? 3 : 0) : (acc ? 2 : 1), 1, nfi, N, N * N, s);
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "merge_adjoint: launch");
}

int spfel_weighted_residual(spfel_plan plan, const void *slices,
                            const void *images, const float *weights,
                            int64_t count, float scale, const float *scale_dev,
                            void *residual, double *loss, void *stream) {
  clear_error();
  Plan *p = reinterpret_cast<Plan *>(plan);
  if (!live(p)) return fail(SPFEL_ESTATE, "weighted_residual: not a live plan");
  if (count < 0) return fail(SPFEL_EINVAL, "weighted_residual: negative count");
  if (!residual && !loss) return fail(SPFEL_EINVAL, "weighted_residual: no output requested");
  if (count == 0) return SPFEL_OK;
  const bool cplx = p->domain == SPFEL_COMPLEX;
  if (!slices || !images) return fail(SPFEL_EINVAL, "weighted_residual: NULL input");
  const size_t a = cplx ? 8 : 4;
  if (!aligned(slices, a) || !aligned(images, a) || (residual && !aligned(residual, a)) ||
      (weights && !aligned(weights, 4)) || (loss && !aligned(loss, 8)) ||
      (scale_dev && !aligned(scale_dev, 4)))
    return fail(SPFEL_EINVAL, "weighted_residual: misaligned pointer");
  DeviceGuard g(p->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "weighted_residual: hipSetDevice");
  hipError_t e = launch_residual(cplx, slices, images, weights, count, scale, scale_dev, residual,
                                 p->partials, loss, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SPFEL_OK : hip_fail(e, "weighted_residual: launch");
}

}  // extern "C"
