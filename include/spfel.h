/*
 * spfel.h - C ABI of the MI355X slice-and-match library.
 *
 * The operations are those of the Cartesian-NUFFT M-TIP reconstruction of
 * SpiniFEL (arXiv 2109.05339):
 *   - slicing (section II-A): M model images on a fixed set of orientations,
 *     the type-2 (uniform -> nonuniform) NUFFT of the model coefficients at
 *     the detector's Ewald-sphere points rotated by each orientation;
 *   - orientation matching (section II-B): every experimental image against
 *     every model image in Euclidean distance, O(MN), nearest model wins;
 *   - merging (section II-C, Eq. (1)-(2)): the type-1 NUFFT A* of the
 *     (weighted) oriented data, the right-hand side A* D b of Eq. (2) and the
 *     adjoint of slicing.
 *
 * Conventions shared by every call
 *   Model: N odd, h = (N-1)/2, array model[i0][i1][i2] (C order, i2 fastest)
 *     holds mode k = (i0-h, i1-h, i2-h).  REAL domain: float32 coefficients,
 *     slice value s(x) = sum_k m_k cos(k.x).  COMPLEX domain: interleaved
 *     complex64 (re, im), s(x) = sum_k m_k exp(+i k.x).
 *   Points: x = R(q) q_p in radians per voxel; R(q) is the rotation of the
 *     unit quaternion q = (w, x, y, z) (Hamilton convention; the library
 *     renormalises, so q and -q give the same slice).  det_q is P x 3 float32.
 *     s is 2 pi periodic in each coordinate of x.
 *   NUFFT: exponential-of-semicircle kernel psi(tau) = exp(beta(sqrt(1 -
 *     (2 tau / w)^2) - 1)) of width w cells, beta = beta_over_w * w,
 *     fine grid n_f = 2N per axis, support cells t - w/2 <= l < t + w/2 with
 *     t = x n_f / (2 pi).
 *   Memory: every pointer argument is a device pointer on the plan's device
 *     (or on the current device for plan-less calls), owned by the caller,
 *     4-byte aligned (8-byte for complex64, 16-byte preferred).
 *   Streams: `stream` is a hipStream_t (NULL = default stream).  Every call
 *     only enqueues work on it and returns; nothing synchronises the device.
 *     Calls on one plan share its device buffers (fine grid, accumulator,
 *     rotation table): work they enqueue on different streams must not
 *     overlap.
 *   Errors: every call returns an spfel_status; on failure nothing has been
 *     enqueued (validation runs before any launch) unless the status is
 *     SPFEL_EHIP, and spfel_last_error() describes the failure.  No C++
 *     exception crosses this boundary; a plan stays usable after any error.
 */
#ifndef SPFEL_H
#define SPFEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spfel_plan_s *spfel_plan;
typedef struct spfel_normal_s *spfel_normal;
typedef struct spfel_phase_s *spfel_phase;

typedef enum {
  SPFEL_OK = 0,
  SPFEL_EINVAL = -1,        /* invalid argument (null, size, alignment) */
  SPFEL_ERANGE = -2,        /* size beyond what the library supports */
  SPFEL_ENOMEM = -3,        /* device allocation failed */
  SPFEL_EHIP = -4,          /* a HIP call or kernel launch failed */
  SPFEL_ESTATE = -5,        /* destroyed plan, or model not set */
  SPFEL_EUNSUPPORTED = -6   /* valid but unsupported parameter combination */
} spfel_status;

enum { SPFEL_REAL = 0, SPFEL_COMPLEX = 1 };
enum { SPFEL_F32 = 0, SPFEL_BF16 = 1 };
enum { SPFEL_MATCH_FP32 = 0, SPFEL_MATCH_BF16_RESCORE8 = 1 };
enum { SPFEL_MERGE_ACCUMULATE = 1, SPFEL_MERGE_DEFER = 2 };
enum { SPFEL_PHASE_ER = 0, SPFEL_PHASE_HIO = 1 };

/* Library version (major * 10000 + minor * 100 + patch). */
int spfel_version(void);

/* Description of the last failure on the calling thread ("" if none).
 * Valid until the next spfel call on that thread. */
const char *spfel_last_error(void);

/* Create a plan for model size n_model (odd, >= 3) on HIP device `device`.
 * kernel_width w in 4..8 and w <= n_model; upsampfac must be 2.0 (fine grid
 * n_f = 2N); beta_over_w in (0, 10] (2.30 is the usual value at upsampling
 * 2); domain SPFEL_REAL or SPFEL_COMPLEX.  All device memory the plan needs
 * (fine grid, transform tables, spreading accumulator, intermediates) is
 * allocated here; later calls allocate nothing.  *out receives the handle. */
int spfel_plan_create(spfel_plan *out, int n_model, int kernel_width,
                      double upsampfac, double beta_over_w, int domain,
                      int device);

/* Release a plan and its device memory.  Work still queued on a stream that
 * uses the plan must have completed.  A destroyed handle is rejected with
 * SPFEL_ESTATE by every later call. */
int spfel_plan_destroy(spfel_plan plan);

/* Plan facts: fine-grid size per axis and device bytes held (either pointer
 * may be NULL). */
int spfel_plan_info(spfel_plan plan, int *n_fine, size_t *device_bytes);

/* Register the detector template (section II-A: the model images are
 * computed on a predetermined geometry; section IV-A: one flat detector).
 * det_q: P x 3 float32 device points.  The plan keeps a copy sorted along a
 * Hilbert curve on the points' principal plane, so runs of 256 consecutive
 * points are compact patches,
 * and spfel_slice / spfel_merge_adjoint called with det_q = NULL (and the
 * same P) use it: each (orientation, patch) then stages its fine-grid brick
 * in LDS.  Outputs stay in the caller's pixel order.  This call copies the
 * points to the host (it synchronises `stream`) and allocates device memory;
 * it replaces any earlier registration, including the binned merge's
 * staging (two sets of up to 2^27 points, 20 or 24 bytes each). */
int spfel_set_detector(spfel_plan plan, const float *det_q, int64_t P,
                       void *stream);

/* Section II-A, the model-side half of the type-2 NUFFT: deconvolve the
 * model by the kernel's Fourier transform, zero-pad to n_f^3 and transform
 * to the oversampled grid the interpolation reads.  `model` is N^3 float32
 * (REAL) or complex64 (COMPLEX).  The plan keeps the grid until the next
 * set_model; `model` may be reused as soon as the stream reaches this call. */
int spfel_set_model(spfel_plan plan, const void *model, void *stream);

/* Section II-A: slice the model at M orientations.  quats: M x 4 float32;
 * det_q: P x 3 float32, or NULL for the registered detector (P must then
 * equal the registered size).  Outputs (either may be NULL, not both):
 *   out       M x P row-major, float32 (REAL) or complex64 (COMPLEX);
 *   out_norm2 M float32 squared norms |s_m|^2 (sum of |s|^2 over P; needs
 *             out).
 * Requires spfel_set_model.  M = 0 or P = 0 is valid (norms become 0). */
int spfel_slice(spfel_plan plan, const float *quats, int64_t M,
                const float *det_q, int64_t P, void *out, float *out_norm2,
                void *stream);

/* Squared row norms of a rows x cols matrix, float32 (dtype SPFEL_F32) or
 * bfloat16 values (SPFEL_BF16), accumulated in float32 in a fixed order
 * (each row: 256 strided partial sums, then a pairwise tree). */
int spfel_row_norm2(const void *x, int dtype, int64_t rows, int64_t cols,
                    float *out, void *stream);

/* Per-pixel centre for the BF16 matcher: out[p] = the mean over the rows
 * of x[r][p] (x: rows x cols float32; float32 sums in a fixed order), rounded
 * to the nearest integer (ties to even) when round_to_integer is nonzero,
 * so that centred photon counts stay integers.  rows >= 1. */
int spfel_column_mean(const float *x, int64_t rows, int64_t cols,
                      int round_to_integer, float *out, void *stream);

/* Operands of the BF16 matcher (section II-B, precision form).  For each
 * row r of x (rows x cols float32) and the per-pixel centre c (cols float32,
 * or NULL for zero):
 *   out[r][p] = bf16(x[r][p] - c[p])  (float32 subtraction, then round to
 *               nearest even);
 *   norm2[r]  = sum_p out[r][p]^2, float32 in a fixed order (may be NULL);
 *   err[r]    >= |out_r - (x_r - c)| with x - c exact: an upper bound on
 *               the row's rounding-error norm (may be NULL).
 * Subtracting one centre from model images and images leaves every distance
 * unchanged; it removes the intensity they share, so the BF16 values carry
 * the part that tells orientations apart. */
int spfel_bf16_centred(const float *x, int64_t rows, int64_t cols,
                       const float *centre, uint16_t *out, float *norm2,
                       float *err, void *stream);

/* Per-pixel weights of the distance (section II-C: the weights D of Eq. (2);
 * a beam stop's missing detector centre is weight 0): out[r][p] =
 * x[r][p] * g[p] for rows x cols float32 x and g[p] = sqrt(w_p).  Matching
 * rows scaled this way (model images and images alike) gives the weighted
 * distance sum_p w_p (s_p - d_p)^2 in every matcher mode.  out may equal x. */
int spfel_scale_columns(const float *x, int64_t rows, int64_t cols,
                        const float *g, float *out, void *stream);

/* Bytes of device workspace spfel_match needs for these sizes and mode. */
size_t spfel_match_workspace_bytes(int64_t M, int64_t n_img, int64_t P,
                                   int mode);

/* Section II-B: for each image n, the model image m minimising the
 * Euclidean distance D[m, n] = |s_m - d_n|^2 (lowest m on ties), merged into
 * the caller's running best: best_idx/best_dist (n_img each) are read and
 * updated, so chunks of model images can be streamed with m_offset = index
 * of the chunk's first model image.  Initialise best_idx = -1 and
 * best_dist = +inf.
 *   mode SPFEL_MATCH_FP32: slices/images float32 M x P / n_img x P;
 *     slice_norm2/image_norm2 their float32 squared norms
 *     (spfel_row_norm2); D = |s|^2 + |d|^2 - 2 s.d in float32, each a chain
 *     of at most 36 + ceil(P/32) roundings.  slices_f32, images_f32,
 *     slice_err, image_err and flags are ignored.
 *   mode SPFEL_MATCH_BF16_RESCORE8: slices/images are the bfloat16 centred
 *     rows of spfel_bf16_centred (one centre for both), slice_norm2/
 *     image_norm2 and slice_err/image_err its norm2 and err outputs;
 *     slices_f32/images_f32 the float32 rows themselves (uncentred).  The
 *     BF16 products accumulate in float32 into the proxy b = |s^ - d^|^2 of
 *     the rounded rows, and each image keeps the 8 smallest proxies.  Every
 *     candidate whose bound |sqrt(D) - sqrt(b)| <= e_m + f_n (widened by the
 *     proxy's float32 accumulation bound) leaves it able to beat the running
 *     best is rescored in float32 as a direct sum of (s_p - d_p)^2 (a chain
 *     of at most P/64 + 16 roundings).  The image is certified when every
 *     model image outside the 8 is bounded away from the running best;
 *     otherwise it is rescored against all M model images in float32 the
 *     same way and flags[n] |= 1 (flags: n_img int32 or NULL).  best_dist
 *     holds the float32 direct sum.
 * workspace: at least spfel_match_workspace_bytes bytes, 256-byte aligned. */
int spfel_match(const void *slices, const float *slice_norm2,
                const void *images, const float *image_norm2, int64_t M,
                int64_t n_img, int64_t P, int64_t m_offset, int mode,
                const float *slices_f32, const float *images_f32,
                const float *slice_err, const float *image_err,
                int32_t *best_idx, float *best_dist, int32_t *flags,
                void *workspace, size_t workspace_bytes, void *stream);

/* Size of the per-device scratch array spfel_match_noalloc uses. */
#define SPFEL_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as spfel_match, without the workspace
 * arguments.  The workspace lives in a 64 MiB array each GPU holds from the
 * library's first call on it until the process ends; sizes whose
 * spfel_match_workspace_bytes exceeds SPFEL_NOALLOC_SCRATCH_BYTES are
 * rejected with SPFEL_ERANGE.  The call allocates nothing.  Every call on
 * one GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other threads) race; calls queued on one stream do not.  Runs on
 * the current device. */
int spfel_match_noalloc(const void *slices, const float *slice_norm2,
                        const void *images, const float *image_norm2,
                        int64_t M, int64_t n_img, int64_t P, int64_t m_offset,
                        int mode, const float *slices_f32,
                        const float *images_f32, const float *slice_err,
                        const float *image_err, int32_t *best_idx,
                        float *best_dist, int32_t *flags, void *stream);

/* Bytes of workspace spfel_orient needs for this chunk length. */
size_t spfel_orient_workspace_bytes(int64_t chunk, int64_t n_img, int64_t P,
                                    int mode);

/* Sections II-A and II-B as one pipeline: slice the M model orientations in
 * chunks of `chunk` and match every image against each chunk, folding into
 * the running best (best_idx/best_dist, initialised by the caller as for
 * spfel_match).  Each chunk's slices are computed on `aux_stream` into one of
 * two workspace buffers while the previous chunk is matched on `stream`; the
 * model slices are never stored in full.  The result equals spfel_slice of
 * each chunk (and, in BF16 mode, spfel_bf16_centred of it with `centre`)
 * followed by spfel_match with m_offset = chunk start; pixel_scale (P
 * float32 or NULL) scales each chunk's columns as spfel_scale_columns before
 * the norms and the centring, for weighted distances (the images must be
 * scaled the same way by the caller).  REAL plans only;
 * requires spfel_set_model.  FP32 mode: images n_img x P float32 with their
 * norms; centre, images_f32, image_err and flags ignored.  BF16 mode: images,
 * image_norm2, image_err from spfel_bf16_centred of images_f32 with
 * `centre`, flags as in spfel_match.  Work queued on `stream` before the
 * call is complete before any slice starts; every result is ordered before
 * work later queued on `stream`.  `aux_stream` may equal `stream` (no
 * overlap).  workspace: spfel_orient_workspace_bytes, 256-byte aligned;
 * calls that overlap on the same plan race. */
int spfel_orient(spfel_plan plan, const float *quats, int64_t M,
                 const float *det_q, int64_t P, const float *pixel_scale,
                 const void *images, const float *image_norm2,
                 const float *images_f32, const float *image_err,
                 const float *centre, int64_t n_img, int mode, int64_t chunk,
                 int32_t *best_idx, float *best_dist, int32_t *flags,
                 void *workspace, size_t workspace_bytes, void *stream,
                 void *aux_stream);

/* Section II-C, Eq. (2) right-hand side: the type-1 NUFFT (adjoint of
 * slicing) of values at the points R(quats[n]) det_q[p] (det_q NULL: the
 * registered detector, values still in the caller's pixel order):
 *   REAL:    out_k = sum_{n,p} y_np cos(k . x_np)
 *   COMPLEX: out_k = sum_{n,p} y_np exp(-i k . x_np)
 * with y = values (n_img x P, float32 or complex64) times weights (n_img x P
 * float32, or NULL for 1).  out is N^3 float32 / complex64.  flags:
 *   SPFEL_MERGE_ACCUMULATE  out += result instead of out = result;
 *   SPFEL_MERGE_DEFER       only spread into the plan's accumulator; the
 *                           next call without DEFER finishes the sum of all
 *                           deferred calls and writes out (out may be NULL
 *                           with DEFER).
 * Spreading uses float32 atomics, so the summation order (and the last bits
 * of the result) can vary between runs.  With the registered detector the
 * points are binned in batches of up to 2^27 on a stream the plan owns
 * (ordered after the work already on `stream`, and before the work queued
 * on `stream` after this call) while the previous batch spreads on
 * `stream`. */
int spfel_merge_adjoint(spfel_plan plan, const float *quats, int64_t n_img,
                        const float *det_q, int64_t P, const void *values,
                        const float *weights, void *out, int flags,
                        void *stream);

/* Weighted residual of slices against images (the gradient's spread input
 * for the weighted loss of Eq. (2)'s D-weighted least squares):
 *   residual[i] = scale * (*scale_dev) * w_i * (s_i - d_i)   (may be NULL)
 *   *loss += sum_i w_i |s_i - d_i|^2                         (may be NULL)
 * over `count` elements (float32 or complex64 per the plan's domain;
 * weights NULL means 1; scale_dev a device float32 scalar or NULL for 1, so
 * a factor computed on the device needs no host round trip).  The loss is a
 * device float64 scalar accumulated in float64 in a fixed order. */
int spfel_weighted_residual(spfel_plan plan, const void *slices,
                            const void *images, const float *weights,
                            int64_t count, float scale, const float *scale_dev,
                            void *residual, double *loss, void *stream);

/* ---- Regularised merging: the normal equations of Eq. (2) ----
 * Section II-C: the autocorrelation solves
 *     (A* D A + lambda I) x = A* D b + lambda x0,
 * with A the type-2 operator of the plan's convention (REAL: cos, COMPLEX:
 * exp(+i k.x)), D the per-point weights, x0 the initial guess.  A* D A is a
 * convolution on the mode grid (the Toeplitz method): its (k, k') entry is
 * T[k - k'] with T the type-1 transform of the weights on (2N - 1)^3 modes,
 *   COMPLEX: T[m] = sum_j d_j exp(-i m.x_j),
 *   REAL:    C[m] = sum_j d_j cos(m.x_j), and A^T D A x = C * even(x),
 *            even(x)[k] = (x[k] + x[-k]) / 2 (the cos operator only sees the
 *            even part of x).
 * Both are spfel_merge_adjoint of the weights (values 1, weights d) on a
 * plan with n_model = 2N - 1 and the same points; A* D b is
 * spfel_merge_adjoint of b with weights d on the size-N plan.  One
 * application is three DFT contractions to L = 2N cells per axis (the
 * circular convolution then equals the linear one), a pointwise product with
 * the transformed kernel and three contractions back; conjugate gradients
 * solve up to 16 systems (one per lambda) at once, sharing every launch.
 *
 * An spfel_normal object holds the DFT tables, the transformed kernel and
 * the CG vectors for up to max_systems systems (all allocated at create;
 * later calls allocate nothing).  Vectors are N^3 float32 (REAL) or complex64
 * (COMPLEX) in the model layout; a batch of n systems is n consecutive
 * vectors.  Calls on one object share its buffers: work on different
 * streams must not overlap.  Calculations are float32; the step sizes of CG
 * stay on the device (no host synchronisation). */

/* n_model odd in 3..511, domain SPFEL_REAL or SPFEL_COMPLEX, max_systems
 * 1..16, on HIP device `device`.  SPFEL_ENOMEM if the buffers (about
 * 8 (2N)^3 (max_systems + 1) bytes) do not fit. */
int spfel_normal_create(spfel_normal *out, int n_model, int domain,
                        int max_systems, int device);

/* Release the object (queued work that uses it must have completed). */
int spfel_normal_destroy(spfel_normal nm);

/* Set the Toeplitz kernel: psf is (2N - 1)^3 float32 (REAL: C) or complex64
 * (COMPLEX: T), index (m0 + N - 1, m1 + N - 1, m2 + N - 1) for mode m.
 * psf may be reused as soon as the stream reaches this call. */
int spfel_normal_set_psf(spfel_normal nm, const void *psf, void *stream);

/* y[s] = A* D A x[s] + lambdas[s] x[s] for s < n (n <= max_systems);
 * lambdas: n host floats, finite and >= 0.  x and y are n vectors each and
 * must not overlap. */
int spfel_normal_apply(spfel_normal nm, const void *x, int n,
                       const float *lambdas, void *y, void *stream);

/* `iters` CG steps on system s: (A* D A + lambdas[s]) x = rhs + lambdas[s]
 * x0, started at x = x0, for s < n.  rhs = A* D b and x0 are one vector
 * each (shared by all systems); x_out receives n vectors.  residuals (n x
 * (iters + 1) device floats, or NULL) receives |r_i| per system and step
 * (i = 0 is the starting residual).  A system whose residual reaches 0 stops
 * moving. */
int spfel_normal_solve(spfel_normal nm, const void *rhs, const void *x0,
                       int n, const float *lambdas, int iters, void *x_out,
                       float *residuals, void *stream);

/* The L-curve over the n solutions x (as written by spfel_normal_solve for
 * the same lambdas, which must be uniformly spaced in log lambda):
 *   rho_s = |D^(1/2) (A x_s - b)|^2 = x_s.(A* D A x_s) - 2 Re x_s.rhs + bdb,
 *   eta_s = |x_s - x0|^2,
 * with bdb = b* D b given by the caller; rho_eta (2n device floats) receives
 * (rho_s, eta_s).  corner (device int32, or NULL) receives the index of the
 * largest curvature of (log rho, log eta) as functions of log lambda (central
 * differences, end points excluded; 0 when n < 3).  With n >= 3 every
 * lambda must be > 0. */
int spfel_normal_lcurve(spfel_normal nm, const void *x, const void *rhs,
                        const void *x0, int n, const float *lambdas,
                        double bdb, float *rho_eta, int32_t *corner,
                        void *stream);

/* ---- Phasing (section II-D) ----
 * The density rho (real, N^3 float32, C order) and its 3D DFT
 * F[k] = sum_r rho[r] exp(-2 pi i k.r / N) (numpy's convention and standard
 * index order for k) are driven between the real-space constraints and the
 * measured amplitudes:
 *   reciprocal space: where measured[k] (all k if measured is NULL),
 *     F[k] <- amp[k] F[k] / |F[k]| (amp[k] where F[k] = 0); elsewhere F[k]
 *     is kept; rho' = Re IFFT(F);
 *   real space: where the constraint holds (support[r] != 0, and rho'[r]
 *     >= 0 when positivity is set) rho <- rho'; elsewhere rho <- 0 (error
 *     reduction, ER) or rho - beta rho' (hybrid input-output, HIO);
 *   error of an iteration: sum over measured k of (|F| - amp)^2 / sum of
 *     amp^2, from the transform of the iterate the iteration starts from.
 * Shrinkwrap replaces the support by the cells where the periodic Gaussian
 * blur (standard deviation sigma cells, unit sum, separable circular
 * convolution) of |rho| reaches tau times its maximum.
 * The transforms are separable DFT contractions (float32).  An spfel_phase
 * object holds the tables and intermediates for one N (about 28 N^3 bytes,
 * allocated at create; later calls allocate nothing); calls on one object
 * share them, so work on different streams must not overlap. */

/* n in 2..1024 cells per axis, on HIP device `device`. */
int spfel_phase_create(spfel_phase *out, int n, int device);

/* Release the object (queued work that uses it must have completed). */
int spfel_phase_destroy(spfel_phase ph);

/* n_iter iterations of mode SPFEL_PHASE_ER or SPFEL_PHASE_HIO (beta used by
 * HIO) on rho in place.  amp: N^3 float32 amplitudes; measured, support:
 * N^3 bytes (0 / nonzero; measured may be NULL); err: n_iter device
 * floats or NULL, receives each iteration's error. */
int spfel_phase_iterate(spfel_phase ph, float *rho, const float *amp,
                        const uint8_t *measured, const uint8_t *support,
                        int n_iter, int mode, float beta, int positivity,
                        float *err, void *stream);

/* Shrinkwrap: support (N^3 bytes) <- blur(|rho|, sigma) >= tau max, sigma
 * > 0, tau in [0, 1]; blurred (N^3 float32, or NULL) receives the blurred
 * |rho|. */
int spfel_phase_shrinkwrap(spfel_phase ph, const float *rho, float sigma,
                           float tau, uint8_t *support, float *blurred,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPFEL_H */
