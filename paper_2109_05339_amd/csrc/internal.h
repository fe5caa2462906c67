// Internal declarations of libspfel: the plan, status plumbing and the
// host-side launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "spfel.h"

namespace spfel {

// A plan owns everything slicing and merging need for one model size.
struct Plan {
  int device = 0;
  int N = 0;          // model modes per axis (odd)
  int nf = 0;         // fine grid cells per axis (2N)
  int w = 0;          // kernel width in cells
  int domain = SPFEL_REAL;
  double beta = 0.0;  // kernel shape
  // Fine grid the interpolation reads: nf^3 float (REAL) or float2
  // (COMPLEX), centred storage: cell l at index (l + nf/2) mod nf per axis.
  void *u = nullptr;
  // Separable transform tables, float2, row-major [L][K] for a contraction
  // over L producing K:
  //   wpos [N][nf]: exp(+2 pi i k (l - nf/2) / nf) / psi_hat(k)  (model -> centred grid)
  //   wneg [nf][N]: exp(-2 pi i k l / nf) / psi_hat(k)   (grid -> modes)
  float2 *wpos = nullptr;
  float2 *wneg = nullptr;
  // Intermediates of the separable transforms, 4 N^3 float2 each.
  float2 *t1 = nullptr;
  float2 *t2 = nullptr;
  // Spreading accumulator: nf^3 float (REAL) or float2 (COMPLEX).
  void *acc = nullptr;
  // Per-block partial sums of the weighted-residual loss.
  double *partials = nullptr;
  // Scaled rotations of up to kRotCap orientations of one slicing launch:
  // rot[9 m + 3 d + e] = R(q_m)[d][e] n_f / (2 pi), float64.
  double *rot = nullptr;
  // Registered detector template (spfel_set_detector): points sorted along
  // a Hilbert curve on their principal plane so that every run of kTile
  // consecutive points is a compact patch; det_perm maps a sorted position
  // to the caller's pixel.
  float *det_sorted = nullptr;   // det_P x 3
  int32_t *det_perm = nullptr;   // det_P
  int64_t det_P = 0;
  // Binned spreading over the registered detector (allocated with it):
  // points of up to bin_batch images at a time, grouped by the fine-grid
  // bin of their support origin and their axis-1 origin (the key).  Two
  // sets of what the spread reads: batch b + 1 is binned into one while
  // batch b spreads from the other.
  float4 *bin_pts[2] = {nullptr, nullptr};    // bin_cap: value (re), three kernel offsets
  uint2 *bin_aux[2] = {nullptr, nullptr};     // bin_cap: packed origin in the brick, value (im) bits
  int32_t *bin_off[2] = {nullptr, nullptr};   // keys + 1: counts, then exclusive offsets
  int32_t *bin_cur = nullptr;                 // keys: scatter cursors
  int32_t *bin_part = nullptr;                // scan block totals
  int4 *bin_sub[2] = {nullptr, nullptr};      // subproblems (bin, first point, end)
  int32_t *bin_nsub[2] = {nullptr, nullptr};  // number of subproblems
  int64_t bin_cap = 0;           // points per batch
  int64_t bin_batch = 0;         // images per batch
  size_t bin_bytes = 0;
  bool model_set = false;
  bool pending = false;  // deferred spreads are waiting in acc
  size_t bytes = 0;
  // Events of the two-stream orientation pipeline (spfel_orient): the main
  // stream's start, each slice buffer's fill and release.
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_sliced[2] = {nullptr, nullptr};
  hipEvent_t ev_matched[2] = {nullptr, nullptr};
  // The binned merge's own stream (default priority) for the binning of
  // the next batch, and its events: the caller's stream at entry, each
  // buffer set binned, each buffer set spread.
  hipStream_t bin_stream = nullptr;
  hipEvent_t ev_bin_start = nullptr;
  hipEvent_t ev_binned[2] = {nullptr, nullptr};
  hipEvent_t ev_spread[2] = {nullptr, nullptr};
};

// Points per detector tile of the tiled slicing/spreading kernels.
constexpr int kTile = 256;
// Orientations per slicing launch (size of Plan::rot).
constexpr int64_t kRotCap = 65536;
// Binned spreading: brick side (cells), points per subproblem, points per
// batch of images (2^27: 3.2 GB of staged points; every batch flushes each
// occupied bin once, so larger batches flush less).
constexpr int kBrick = 16;
constexpr int kSubMax = 8192;
constexpr int64_t kBinBatchPoints = (int64_t)1 << 27;
size_t bin_keys(int nf, int w);
size_t bin_max_subproblems(int nf, int w, int64_t cap);

// Status helpers: set the thread-local message and return the code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
void clear_error();

// psi_hat(k) for k = -h..h (host, float64): Fourier transform of the kernel
// at mode k on a grid of nf cells.
void kernel_transform(int N, int nf, int w, double beta, double *out);

constexpr int kMaxPartials = 1024;

// ---- launchers (return hipSuccess or the launch error) ----
// Y[a][k][b] = sum_l X[a][l][b] W[l][k] (X float or float2 per x_complex);
// out_mode: 0 store float2, 1 store real part (float), 2 add real part,
// 3 add float2.
hipError_t launch_contract(const void *X, bool x_complex, const float2 *W,
                           void *Y, int out_mode, int A, int L, int K, int B,
                           hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

// detq == nullptr selects the plan's registered detector (tiled kernel).
hipError_t launch_interp(const Plan &pl, const float *quats, int64_t M,
                         const float *detq, int64_t P, void *out, hipStream_t s);
// rot[9 m + 3 d + e] = R(quats[m])[d][e] * scale (float64; NaN for a zero
// or non-finite quaternion), M <= kRotCap.
hipError_t launch_rotations(const float *quats, int64_t M, double scale, double *rot,
                            hipStream_t s);
hipError_t launch_row_norm2(const void *x, bool bf16, int64_t rows,
                            int64_t cols, float *out, hipStream_t s);

// detq == nullptr selects the plan's registered detector (binned spread).
hipError_t launch_spread(const Plan &pl, const float *quats, int64_t n_img,
                         const float *detq, int64_t P, const void *values,
                         const float *weights, hipStream_t s);
hipError_t launch_spread_binned(const Plan &pl, const float *quats, int64_t n_img,
                                int64_t P, const void *values, const float *weights,
                                hipStream_t s);

hipError_t launch_pack_keys(const int32_t *idx, const float *dist,
                            unsigned long long *keys, int64_t n,
                            hipStream_t s);
hipError_t launch_unpack_keys(const unsigned long long *keys, int32_t *idx,
                              float *dist, int64_t n, hipStream_t s);
// workspace: packed keys (N u64) first, then split-K counters and partial
// tiles when the launch splits K (match_f32_workspace_bytes).
int match_f32_splits(int64_t M, int64_t N, int64_t P);
size_t match_f32_workspace_bytes(int64_t M, int64_t N, int64_t P);
hipError_t launch_match_f32(const float *S, const float *D, const float *sn,
                            const float *dn, int64_t M, int64_t N, int64_t P,
                            int64_t m_offset, void *workspace, hipStream_t s);
// The candidate buffer holds 8 words per image per tile of tile_rows model
// images (128 or 256, match_bf16_tile_rows); its size is that of the
// 128-row tiling.
int match_bf16_tile_rows(int64_t M, int64_t N, int64_t P, const void *S, const void *D);
size_t match_bf16_candidate_bytes(int64_t M, int64_t N);
hipError_t launch_match_bf16(const uint16_t *S, const uint16_t *D,
                             const float *sn, const float *dn, int64_t M,
                             int64_t N, int64_t P, uint32_t *cand, hipStream_t s);
// Certified rescore and fallback of the BF16 matcher.  scratch:
// match_rescore_bytes(N) bytes, 256-byte aligned (chunk maxima, fallback
// count, list and keys).
size_t match_rescore_bytes(int64_t N);
hipError_t launch_rescore(const uint32_t *cand, int tile_rows, int64_t M, int64_t N,
                          int64_t P, int64_t m_offset, const float *S32,
                          const float *D32, const float *sn, const float *dn,
                          const float *se, const float *de, int32_t *best_idx,
                          float *best_dist, int32_t *flags, void *scratch,
                          hipStream_t s);
// Matcher operands (centre.hip).
hipError_t launch_column_mean(const float *x, int64_t rows, int64_t cols,
                              int round_int, float *out, hipStream_t s);
hipError_t launch_bf16_centred(const float *x, int64_t rows, int64_t cols,
                               const float *c, uint16_t *out, float *norm2,
                               float *err, hipStream_t s);
hipError_t launch_scale_columns(const float *x, int64_t rows, int64_t cols,
                                const float *g, float *out, hipStream_t s);

hipError_t launch_residual(bool cplx, const void *s, const void *d,
                           const float *w, int64_t count, float scale,
                           const float *scale_dev, void *r, double *partials,
                           double *loss, hipStream_t st);

}  // namespace spfel
