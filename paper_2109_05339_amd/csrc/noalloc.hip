// spfel_match_noalloc: spfel_match with its workspace in a file-scope device
// array instead of a caller-provided buffer, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
//
// Each GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never passes the array's name to a kernel (on
// the host it is a stand-in, not a device address): the device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept in scratch_ptr[device].
#include <mutex>

#include "internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[SPFEL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void *scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_of(int device, void **out) {
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[device] = p;
  }
  *out = scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

int spfel_match_noalloc(const void *slices, const float *slice_norm2, const void *images,
                        const float *image_norm2, int64_t M, int64_t n_img, int64_t P,
                        int64_t m_offset, int mode, const float *slices_f32,
                        const float *images_f32, const float *slice_err, const float *image_err,
                        int32_t *best_idx, float *best_dist, int32_t *flags, void *stream) {
  spfel::clear_error();
  if (M < 0 || n_img < 0 || P < 0) return spfel::fail(SPFEL_EINVAL, "match_noalloc: negative size");
  const size_t need = spfel_match_workspace_bytes(M, n_img, P, mode);
  if (need > (size_t)SPFEL_NOALLOC_SCRATCH_BYTES)
    return spfel::fail(SPFEL_ERANGE, "match_noalloc: these sizes need " + std::to_string(need) +
                                         " bytes of workspace, more than the " +
                                         std::to_string((size_t)SPFEL_NOALLOC_SCRATCH_BYTES) +
                                         "-byte scratch array; use spfel_match");
  if (M == 0 || n_img == 0) return SPFEL_OK;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return spfel::hip_fail(e, "match_noalloc: hipGetDevice");
  if (device < 0 || device >= kMaxDevices)
    return spfel::fail(SPFEL_ERANGE, "match_noalloc: device index beyond the supported 64");
  void *ws = nullptr;
  e = scratch_of(device, &ws);
  if (e != hipSuccess) return spfel::hip_fail(e, "match_noalloc: hipGetSymbolAddress");
  return spfel_match(slices, slice_norm2, images, image_norm2, M, n_img, P, m_offset, mode,
                     slices_f32, images_f32, slice_err, image_err, best_idx, best_dist, flags, ws,
                     (size_t)SPFEL_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
