// Error reporting, version and the volume handle of libfovol.
#include <cstdio>
#include <string>

#include "common.h"

namespace fv {

static thread_local std::string g_err;

fv_status fail(fv_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

void clear_error() { g_err.clear(); }

fv_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return FV_OK;
  return fail(FV_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Fills the padded copy: every destination element (including the apron)
// reads the clamped source voxel.  One thread per destination element.
template <typename T>
__global__ void __launch_bounds__(256) k_pad_copy(const T* __restrict__ src, T* __restrict__ dst,
                                                  int nx, int ny, int nz, int64_t px, int64_t py,
                                                  int64_t total) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int64_t i = e % px, r = e / px;
  int64_t j = r % py, k = r / py;
  int64_t si = min(max(i - 2, (int64_t)0), (int64_t)nx - 1);
  int64_t sj = min(max(j - 2, (int64_t)0), (int64_t)ny - 1);
  int64_t sk = min(max(k - 2, (int64_t)0), (int64_t)nz - 1);
  dst[e] = src[(sk * ny + sj) * nx + si];
}

}  // namespace fv

extern "C" {

const char* fv_last_error(void) { return fv::g_err.c_str(); }

int fv_abi_version(void) { return FV_ABI_VERSION; }

fv_status fv_volume_create(const void* dev_data, int nx, int ny, int nz, fv_dtype dt,
                           void* stream, fv_volume** out) {
  fv::clear_error();
  if (!dev_data || !out) return fv::fail(FV_ERR_INVALID_ARG, "fv_volume_create: null pointer");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_volume_create: dims %d x %d x %d outside [1, 4096]",
                    nx, ny, nz);
  if (dt != FV_U8 && dt != FV_F16 && dt != FV_F32)
    return fv::fail(FV_ERR_UNSUPPORTED, "fv_volume_create: unknown dtype %d", (int)dt);
  fv_volume* v = new fv_volume();
  v->n[0] = nx;
  v->n[1] = ny;
  v->n[2] = nz;
  v->dt = dt;
  v->px = nx + 4;
  v->py = ny + 4;
  v->pz = nz + 4;
  if (hipGetDevice(&v->device) != hipSuccess) {
    delete v;
    return fv::fail(FV_ERR_DEVICE, "fv_volume_create: hipGetDevice failed");
  }
  int64_t total = v->px * v->py * v->pz;
  size_t bytes = (size_t)total * fv::dtype_bytes(dt);
  if (bytes >= ((size_t)1 << 32) - 1) {
    delete v;
    return fv::fail(FV_ERR_UNSUPPORTED,
                    "fv_volume_create: the padded copy must be < 4 GiB "
                    "((nx+4)(ny+4)(nz+4) x bytes per voxel)");
  }
  if (hipMalloc(&v->data, bytes) != hipSuccess) {
    delete v;
    return fv::fail(FV_ERR_NOMEM, "fv_volume_create: cannot allocate %zu bytes", bytes);
  }
  hipStream_t s = (hipStream_t)stream;
  unsigned grid = (unsigned)((total + 255) / 256);
  switch (dt) {
    case FV_U8:
      fv::k_pad_copy<uint8_t><<<grid, 256, 0, s>>>((const uint8_t*)dev_data, (uint8_t*)v->data,
                                                    nx, ny, nz, v->px, v->py, total);
      break;
    case FV_F16:
      fv::k_pad_copy<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)dev_data,
                                                     (uint16_t*)v->data, nx, ny, nz, v->px,
                                                     v->py, total);
      break;
    default:
      fv::k_pad_copy<float><<<grid, 256, 0, s>>>((const float*)dev_data, (float*)v->data, nx, ny,
                                                  nz, v->px, v->py, total);
  }
  fv_status st = fv::launch_status("fv_volume_create: copy kernel");
  if (st == FV_OK) st = fv::hip_status(hipStreamSynchronize(s), "fv_volume_create: sync");
  if (st != FV_OK) {
    (void)hipFree(v->data);
    delete v;
    return st;
  }
  *out = v;
  return FV_OK;
}

fv_status fv_volume_destroy(fv_volume* v) {
  fv::clear_error();
  if (!v) return FV_OK;
  fv_status st = FV_OK;
  if (v->data) st = fv::hip_status(hipFree(v->data), "fv_volume_destroy: hipFree");
  delete v;
  return st;
}

}  // extern "C"
