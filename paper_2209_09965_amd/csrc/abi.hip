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

// Fills the bricked copy: every destination element reads its clamped source
// voxel.  One thread per destination element.
template <typename T>
__global__ void __launch_bounds__(256) k_brick_copy(const T* __restrict__ src,
                                                    T* __restrict__ dst, int nx, int ny, int nz,
                                                    int nbx, int nby, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t b = e / kBrickVox;
  const int r = (int)(e - b * kBrickVox);
  const int sx = r % kBrickRow, sy = (r / kBrickRow) % kBrickRow, sz = r / (kBrickRow * kBrickRow);
  const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby), bz = (int)(b / ((int64_t)nbx * nby));
  const int64_t i = min(max(kBrick * bx - 2 + sx, 0), nx - 1);
  const int64_t j = min(max(kBrick * by - 2 + sy, 0), ny - 1);
  const int64_t k = min(max(kBrick * bz - 2 + sz, 0), nz - 1);
  dst[e] = src[(k * ny + j) * nx + i];
}

fv_status volume_create(const void* dev_data, int nx, int ny, int nz, fv_dtype dt, int brick,
                        void* stream, fv_volume** out, const char* fn) {
  clear_error();
  if (!dev_data || !out) return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
    return fail(FV_ERR_INVALID_ARG, "%s: dims %d x %d x %d outside [1, 4096]", fn, nx, ny, nz);
  if (dt != FV_U8 && dt != FV_F16 && dt != FV_F32)
    return fail(FV_ERR_UNSUPPORTED, "%s: unknown dtype %d", fn, (int)dt);
  fv_volume* v = new fv_volume();
  v->n[0] = nx;
  v->n[1] = ny;
  v->n[2] = nz;
  v->dt = dt;
  v->px = nx + 4;
  v->py = ny + 4;
  v->pz = nz + 4;
  v->brick = brick;
  for (int a = 0; a < 3; ++a) v->nb[a] = (v->n[a] + 1 + kBrick - 1) / kBrick;
  if (hipGetDevice(&v->device) != hipSuccess) {
    delete v;
    return fail(FV_ERR_DEVICE, "%s: hipGetDevice failed", fn);
  }
  const int64_t total = brick ? (int64_t)v->nb[0] * v->nb[1] * v->nb[2] * kBrickVox
                              : v->px * v->py * v->pz;
  const size_t bytes = (size_t)total * dtype_bytes(dt);
  if (bytes >= ((size_t)1 << 32) - 1) {
    delete v;
    return fail(FV_ERR_UNSUPPORTED, "%s: the volume copy must be < 4 GiB (%zu bytes)", fn, bytes);
  }
  v->bytes = bytes;
  if (hipMalloc(&v->data, bytes) != hipSuccess) {
    delete v;
    return fail(FV_ERR_NOMEM, "%s: cannot allocate %zu bytes", fn, bytes);
  }
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = (unsigned)((total + 255) / 256);
  auto launch = [&](auto tag) {
    using T = decltype(tag);
    if (brick)
      k_brick_copy<T><<<grid, 256, 0, s>>>((const T*)dev_data, (T*)v->data, nx, ny, nz,
                                           v->nb[0], v->nb[1], total);
    else
      k_pad_copy<T><<<grid, 256, 0, s>>>((const T*)dev_data, (T*)v->data, nx, ny, nz, v->px,
                                         v->py, total);
  };
  switch (dt) {
    case FV_U8:
      launch(uint8_t{});
      break;
    case FV_F16:
      launch(uint16_t{});
      break;
    default:
      launch(float{});
  }
  fv_status st = launch_status("volume copy kernel");
  if (st == FV_OK) st = hip_status(hipStreamSynchronize(s), "volume copy: sync");
  if (st != FV_OK) {
    (void)hipFree(v->data);
    delete v;
    return st;
  }
  *out = v;
  return FV_OK;
}

}  // namespace fv

extern "C" {

const char* fv_last_error(void) { return fv::g_err.c_str(); }

int fv_abi_version(void) { return FV_ABI_VERSION; }

fv_status fv_volume_create(const void* dev_data, int nx, int ny, int nz, fv_dtype dt,
                           void* stream, fv_volume** out) {
  return fv::volume_create(dev_data, nx, ny, nz, dt, 0, stream, out, "fv_volume_create");
}

fv_status fv_volume_create_bricked(const void* dev_data, int nx, int ny, int nz, fv_dtype dt,
                                   void* stream, fv_volume** out) {
  return fv::volume_create(dev_data, nx, ny, nz, dt, 1, stream, out, "fv_volume_create_bricked");
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
