// Reconstruction network state: checkpoint blobs (FP32 master weights, Adam
// moments and step), an externally supplied gradient, and the FP8 scales of
// a calibrated handle.
#include <cstring>
#include <vector>

#include "net.h"

namespace fv {
namespace net {

namespace {

// Checkpoint blob layout (little-endian, as written by fv_net_save).
struct BlobHeader {
  char magic[8];       // "FOVOLNET"
  uint32_t version;    // 1
  uint32_t recurrent;  // 0 plain form, 1 recurrent form
  uint64_t n_params;   // external parameter count of the form
  int64_t step;        // Adam steps taken
  uint8_t reserved[32];
};
static_assert(sizeof(BlobHeader) == 64, "blob header is 64 bytes");
constexpr char kMagic[8] = {'F', 'O', 'V', 'O', 'L', 'N', 'E', 'T'};
constexpr uint32_t kBlobVersion = 1;

size_t blob_bytes(int recurrent) {
  return sizeof(BlobHeader) + 3 * (size_t)external_param_count(recurrent) * sizeof(float);
}

// Gradient in the external layout of the handle's form -> internal layout.
// The plain form's first conv has 5 input channels outside the library and
// 8 inside (the last 3, the fed-back O_d of the recurrent form, carry zero
// weights): their gradient slots are zero.
__global__ void __launch_bounds__(256) k_grad_to_internal(const float* __restrict__ ext,
                                                          float* __restrict__ in, int64_t n,
                                                          int recurrent, int co0, int ci0,
                                                          int fed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (recurrent) {
    in[i] = ext[i];
    return;
  }
  const int64_t wi = (int64_t)co0 * ci0 * 9;   // internal first-conv weights
  const int ce = ci0 - fed;                     // external input channels
  if (i < wi) {
    const int o = (int)(i / (ci0 * 9)), r = (int)(i % (ci0 * 9));
    const int c = r / 9, t = r % 9;
    in[i] = c < ce ? ext[((int64_t)o * ce + c) * 9 + t] : 0.0f;
  } else {
    in[i] = ext[i - (int64_t)co0 * fed * 9];
  }
}

}  // namespace
}  // namespace net
}  // namespace fv

using namespace fv;
using namespace fv::net;

extern "C" {

fv_status fv_net_save(const fv_net* n, void* host_blob, size_t* bytes) {
  clear_error();
  if (!n || !bytes) return fail(FV_ERR_INVALID_ARG, "fv_net_save: null pointer");
  const size_t need = blob_bytes(n->recurrent);
  if (!host_blob) {
    *bytes = need;
    return FV_OK;
  }
  if (*bytes < need)
    return fail(FV_ERR_CAPACITY, "fv_net_save: buffer of %zu bytes, the blob needs %zu", *bytes,
                need);
  const int64_t P = param_count(), E = external_param_count(n->recurrent);
  std::vector<float> internal((size_t)P);
  BlobHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, sizeof kMagic);
  h.version = kBlobVersion;
  h.recurrent = (uint32_t)n->recurrent;
  h.n_params = (uint64_t)E;
  h.step = n->step;
  uint8_t* out = (uint8_t*)host_blob;
  std::memcpy(out, &h, sizeof h);
  const float* src[3] = {n->master, n->adam_m, n->adam_v};
  for (int k = 0; k < 3; ++k) {
    fv_status st = hip_status(hipMemcpy(internal.data(), src[k], (size_t)P * sizeof(float),
                                        hipMemcpyDeviceToHost), "fv_net_save: read state");
    if (st != FV_OK) return st;
    params_to_external(internal.data(), n->recurrent,
                       (float*)(out + sizeof h + (size_t)k * E * sizeof(float)));
  }
  *bytes = need;
  return FV_OK;
}

fv_status fv_net_load(const void* host_blob, size_t bytes, fv_net** out) {
  clear_error();
  if (!host_blob || !out) return fail(FV_ERR_INVALID_ARG, "fv_net_load: null pointer");
  *out = nullptr;
  BlobHeader h;
  if (bytes < sizeof h) return fail(FV_ERR_INVALID_ARG, "fv_net_load: %zu bytes, no header", bytes);
  std::memcpy(&h, host_blob, sizeof h);
  if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0)
    return fail(FV_ERR_INVALID_ARG, "fv_net_load: not a network checkpoint");
  if (h.version != kBlobVersion)
    return fail(FV_ERR_UNSUPPORTED, "fv_net_load: blob version %u (this library reads %u)",
                h.version, kBlobVersion);
  if (h.recurrent > 1 || h.n_params != (uint64_t)external_param_count((int)h.recurrent))
    return fail(FV_ERR_INVALID_ARG, "fv_net_load: %llu parameters for form %u",
                (unsigned long long)h.n_params, h.recurrent);
  if (h.step < 0) return fail(FV_ERR_INVALID_ARG, "fv_net_load: negative step");
  if (bytes < blob_bytes((int)h.recurrent))
    return fail(FV_ERR_INVALID_ARG, "fv_net_load: %zu bytes, the blob needs %zu", bytes,
                blob_bytes((int)h.recurrent));
  const uint8_t* in = (const uint8_t*)host_blob + sizeof h;
  const int64_t E = (int64_t)h.n_params, P = param_count();
  // the blob is not necessarily float-aligned: copy each section out
  std::vector<float> ext((size_t)E), internal((size_t)P);
  std::memcpy(ext.data(), in, (size_t)E * sizeof(float));
  fv_net* n = nullptr;
  fv_status st = fv_net_create(ext.data(), (size_t)E, &n);
  if (st != FV_OK) return st;
  float* dst[2] = {n->adam_m, n->adam_v};
  for (int k = 0; k < 2 && st == FV_OK; ++k) {
    std::memcpy(ext.data(), in + (size_t)(k + 1) * E * sizeof(float), (size_t)E * sizeof(float));
    params_to_internal(ext.data(), n->recurrent, internal.data());
    st = hip_status(hipMemcpy(dst[k], internal.data(), (size_t)P * sizeof(float),
                              hipMemcpyHostToDevice), "fv_net_load: upload Adam state");
  }
  if (st != FV_OK) {
    fv_net_destroy(n);
    return st;
  }
  n->step = h.step;
  *out = n;
  return FV_OK;
}

fv_status fv_net_set_grad(fv_net* n, const float* grad, size_t n_params, void* stream) {
  clear_error();
  if (!n || !grad) return fail(FV_ERR_INVALID_ARG, "fv_net_set_grad: null pointer");
  if (n_params != (size_t)external_param_count(n->recurrent))
    return fail(FV_ERR_INVALID_ARG, "fv_net_set_grad: size %zu, the network has %lld", n_params,
                (long long)external_param_count(n->recurrent));
  const int64_t P = param_count();
  k_grad_to_internal<<<(unsigned)((P + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      grad, n->grad, P, n->recurrent, kLayers[0].co, kLayers[0].ci, kFedBack);
  return launch_status("fv_net_set_grad");
}

fv_status fv_net_fp8_scales(const fv_net* n, float* host_scales, int count) {
  clear_error();
  if (!n || !host_scales) return fail(FV_ERR_INVALID_ARG, "fv_net_fp8_scales: null pointer");
  if (count != FV_NET_FP8_TENSORS)
    return fail(FV_ERR_INVALID_ARG, "fv_net_fp8_scales: count %d, expected %d", count,
                FV_NET_FP8_TENSORS);
  if (!n->fp8_ready)
    return fail(FV_ERR_INVALID_ARG, "fv_net_fp8_scales: the network is not calibrated");
  host_scales[0] = n->act_scale[T_IN];
  for (int l = 0; l < kNumConv; ++l) host_scales[1 + l] = n->act_scale[kLayerIO[l][2]];
  return FV_OK;
}

}  // extern "C"
