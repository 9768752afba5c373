// Internal helpers of libfovol (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>

#include "fovol.h"

namespace fv {

// Records a message for fv_last_error() on this thread and returns `s`.
fv_status fail(fv_status s, const char* fmt, ...);
// Clears the thread's error message (start of every entry point).
void clear_error();
// Maps a HIP error to FV_ERR_DEVICE with a message, FV_OK otherwise.
fv_status hip_status(hipError_t e, const char* what);
// Checks the launch that was just enqueued.
inline fv_status launch_status(const char* what) { return hip_status(hipGetLastError(), what); }

constexpr int kWave = 64;

// Voxel element conversion to float: u8 -> v/255, f16 and f32 as stored.
template <int DT> struct Voxel;
template <> struct Voxel<FV_U8> {
  using T = uint8_t;
  static __device__ __forceinline__ float f(T v) { return (float)v * (1.0f / 255.0f); }
};
template <> struct Voxel<FV_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float f(T v) { return (float)v; }
};
template <> struct Voxel<FV_F32> {
  using T = float;
  static __device__ __forceinline__ float f(T v) { return v; }
};

inline size_t dtype_bytes(fv_dtype d) { return d == FV_U8 ? 1 : d == FV_F16 ? 2 : 4; }

// Pull-push reconstruction (pullpush.hip), also reached through
// fv_reconstruct with FV_RECON_PULLPUSH.
size_t pullpush_workspace_bytes(int views, int W, int H);
fv_status pullpush_run(const float* frame_rgba, const uint8_t* mask, int views, int W, int H,
                       float* out_rgb, void* workspace, size_t ws_bytes, hipStream_t s,
                       const char* fn);

}  // namespace fv

// Library-owned volume copy, clamp-to-edge built in (no index clamps when
// sampling).  Two layouts:
//  linear  the grid with a 2-voxel apron of replicated edge voxels on every
//          side, x fastest: element (i, j, k), i in [-2, nx+1], at
//          data[((k + 2) * py + (j + 2)) * px + (i + 2)], px = nx + 4, py = ny + 4;
//  bricks  cells j = i + 1 in [0, n] grouped 16 per axis into bricks, each
//          stored whole with the voxels its cells' stencils read: brick b
//          holds voxels [16 b - 2, 16 b + 17) per axis (clamped to the grid),
//          19^3 elements x fastest, bricks in (bz, by, bx) order.  Every
//          sample's 4^3 stencil lies inside one brick, so the gather keeps
//          uniform row / slice strides (19, 361 elements).
constexpr int kBrick = 16;       // cells per brick edge
constexpr int kBrickRow = kBrick + 3;  // stored voxels per brick edge
constexpr int kBrickVox = kBrickRow * kBrickRow * kBrickRow;
struct fv_volume {
  int n[3];
  fv_dtype dt;
  int device;
  void* data;
  int64_t px, py, pz;  // linear layout pitches
  int brick;           // 1: the bricked layout
  int nb[3];           // bricks per axis (bricked layout)
  uint64_t bytes;      // size of the copy
};
