// Sample map + ordered stream compaction (paper: "Sample Maps", Eq. (1)-(2);
// "Stream Compaction").
//
// Three launches on the caller's stream, no host synchronisation:
//   k_mask_count   one wave per 8x8 screen tile (16 tiles per 256-thread
//                  block): hash -> threshold -> wave ballot -> block count
//   k_block_scan   one workgroup: exclusive scan of the block counts, total
//                  written to *count
//   k_mask_scatter recomputes the mask bits (cheaper than re-reading them),
//                  ranks each selected lane inside its wave with a masked
//                  popcount and writes ray_idx in tile order; writes the mask.
// The threshold table is built on the host in IEEE double and cached in
// device memory per (device, sigma, p_floor, mode, W, H).
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace fv {
namespace {

constexpr int kTilesPerBlock = 16;  // 4 waves x 4 tiles
constexpr int kMaxDim = 65535;
constexpr double kOne24 = 16777216.0;

// ---------------------------------------------------------------- host table

double tau_of(double R, double sigma, double pf, int mode) {
  const double g = std::exp(-(R / 4.0) / (2.0 * sigma * sigma));
  return mode == FV_FOVEA_LERP ? (1.0 - pf) * g + pf : (g > pf ? g : pf);
}

uint32_t quantise(double tau) {
  double t = std::floor(tau * kOne24);
  if (t > kOne24) t = kOne24;
  if (t < 0.0) t = 0.0;
  return (uint32_t)t;
}

struct Table {
  std::vector<uint32_t> lut;
  int shift = 0;
  uint32_t t_inf = 0;
};

bool build_table(const fv_fovea_params& p, int W, int H, Table* out) {
  const int64_t mx = 2 * (int64_t)W - 1, my = 2 * (int64_t)H - 1;
  const int64_t r_max = mx * mx + my * my;
  const uint32_t t_inf = quantise((double)p.p_floor);
  for (int sh = 0; sh < 63; ++sh) {
    const int64_t cap = (r_max >> sh) + 1;
    int64_t n = 0;
    for (; n < cap && n <= FV_LUT_MAX; ++n)
      if (quantise(tau_of((double)(n << sh), p.sigma_px, p.p_floor, p.mode)) == t_inf) break;
    if (n > FV_LUT_MAX) continue;
    out->lut.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k)
      out->lut[(size_t)k] = quantise(tau_of((double)(k << sh), p.sigma_px, p.p_floor, p.mode));
    out->shift = sh;
    out->t_inf = t_inf;
    return true;
  }
  return false;
}

fv_status check_params(const fv_fovea_params* p, int W, int H, const char* fn) {
  if (!p) return fail(FV_ERR_INVALID_ARG, "%s: null params", fn);
  if (W <= 0 || H <= 0 || W > kMaxDim || H > kMaxDim)
    return fail(FV_ERR_INVALID_ARG, "%s: frame %d x %d outside [1, %d]", fn, W, H, kMaxDim);
  if (p->mode != FV_FOVEA_CLAMP && p->mode != FV_FOVEA_LERP)
    return fail(FV_ERR_UNSUPPORTED, "%s: unknown fovea mode %d", fn, (int)p->mode);
  if (!(std::isfinite(p->sigma_px) && p->sigma_px > 0.0f))
    return fail(FV_ERR_INVALID_ARG, "%s: sigma_px must be finite and > 0", fn);
  if (!(p->p_floor >= 0.0f && p->p_floor <= 1.0f))
    return fail(FV_ERR_INVALID_ARG, "%s: p_floor must be in [0, 1]", fn);
  if (!(p->focus_x >= 0.0f && p->focus_x <= (float)W && p->focus_y >= 0.0f &&
        p->focus_y <= (float)H))
    return fail(FV_ERR_INVALID_ARG, "%s: focus (%g, %g) outside the frame", fn,
                (double)p->focus_x, (double)p->focus_y);
  return FV_OK;
}

// ------------------------------------------------------ device table cache

struct CachedTable {
  int device, mode, W, H;
  uint32_t sigma_bits, pf_bits;
  uint32_t* dev_lut;
  int n, shift;
  uint32_t t_inf;
};

std::mutex g_cache_mu;
std::vector<CachedTable> g_cache;
constexpr size_t kCacheMax = 32;

uint32_t bits_of(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

fv_status get_device_table(const fv_fovea_params& p, int W, int H, CachedTable* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FV_ERR_DEVICE, "fv_fovea_mask: hipGetDevice");
  std::lock_guard<std::mutex> lock(g_cache_mu);
  for (const auto& c : g_cache)
    if (c.device == dev && c.mode == p.mode && c.W == W && c.H == H &&
        c.sigma_bits == bits_of(p.sigma_px) && c.pf_bits == bits_of(p.p_floor)) {
      *out = c;
      return FV_OK;
    }
  Table t;
  if (!build_table(p, W, H, &t)) return fail(FV_ERR_INVALID_ARG, "fv_fovea_mask: no table fits");
  CachedTable c{dev, p.mode, W, H, bits_of(p.sigma_px), bits_of(p.p_floor), nullptr,
                (int)t.lut.size(), t.shift, t.t_inf};
  const size_t bytes = sizeof(uint32_t) * (t.lut.empty() ? 1 : t.lut.size());
  if (hipMalloc(&c.dev_lut, bytes) != hipSuccess)
    return fail(FV_ERR_NOMEM, "fv_fovea_mask: table allocation");
  if (!t.lut.empty()) {
    fv_status st = hip_status(hipMemcpy(c.dev_lut, t.lut.data(), bytes, hipMemcpyHostToDevice),
                              "fv_fovea_mask: table upload");
    if (st != FV_OK) {
      (void)hipFree(c.dev_lut);
      return st;
    }
  }
  if (g_cache.size() >= kCacheMax) {
    // the evicted table may still be read by enqueued work on its device
    int cur = dev;
    (void)hipSetDevice(g_cache.front().device);
    (void)hipDeviceSynchronize();
    (void)hipFree(g_cache.front().dev_lut);
    (void)hipSetDevice(cur);
    g_cache.erase(g_cache.begin());
  }
  g_cache.push_back(c);
  *out = c;
  return FV_OK;
}

// ------------------------------------------------------------------ device

struct MaskArgs {
  const uint32_t* lut;
  int n, shift;
  uint32_t t_inf;
  uint32_t seed_lo, seed_hi, frame;
  int W, H, tiles_x, tiles_per_view;
  int64_t total_tiles;
  int64_t f2x, f2y;
  // noise tiles instead of the hash (NULL: hash): tcount tiles of tw x th
  // 24-bit values, tile (frame + view) mod tcount, repeated over the frame
  const uint32_t* noise;
  int tw, th, tcount;
};

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Mask bit of this lane's pixel in tile `t`; also returns its linear index.
__device__ __forceinline__ bool mask_bit(const MaskArgs& a, int64_t t, int lane, uint32_t* lin) {
  if (t >= a.total_tiles) return false;
  const int view = (int)(t / a.tiles_per_view);
  const int r = (int)(t - (int64_t)view * a.tiles_per_view);
  const int ty = r / a.tiles_x, tx = r - ty * a.tiles_x;
  const int x = tx * 8 + (lane & 7), y = ty * 8 + (lane >> 3);
  if (x >= a.W || y >= a.H) return false;
  uint32_t u;
  if (a.noise) {
    const uint32_t ti = (a.frame + (uint32_t)view) % (uint32_t)a.tcount;
    const uint32_t ty2 = (uint32_t)y % (uint32_t)a.th, tx2 = (uint32_t)x % (uint32_t)a.tw;
    u = a.noise[((size_t)ti * (uint32_t)a.th + ty2) * (uint32_t)a.tw + tx2];
  } else {
    uint32_t h = 0x6A09E667u;
    h = fmix32(h ^ a.seed_lo);
    h = fmix32(h ^ a.seed_hi);
    h = fmix32(h ^ a.frame);
    h = fmix32(h ^ (uint32_t)view);
    h = fmix32(h ^ (uint32_t)y);
    h = fmix32(h ^ (uint32_t)x);
    u = h >> 8;
  }
  const int64_t dx = 2 * (int64_t)x + 1 - a.f2x, dy = 2 * (int64_t)y + 1 - a.f2y;
  const int64_t k = (dx * dx + dy * dy) >> a.shift;
  const uint32_t T = k < a.n ? a.lut[k] : a.t_inf;
  *lin = (uint32_t)view * (uint32_t)a.W * (uint32_t)a.H + (uint32_t)y * (uint32_t)a.W + (uint32_t)x;
  return u < T;
}

__global__ void __launch_bounds__(256) k_mask_count(MaskArgs a, uint32_t* __restrict__ counts) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kTilesPerBlock + wave * 4;
  uint32_t c = 0;
  for (int i = 0; i < 4; ++i) {
    uint32_t lin;
    const bool m = mask_bit(a, t0 + i, lane, &lin);
    c += (uint32_t)__popcll(__ballot(m));
  }
  if (lane == 0) wsum[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Exclusive scan of `n` block counts by one 1024-thread workgroup.
__global__ void __launch_bounds__(1024) k_block_scan(const uint32_t* __restrict__ counts,
                                                     uint32_t* __restrict__ offsets, int64_t n,
                                                     uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t i = base + tid;
    const uint32_t v = i < n ? counts[i] : 0u;
    // inclusive scan inside the wave
    uint32_t s = v;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(s, d, 64);
      if (lane >= d) s += o;
    }
    if (lane == 63) wsum[wave] = s;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wsum[w];
    const uint32_t c = carry;
    if (i < n) offsets[i] = c + wpre + s - v;
    __syncthreads();
    if (tid == 1023) carry = c + wpre + s;
    __syncthreads();
  }
  if (tid == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_mask_scatter(MaskArgs a,
                                                      const uint32_t* __restrict__ offsets,
                                                      uint8_t* __restrict__ mask,
                                                      uint32_t* __restrict__ ray_idx) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kTilesPerBlock + wave * 4;
  uint64_t bal[4];
  bool bit[4];
  uint32_t lin[4];
  uint32_t c = 0;
  for (int i = 0; i < 4; ++i) {
    lin[i] = 0xffffffffu;
    bit[i] = mask_bit(a, t0 + i, lane, &lin[i]);
    bal[i] = __ballot(bit[i]);
    c += (uint32_t)__popcll(bal[i]);
  }
  if (lane == 0) wsum[wave] = c;
  __syncthreads();
  uint32_t base = offsets[blockIdx.x];
  for (int w = 0; w < wave; ++w) base += wsum[w];
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int i = 0; i < 4; ++i) {
    if (bit[i]) ray_idx[base + (uint32_t)__popcll(bal[i] & lt)] = lin[i];
    if (mask && lin[i] != 0xffffffffu) mask[lin[i]] = (uint8_t)bit[i];
    base += (uint32_t)__popcll(bal[i]);
  }
}

int64_t num_blocks(int W, int H, int views) {
  const int64_t tiles = (int64_t)((W + 7) / 8) * ((H + 7) / 8) * views;
  return (tiles + kTilesPerBlock - 1) / kTilesPerBlock;
}

// ------------------------------------------- allocation-free variant's memory
// fv_fovea_mask_noalloc keeps the threshold table and the per-block counts
// and offsets of the scan in this array instead of library allocations and a
// workspace: [table: FV_LUT_MAX words][counts: kNoAllocBlocks][offsets:
// kNoAllocBlocks].  Each device holds its own copy for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is not a device address there).
constexpr int64_t kNoAllocBlocks = FV_MASK_NOALLOC_MAX_BLOCKS;
constexpr size_t kScratchWords = (size_t)FV_LUT_MAX + 2 * (size_t)kNoAllocBlocks;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

struct NoAllocDevice {
  uint32_t* ptr = nullptr;  // this device's scratch
  bool has_table = false;   // which table the scratch holds
  int mode = 0, W = 0, H = 0;
  uint32_t sigma_bits = 0, pf_bits = 0;
  Table table;              // its host copy (the source of the last upload)
};
std::mutex g_noalloc_mu;
constexpr int kMaxDevices = 64;
NoAllocDevice g_noalloc[kMaxDevices];

}  // namespace
}  // namespace fv

extern "C" {

fv_status fv_fovea_lut(const fv_fovea_params* p, int width, int height, uint32_t* host_lut,
                       int* n_entries, int* shift, uint32_t* t_inf) {
  fv::clear_error();
  fv_status st = fv::check_params(p, width, height, "fv_fovea_lut");
  if (st != FV_OK) return st;
  if (!host_lut || !n_entries || !shift || !t_inf)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_fovea_lut: null output pointer");
  fv::Table t;
  if (!fv::build_table(*p, width, height, &t))
    return fv::fail(FV_ERR_INVALID_ARG, "fv_fovea_lut: no table fits");
  for (size_t k = 0; k < t.lut.size(); ++k) host_lut[k] = t.lut[k];
  *n_entries = (int)t.lut.size();
  *shift = t.shift;
  *t_inf = t.t_inf;
  return FV_OK;
}

fv_status fv_fovea_mask_workspace(int width, int height, int views, size_t* bytes) {
  fv::clear_error();
  if (!bytes) return fv::fail(FV_ERR_INVALID_ARG, "fv_fovea_mask_workspace: null bytes");
  if (width <= 0 || height <= 0 || views <= 0)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_fovea_mask_workspace: non-positive size");
  const int64_t nb = fv::num_blocks(width, height, views);
  *bytes = (size_t)(((2 * nb * 4) + 255) / 256 * 256);
  return FV_OK;
}

static fv_status launch_mask(const fv_fovea_params* p, const uint32_t* tiles, int tile_w,
                             int tile_h, int tile_count, int width, int height, int views,
                             uint8_t* mask, uint32_t* ray_idx, uint32_t* count,
                             const uint32_t* lut, int n, int shift, uint32_t t_inf,
                             uint32_t* counts, uint32_t* offsets, hipStream_t s);

// Host-side checks shared by the entry points (everything but the workspace).
static fv_status check_mask_args(const char* fn, const fv_fovea_params* p, int width,
                                 int height, int views, const uint32_t* ray_idx,
                                 uint32_t capacity, const uint32_t* count) {
  fv_status st = fv::check_params(p, width, height, fn);
  if (st != FV_OK) return st;
  if (views <= 0) return fv::fail(FV_ERR_INVALID_ARG, "%s: views must be > 0", fn);
  const uint64_t total = (uint64_t)views * (uint64_t)width * (uint64_t)height;
  if (total >= (1ull << 32))
    return fv::fail(FV_ERR_INVALID_ARG, "%s: views*W*H must be < 2^32", fn);
  if (!ray_idx || !count) return fv::fail(FV_ERR_INVALID_ARG, "%s: null ray_idx or count", fn);
  if ((uint64_t)capacity < total)
    return fv::fail(FV_ERR_CAPACITY, "%s: capacity %u < views*W*H = %llu", fn, capacity,
                    (unsigned long long)total);
  return FV_OK;
}

static fv_status mask_entry(const char* fn, const fv_fovea_params* p, const uint32_t* tiles,
                            int tile_w, int tile_h, int tile_count, int width, int height,
                            int views, uint8_t* mask, uint32_t* ray_idx, uint32_t capacity,
                            uint32_t* count, void* workspace, size_t ws_bytes, void* stream) {
  fv::clear_error();
  fv_status st = check_mask_args(fn, p, width, height, views, ray_idx, capacity, count);
  if (st != FV_OK) return st;
  if (!workspace) return fv::fail(FV_ERR_INVALID_ARG, "%s: null workspace", fn);
  size_t need = 0;
  fv_fovea_mask_workspace(width, height, views, &need);
  if (ws_bytes < need)
    return fv::fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, need);
  if ((uintptr_t)workspace % 256)
    return fv::fail(FV_ERR_INVALID_ARG, "%s: workspace not 256-byte aligned", fn);
  fv::CachedTable tab;
  st = fv::get_device_table(*p, width, height, &tab);
  if (st != FV_OK) return st;
  const int64_t nb = fv::num_blocks(width, height, views);
  uint32_t* counts = (uint32_t*)workspace;
  return launch_mask(p, tiles, tile_w, tile_h, tile_count, width, height, views, mask, ray_idx,
                     count, tab.dev_lut, tab.n, tab.shift, tab.t_inf, counts, counts + nb,
                     (hipStream_t)stream);
}

// The three launches over a device table (lut, n, shift, t_inf) and the
// scan's block counts / offsets (num_blocks words each).
static fv_status launch_mask(const fv_fovea_params* p, const uint32_t* tiles, int tile_w,
                             int tile_h, int tile_count, int width, int height, int views,
                             uint8_t* mask, uint32_t* ray_idx, uint32_t* count,
                             const uint32_t* lut, int n, int shift, uint32_t t_inf,
                             uint32_t* counts, uint32_t* offsets, hipStream_t s) {
  fv_status st;
  fv::MaskArgs a;
  a.lut = lut;
  a.n = n;
  a.shift = shift;
  a.t_inf = t_inf;
  a.seed_lo = (uint32_t)(p->seed & 0xffffffffu);
  a.seed_hi = (uint32_t)(p->seed >> 32);
  a.frame = p->frame;
  a.W = width;
  a.H = height;
  a.tiles_x = (width + 7) / 8;
  a.tiles_per_view = a.tiles_x * ((height + 7) / 8);
  a.total_tiles = (int64_t)a.tiles_per_view * views;
  a.f2x = (int64_t)llround(2.0 * (double)p->focus_x);
  a.f2y = (int64_t)llround(2.0 * (double)p->focus_y);
  a.noise = tiles;
  a.tw = tile_w;
  a.th = tile_h;
  a.tcount = tile_count;

  const int64_t nb = fv::num_blocks(width, height, views);
  fv::k_mask_count<<<(unsigned)nb, 256, 0, s>>>(a, counts);
  if ((st = fv::launch_status("count kernel")) != FV_OK) return st;
  fv::k_block_scan<<<1, 1024, 0, s>>>(counts, offsets, nb, count);
  if ((st = fv::launch_status("scan kernel")) != FV_OK) return st;
  fv::k_mask_scatter<<<(unsigned)nb, 256, 0, s>>>(a, offsets, mask, ray_idx);
  return fv::launch_status("scatter kernel");
}

fv_status fv_fovea_mask(const fv_fovea_params* p, int width, int height, int views,
                        uint8_t* mask, uint32_t* ray_idx, uint32_t capacity, uint32_t* count,
                        void* workspace, size_t ws_bytes, void* stream) {
  return mask_entry("fv_fovea_mask", p, nullptr, 0, 0, 0, width, height, views, mask, ray_idx,
                    capacity, count, workspace, ws_bytes, stream);
}

fv_status fv_fovea_mask_noalloc(const fv_fovea_params* p, int width, int height, int views,
                                uint8_t* mask, uint32_t* ray_idx, uint32_t capacity,
                                uint32_t* count, void* stream) {
  const char* fn = "fv_fovea_mask_noalloc";
  fv::clear_error();
  fv_status st = check_mask_args(fn, p, width, height, views, ray_idx, capacity, count);
  if (st != FV_OK) return st;
  const int64_t nb = fv::num_blocks(width, height, views);
  if (nb > fv::kNoAllocBlocks)
    return fv::fail(FV_ERR_CAPACITY,
                    "%s: %lld blocks of 16 8x8 tiles, at most %d without a workspace", fn,
                    (long long)nb, (int)fv::kNoAllocBlocks);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fv::fail(FV_ERR_DEVICE, "%s: hipGetDevice", fn);
  if (dev < 0 || dev >= fv::kMaxDevices)
    return fv::fail(FV_ERR_UNSUPPORTED, "%s: device %d", fn, dev);
  std::lock_guard<std::mutex> lock(fv::g_noalloc_mu);
  fv::NoAllocDevice& d = fv::g_noalloc[dev];
  if (!d.ptr) {
    // once per device, with that device current: the address of its copy
    void* addr = nullptr;
    st = fv::hip_status(hipGetSymbolAddress(&addr, HIP_SYMBOL(fv::scratch)),
                        "fv_fovea_mask_noalloc: scratch address");
    if (st != FV_OK) return st;
    d.ptr = (uint32_t*)addr;
  }
  hipStream_t s = (hipStream_t)stream;
  // the table: uploaded into the scratch when the parameters it depends on
  // change (ordered on the stream after earlier calls' kernels)
  if (!d.has_table || d.mode != p->mode || d.W != width || d.H != height ||
      d.sigma_bits != fv::bits_of(p->sigma_px) || d.pf_bits != fv::bits_of(p->p_floor)) {
    fv::Table t;
    if (!fv::build_table(*p, width, height, &t))
      return fv::fail(FV_ERR_INVALID_ARG, "%s: no table fits", fn);
    d.has_table = false;
    d.table = std::move(t);
    if (!d.table.lut.empty()) {
      st = fv::hip_status(hipMemcpyAsync(d.ptr, d.table.lut.data(),
                                         d.table.lut.size() * sizeof(uint32_t),
                                         hipMemcpyHostToDevice, s),
                          "fv_fovea_mask_noalloc: table upload");
      if (st != FV_OK) return st;
    }
    d.has_table = true;
    d.mode = p->mode;
    d.W = width;
    d.H = height;
    d.sigma_bits = fv::bits_of(p->sigma_px);
    d.pf_bits = fv::bits_of(p->p_floor);
  }
  uint32_t* counts = d.ptr + FV_LUT_MAX;
  return launch_mask(p, nullptr, 0, 0, 0, width, height, views, mask, ray_idx, count, d.ptr,
                     (int)d.table.lut.size(), d.table.shift, d.table.t_inf, counts,
                     counts + fv::kNoAllocBlocks, s);
}

fv_status fv_fovea_mask_tiles(const fv_fovea_params* p, const uint32_t* tiles, int tile_w,
                              int tile_h, int tile_count, int width, int height, int views,
                              uint8_t* mask, uint32_t* ray_idx, uint32_t capacity,
                              uint32_t* count, void* workspace, size_t ws_bytes, void* stream) {
  if (!tiles || tile_w <= 0 || tile_h <= 0 || tile_count <= 0 ||
      (uint64_t)tile_w * tile_h * tile_count >= (1ull << 31)) {
    fv::clear_error();
    return fv::fail(FV_ERR_INVALID_ARG, "fv_fovea_mask_tiles: bad tile stack");
  }
  return mask_entry("fv_fovea_mask_tiles", p, tiles, tile_w, tile_h, tile_count, width, height,
                    views, mask, ray_idx, capacity, count, workspace, ws_bytes, stream);
}

}  // extern "C"
