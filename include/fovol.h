/*
 * fovol.h -- C ABI of libfovol.so: foveated sparse direct volume rendering
 * with neural full-frame reconstruction on AMD Instinct MI355X (gfx950).
 *
 * Method: FoVolNet (Bauer, Wu, Ma; arXiv 2209.09965).  The pipeline renders
 * only the pixels selected by a fovea-weighted sample map, packs them with
 * stream compaction, ray-marches the packed list, scatters the results back
 * to the full frame and lets a small network reconstruct the missing pixels
 * (paper: Methods, "Foveated Rendering", "Sample Maps", "Stream Compaction",
 * "Reconstruction Network").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Plain C: no C++ types, no exceptions cross this boundary.
 *  - Every data pointer documented "dev" is caller-owned device memory
 *    (hipMalloc or a framework allocator).  The library never frees or keeps
 *    a caller pointer beyond the work it enqueues.  "host" pointers are read
 *    (or written) synchronously during the call.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    All compute calls only enqueue work and return; results are valid after
 *    the caller synchronises that stream.
 *  - Argument errors are detected on the host before anything is enqueued;
 *    the call then returns a negative fv_status and fv_last_error() holds a
 *    message.  A launch failure reported by the HIP runtime returns
 *    FV_ERR_DEVICE.
 *  - Pixel index convention: a pixel (x, y) of view v in a views x H x W
 *    frame stack has linear index  idx = v*W*H + y*W + x.  Frame buffers are
 *    "pixel-major": frame_rgba[idx*4 + c], frame_depth[idx].
 *  - Thread safety: separate handles may be used from different host
 *    threads; one handle must not be used by two calls at the same time.
 */
#ifndef FOVOL_H
#define FOVOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FV_ABI_VERSION 2

typedef enum {
  FV_OK = 0,
  FV_ERR_INVALID_ARG = -1, /* null pointer, bad size, out-of-range parameter */
  FV_ERR_CAPACITY = -2,    /* an output capacity is too small                 */
  FV_ERR_UNSUPPORTED = -3, /* unknown dtype / mode / precision                */
  FV_ERR_DEVICE = -4,      /* the HIP runtime reported an error               */
  FV_ERR_NOMEM = -5        /* a library-owned allocation failed               */
} fv_status;

/* Message for the last failing call on this host thread ("" if none).  The
 * pointer stays valid until the next call on the same thread. */
const char* fv_last_error(void);
int fv_abi_version(void);

typedef enum { FV_U8 = 0, FV_F16 = 1, FV_F32 = 2 } fv_dtype;

/* ------------------------------------------------------------------------
 * 1. Sample map and stream compaction
 *    (paper: "Sample Maps", Eq. (1) and (2); "Stream Compaction")
 * ------------------------------------------------------------------------
 * The sample map is M(x,y) = [N(x,y) < tau(x,y)].
 *
 *  N   Seeded white noise: u = H32(seed, frame, view, y, x) >> 8, a 24-bit
 *      integer, where H32 chains the MurmurHash3 32-bit finaliser over the
 *      key words (seed low, seed high, frame, view, y, x), starting from
 *      0x6A09E667: h = fmix32(h ^ word) for each word in that order.  The
 *      paper draws N from pre-computed spatio-temporal blue-noise tiles; a
 *      counter-based hash stands in for them (random access, reproducible
 *      from the seed, a new pattern every frame).
 *  tau The fovea density (Eq. 1) is read as a Gaussian fall-off of the
 *      pixel's distance r to the focal point, g = exp(-r^2 / (2 s^2)) with
 *      s = sigma_px.  It is combined with the base density p = p_floor by
 *      either  FV_FOVEA_LERP:  tau = (1 - p) g + p      (Eq. 2), or
 *              FV_FOVEA_CLAMP: tau = max(g, p).
 *  Quantisation (makes the mask bit-reproducible on host and device):
 *      distances use doubled pixel coordinates, R = (2x+1-F2x)^2 +
 *      (2y+1-F2y)^2 with F2 = llround(2*focus) (R/4 = r^2 in px^2).
 *      T(R) = min(2^24, floor(tau(R) * 2^24)) evaluated in IEEE double,
 *      T_inf = min(2^24, floor(p * 2^24)).  The table holds T_k = T(k << sh)
 *      for k < n; bins k >= n use T_inf.  sh is the smallest shift for which
 *      n <= FV_LUT_MAX, where n = the first k with T(k << sh) == T_inf,
 *      capped at (R_max >> sh) + 1 with R_max = (2W-1)^2 + (2H-1)^2 (the
 *      largest R of any pixel for any focus in the frame).  The table thus
 *      depends on (sigma_px, p_floor, mode, W, H) and not on the focus.
 *      M = [u < T_{R >> sh}]   (strict, as in the paper's N < tau).
 *  Compaction order: view-major, then 8x8 screen tiles in row-major tile
 *      order, then row-major inside a tile (edge tiles are clipped to the
 *      frame).  ray_idx[i] is the linear pixel index of the i-th selected
 *      pixel in that order; count = number of selected pixels.
 */
#define FV_LUT_MAX 16384

typedef enum { FV_FOVEA_CLAMP = 0, FV_FOVEA_LERP = 1 } fv_fovea_mode;

typedef struct {
  uint64_t seed;
  uint32_t frame;   /* animation frame, part of the noise key              */
  int32_t mode;     /* fv_fovea_mode                                       */
  float focus_x;    /* focal point in pixels; pixel (x,y) spans [x,x+1)    */
  float focus_y;    /*   x [y,y+1); the frame centre is (W/2, H/2)         */
  float sigma_px;   /* s > 0, Gaussian fall-off in pixels                  */
  float p_floor;    /* base density p in [0, 1]                            */
} fv_fovea_params;

/* Threshold table of the sample map (host; a test hook and a diagnostic).
 * host_lut must hold FV_LUT_MAX entries; n_entries, shift and t_inf receive
 * n, sh and T_inf.  Errors: FV_ERR_INVALID_ARG for null pointers, width or
 * height <= 0, sigma_px <= 0 or not finite, p_floor outside [0,1], focus not
 * finite or outside [0,W]x[0,H]; FV_ERR_UNSUPPORTED for an unknown mode. */
fv_status fv_fovea_lut(const fv_fovea_params* p, int width, int height,
                       uint32_t* host_lut, int* n_entries, int* shift,
                       uint32_t* t_inf);

/* Bytes of device workspace fv_fovea_mask needs for this frame stack. */
fv_status fv_fovea_mask_workspace(int width, int height, int views,
                                  size_t* bytes);

/* Sample map + ordered stream compaction for `views` frames of W x H that
 * share the fovea parameters (the view index is part of the noise key).
 *   mask      dev uint8 [views*H*W] (1 = sampled) or NULL to skip
 *   ray_idx   dev uint32 [capacity]; entries [0, count) are written
 *   capacity  must be >= views*W*H (so the device can never overflow it);
 *             otherwise FV_ERR_CAPACITY
 *   count     dev uint32 [1]; written, stays on the device
 *   workspace dev, >= fv_fovea_mask_workspace() bytes, 256-byte aligned;
 *             contents on entry are ignored
 * Errors: as fv_fovea_lut, plus views <= 0, views*W*H >= 2^32, null ray_idx,
 * count or workspace, and a workspace that is too small (FV_ERR_CAPACITY). */
fv_status fv_fovea_mask(const fv_fovea_params* p, int width, int height,
                        int views, uint8_t* mask, uint32_t* ray_idx,
                        uint32_t capacity, uint32_t* count, void* workspace,
                        size_t ws_bytes, void* stream);

/* fv_fovea_mask without a workspace and without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Outputs, arguments and errors are
 * those of fv_fovea_mask minus the workspace.  The scan's block counts and
 * the threshold table live in one library array per device, held until the
 * process ends: FV_LUT_MAX + 2 * FV_MASK_NOALLOC_MAX_BLOCKS 32-bit words
 * (320 KiB).  A frame stack of more than FV_MASK_NOALLOC_MAX_BLOCKS blocks
 * (a block = 16 tiles of 8 x 8 pixels of one view, so about 33.5 million
 * pixels) is refused with FV_ERR_CAPACITY.  The table is uploaded into the
 * array, on `stream`, when its parameters (sigma_px, p_floor, mode, W, H)
 * differ from the previous call's on the device.  Every call on a device
 * shares that array: calls that overlap on one device (other streams, other
 * host threads) race and must be ordered by the caller. */
#define FV_MASK_NOALLOC_MAX_BLOCKS 32768
fv_status fv_fovea_mask_noalloc(const fv_fovea_params* p, int width, int height,
                                int views, uint8_t* mask, uint32_t* ray_idx,
                                uint32_t capacity, uint32_t* count, void* stream);

/* Sample map from a stack of noise tiles (paper Sec. 3.1.1: tileable noise
 * textures, a different tile each frame, looping over the stack) in place of
 * the seeded hash: pixel (x, y) of view v in frame f draws
 *   u = tiles[((f + v) mod tile_count) * tile_h + y mod tile_h][x mod tile_w]
 * and is sampled when u < T (the same quantised density as fv_fovea_mask;
 * the seed is not used).  Everything else, outputs and workspace included,
 * is as fv_fovea_mask.
 *   tiles  dev uint32 [tile_count][tile_h][tile_w], values in [0, 2^24)
 *          (a value v of an 8-bit noise texture maps to v * 2^16 + 2^15)
 * Errors: as fv_fovea_mask, plus a null tile stack, non-positive tile sizes
 * or a stack of 2^31 values or more. */
fv_status fv_fovea_mask_tiles(const fv_fovea_params* p, const uint32_t* tiles,
                              int tile_w, int tile_h, int tile_count,
                              int width, int height, int views, uint8_t* mask,
                              uint32_t* ray_idx, uint32_t capacity,
                              uint32_t* count, void* workspace,
                              size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * 2. Volume
 * ------------------------------------------------------------------------
 * World space: the volume's box is centred at the origin and its longest
 * side has length 1, so a voxel has edge h = 1/max(nx,ny,nz); voxel (i,j,k)
 * has its centre at ((i+0.5)h - nx*h/2, (j+0.5)h - ny*h/2, (k+0.5)h - nz*h/2).
 * Scalars: u8 maps to v/255, f16 and f32 are taken as they are.
 *
 * fv_volume_create copies a caller-owned linear device array (x fastest,
 * then y, then z; nx*ny*nz elements of `dt`) into a library-owned
 * layout on the stream, then synchronises that stream.  The handle owns that copy until
 * fv_volume_destroy.  Errors: null pointers, any dimension < 1 or > 4096,
 * unknown dtype or a padded copy of 4 GiB or more, i.e.
 * (nx+4)(ny+4)(nz+4) x bytes per voxel >= 2^32 (FV_ERR_UNSUPPORTED),
 * allocation failure (FV_ERR_NOMEM). */
typedef struct fv_volume fv_volume;

fv_status fv_volume_create(const void* dev_data, int nx, int ny, int nz,
                           fv_dtype dt, void* stream, fv_volume** out);
/* The same volume in the bricked layout: cells grouped in 16^3 bricks, each
 * stored whole with the apron its samples' stencils read (19^3 voxels, x
 * fastest), bricks in z, y, x order; (ceil((n+1)/16))^3 x 19^3 elements,
 * about 1.7 x the grid.  A sample's voxels then lie within one brick: fewer
 * cache lines per sample and neighbouring samples on the same lines, for
 * volumes beyond the caches.  Every march reads the same voxel values in
 * either layout (bit-identical results).  Errors as fv_volume_create (the
 * bricked copy must be < 4 GiB). */
fv_status fv_volume_create_bricked(const void* dev_data, int nx, int ny, int nz,
                                   fv_dtype dt, void* stream, fv_volume** out);
fv_status fv_volume_destroy(fv_volume* v);

/* ------------------------------------------------------------------------
 * 3. Ray marching (paper: "Foveated Rendering", "Rendering", "Stream
 *    Compaction" -- the renderer that samples the packed pixel list)
 * ------------------------------------------------------------------------
 * Per pixel ray (pinhole camera):
 *   f = normalize(target-eye), r = normalize(f x up), u = r x f,
 *   px = (2(x+0.5)/W - 1) tan(fovy/2) W/H,  py = (1 - 2(y+0.5)/H) tan(fovy/2),
 *   d = normalize(f + px r + py u),  origin = eye + eye_offset * r.
 * Box entry/exit by the slab method: [t0, t1], t0 clamped to >= 0; a miss
 * (t1 <= t0) gives RGB = bg, A = 0, depth = 0.
 * Segments: L = (t1-t0)/h voxel lengths are cut into N = ceil(L/step_vox)
 * segments [k*step, min((k+1)*step, L)]; segment k (length l_k) is sampled at
 * its midpoint.  Sampling: clamp-to-edge trilinear interpolation in voxel
 * index space.  Transfer function: 256 x (r, g, b, sigma) float entries,
 * looked up with linear interpolation at x = clamp(v,0,1)*255; sigma is an
 * extinction per voxel length and the segment opacity is
 * alpha_k = 1 - exp(-sigma * l_k).
 * Shading (shading != 0): gradient by one-voxel central differences of the
 * interpolated field, n = -grad / max(|grad|, 1e-4), L = normalize(light_dir),
 * V = -d, Hv = normalize(L + V),
 * c = rgb (ka + kd |n.L|) + ks |n.Hv|^shininess, the power computed as
 * exp2(shininess log2 x) with the hardware exp2/log2 (relative error a few
 * 1e-6 at shininess 32).
 * Global shadows (shading != 0 and shadow_step > 0; paper "Foveated
 * Rendering": one shadow ray per sample towards the light at a lower sample
 * rate): from the sample's position q (voxel index space, where the box is
 * [-1/2, n-1/2] per axis) a ray along L runs to the box exit, L_s voxel
 * lengths away, in ceil(L_s/shadow_step) midpoint-sampled segments (the last
 * shorter); with tau = sum sigma_j len_j over them,
 * c = rgb (ka + e^-tau kd |n.L|) + e^-tau ks |n.Hv|^shininess.
 * Compositing front to back in FP32 with early termination:
 *   w = T alpha_k; C += w c; D += w t_k; T *= (1 - alpha_k);
 *   stop once 1 - T >= alpha_stop.
 * Output RGB = C + T bg, A = 1 - T, depth = D (world units, premultiplied by
 * opacity).
 *
 * The dense and the sparse march run the same per-ray device code, so a
 * sparse pixel equals the dense pixel at the same index bit for bit.
 */
typedef struct {
  float eye[3];
  float target[3];
  float up[3];
  float fovy_deg;    /* vertical field of view, (0, 180)                  */
  float eye_offset;  /* origin shift along the camera's right axis        */
} fv_camera;

typedef struct {
  float step_vox;    /* segment length in voxels, in [1/64, 64]           */
  float alpha_stop;  /* early-termination opacity, in (0, 1]              */
  int32_t shading;   /* 0 = emission-absorption only, 1 = Blinn-Phong     */
  float light_dir[3];/* direction towards the light (non-zero)            */
  float ka, kd, ks;
  float shininess;   /* specular exponent, in [0, 1024] when shading      */
  float bg[3];       /* background colour                                 */
  float shadow_step; /* global shadows (shading only): 0 = none, else the
                        shadow-ray segment length in voxels, in [1/64, 64];
                        the paper's renderer uses 4 x step_vox           */
  int32_t lanes_per_ray; /* sparse march: 0 = chosen per launch from the
                        rays that reach the volume and the resident lanes;
                        1, 2, 4 or 8 forces that many lanes per ray (for
                        timing; every choice gives the same pixels)      */
} fv_march_params;

#define FV_TF_ENTRIES 256

/* Full-frame march: every pixel of `views` frames.
 *   tf_rgba      dev float [256*4]  (r, g, b, sigma) per entry
 *   cams         host [views] cameras
 *   frame_rgba   dev float [views*H*W*4]
 *   frame_depth  dev float [views*H*W] or NULL
 *   sample_count dev uint64 [1] or NULL; if given, the number of composited
 *                samples (segments, counting the terminating one) is ADDED
 *                to it (the caller clears it)
 * Errors: null v/tf/cams/params/frame_rgba, width/height/views <= 0,
 * views > 8, views*W*H >= 2^32, W or H > 65535, tf_n != 256, step_vox
 * outside [1/64, 64], alpha_stop outside (0,1], a zero light_dir or a
 * shininess outside [0, 1024] with shading, shadow_step not 0 and outside
 * [1/64, 64], lanes_per_ray not 0, 1, 2, 4 or 8, shading not 0/1
 * (FV_ERR_UNSUPPORTED), non-finite camera, fovy outside (0,180), eye ==
 * target or up parallel to the view direction. */
fv_status fv_raymarch_dense(const fv_volume* v, const float* tf_rgba, int tf_n,
                            const fv_camera* cams, int views, int width,
                            int height, const fv_march_params* mp,
                            float* frame_rgba, float* frame_depth,
                            uint64_t* sample_count, void* stream);

/* Naive rejection (paper Sec. 3.1.5, the alternative to stream compaction):
 * the full-frame launch of fv_raymarch_dense, in which the thread of a pixel
 * whose sample-map entry is 0 returns at once and the others march their ray
 * exactly as fv_raymarch_dense does (the same results, bit for bit).  It is
 * the baseline that stream compaction is measured against: a wave runs as
 * long as its slowest sampled pixel however few of its pixels are sampled.
 *   mask         dev uint8 [views*H*W], nonzero = march this pixel (the
 *                layout fv_fovea_mask writes)
 *   frame_rgba, frame_depth, sample_count  as fv_raymarch_dense; pixels with
 *                mask 0 are left untouched
 * Errors: as fv_raymarch_dense, plus a null mask. */
fv_status fv_raymarch_masked(const fv_volume* v, const float* tf_rgba,
                             int tf_n, const fv_camera* cams, int views,
                             int width, int height, const fv_march_params* mp,
                             const uint8_t* mask, float* frame_rgba,
                             float* frame_depth, uint64_t* sample_count,
                             void* stream);

/* Bytes of device workspace fv_raymarch_sparse needs for a list of up to
 * `capacity` rays: a claim counter and the per-ray set-up (the camera ray's
 * box entry, sample step and segment count, 88 bytes a ray), which a first
 * kernel computes once per listed ray.  Errors: null bytes, capacity 0. */
fv_status fv_raymarch_sparse_workspace(uint32_t capacity, size_t* bytes);

/* Sparse march over the compacted list written by fv_fovea_mask.  `count`
 * is read on the device (no host synchronisation).  For i < *count the ray
 * of pixel ray_idx[i] is marched; its result goes to
 *   rgba_compact[i*4..]/depth_compact[i]   (dev, [capacity*4]/[capacity], or NULL)
 *   frame_rgba[ray_idx[i]*4..]/frame_depth[ray_idx[i]]  (dev, full frame, or NULL)
 * (back-projection).  Frame pixels not in the list are left untouched: clear
 * the frame first to get the sparse image.  Entries of ray_idx must be
 * < views*W*H (they are checked on the device; a bad entry is skipped).
 *   workspace  dev, >= fv_raymarch_sparse_workspace(capacity) bytes,
 *              256-byte aligned
 * Errors: as fv_raymarch_dense, plus null ray_idx/count/workspace, capacity
 * == 0 or > views*W*H, and all four outputs NULL. */
fv_status fv_raymarch_sparse(const fv_volume* v, const float* tf_rgba,
                             int tf_n, const fv_camera* cams, int views,
                             int width, int height, const fv_march_params* mp,
                             const uint32_t* ray_idx, const uint32_t* count,
                             uint32_t capacity, float* rgba_compact,
                             float* depth_compact, float* frame_rgba,
                             float* frame_depth, uint64_t* sample_count,
                             void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * 4. Reconstruction network (paper: "Reconstruction Network", "Model
 *    Precision & Optimization")
 * ------------------------------------------------------------------------
 * A 4-level U-Net (32/48/64/96 channels, two 3x3 conv + ReLU per block, 2x2
 * average pooling, bilinear x2 upsampling with half-pixel centres, skips
 * concatenated after the upsampled features) whose last decoder state H_d
 * feeds two 1x1 heads: the direct prediction O_d (3 channels, linear) and 25
 * kernel logits; the softmax of the logits is a per-pixel 5x5 kernel applied
 * to O_d with replicated borders (tap k = 5 (dy+2) + (dx+2)).
 * Input per pixel: [M r, M g, M b, M, M depth/2] from the back-projected
 * sparse frame (M = sample map).
 *
 * Parameters: FV_NET_PARAMS floats in canonical layer order e0a e0b e1a e1b
 * e2a e2b e3a e3b d2a d2b d1a d1b d0a d0b hd hk; per layer the weight
 * [Co][Ci][k][k] then the bias [Co].  Concatenated inputs list the
 * upsampled channels first.  The handle keeps FP32 master weights, Adam
 * state, a BF16 copy (training, BF16 inference) and an FP8 E4M3 copy.
 *
 * Precision:
 *  FV_PREC_BF16  activations and weights BF16, MFMA with FP32 accumulation.
 *  FV_PREC_FP8   activations and weights FP8 E4M3 (OCP: 4 exponent bits,
 *                bias 7, 3 mantissa bits, largest finite 448), FP32
 *                accumulation, post-training quantisation:
 *    Activation scales: fv_net_calibrate runs the BF16 network over its
 *      frames and takes, for every tensor t with a scale (the packed input
 *      and the output of each 3x3 conv, after its ReLU), the largest
 *      magnitude m_t as computed before the tensor is rounded for storage:
 *      s_t = FV_FP8_HEADROOM max(m_t, 1e-6) / 448 (the headroom keeps
 *      frames brighter than the calibration frames from saturating).  A
 *      value a of t is stored as the code q = E4M3(a / s_t), saturated at
 *      +-448, rounded to nearest even.  A
 *      pooled tensor stores E4M3 of the mean of four codes and an upsampled
 *      one E4M3 of the bilinear blend of the codes; both keep their source's
 *      scale.
 *    Weight scales: for a 3x3 layer whose input channel c comes from a
 *      tensor of scale s_in(c), W'[o][c][t] = W[o][c][t] s_in(c),
 *      omega_o = max over c, t of |W'[o][c][t]| / 448 (1 for an all-zero
 *      channel), weight codes Wq = E4M3(W' / omega_o).
 *    Epilogue: acc_o = sum of Wq q over the 3x3 taps and channels (FP32
 *      accumulation), stored q_out = E4M3(min(max(acc_o (omega_o / s_out) +
 *      B_o / s_out, 0), 448)), the two factors in FP32 (ReLU and
 *      saturation in one clamp).
 *    First layer: the packed input (the sampled colours, and the fed-back
 *      O_d of the recurrent form) is not quantised to E4M3, whose 6 % steps
 *      the output would inherit: e0a reads it in BF16 with BF16 weights
 *      (FP32 accumulation) and stores q = E4M3(min(max(acc / s_e0a +
 *      B / s_e0a, 0), 448)); the input's scale s_in is measured but unused.
 *    Heads: the codes of the last decoder tensor with the head weights
 *      BF16(W s_d0b), FP32 bias and accumulation.
 *  The two 1x1 heads run on MFMA with BF16 operands (FP8 activations are
 *  widened) and FP32 accumulation; softmax and the kernel application run
 *  in FP32.
 */
#define FV_FP8_HEADROOM 2.0f
#define FV_NET_PARAMS 480060

/* Recurrent form (paper Sec. 3.2.4, the feedback of the direct prediction):
 * the first conv (e0a) reads 8 channels, the 5 above followed by the
 * previous frame's direct prediction O_d (r, g, b, FP32, unmasked), so its
 * weight is [32][8][3][3] and the vector has 32 * 3 * 9 = 864 more entries.
 * The first frame of a sequence is run with a zero O_d.  Under FP8 the
 * first conv reads the input in BF16 as in the plain form.  The recurrent
 * decoder hidden states of the
 * paper's network are not part of this form.
 * fv_net_create tells the two forms apart by n_params. */
#define FV_NET_PARAMS_RECURRENT 480924

/* FV_RECON_PULLPUSH selects the reconstruction without a network (section
 * 4b below) in fv_reconstruct and fv_reconstruct_workspace; the network
 * handle may then be NULL and frame_depth is ignored. */
typedef enum { FV_PREC_BF16 = 1, FV_PREC_FP8 = 2, FV_RECON_PULLPUSH = 3 } fv_precision;

typedef struct fv_net fv_net;

/* FV_NET_PARAMS (the plain form). */
size_t fv_net_param_count(void);
/* Input channels of the handle's network: 5 (plain) or 8 (recurrent); -1
 * for a null handle. */
int fv_net_input_channels(const fv_net* n);

/* Uploads host FP32 parameters (n_params == FV_NET_PARAMS for the plain
 * form, FV_NET_PARAMS_RECURRENT for the recurrent one), zeroes the Adam
 * state and builds the BF16 copy; synchronises the device.  FP8 is not
 * usable until fv_net_calibrate.  Errors: null pointers, wrong n_params,
 * allocation failure (FV_ERR_NOMEM). */
fv_status fv_net_create(const float* host_params, size_t n_params, fv_net** out);
fv_status fv_net_destroy(fv_net* n);
/* Copies the FP32 master parameters to / from host memory (synchronous);
 * n_params must be the handle's form's count.  fv_net_set_params
 * invalidates the FP8 copy. */
fv_status fv_net_get_params(const fv_net* n, float* host_params, size_t n_params);
fv_status fv_net_set_params(fv_net* n, const float* host_params, size_t n_params);

/* Device workspace for fv_reconstruct at this size and precision. */
fv_status fv_reconstruct_workspace(const fv_net* n, int precision, int views,
                                   int width, int height, size_t* bytes);

/* Full-frame reconstruction of `views` sparse frames.
 *   frame_rgba  dev float [views*H*W*4]  back-projected sparse march output
 *               (only pixels with mask != 0 are read)
 *   mask        dev uint8 [views*H*W]
 *   frame_depth dev float [views*H*W] or NULL (depth channel = 0)
 *   out_rgb     dev float [views*H*W*3]  reconstructed frame
 *   out_direct  dev float [views*H*W*3] or NULL: the direct prediction O_d
 *   workspace   dev, >= fv_reconstruct_workspace() bytes, 256-byte aligned
 * Errors: null pointers, W or H not a multiple of 8 (three poolings) or
 * outside [8, 16384], unknown precision (FV_ERR_UNSUPPORTED), FP8 before
 * calibration, workspace too small (FV_ERR_CAPACITY). */
fv_status fv_reconstruct(const fv_net* n, int precision, const float* frame_rgba,
                         const uint8_t* mask, const float* frame_depth, int views,
                         int width, int height, float* out_rgb, float* out_direct,
                         void* workspace, size_t ws_bytes, void* stream);

/* fv_reconstruct for the recurrent form (Sec. 3.2.4): frame t of a sequence
 * reads the direct prediction of frame t-1 of the same view.
 *   prev_direct dev float [views*H*W*3] or NULL (zero: the first frame), the
 *               out_direct of the previous call; it may be the same buffer
 *               as this call's out_direct (it is read before O_d is written)
 * fv_reconstruct on a recurrent network is this call with a NULL
 * prev_direct.  Errors: those of fv_reconstruct, and a non-NULL prev_direct
 * for a plain network (FV_ERR_INVALID_ARG). */
fv_status fv_reconstruct_recurrent(const fv_net* n, int precision, const float* frame_rgba,
                                   const uint8_t* mask, const float* frame_depth,
                                   const float* prev_direct, int views, int width, int height,
                                   float* out_rgb, float* out_direct, void* workspace,
                                   size_t ws_bytes, void* stream);

/* Post-training quantisation to FP8: runs one BF16 forward pass over the
 * given frames, records the largest magnitude of every activation tensor
 * (scale = max / 448), folds the scales into per-output-channel E4M3
 * weights and stores them in the handle.  Synchronises `stream`.  The
 * workspace must hold the BF16 plan (fv_reconstruct_workspace with
 * FV_PREC_BF16). */
fv_status fv_net_calibrate(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                           const float* frame_depth, int views, int width, int height,
                           void* workspace, size_t ws_bytes, void* stream);
/* The same with the fed-back O_d of the recurrent form in the calibration
 * pass (prev_direct as in fv_reconstruct_recurrent, NULL for zeros), so the
 * activation scales reflect the fed-back input. */
fv_status fv_net_calibrate_recurrent(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                                     const float* frame_depth, const float* prev_direct,
                                     int views, int width, int height, void* workspace,
                                     size_t ws_bytes, void* stream);

/* The FP8 scales of a calibrated network (a test hook and a diagnostic):
 * host_scales[0] = s_in of the packed input, host_scales[1 + l] = the scale
 * of the output of 3x3 conv l in canonical order (e0a, e0b, ..., d0b); 15
 * values.  Errors: null pointers, count != FV_NET_FP8_TENSORS, a network
 * that has not been calibrated (FV_ERR_INVALID_ARG). */
#define FV_NET_FP8_TENSORS 15
fv_status fv_net_fp8_scales(const fv_net* n, float* host_scales, int count);

/* FP8 from scales calibrated elsewhere (offline, over many frames, or by a
 * reference): host_scales in the order fv_net_fp8_scales returns them; the
 * handle then quantises its weights exactly as fv_net_calibrate does after
 * measuring them.  Synchronises `stream`.  Errors: null pointers, count !=
 * FV_NET_FP8_TENSORS, a scale that is not finite and positive. */
fv_status fv_net_set_fp8_scales(fv_net* n, const float* host_scales, int count, void* stream);

/* Test hooks: the forward pass one step at a time (paper Sec. 3.2, the
 * network's layers; Sec. 3.4, its reduced-precision storage), so that a test
 * can hold each layer's kernel to a reference on inputs of the test's
 * choosing.
 *
 * Activation tensors of a forward pass, in this order (index: name,
 * channels, resolution level; level l is (H >> l) x (W >> l)):
 *   0 packed input 8, 0    1 e0a 32, 0    2 e0b 32, 0    3 pool(e0b) 32, 1
 *   4 e1a 48, 1            5 e1b 48, 1    6 pool(e1b) 48, 2
 *   7 e2a 64, 2            8 e2b 64, 2    9 pool(e2b) 64, 3
 *  10 e3a 96, 3           11 e3b 96, 3
 *  12 d2a 64, 2  13 d2b 64, 2  14 d1a 48, 1  15 d1b 48, 1  16 d0a 32, 0
 *  17 d0b 32, 0
 * Each lives in the workspace of fv_reconstruct at a fixed byte offset as
 * views x h x w x channels (channel fastest), one element per value in the
 * precision's storage format: FP8 the E4M3 code q of the scheme above (the
 * value is q times the tensor's scale; a pooled tensor has the scale of its
 * source), BF16 the bfloat16 value.  An upsampled source is not stored: a
 * decoder conv computes it from the lower level on the fly.
 *
 * fv_reconstruct_tensor: offset (bytes from the workspace start), channels
 * and level of tensor `tensor` at this frame size and precision.  Errors:
 * null pointers, tensor outside 0 .. 17, precision not BF16 / FP8, a frame
 * size fv_reconstruct rejects. */
#define FV_NET_TENSORS 18
fv_status fv_reconstruct_tensor(int precision, int views, int width, int height, int tensor,
                                size_t* offset, int* channels, int* level);

/* fv_reconstruct (or fv_reconstruct_recurrent: prev_direct) restricted to
 * steps first .. last of its forward pass: step l in 0 .. 13 is 3x3 conv l
 * in canonical order (writing its output tensor, and for l = 1, 3, 5 also
 * the pooled tensor after it), step 14 the heads (out_rgb, out_direct).
 * Steps 0 and 1 run as one fused kernel that computes the packed input and
 * e0a from the frame without storing them (tensors 0 and 1 are not
 * written); a range that starts at 0 or 1 runs both.  A step reads its
 * input tensors from the workspace as an earlier step (or the caller)
 * left them.  frame_rgba and mask may be NULL when first >= 2, out_rgb when
 * last < 14.  Errors: those of fv_reconstruct, first < 0, last > 14,
 * first > last. */
fv_status fv_reconstruct_steps(const fv_net* n, int precision, int first, int last,
                               const float* frame_rgba, const uint8_t* mask,
                               const float* frame_depth, const float* prev_direct, int views,
                               int width, int height, float* out_rgb, float* out_direct,
                               void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * 4b. Reconstruction without a network: pull-push
 * ------------------------------------------------------------------------
 * The baseline against which the learned reconstruction (paper Sec. 3.2) is
 * measured, and a full-frame fill that needs no weights: the pull-push
 * scattered-data interpolation of Gortler et al. ("The Lumigraph", 1996,
 * Sec. 3.3) on an image pyramid, per view.  Level l+1 has ceil(H_l/2) x
 * ceil(W_l/2) pixels, down to 1 x 1; level 0 holds c_0 = the sampled RGB and
 * w_0 = M (the sample map).
 *   Pull: with t = min(w, 1) for each of the (up to) four children q of a
 *     coarse pixel, w' = sum t(q), c' = sum t(q) c(q) / w' (0 if w' = 0).
 *   Push: f_top = c_top; f_l(q) = t_l(q) c_l(q) + (1 - t_l(q)) u(q), where
 *     u is f_{l+1} interpolated bilinearly at (q + 1/2)/2 - 1/2 per axis,
 *     clamped to the coarser level's pixel range.
 * out = f_0: sampled pixels keep their colour exactly; a frame without any
 * sample gives 0.  FP32 arithmetic.
 *   frame_rgba  dev float [views*H*W*4]; only pixels with mask != 0 are read
 *   mask        dev uint8 [views*H*W]
 *   out_rgb     dev float [views*H*W*3]
 *   workspace   dev, >= fv_pullpush_workspace() bytes (the pulled pyramid
 *               levels 1.., a float4 per pixel), 256-byte aligned
 * Any frame size with views*W*H < 2^32 and W, H <= 65535.  Errors: null
 * pointers, bad sizes (FV_ERR_INVALID_ARG), workspace too small
 * (FV_ERR_CAPACITY). */
fv_status fv_pullpush_workspace(int views, int width, int height, size_t* bytes);
fv_status fv_reconstruct_pullpush(const float* frame_rgba, const uint8_t* mask, int views,
                                  int width, int height, float* out_rgb, void* workspace,
                                  size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * 4c. The foveated frame in one call, with the dense march as quality
 *     reference and fallback
 * ------------------------------------------------------------------------
 * The paper's pipeline (Sec. 3, Fig. 2): sample map and compaction
 * (fv_fovea_mask), sparse march with back-projection (fv_raymarch_sparse),
 * full-frame reconstruction (fv_reconstruct with the policy's precision).
 * The conventional renderer it replaces, the dense march, stays available
 * as the quality reference of the reconstruction and as its fallback:
 *   - frame f is a check frame when check_every > 0 and f mod check_every
 *     == 0 (f counts the renderer's frames from 0); a check frame renders
 *     the foveated frame and the dense frame and scores the reconstruction
 *     by PSNR = 10 log10(1 / MSE), MSE over all pixels and RGB channels of
 *     values clamped to [0, 1] (FP64 sums in a fixed order), then
 *     synchronises the stream once to read it;
 *   - a check frame scoring below min_psnr_db (or NaN) puts the renderer in
 *     fallback and its output is the dense frame's RGB; one scoring at or
 *     above the threshold takes it out of fallback;
 *   - in fallback, frames between checks are dense frames (no sample map,
 *     no reconstruction).
 * The renderer owns every intermediate buffer (about 37 bytes a pixel plus
 * the march and network workspaces); it is single-stream like the other
 * handles.  Calls on one renderer must not overlap. */
typedef struct {
  int32_t precision;    /* FV_PREC_FP8, FV_PREC_BF16 or FV_RECON_PULLPUSH     */
  int32_t check_every;  /* >= 0; 0 = never check (never falls back)           */
  float min_psnr_db;    /* fallback threshold, finite                         */
} fv_render_policy;

typedef struct {
  uint64_t frame;       /* this frame's index in the renderer's sequence      */
  int32_t checked;      /* 1: the dense frame was marched and compared        */
  int32_t dense;        /* 1: out_rgb is the dense frame (fallback)           */
  int32_t fallback;     /* the renderer's state after this frame              */
  float psnr_db;        /* the reconstruction's PSNR on a check frame, else NaN */
} fv_frame_info;

typedef struct fv_renderer fv_renderer;

/* Errors: null pointers, views outside [1, 8], W or H not a multiple of 8 in
 * [8, 16384], views*W*H >= 2^32, check_every < 0 or a non-finite threshold
 * (FV_ERR_INVALID_ARG), an unknown precision (FV_ERR_UNSUPPORTED),
 * allocation failure (FV_ERR_NOMEM). */
fv_status fv_renderer_create(int views, int width, int height, const fv_render_policy* policy,
                             fv_renderer** out);
fv_status fv_renderer_destroy(fv_renderer* r);

/* One frame of the renderer's views: cams[views], the fovea parameters of
 * fv_fovea_mask, and the march parameters and transfer function of the
 * march calls.
 *   net      the reconstruction network (FP8 needs fv_net_calibrate first);
 *            may be NULL for FV_RECON_PULLPUSH
 *   out_rgb  dev float [views*H*W*3]
 *   info     host, filled on return
 * Errors: those of the calls it makes, and a NULL network for a network
 * precision (FV_ERR_INVALID_ARG). */
fv_status fv_render_frame(fv_renderer* r, const fv_volume* vol, const float* tf_rgba, int tf_n,
                          const fv_camera* cams, const fv_march_params* mp,
                          const fv_fovea_params* fp, const fv_net* net, float* out_rgb,
                          fv_frame_info* info, void* stream);

/* ------------------------------------------------------------------------
 * 4d. The two-stage W-Net (paper Sec. 3.2.1-3.2.3, Sec. 3.5.1), inference in
 *     BF16
 * ------------------------------------------------------------------------
 * Network D: a U-Net of 3x3 convs + ReLU with the paper's depth progression
 * e64-e64-e80-d96-d80-d64-d64 read as encoder 64/64/80/96 (two convs per
 * level, 2x2 average pooling between levels) and decoder 80/64/64 (bilinear
 * x2 upsampling with half-pixel centres, [upsampled, encoder skip]
 * concatenated); its last decoder state gives the direct prediction O_d by a
 * 1x1 conv (linear).  Network K: 1x1 convs on D's hidden states H_0..H_3 (the
 * decoder states at 1, 1/2, 1/4 resolution and the 1/8 bottleneck).  Its
 * encoder filters J_0 = O_d at level 0 with the softmax of 25 predicted
 * logits as a 5x5 kernel (replicated border, tap k = 5 (dy+2) + (dx+2)), pools
 * the result 2x2 into J_1, and so on to level 3; its decoder at level l
 * (2, 1, 0) predicts 25 logits and a blend logit z, forms
 * B = (1 - sigmoid(z)) Je_l + sigmoid(z) up(J_(l+1)) from the encoder's
 * filtered image Je_l and the upsampled coarser result, and filters B with
 * its kernel; the output is J_0.  The input is the 5-channel packed sparse
 * frame of section 4.
 * D runs on MFMA with BF16 operands and stored activations, FP32
 * accumulation; O_d and K in FP32.
 *
 * Parameters: FV_WNET_PARAMS floats, per layer the weight [Co][Ci][k][k]
 * then the bias [Co], in the order e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b
 * d1a d1b d0a d0b (3x3), hd (64 -> 3), ke0 ke1 ke2 ke3 (64/64/80/96 -> 25),
 * kd2 kd1 kd0 (80/64/64 -> 26, the 26th the blend logit). */
#define FV_WNET_PARAMS 798341
typedef struct fv_wnet fv_wnet;
size_t fv_wnet_param_count(void);
/* Uploads host FP32 parameters and builds D's BF16 weights; synchronises the
 * device.  Errors: null pointers, n_params neither FV_WNET_PARAMS nor
 * FV_WNET_PARAMS_RECURRENT (the recurrent form, below), allocation failure
 * (FV_ERR_NOMEM). */
fv_status fv_wnet_create(const float* host_params, size_t n_params, fv_wnet** out);
fv_status fv_wnet_destroy(fv_wnet* n);
/* Device workspace of fv_wnet_reconstruct at this size. */
fv_status fv_wnet_workspace(int views, int width, int height, size_t* bytes);
/* Full-frame reconstruction by the W-Net; arguments, layouts and errors as
 * fv_reconstruct (out_direct: O_d or NULL).  Error for a recurrent handle. */
fv_status fv_wnet_reconstruct(const fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                              const float* frame_depth, int views, int width, int height,
                              float* out_rgb, float* out_direct, void* workspace,
                              size_t ws_bytes, void* stream);

/* The recurrent W-Net (paper Sec. 3.2.4): a state carried from frame to
 * frame.  D's first conv also reads the previous frame's O_d (packed input
 * channels 5-7, as fv_reconstruct_recurrent), and the first conv of each
 * decoder block (d2, d1, d0) also reads that block's own output of the
 * previous frame, concatenated after [upsampled, skip]; the state is zero at
 * a sequence start.
 * Parameters: FV_WNET_PARAMS_RECURRENT floats, the order of the plain form
 * with e0a's Ci = 8 (the 5 frame channels, then O_d,prev RGB) and the
 * decoders' first convs reading [upsampled, skip, fed-back]: d2a 96+80+80,
 * d1a 80+64+64, d0a 64+64+64 input channels.  fv_wnet_create takes either
 * count and builds the form it names; fv_wnet_is_recurrent tells which.
 *
 * State: caller-owned device memory of fv_wnet_state_bytes, 256-byte
 * aligned, one per sequence (views x W x H).  Layout (fv_wnet_state_layout
 * gives the byte offsets): O_d float [views*H*W*3]; then d2b, d1b, d0b as
 * BF16 NHWC at 1/4, 1/2 and full resolution with 80, 64 and 64 channels.
 * fv_wnet_reconstruct_recurrent reads the state, runs the frame and leaves
 * this frame's O_d and decoder outputs in it; reset != 0 zeroes it first (a
 * sequence start).  Calls on one state must be issued in frame order on one
 * stream.  Other arguments as fv_wnet_reconstruct (out_direct: a copy of
 * O_d, or NULL).
 * Errors: as fv_wnet_reconstruct; a null or unaligned state; state_bytes too
 * small (FV_ERR_CAPACITY); a plain handle. */
#define FV_WNET_PARAMS_RECURRENT 931397
size_t fv_wnet_param_count_recurrent(void);
int fv_wnet_is_recurrent(const fv_wnet* n);
fv_status fv_wnet_state_bytes(int views, int width, int height, size_t* bytes);
fv_status fv_wnet_state_layout(int views, int width, int height, size_t* od_offset,
                               size_t* d2_offset, size_t* d1_offset, size_t* d0_offset);
fv_status fv_wnet_reconstruct_recurrent(const fv_wnet* n, const float* frame_rgba,
                                        const uint8_t* mask, const float* frame_depth,
                                        void* state, size_t state_bytes, int reset, int views,
                                        int width, int height, float* out_rgb,
                                        float* out_direct, void* workspace, size_t ws_bytes,
                                        void* stream);

/* Training of the (plain) W-Net on the GPU, BF16 like fv_train_step: the
 * forward keeps D's activations and K's per-level kernels, blend weights and
 * blends; the loss is fv_net_loss's (0.9 (1 - SSIM) + 0.1 L1); the backward
 * pass computes every parameter's gradient (D's convs on MFMA as
 * fv_net_backward; K's 5x5 applications, softmax, blends, pooling,
 * upsampling and 1x1 predictors in FP32), and fv_wnet_adam takes one Adam
 * step on the FP32 master (then rebuilds D's BF16 copies).  Reductions use
 * fixed orders, so a step is deterministic.  Frames at least 16 x 16,
 * multiples of 8.  Arguments and layouts as the fv_net training calls
 * (grad_out: dev float [the handle's parameter count] or NULL).  Errors:
 * those of the fv_net training calls; the state-less calls refuse a
 * recurrent handle (it has its own, below).
 * fv_wnet_get_params / fv_wnet_set_params copy the FP32 master to / from
 * the host (set rebuilds the BF16 copies and synchronises). */
fv_status fv_wnet_train_workspace(const fv_wnet* n, int batch, int width, int height,
                                  size_t* bytes);
fv_status fv_wnet_forward_train(fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                                const float* frame_depth, int batch, int width, int height,
                                float* out_rgb, void* workspace, size_t ws_bytes, void* stream);
fv_status fv_wnet_backward(fv_wnet* n, const float* dloss_dout, int batch, int width,
                           int height, float* grad_out, void* workspace, size_t ws_bytes,
                           void* stream);
fv_status fv_wnet_adam(fv_wnet* n, float lr, float beta1, float beta2, float eps, void* stream);
fv_status fv_wnet_train_step(fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                             const float* frame_depth, const float* target_rgba, int batch,
                             int width, int height, float lr, float* loss3, void* workspace,
                             size_t ws_bytes, void* stream);
/* The recurrent form trains on frames with their fed-back state given as
 * an input (the state is carried over one step, detached, as the
 * single-stage network's recurrent training): state has the layout of
 * fv_wnet_state_layout for `batch` views, entry b the state frame b reads;
 * it is only read, and must be passed unchanged to the backward call.
 * fv_wnet_loss (fv_wnet_loss_temporal) is fv_net_loss (fv_net_loss_temporal)
 * on the W-Net's training workspace (either form).  Errors: those above; a state for a plain handle or none for a
 * recurrent one. */
fv_status fv_wnet_forward_train_recurrent(fv_wnet* n, const float* frame_rgba,
                                          const uint8_t* mask, const float* frame_depth,
                                          const void* state, size_t state_bytes, int batch,
                                          int width, int height, float* out_rgb,
                                          void* workspace, size_t ws_bytes, void* stream);
fv_status fv_wnet_backward_recurrent(fv_wnet* n, const float* dloss_dout, const void* state,
                                     size_t state_bytes, int batch, int width, int height,
                                     float* grad_out, void* workspace, size_t ws_bytes,
                                     void* stream);
fv_status fv_wnet_loss(const fv_wnet* n, const float* out_rgb, const float* target_rgba,
                       int batch, int width, int height, float* loss3, float* dloss_dout,
                       void* workspace, size_t ws_bytes, void* stream);
/* fv_net_loss_temporal on the W-Net's training workspace. */
fv_status fv_wnet_loss_temporal(const fv_wnet* n, const float* out_rgb,
                                const float* target_rgba, int batch, int width, int height,
                                float weight, float* loss, float* dloss_dout, void* workspace,
                                size_t ws_bytes, void* stream);
fv_status fv_wnet_get_params(const fv_wnet* n, float* host_out, size_t n_params);
fv_status fv_wnet_set_params(fv_wnet* n, const float* host_params, size_t n_params);

/* ------------------------------------------------------------------------
 * 5. Training of the reconstruction network (paper: "Loss", "Training")
 * ------------------------------------------------------------------------
 * One workspace (fv_train_workspace) serves the four steps of a training
 * iteration on a batch of `batch` frames of W x H (multiples of 8, >= 16):
 *   fv_net_forward_train  BF16 forward that keeps every activation;
 *   fv_net_loss           L = 0.9 (1 - SSIM) + 0.1 L1 against the target
 *                         frames (the paper's 0.9 / 0.1 weights with SSIM in
 *                         place of the VGG19-LPIPS term), and d L / d out;
 *   fv_net_backward       gradient of sum(dloss_dout * out) w.r.t. all
 *                         parameters into the handle (and grad_out if given),
 *                         using the activations of the last forward_train;
 *   fv_net_adam           one Adam step on the FP32 master weights, then the
 *                         BF16 copy is rebuilt (the FP8 copy is invalidated).
 * SSIM: 11x11 Gaussian window (sigma 1.5), K1 = 0.01, K2 = 0.03, L = 1,
 * valid region, mean over pixels, channels and batch.  Reductions use fixed
 * orders, so a step is deterministic.  Calls that share a workspace must
 * be issued on one stream.
 *   out_rgb / dloss_dout   dev float [batch*H*W*3]
 *   target_rgba            dev float [batch*H*W*4] (dense frames; RGB used)
 *   loss3                  dev float [3] = {loss, SSIM, L1}
 *   grad_out               dev float [FV_NET_PARAMS or FV_NET_PARAMS_RECURRENT,
 *                          the handle's form] or NULL
 * Errors: null pointers, bad sizes, workspace too small (FV_ERR_CAPACITY),
 * hyper-parameters out of range (Adam: lr >= 0, betas in [0,1), eps > 0). */
fv_status fv_train_workspace(const fv_net* n, int batch, int width, int height,
                             size_t* bytes);
fv_status fv_net_forward_train(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                               const float* frame_depth, int batch, int width, int height,
                               float* out_rgb, void* workspace, size_t ws_bytes,
                               void* stream);
/* fv_net_forward_train for the recurrent form: entry b of the batch reads
 * prev_direct[b] (dev float [batch*H*W*3], or NULL for zeros) as its
 * previous frame's O_d.  The feedback is an input: fv_net_backward gives
 * no gradient through it (the state is carried over one step, detached).
 * Errors: those of fv_net_forward_train, and a non-NULL prev_direct for a
 * plain network. */
fv_status fv_net_forward_train_recurrent(fv_net* n, const float* frame_rgba,
                                         const uint8_t* mask, const float* frame_depth,
                                         const float* prev_direct, int batch, int width,
                                         int height, float* out_rgb, void* workspace,
                                         size_t ws_bytes, void* stream);
fv_status fv_net_loss(const fv_net* n, const float* out_rgb, const float* target_rgba,
                      int batch, int width, int height, float* loss3, float* dloss_dout,
                      void* workspace, size_t ws_bytes, void* stream);
/* Temporal loss, the finite-difference term of the paper's temporal loss
 * (Sec. 3.3.2; the optical-flow term is not included): batch entries
 * (2i, 2i+1) are consecutive frames t-1 and t of one sequence, and
 *   L_t = mean |(out_2i+1 - out_2i) - (target_2i+1 - target_2i)|
 * over pairs, pixels and RGB channels.  Writes L_t to loss[0] (dev float
 * [1]) and ADDS weight * d L_t / d out to dloss_dout, so it is called after
 * fv_net_loss (which writes dloss_dout), on the same stream and workspace.
 * Errors: as fv_net_loss, plus an odd batch and a negative or non-finite
 * weight. */
fv_status fv_net_loss_temporal(const fv_net* n, const float* out_rgb,
                               const float* target_rgba, int batch, int width,
                               int height, float weight, float* loss,
                               float* dloss_dout, void* workspace,
                               size_t ws_bytes, void* stream);
fv_status fv_net_backward(fv_net* n, const float* dloss_dout, int batch, int width,
                          int height, float* grad_out, void* workspace, size_t ws_bytes,
                          void* stream);
fv_status fv_net_adam(fv_net* n, float lr, float beta1, float beta2, float eps,
                      void* stream);
/* Replaces the handle's parameter gradient with a caller-supplied one:
 *   grad  dev float [n_params], the external layout of the handle's form
 *         (the layout of fv_net_backward's grad_out)
 * enqueued on `stream`; the next fv_net_adam applies it.  This is where a
 * gradient that was reduced outside the library (for instance over
 * data-parallel replicas) re-enters the handle.  Errors: null pointers,
 * n_params not the form's count. */
fv_status fv_net_set_grad(fv_net* n, const float* grad, size_t n_params, void* stream);

/* Checkpoints of the training state (the paper exports its trained network
 * for deployment, Sec. 3.4; here the blob also carries what training needs
 * to resume).  Blob layout, little-endian:
 *   64-byte header: the 8 characters "FOVOLNET", u32 version (1), u32 form
 *     (0 plain, 1 recurrent), u64 n_params, i64 Adam step, 32 zero bytes;
 *   then FP32 master weights, Adam first moments m and second moments v,
 *     n_params each, in the external parameter layout of the form.
 * fv_net_save with host_blob NULL stores the blob size in *bytes; otherwise
 * *bytes is the buffer size on entry (FV_ERR_CAPACITY if too small) and the
 * blob size on return.  It reads the device state synchronously, so the
 * caller first synchronises the streams that updated the handle.
 * fv_net_load creates a handle from a blob, as fv_net_create does, with the
 * Adam moments and step restored: training resumes exactly where the saved
 * handle stood (the FP8 copy needs fv_net_calibrate again).  Errors: null
 * pointers, a short blob, a bad magic, form or parameter count, a negative
 * step (FV_ERR_INVALID_ARG), an unknown version (FV_ERR_UNSUPPORTED),
 * allocation failure (FV_ERR_NOMEM). */
fv_status fv_net_save(const fv_net* n, void* host_blob, size_t* bytes);
fv_status fv_net_load(const void* host_blob, size_t bytes, fv_net** out);

/* forward_train + loss + backward + Adam (beta 0.9 / 0.999, eps 1e-8).  A
 * recurrent network is trained here with a zero fed-back O_d. */
fv_status fv_train_step(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                        const float* frame_depth, const float* target_rgba, int batch,
                        int width, int height, float lr, float* loss3, void* workspace,
                        size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FOVOL_H */
