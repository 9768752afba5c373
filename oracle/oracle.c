/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the foveated sample map,
 * stream compaction and the direct-volume ray marcher.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; it is written
 * from the definitions of the method (FoVolNet, arXiv 2209.09965) and the
 * readings listed with each function.
 *
 * Everything is IEEE double.  Inputs that the GPU receives as float32
 * (camera, transfer function, parameters) are passed here already widened,
 * so both sides start from identical values.
 *
 * Built with gcc (no -ffast-math), OpenMP over independent pixels.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ noise */

/* MurmurHash3 32-bit finaliser (Appleby, public domain). */
uint32_t or_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* The noise N(u,v) that drives the sample map ("Noise Patterns"): the paper
 * uses pre-computed blue-noise tiles; here it is seeded white noise, a 24-bit
 * integer from a hash of the key (seed, frame, view, y, x).  The frame is in
 * the key so the pattern changes every frame, as the paper requires. */
uint32_t or_noise24(uint64_t seed, uint32_t frame, uint32_t view, uint32_t y,
                    uint32_t x) {
  uint32_t words[6];
  words[0] = (uint32_t)(seed & 0xffffffffu);
  words[1] = (uint32_t)(seed >> 32);
  words[2] = frame;
  words[3] = view;
  words[4] = y;
  words[5] = x;
  uint32_t h = 0x6A09E667u;
  for (int i = 0; i < 6; ++i) h = or_fmix32(h ^ words[i]);
  return h >> 8;
}

/* ------------------------------------------------------ threshold (tau) */

#define OR_LUT_MAX 16384
#define OR_ONE24 16777216.0 /* 2^24 */

/* tau as a function of R, the squared distance to the focus in doubled
 * pixel units (R/4 = r^2 px^2).
 * Eq. (1): fovea density, read as a Gaussian of the distance to the focus
 *          whose spread is sigma: g = exp(-r^2 / (2 sigma^2)).
 * Eq. (2): tau = (1 - P_b) P_f + P_b          (mode 1, "lerp")
 * clamp:   tau = max(P_f, P_b)                (mode 0) */
static double or_tau(double R, double sigma, double p_floor, int mode) {
  double r2 = R / 4.0;
  double g = exp(-r2 / (2.0 * sigma * sigma));
  if (mode == 1) return (1.0 - p_floor) * g + p_floor;
  return g > p_floor ? g : p_floor;
}

/* Threshold quantised to the noise's 24-bit range. */
static uint32_t or_tau_q(double R, double sigma, double p_floor, int mode) {
  double t = floor(or_tau(R, sigma, p_floor, mode) * OR_ONE24);
  if (t > OR_ONE24) t = OR_ONE24;
  if (t < 0.0) t = 0.0;
  return (uint32_t)t;
}

static int64_t or_round_half_away(double v) { return (int64_t)llround(v); }

/* Bound on R for any pixel centre of a W x H frame and any focus inside
 * [0,W]x[0,H]: |2x+1-F2x| <= 2W-1 and |2y+1-F2y| <= 2H-1. */
static int64_t or_rmax(int W, int H) {
  int64_t mx = (int64_t)2 * W - 1, my = (int64_t)2 * H - 1;
  return mx * mx + my * my;
}

/* Builds the threshold table exactly as the library's ABI header defines
 * it.  Returns 0 on success, -1 if no shift fits (cannot happen for frames
 * up to 2^31 px across). */
int or_fovea_lut(int W, int H, double focus_x, double focus_y, double sigma,
                 double p_floor, int mode, uint32_t* lut, int* n_out,
                 int* sh_out, uint32_t* tinf_out) {
  (void)focus_x;
  (void)focus_y; /* the table does not depend on the focus */
  int64_t rmax = or_rmax(W, H);
  double tinf_d = floor(p_floor * OR_ONE24);
  if (tinf_d > OR_ONE24) tinf_d = OR_ONE24;
  uint32_t tinf = (uint32_t)tinf_d;
  for (int sh = 0; sh < 63; ++sh) {
    int64_t cap = (rmax >> sh) + 1;
    int64_t n = 0;
    while (n < cap && n <= OR_LUT_MAX) {
      uint32_t t = or_tau_q((double)(n << sh), sigma, p_floor, mode);
      if (t == tinf) break;
      ++n;
    }
    if (n <= OR_LUT_MAX) {
      for (int64_t k = 0; k < n; ++k)
        lut[k] = or_tau_q((double)(k << sh), sigma, p_floor, mode);
      *n_out = (int)n;
      *sh_out = sh;
      *tinf_out = tinf;
      return 0;
    }
  }
  return -1;
}

/* ---------------------------------------------- sample map + compaction */

/* Sample map M = [N < tau] ("Sample Maps") followed by stream compaction
 * ("Stream Compaction"): the selected pixels are listed in the order view,
 * 8x8 tile (row-major over tiles), row-major inside the tile.  mask may be
 * NULL; idx must hold views*W*H entries.  Returns the count, or -1. */
/* Sample map + compaction.  The uniform number of each pixel is the seeded
 * hash, or, when `tiles` is given, the entry of the noise tile stack that
 * the paper's tileable textures stand for (Sec. 3.1.1): tile
 * (frame + view) mod tile_count, repeated over the frame. */
int64_t or_fovea_mask_src(uint64_t seed, uint32_t frame, int W, int H, int views,
                          double focus_x, double focus_y, double sigma,
                          double p_floor, int mode, const uint32_t* tiles, int tw,
                          int th, int tcount, uint8_t* mask, uint32_t* idx) {
  uint32_t* lut = (uint32_t*)malloc(sizeof(uint32_t) * OR_LUT_MAX);
  int n, sh;
  uint32_t tinf;
  if (!lut) return -1;
  if (or_fovea_lut(W, H, focus_x, focus_y, sigma, p_floor, mode, lut, &n, &sh,
                   &tinf) != 0) {
    free(lut);
    return -1;
  }
  int64_t f2x = or_round_half_away(2.0 * focus_x);
  int64_t f2y = or_round_half_away(2.0 * focus_y);
  int64_t count = 0;
  int tiles_x = (W + 7) / 8, tiles_y = (H + 7) / 8;
  for (int v = 0; v < views; ++v)
    for (int ty = 0; ty < tiles_y; ++ty)
      for (int tx = 0; tx < tiles_x; ++tx)
        for (int y = ty * 8; y < ty * 8 + 8 && y < H; ++y)
          for (int x = tx * 8; x < tx * 8 + 8 && x < W; ++x) {
            int64_t dx = (int64_t)2 * x + 1 - f2x, dy = (int64_t)2 * y + 1 - f2y;
            int64_t R = dx * dx + dy * dy;
            int64_t k = R >> sh;
            uint32_t T = k < n ? lut[k] : tinf;
            uint32_t u;
            if (tiles) {
              uint32_t ti = (frame + (uint32_t)v) % (uint32_t)tcount;
              u = tiles[((size_t)ti * th + (size_t)(y % th)) * tw + (size_t)(x % tw)];
            } else {
              u = or_noise24(seed, frame, (uint32_t)v, (uint32_t)y, (uint32_t)x);
            }
            int m = u < T;
            uint64_t lin = (uint64_t)v * W * H + (uint64_t)y * W + x;
            if (mask) mask[lin] = (uint8_t)m;
            if (m) idx[count++] = (uint32_t)lin;
          }
  free(lut);
  return count;
}

int64_t or_fovea_mask(uint64_t seed, uint32_t frame, int W, int H, int views,
                      double focus_x, double focus_y, double sigma,
                      double p_floor, int mode, uint8_t* mask, uint32_t* idx) {
  return or_fovea_mask_src(seed, frame, W, H, views, focus_x, focus_y, sigma, p_floor,
                           mode, NULL, 0, 0, 0, mask, idx);
}

/* Mean of tau over the frame: C_max of Eq. (3), the expected sampled
 * fraction (the sum's bounds are read as the h*w pixels).  Unquantised. */
double or_cmax(int W, int H, double focus_x, double focus_y, double sigma,
               double p_floor, int mode) {
  int64_t f2x = or_round_half_away(2.0 * focus_x);
  int64_t f2y = or_round_half_away(2.0 * focus_y);
  double s = 0.0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t dx = (int64_t)2 * x + 1 - f2x, dy = (int64_t)2 * y + 1 - f2y;
      s += or_tau((double)(dx * dx + dy * dy), sigma, p_floor, mode);
    }
  return s / ((double)W * H);
}

/* --------------------------------------------------------------- volume */

/* IEEE 754 binary16 -> double, from the format's definition. */
static double or_half(uint16_t b) {
  int s = (b >> 15) & 1, e = (b >> 10) & 31, m = b & 1023;
  double v;
  if (e == 0)
    v = ldexp((double)m, -24);
  else if (e == 31)
    v = m ? NAN : INFINITY;
  else
    v = ldexp(1024.0 + m, e - 25);
  return s ? -v : v;
}

typedef struct {
  const void* data;
  int n[3];
  int dtype; /* 0 u8, 1 f16, 2 f32 */
  double h;  /* voxel edge */
} or_vol;

static double or_voxel(const or_vol* V, int i, int j, int k) {
  /* clamp-to-edge */
  if (i < 0) i = 0;
  if (i > V->n[0] - 1) i = V->n[0] - 1;
  if (j < 0) j = 0;
  if (j > V->n[1] - 1) j = V->n[1] - 1;
  if (k < 0) k = 0;
  if (k > V->n[2] - 1) k = V->n[2] - 1;
  size_t lin = ((size_t)k * V->n[1] + j) * V->n[0] + i;
  if (V->dtype == 0) return ((const uint8_t*)V->data)[lin] / 255.0;
  if (V->dtype == 1) return or_half(((const uint16_t*)V->data)[lin]);
  return (double)((const float*)V->data)[lin];
}

/* Trilinear interpolation at q (voxel index space: voxel centres at
 * integers), sum over the 8 corners of the product of 1-D weights. */
static double or_trilinear(const or_vol* V, const double q[3]) {
  double fl[3], w[3];
  int i0[3];
  for (int a = 0; a < 3; ++a) {
    fl[a] = floor(q[a]);
    i0[a] = (int)fl[a];
    w[a] = q[a] - fl[a];
  }
  double v = 0.0;
  for (int c = 0; c < 8; ++c) {
    int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    double wt = (cx ? w[0] : 1.0 - w[0]) * (cy ? w[1] : 1.0 - w[1]) *
                (cz ? w[2] : 1.0 - w[2]);
    v += wt * or_voxel(V, i0[0] + cx, i0[1] + cy, i0[2] + cz);
  }
  return v;
}

/* --------------------------------------------------------------- camera */

typedef struct {
  double eye[3], target[3], up[3], fovy_deg, eye_offset;
} or_cam;

static void or_cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double or_dot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void or_normalize(double a[3]) {
  double l = sqrt(or_dot(a, a));
  a[0] /= l;
  a[1] /= l;
  a[2] /= l;
}

/* Pinhole ray through the centre of pixel (x, y). */
static void or_ray(const or_cam* c, int W, int H, int x, int y, double o[3],
                   double d[3]) {
  double f[3], r[3], u[3];
  for (int a = 0; a < 3; ++a) f[a] = c->target[a] - c->eye[a];
  or_normalize(f);
  or_cross(f, c->up, r);
  or_normalize(r);
  or_cross(r, f, u);
  double th = tan(c->fovy_deg * M_PI / 360.0);
  double px = (2.0 * (x + 0.5) / W - 1.0) * th * ((double)W / H);
  double py = (1.0 - 2.0 * (y + 0.5) / H) * th;
  for (int a = 0; a < 3; ++a) d[a] = f[a] + px * r[a] + py * u[a];
  or_normalize(d);
  for (int a = 0; a < 3; ++a) o[a] = c->eye[a] + c->eye_offset * r[a];
}

/* Slab test against the box [-n_a h/2, n_a h/2]; returns 0 on a miss. */
static int or_slab(const or_vol* V, const double o[3], const double d[3],
                   double* t0, double* t1) {
  double tn = -INFINITY, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double b = V->n[a] * V->h / 2.0;
    if (d[a] == 0.0) {
      if (o[a] < -b || o[a] > b) return 0;
      continue;
    }
    double ta = (-b - o[a]) / d[a], tb = (b - o[a]) / d[a];
    double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
    if (lo > tn) tn = lo;
    if (hi < tf) tf = hi;
  }
  if (tn < 0.0) tn = 0.0;
  if (!(tf > tn)) return 0;
  *t0 = tn;
  *t1 = tf;
  return 1;
}

/* ---------------------------------------------------------------- march */

typedef struct {
  double step, alpha_stop;
  int shading;
  double light[3], ka, kd, ks, shininess, bg[3];
  double shadow_step; /* shadow-ray segment length in voxels, 0 = no shadows */
} or_mp;

/* TF opacity channel (sigma) at value v: linear interpolation between the
 * 256 entries at clamp(v, 0, 1) * 255. */
static double or_tf_sigma(const double* tf, double v) {
  double xv = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
  xv *= 255.0;
  int j = (int)floor(xv);
  if (j > 254) j = 254;
  double f = xv - j;
  return (1.0 - f) * tf[j * 4 + 3] + f * tf[(j + 1) * 4 + 3];
}

/* Global ray-marched shadow (paper Sec. 3.1 "Foveated Rendering": one shadow
 * ray per sample, towards the light, at a lower sample rate).  Reading: a
 * directional light; the shadow ray leaves the sample point p (voxel index
 * space, where the box is [-1/2, n_a - 1/2] on axis a) along the unit light
 * direction lhat and ends where it leaves the box, after L voxel lengths.
 * It is cut into ceil(L / ds) segments of length ds (the last one shorter),
 * each sampled at its midpoint like the primary ray, and the light reaching
 * p is attenuated by the transmittance exp(-sum sigma_j len_j). */
static double or_shadow(const or_vol* V, const double* tf, const double q[3],
                        const double lhat[3], double ds) {
  double L = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (lhat[a] == 0.0) continue;
    double face = lhat[a] > 0.0 ? V->n[a] - 0.5 : -0.5;
    double t = (face - q[a]) / lhat[a];
    if (t < L) L = t;
  }
  if (!(L > 0.0)) return 1.0;
  int64_t N = (int64_t)ceil(L / ds);
  double tau = 0.0;
  for (int64_t j = 0; j < N; ++j) {
    double a0 = j * ds, b0 = (j + 1) * ds;
    if (b0 > L) b0 = L;
    double m = 0.5 * (a0 + b0), qs[3];
    for (int a = 0; a < 3; ++a) qs[a] = q[a] + m * lhat[a];
    tau += or_tf_sigma(tf, or_trilinear(V, qs)) * (b0 - a0);
  }
  return exp(-tau);
}

typedef struct {
  double rgba[4];
  double depth;
  int64_t samples;
} or_px;

/* One ray, front-to-back emission-absorption compositing with early
 * termination at threshold `stop`.  The paper gives the renderer only as a
 * ray marcher; the sampling, transfer function, shading and compositing
 * rules are the readings documented in the library header. */
static void or_march_ray(const or_vol* V, const double* tf, const or_mp* mp,
                         const double o[3], const double d[3], double stop,
                         or_px* out) {
  double t0, t1;
  out->depth = 0.0;
  out->samples = 0;
  if (!or_slab(V, o, d, &t0, &t1)) {
    out->rgba[0] = mp->bg[0];
    out->rgba[1] = mp->bg[1];
    out->rgba[2] = mp->bg[2];
    out->rgba[3] = 0.0;
    return;
  }
  double h = V->h;
  double L = (t1 - t0) / h; /* in voxel lengths */
  int64_t N = (int64_t)ceil(L / mp->step);
  double Lhat[3], Vv[3], Hv[3];
  if (mp->shading) {
    for (int a = 0; a < 3; ++a) Lhat[a] = mp->light[a];
    or_normalize(Lhat);
    for (int a = 0; a < 3; ++a) {
      Vv[a] = -d[a];
      Hv[a] = Lhat[a] + Vv[a];
    }
    double hl = sqrt(or_dot(Hv, Hv));
    if (hl < 1e-30) hl = 1e-30;
    for (int a = 0; a < 3; ++a) Hv[a] /= hl;
  }
  double C[3] = {0, 0, 0}, T = 1.0, D = 0.0;
  for (int64_t k = 0; k < N; ++k) {
    double a0 = k * mp->step;
    double b0 = (k + 1) * mp->step;
    if (b0 > L) b0 = L;
    double len = b0 - a0;
    double m = 0.5 * (a0 + b0);
    double t = t0 + h * m;
    double p[3], q[3];
    for (int a = 0; a < 3; ++a) {
      p[a] = o[a] + d[a] * t;
      q[a] = (p[a] + V->n[a] * h / 2.0) / h - 0.5;
    }
    double v = or_trilinear(V, q);
    /* transfer function, linear interpolation between entries */
    double xv = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    xv *= 255.0;
    int j = (int)floor(xv);
    if (j > 254) j = 254;
    double f = xv - j;
    double c4[4];
    for (int ch = 0; ch < 4; ++ch)
      c4[ch] = (1.0 - f) * tf[j * 4 + ch] + f * tf[(j + 1) * 4 + ch];
    double alpha = 1.0 - exp(-c4[3] * len);
    double col[3] = {c4[0], c4[1], c4[2]};
    if (mp->shading) {
      double g[3];
      for (int a = 0; a < 3; ++a) {
        double qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
        qp[a] += 1.0;
        qm[a] -= 1.0;
        g[a] = (or_trilinear(V, qp) - or_trilinear(V, qm)) / 2.0;
      }
      double gl = sqrt(or_dot(g, g));
      if (gl < 1e-4) gl = 1e-4;
      double nrm[3] = {-g[0] / gl, -g[1] / gl, -g[2] / gl};
      double ndl = fabs(or_dot(nrm, Lhat));
      double ndh = fabs(or_dot(nrm, Hv));
      double spec = mp->ks * pow(ndh, mp->shininess);
      /* with shadows, the light reaching the sample (diffuse and specular
       * terms) is attenuated; the ambient term is not */
      double ts = mp->shadow_step > 0.0 ? or_shadow(V, tf, q, Lhat, mp->shadow_step) : 1.0;
      for (int ch = 0; ch < 3; ++ch)
        col[ch] = c4[ch] * (mp->ka + ts * (mp->kd * ndl)) + ts * spec;
    }
    double w = T * alpha;
    for (int ch = 0; ch < 3; ++ch) C[ch] += w * col[ch];
    D += w * t;
    T *= (1.0 - alpha);
    out->samples++;
    if (1.0 - T >= stop) break;
  }
  for (int ch = 0; ch < 3; ++ch) out->rgba[ch] = C[ch] + T * mp->bg[ch];
  out->rgba[3] = 1.0 - T;
  out->depth = D;
}

/* March a list of pixels.
 *   vol    raw volume, x fastest (dtype 0 u8, 1 f16, 2 f32)
 *   tf     256*4 doubles (r, g, b, sigma)
 *   cams   views*11 doubles: eye[3] target[3] up[3] fovy_deg eye_offset
 *   mpv    14 doubles: step alpha_stop shading light[3] ka kd ks shininess bg[3]
 *          shadow_step (0 = no shadows)
 *   idx    pixel indices (v*W*H + y*W + x), or NULL for all pixels in order
 *   rgba   n*4, depth n, samples n (any of these may be NULL)
 *   flags, rgba_lo, rgba_hi: if non-NULL, the ray is also marched with the
 *          threshold moved by -eps and +eps; flags[i] = 1 when the number of
 *          samples differs, i.e. the early-termination decision sits within
 *          eps of the threshold and either branch is a correct result. */
int or_march(const void* vol, int nx, int ny, int nz, int dtype,
             const double* tf, const double* cams, int views, int W, int H,
             const double* mpv, const uint32_t* idx, int64_t n, double* rgba,
             double* depth, int64_t* samples, uint8_t* flags, double* rgba_lo,
             double* rgba_hi, double eps) {
  or_vol V;
  V.data = vol;
  V.n[0] = nx;
  V.n[1] = ny;
  V.n[2] = nz;
  V.dtype = dtype;
  int nmax = nx > ny ? nx : ny;
  if (nz > nmax) nmax = nz;
  V.h = 1.0 / nmax;
  or_mp mp;
  mp.step = mpv[0];
  mp.alpha_stop = mpv[1];
  mp.shading = mpv[2] != 0.0;
  for (int a = 0; a < 3; ++a) mp.light[a] = mpv[3 + a];
  mp.ka = mpv[6];
  mp.kd = mpv[7];
  mp.ks = mpv[8];
  mp.shininess = mpv[9];
  for (int a = 0; a < 3; ++a) mp.bg[a] = mpv[10 + a];
  mp.shadow_step = mpv[13];
  int64_t total = (int64_t)views * W * H;
  if (!idx) n = total;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t lin = idx ? (int64_t)idx[i] : i;
    if (lin < 0 || lin >= total) continue;
    int v = (int)(lin / ((int64_t)W * H));
    int64_t rem = lin % ((int64_t)W * H);
    int y = (int)(rem / W), x = (int)(rem % W);
    or_cam c;
    const double* cv = cams + (size_t)v * 11;
    for (int a = 0; a < 3; ++a) {
      c.eye[a] = cv[a];
      c.target[a] = cv[3 + a];
      c.up[a] = cv[6 + a];
    }
    c.fovy_deg = cv[9];
    c.eye_offset = cv[10];
    double o[3], d[3];
    or_ray(&c, W, H, x, y, o, d);
    or_px px;
    or_march_ray(&V, tf, &mp, o, d, mp.alpha_stop, &px);
    if (rgba)
      for (int ch = 0; ch < 4; ++ch) rgba[i * 4 + ch] = px.rgba[ch];
    if (depth) depth[i] = px.depth;
    if (samples) samples[i] = px.samples;
    if (flags) {
      or_px lo, hi;
      or_march_ray(&V, tf, &mp, o, d, mp.alpha_stop - eps, &lo);
      or_march_ray(&V, tf, &mp, o, d, mp.alpha_stop + eps, &hi);
      flags[i] = (uint8_t)(lo.samples != hi.samples);
      if (rgba_lo)
        for (int ch = 0; ch < 4; ++ch) rgba_lo[i * 4 + ch] = lo.rgba[ch];
      if (rgba_hi)
        for (int ch = 0; ch < 4; ++ch) rgba_hi[i * 4 + ch] = hi.rgba[ch];
    }
  }
  return 0;
}

/* Shadow transmittance at voxel-index position q towards the light
 * direction (normalised here), exposed for pin tests. */
double or_shadow_at(const void* vol, int nx, int ny, int nz, int dtype, const double* tf,
                    double qx, double qy, double qz, double lx, double ly, double lz,
                    double ds) {
  or_vol V;
  V.data = vol;
  V.n[0] = nx;
  V.n[1] = ny;
  V.n[2] = nz;
  V.dtype = dtype;
  int nmax = nx > ny ? nx : ny;
  if (nz > nmax) nmax = nz;
  V.h = 1.0 / nmax;
  double l[3] = {lx, ly, lz}, q[3] = {qx, qy, qz};
  or_normalize(l);
  return or_shadow(&V, tf, q, l, ds);
}

/* Single trilinear sample, exposed for pin tests. */
double or_sample(const void* vol, int nx, int ny, int nz, int dtype, double qx,
                 double qy, double qz) {
  or_vol V;
  V.data = vol;
  V.n[0] = nx;
  V.n[1] = ny;
  V.n[2] = nz;
  V.dtype = dtype;
  V.h = 1.0;
  double q[3] = {qx, qy, qz};
  return or_trilinear(&V, q);
}

/* Back-projection and network input ("Stream Compaction": the compact
 * results go back to their pixels; the network sees the sparse frame).
 * in5 = [M*r, M*g, M*b, M, M*depth/2] per pixel, pixel-major (idx*5 + c). */
void or_pack_input(const double* frame_rgba, const uint8_t* mask,
                   const double* frame_depth, int64_t npx, double* in5) {
  for (int64_t i = 0; i < npx; ++i) {
    double m = mask[i] ? 1.0 : 0.0;
    in5[i * 5 + 0] = m * frame_rgba[i * 4 + 0];
    in5[i * 5 + 1] = m * frame_rgba[i * 4 + 1];
    in5[i * 5 + 2] = m * frame_rgba[i * 4 + 2];
    in5[i * 5 + 3] = m;
    in5[i * 5 + 4] = m * frame_depth[i] / 2.0;
  }
}
