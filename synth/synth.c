/*
 * Seeded synthetic inputs for the densification hot path: scene-like RGB views
 * and 3D Gaussian sets with a split-selection mask.
 *
 * This module is an input source only. It holds none of the method's
 * arithmetic (no grayscale, blur, gradient, suppression, median or split
 * step); it is the one piece of code that both the CPU oracle and the GPU
 * path may use, so that both see the very same bytes.
 *
 * Image recipe (one view, W x H, values in DN):
 *   background : linear blend between two random colours along a random
 *                direction theta, t clipped to [0, 1];
 *   polygons   : n_poly random star-shaped polygons (3..8 vertices, radius
 *                U[0.03, 0.25] * min(W, H)), filled by the even-odd rule at
 *                pixel centres in painter's order with a uniform random
 *                colour; with texture on, even-indexed polygons also get
 *                amp * sin(2 pi f (x cos a + y sin a) + phi), f ~ U[1/64, 1/8];
 *   noise      : N(0, sigma^2) per channel, then round-to-nearest, clip to
 *                [0, 255].
 * Gaussians: means U[-1,1]^3, log-scales N(mu, sd^2) per axis, quaternion
 * normalise(N(0,1)^4) stored (w,x,y,z), opacity u ~ U(0,1) stored as
 * logit(u); mask: exactly K distinct rows by a partial Fisher-Yates shuffle.
 *
 * Every random draw comes from SplitMix64 (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014), used in two ways:
 * as a sequential stream for the few per-view scene parameters, and as a
 * counter-based hash (key, index) for the per-pixel noise, so that output
 * bytes do not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_PI 3.14159265358979323846

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline uint64_t rng_next(rng_t* r) {
  r->s += 0x9E3779B97F4A7C15ULL;
  return mix64(r->s);
}
/* uniform double in [0, 1) with 53 random bits */
static inline double rng_u01(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
static inline double rng_uniform(rng_t* r, double a, double b) { return a + (b - a) * rng_u01(r); }
/* uniform integer in [lo, hi] (inclusive); modulo bias is below 2^-40 here */
static inline int64_t rng_int(rng_t* r, int64_t lo, int64_t hi) {
  return lo + (int64_t)(rng_next(r) % (uint64_t)(hi - lo + 1));
}
/* standard normal, Box-Muller (one of the pair; simple and plain) */
static double rng_normal(rng_t* r) {
  double u1 = 1.0 - rng_u01(r); /* (0, 1] */
  double u2 = rng_u01(r);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * SYN_PI * u2);
}

/* counter-based: uniform in (0,1] and [0,1) from (key, counter) */
static inline double hash_u01(uint64_t key, uint64_t ctr) {
  return (double)(mix64(key ^ mix64(ctr * 0x9E3779B97F4A7C15ULL + 0xD1B54A32D192ED03ULL)) >> 11) * 0x1.0p-53;
}

typedef struct {
  int nv;
  double vx[8], vy[8];
  double col[3];
  int textured;
  double f, ca, sa, phi, amp;
} poly_t;

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/*
 * Render one view into a float working buffer acc[H*W*3] (before noise),
 * then add noise and quantise into out (uint8, HWC, packed rows).
 */
static void render_view(uint64_t seed, int W, int H, int n_poly, int texture, double tex_amp,
                        double noise_sigma, uint8_t* out) {
  rng_t r = {seed * 0x2545F4914F6CDD1DULL + 0x632BE59BD9B4E019ULL};
  (void)rng_next(&r);
  double c0[3], c1[3];
  for (int c = 0; c < 3; ++c) c0[c] = rng_uniform(&r, 0.0, 255.0);
  for (int c = 0; c < 3; ++c) c1[c] = rng_uniform(&r, 0.0, 255.0);
  double th = rng_uniform(&r, 0.0, 2.0 * SYN_PI);
  double ct = cos(th), st = sin(th);
  double den = fabs((double)W * ct) + fabs((double)H * st);

  float* acc = (float*)malloc((size_t)W * H * 3 * sizeof(float));
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      double t = (((x + 0.5) - 0.5 * W) * ct + ((y + 0.5) - 0.5 * H) * st) / den + 0.5;
      if (t < 0.0) t = 0.0;
      if (t > 1.0) t = 1.0;
      float* p = acc + ((size_t)y * W + x) * 3;
      for (int c = 0; c < 3; ++c) p[c] = (float)(c0[c] + (c1[c] - c0[c]) * t);
    }
  }

  double mn = (double)(W < H ? W : H);
  double xs[16];
  for (int k = 0; k < n_poly; ++k) {
    poly_t P;
    double cx = rng_uniform(&r, 0.0, (double)W);
    double cy = rng_uniform(&r, 0.0, (double)H);
    double R = rng_uniform(&r, 0.03, 0.25) * mn;
    P.nv = (int)rng_int(&r, 3, 8);
    double ang[8];
    for (int i = 0; i < P.nv; ++i) ang[i] = rng_uniform(&r, 0.0, 2.0 * SYN_PI);
    qsort(ang, (size_t)P.nv, sizeof(double), cmp_double);
    for (int i = 0; i < P.nv; ++i) {
      double rad = R * rng_uniform(&r, 0.5, 1.0);
      P.vx[i] = cx + rad * cos(ang[i]);
      P.vy[i] = cy + rad * sin(ang[i]);
    }
    for (int c = 0; c < 3; ++c) P.col[c] = rng_uniform(&r, 0.0, 255.0);
    P.textured = texture && (k % 2 == 0);
    P.f = rng_uniform(&r, 1.0 / 64.0, 1.0 / 8.0);
    double a = rng_uniform(&r, 0.0, 2.0 * SYN_PI);
    P.ca = cos(a);
    P.sa = sin(a);
    P.phi = rng_uniform(&r, 0.0, 2.0 * SYN_PI);
    P.amp = tex_amp;

    /* scanline even-odd fill at pixel centres */
    double ymin = P.vy[0], ymax = P.vy[0];
    for (int i = 1; i < P.nv; ++i) {
      if (P.vy[i] < ymin) ymin = P.vy[i];
      if (P.vy[i] > ymax) ymax = P.vy[i];
    }
    int y0 = (int)floor(ymin - 0.5), y1 = (int)ceil(ymax - 0.5);
    if (y0 < 0) y0 = 0;
    if (y1 > H - 1) y1 = H - 1;
    for (int y = y0; y <= y1; ++y) {
      double yc = y + 0.5;
      int nx = 0;
      for (int i = 0; i < P.nv; ++i) {
        int j = (i + 1) % P.nv;
        double ya = P.vy[i], yb = P.vy[j];
        if ((ya <= yc) != (yb <= yc)) {
          xs[nx++] = P.vx[i] + (yc - ya) * (P.vx[j] - P.vx[i]) / (yb - ya);
        }
      }
      qsort(xs, (size_t)nx, sizeof(double), cmp_double);
      for (int s = 0; s + 1 < nx; s += 2) {
        int xa = (int)ceil(xs[s] - 0.5), xb = (int)ceil(xs[s + 1] - 0.5); /* centres in [xs, xe) */
        if (xa < 0) xa = 0;
        if (xb > W) xb = W;
        for (int x = xa; x < xb; ++x) {
          float* p = acc + ((size_t)y * W + x) * 3;
          double tex = 0.0;
          if (P.textured)
            tex = P.amp * sin(2.0 * SYN_PI * P.f * ((x + 0.5) * P.ca + yc * P.sa) + P.phi);
          for (int c = 0; c < 3; ++c) p[c] = (float)(P.col[c] + tex);
        }
      }
    }
  }

  uint64_t nkey = mix64(seed ^ 0xA0761D6478BD642FULL);
  size_t nval = (size_t)W * H * 3;
  for (size_t i = 0; i < nval; i += 2) {
    /* one Box-Muller pair per two consecutive channel values */
    double u1 = 1.0 - hash_u01(nkey, 2 * (i / 2));
    double u2 = hash_u01(nkey, 2 * (i / 2) + 1);
    double rr = sqrt(-2.0 * log(u1));
    double z0 = rr * cos(2.0 * SYN_PI * u2), z1 = rr * sin(2.0 * SYN_PI * u2);
    for (size_t k = 0; k < 2 && i + k < nval; ++k) {
      double v = (double)acc[i + k] + noise_sigma * (k == 0 ? z0 : z1);
      v = floor(v + 0.5);
      if (v < 0.0) v = 0.0;
      if (v > 255.0) v = 255.0;
      out[i + k] = (uint8_t)v;
    }
  }
  free(acc);
}

/* one view, W x H, written to out[H*W*3] */
void syn_image(uint64_t seed, int32_t W, int32_t H, int32_t n_poly, int32_t texture, double tex_amp,
               double noise_sigma, uint8_t* out) {
  render_view(seed, W, H, n_poly, texture, tex_amp, noise_sigma, out);
}

/*
 * Render at (W, H), then 2x2 box-downsample (mean of the four bytes, rounded
 * half up) to (W/2, H/2) written to out.
 */
void syn_image_down2(uint64_t seed, int32_t W, int32_t H, int32_t n_poly, int32_t texture, double tex_amp,
                     double noise_sigma, uint8_t* out) {
  uint8_t* full = (uint8_t*)malloc((size_t)W * H * 3);
  render_view(seed, W, H, n_poly, texture, tex_amp, noise_sigma, full);
  int w = W / 2, h = H / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x)
      for (int c = 0; c < 3; ++c) {
        int s = full[((size_t)(2 * y) * W + 2 * x) * 3 + c] + full[((size_t)(2 * y) * W + 2 * x + 1) * 3 + c] +
                full[((size_t)(2 * y + 1) * W + 2 * x) * 3 + c] + full[((size_t)(2 * y + 1) * W + 2 * x + 1) * 3 + c];
        out[((size_t)y * w + x) * 3 + c] = (uint8_t)((s + 2) / 4);
      }
  free(full);
}

/*
 * A batch of views into one packed buffer. For view v: seeds[v], full size
 * (fw[v], fh[v]), down2[v] != 0 selects the 2x downsample, and the bytes go to
 * out + offsets[v]. Views are rendered in parallel, each by one thread.
 */
void syn_image_batch(int32_t n, const uint64_t* seeds, const int32_t* fw, const int32_t* fh, const int32_t* down2,
                     int32_t n_poly, int32_t texture, double tex_amp, double noise_sigma, const int64_t* offsets,
                     uint8_t* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int v = 0; v < n; ++v) {
    if (down2[v])
      syn_image_down2(seeds[v], fw[v], fh[v], n_poly, texture, tex_amp, noise_sigma, out + offsets[v]);
    else
      render_view(seeds[v], fw[v], fh[v], n_poly, texture, tex_amp, noise_sigma, out + offsets[v]);
  }
}

/* View sizes: W ~ U{wlo..whi}, aspect ~ U[alo, ahi], H = round(W / aspect). */
void syn_view_sizes(uint64_t seed, int32_t n, int32_t wlo, int32_t whi, double alo, double ahi, int32_t* W,
                    int32_t* H) {
  rng_t r = {seed ^ 0x5851F42D4C957F2DULL};
  for (int i = 0; i < n; ++i) {
    W[i] = (int32_t)rng_int(&r, wlo, whi);
    double a = rng_uniform(&r, alo, ahi);
    H[i] = (int32_t)floor((double)W[i] / a + 0.5);
  }
}

/*
 * Gaussian set of N rows (structure of arrays, float32):
 * means[N*3], log_scales[N*3], quats[N*4] (w,x,y,z), opacity_logits[N].
 */
void syn_gaussians(uint64_t seed, int64_t N, double ls_mu, double ls_sd, float* means, float* log_scales,
                   float* quats, float* opac) {
  const int64_t CH = 65536;
  int64_t nch = (N + CH - 1) / CH;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    rng_t r = {mix64(seed * 0x9E3779B97F4A7C15ULL + (uint64_t)c * 0xD1B54A32D192ED03ULL)};
    int64_t e = (c + 1) * CH < N ? (c + 1) * CH : N;
    for (int64_t i = c * CH; i < e; ++i) {
      for (int k = 0; k < 3; ++k) means[i * 3 + k] = (float)rng_uniform(&r, -1.0, 1.0);
      for (int k = 0; k < 3; ++k) log_scales[i * 3 + k] = (float)(ls_mu + ls_sd * rng_normal(&r));
      double q[4], n2 = 0.0;
      do {
        n2 = 0.0;
        for (int k = 0; k < 4; ++k) {
          q[k] = rng_normal(&r);
          n2 += q[k] * q[k];
        }
      } while (n2 < 1e-12);
      double inv = 1.0 / sqrt(n2);
      for (int k = 0; k < 4; ++k) quats[i * 4 + k] = (float)(q[k] * inv);
      double u;
      do { u = rng_u01(&r); } while (u <= 0.0);
      opac[i] = (float)log(u / (1.0 - u));
    }
  }
}

/* Exactly K distinct selected rows among N (partial Fisher-Yates); mask[N] in {0,1}. */
void syn_mask(uint64_t seed, int64_t N, int64_t K, uint8_t* mask) {
  memset(mask, 0, (size_t)N);
  if (K <= 0 || N <= 0) return;
  if (K > N) K = N;
  int32_t* idx = (int32_t*)malloc((size_t)N * sizeof(int32_t));
  for (int64_t i = 0; i < N; ++i) idx[i] = (int32_t)i;
  rng_t r = {seed ^ 0x243F6A8885A308D3ULL};
  for (int64_t i = 0; i < K; ++i) {
    int64_t j = rng_int(&r, i, N - 1);
    int32_t t = idx[i];
    idx[i] = idx[j];
    idx[j] = t;
    mask[idx[i]] = 1;
  }
  free(idx);
}

/* ---------------------------------------------------------------- contributions
 * Synthetic pixel contributions of Gaussians, standing in for what a
 * rasteriser's backward pass knows: Gaussian g covers a disc of integer
 * radius r in [1, 2 * mean_radius - 1] around a uniform centre of one uniform
 * view, clipped to the view, with weight a * exp(-d^2 / (2 (r/2)^2)) for a
 * per-Gaussian opacity a in [0.05, 1). Everything about Gaussian g is drawn
 * from a generator keyed by (seed, g), so the lists of different Gaussians
 * are independent of each other and of the thread count. Order 0 spreads
 * the entries by the bijection i -> (i * P) mod n (P prime, not dividing n),
 * so neighbouring entries belong to different Gaussians; order 1 is the row
 * order below.
 */
typedef struct {
  int32_t v, cx, cy, r;
  double a;
} foot_t;

static foot_t footprint(uint64_t seed, int64_t g, int32_t n_views, const int32_t* W, const int32_t* H,
                        int32_t mean_radius) {
  rng_t rg = {mix64(seed * 0x9E3779B97F4A7C15ULL + (uint64_t)g)};
  foot_t f;
  f.v = (int32_t)rng_int(&rg, 0, n_views - 1);
  f.cx = (int32_t)rng_int(&rg, 0, W[f.v] - 1);
  f.cy = (int32_t)rng_int(&rg, 0, H[f.v] - 1);
  f.r = (int32_t)rng_int(&rg, 1, 2 * mean_radius - 1);
  f.a = rng_uniform(&rg, 0.05, 1.0);
  return f;
}

static int64_t foot_count(const foot_t* f, const int32_t* W, const int32_t* H) {
  int64_t c = 0;
  for (int dy = -f->r; dy <= f->r; ++dy)
    for (int dx = -f->r; dx <= f->r; ++dx) {
      const int x = f->cx + dx, y = f->cy + dy;
      if (dx * dx + dy * dy <= f->r * f->r && x >= 0 && y >= 0 && x < W[f->v] && y < H[f->v]) ++c;
    }
  return c;
}

/* Number of entries for n_gauss Gaussians (first call), then the entries. */
int64_t syn_contrib_count(uint64_t seed, int64_t n_gauss, int32_t n_views, const int32_t* W, const int32_t* H,
                          int32_t mean_radius, int64_t* offsets /* [n_gauss + 1] */) {
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n_gauss; ++g) {
    const foot_t f = footprint(seed, g, n_views, W, H, mean_radius);
    offsets[g + 1] = foot_count(&f, W, H);
  }
  offsets[0] = 0;
  for (int64_t g = 0; g < n_gauss; ++g) offsets[g + 1] += offsets[g];
  return offsets[n_gauss];
}

static int64_t gcd64(int64_t a, int64_t b) {
  while (b) { const int64_t t = a % b; a = b; b = t; }
  return a;
}

/* Row order: entries grouped by (view, row), rows of a view in order, and
 * inside a row by Gaussian (each Gaussian's pixels of that row contiguous,
 * left to right) -- the order a rasteriser walking the image would meet
 * them in, up to the order of Gaussians within a row. */
static void contrib_fill_rows(uint64_t seed, int64_t n_gauss, int32_t n_views, const int32_t* W, const int32_t* H,
                              int32_t mean_radius, int64_t n, int32_t* gauss, int32_t* view, int32_t* pixel,
                              float* weight) {
  int64_t rows = 0;
  int64_t* row0 = (int64_t*)malloc(sizeof(int64_t) * (n_views + 1));
  for (int v = 0; v < n_views; ++v) { row0[v] = rows; rows += H[v]; }
  row0[n_views] = rows;
  int64_t* cur = (int64_t*)calloc(rows + 1, sizeof(int64_t));
  for (int64_t g = 0; g < n_gauss; ++g) {   /* entries per (view, row) */
    const foot_t f = footprint(seed, g, n_views, W, H, mean_radius);
    for (int dy = -f.r; dy <= f.r; ++dy) {
      const int y = f.cy + dy;
      if (y < 0 || y >= H[f.v]) continue;
      for (int dx = -f.r; dx <= f.r; ++dx) {
        const int x = f.cx + dx;
        if (dx * dx + dy * dy <= f.r * f.r && x >= 0 && x < W[f.v]) ++cur[row0[f.v] + y + 1];
      }
    }
  }
  for (int64_t r = 0; r < rows; ++r) cur[r + 1] += cur[r];
  for (int64_t g = 0; g < n_gauss; ++g) {
    const foot_t f = footprint(seed, g, n_views, W, H, mean_radius);
    const double s2 = 2.0 * (0.5 * f.r) * (0.5 * f.r);
    for (int dy = -f.r; dy <= f.r; ++dy) {
      const int y = f.cy + dy;
      if (y < 0 || y >= H[f.v]) continue;
      for (int dx = -f.r; dx <= f.r; ++dx) {
        const int x = f.cx + dx;
        if (dx * dx + dy * dy > f.r * f.r || x < 0 || x >= W[f.v]) continue;
        const int64_t o = cur[row0[f.v] + y]++;
        gauss[o] = (int32_t)g;
        view[o] = f.v;
        pixel[o] = y * W[f.v] + x;
        weight[o] = (float)(f.a * exp(-(double)(dx * dx + dy * dy) / s2));
      }
    }
  }
  (void)n;
  free(cur);
  free(row0);
}

void syn_contrib_fill(uint64_t seed, int64_t n_gauss, int32_t n_views, const int32_t* W, const int32_t* H,
                      int32_t mean_radius, const int64_t* offsets, int32_t order, int32_t* gauss, int32_t* view,
                      int32_t* pixel, float* weight) {
  const int64_t n = offsets[n_gauss];
  if (n == 0) return;
  if (order == 1) {
    contrib_fill_rows(seed, n_gauss, n_views, W, H, mean_radius, n, gauss, view, pixel, weight);
    return;
  }
  int64_t P = 1000003;  /* prime; step to the next prime-ish value until coprime with n */
  while (gcd64(P, n) != 1) P += 2;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t g = 0; g < n_gauss; ++g) {
    const foot_t f = footprint(seed, g, n_views, W, H, mean_radius);
    const double s2 = 2.0 * (0.5 * f.r) * (0.5 * f.r);
    int64_t i = offsets[g];
    for (int dy = -f.r; dy <= f.r; ++dy)
      for (int dx = -f.r; dx <= f.r; ++dx) {
        const int x = f.cx + dx, y = f.cy + dy;
        if (dx * dx + dy * dy > f.r * f.r || x < 0 || y < 0 || x >= W[f.v] || y >= H[f.v]) continue;
        const int64_t o = (int64_t)(((__int128)i * P) % n);
        gauss[o] = (int32_t)g;
        view[o] = f.v;
        pixel[o] = y * W[f.v] + x;
        weight[o] = (float)(f.a * exp(-(double)(dx * dx + dy * dy) / s2));
        ++i;
      }
  }
}
