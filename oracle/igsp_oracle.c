/*
 * CPU ORACLE for the ImprovedGS+ densification hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do. It shares no code, header or constant with the GPU
 * library: it is written from the paper alone, plainly and slowly, so that a
 * reader can check each step against the text by eye.
 *
 * Paper: "ImprovedGS+: A High-Performance C++/CUDA Re-Implementation
 * Strategy for 3D Gaussian Splatting", arXiv 2603.08661.
 *
 * Part 1, edge-score importance map (Sec. 2.1, the three enumerated steps of
 * the distilled Canny pipeline, then median normalisation). Where the paper
 * leaves a detail open, the reading taken is stated at the step. Arithmetic
 * is exact in int64 from the pixels through the gradient magnitude and the
 * orientation bin, then FP64 for the square root, the median and the
 * division.
 *
 * Part 2, Long-Axis-Split (Sec. 2.2, Algorithm 1 with the coordinate
 * transform of Algorithm 2 and the constants alpha, gamma, beta of the
 * paragraph after Algorithm 1), in FP64 on FP32 inputs.
 *
 * Every function here is pinned by tests against facts the paper and the
 * mathematics fix (closed forms, invariants, library routines, brute force);
 * none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Part 1: edge-score importance map                                          */
/* ------------------------------------------------------------------------- */

/*
 * Border rule (reading: reflect-101, the paper names none). An index one or
 * two steps outside [0, n-1] is mirrored about the border pixel without
 * repeating it: -1 -> 1, -2 -> 2, n -> n-2, n+1 -> n-3. Valid for n >= 3.
 */
static int64_t refl(int64_t i, int64_t n) {
  if (i < 0) i = -i;
  if (i > n - 1) i = 2 * (n - 1) - i;
  return i;
}

/*
 * 5-tap Gaussian (reading: the binomial taps 1,4,6,4,1 over 16 per axis,
 * the standard discrete 5x5 Gaussian with sigma near 1; the paper gives the
 * size only, Sec. 2.1 step 1). Kept unnormalised so every value stays an
 * exact integer; the full 5x5 kernel is the outer product, total weight 256.
 */
static const int64_t BLUR_TAPS[5] = {1, 4, 6, 4, 1};

void orc_blur_taps(int64_t* out5) {
  for (int k = 0; k < 5; ++k) out5[k] = BLUR_TAPS[k];
}

/*
 * Step 1a, grayscale (Sec. 2.1 step 1; reading: ITU-R BT.601 luma weights
 * 0.299, 0.587, 0.114 applied to R, G, B bytes, scaled by 1000 so the result
 * is an exact integer). gray = 299 R + 587 G + 114 B.
 */
void orc_gray(const uint8_t* rgb, int32_t W, int32_t H, int64_t* gray) {
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      const uint8_t* p = rgb + (y * W + x) * 3;
      gray[y * W + x] = 299 * (int64_t)p[0] + 587 * (int64_t)p[1] + 114 * (int64_t)p[2];
    }
}

/*
 * Step 1b, 5x5 Gaussian blur (Sec. 2.1 step 1), applied as a horizontal then
 * a vertical pass of the binomial taps with the border rule at each pass.
 * Output b = 256 * (blurred gray), exact.
 */
void orc_blur(const int64_t* gray, int32_t W, int32_t H, int64_t* b) {
  int64_t* h = (int64_t*)malloc(sizeof(int64_t) * (size_t)W * H);
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      int64_t s = 0;
      for (int k = 0; k < 5; ++k) s += BLUR_TAPS[k] * gray[y * W + refl(x + k - 2, W)];
      h[y * W + x] = s;
    }
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      int64_t s = 0;
      for (int k = 0; k < 5; ++k) s += BLUR_TAPS[k] * h[refl(y + k - 2, H) * W + x];
      b[y * W + x] = s;
    }
  free(h);
}

/*
 * Step 2, Sobel gradient (Sec. 2.1 step 2). x runs right, y runs down.
 *   gx = [1 2 1]^T (vertical smoothing) x [-1 0 1] (horizontal difference)
 *   gy = its transpose.
 * Unnormalised (no division by 8; the final map is scale-free).
 */
void orc_sobel(const int64_t* b, int32_t W, int32_t H, int64_t* gx, int64_t* gy) {
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      int64_t ym = refl(y - 1, H), yp = refl(y + 1, H);
      int64_t xm = refl(x - 1, W), xp = refl(x + 1, W);
      gx[y * W + x] = (b[ym * W + xp] - b[ym * W + xm]) + 2 * (b[y * W + xp] - b[y * W + xm]) +
                      (b[yp * W + xp] - b[yp * W + xm]);
      gy[y * W + x] = (b[yp * W + xm] - b[ym * W + xm]) + 2 * (b[yp * W + x] - b[ym * W + x]) +
                      (b[yp * W + xp] - b[ym * W + xp]);
    }
}

/*
 * Orientation of a gradient, quantised to one of four axes mod 180 degrees
 * (Sec. 2.1 step 2; reading: the usual Canny quantisation to the nearest
 * multiple of 45 degrees). Decided exactly in integers: with a = |gx|,
 * c = |gy|, the angle is within 22.5 degrees of horizontal iff
 * c < tan(22.5) a = (sqrt 2 - 1) a, i.e. (a + c)^2 < 2 a^2; symmetric for
 * vertical. sqrt 2 is irrational, so no integer pair sits on a boundary.
 *   0 = horizontal gradient (x axis), 1 = vertical (y axis),
 *   2 = diagonal with gx*gy > 0, 3 = diagonal with gx*gy < 0 (or zero gradient).
 */
int32_t orc_bin(int64_t gx, int64_t gy) {
  int64_t a = gx < 0 ? -gx : gx, c = gy < 0 ? -gy : gy;
  int64_t s = (a + c) * (a + c);
  if (s < 2 * a * a) return 0;
  if (s < 2 * c * c) return 1;
  return ((gx > 0) == (gy > 0)) && gx != 0 && gy != 0 ? 2 : 3;
}

static int64_t sgn(int64_t v) { return (v > 0) - (v < 0); }

/*
 * Unit step d along the gradient for a pixel's bin: horizontal (sgn gx, 0),
 * vertical (0, sgn gy), diagonal (sgn gx, sgn gy).
 */
static void step_of(int64_t gx, int64_t gy, int32_t bin, int64_t* dx, int64_t* dy) {
  if (bin == 0) { *dx = sgn(gx); *dy = 0; }
  else if (bin == 1) { *dx = 0; *dy = sgn(gy); }
  else { *dx = sgn(gx); *dy = sgn(gy); }
}

/*
 * Step 3, non-maximum suppression along the gradient (Sec. 2.1 step 3),
 * without hysteresis or thresholds (only three steps are listed). With the
 * squared magnitude M = gx^2 + gy^2 (exact), a pixel p survives iff
 *   M(p) > M(p - d)  and  M(p) >= M(p + d)  and  M(p) > 0.
 * Reading for ties: strict toward -d, non-strict toward +d, so a blurred
 * ideal step, whose two central pixels have equal magnitude, keeps exactly
 * one of them. Neighbours outside the view use the border rule.
 * Outputs: keep (0/1), and per pixel the decision margin
 *   c(p) = min(|sqrt M(p) - sqrt M(p-d)|, |sqrt M(p) - sqrt M(p+d)|,
 *              ||gy| - t|gx||, ||gx| - t|gy||) / sqrt M(p),   t = sqrt 2 - 1,
 * which is +inf when M(p) = 0: how far the pixel is from any comparison
 * whose outcome would change its decision.
 */
void orc_nms(const int64_t* gx, const int64_t* gy, int32_t W, int32_t H, int64_t* M, uint8_t* bin,
             uint8_t* keep, double* margin) {
  const double t = sqrt(2.0) - 1.0;
  for (int64_t i = 0; i < (int64_t)W * H; ++i) M[i] = gx[i] * gx[i] + gy[i] * gy[i];
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      int64_t i = y * W + x;
      int32_t bn = orc_bin(gx[i], gy[i]);
      int64_t dx, dy;
      step_of(gx[i], gy[i], bn, &dx, &dy);
      int64_t im = refl(y - dy, H) * W + refl(x - dx, W);
      int64_t ip = refl(y + dy, H) * W + refl(x + dx, W);
      if (bin) bin[i] = (uint8_t)bn;
      keep[i] = (uint8_t)(M[i] > M[im] && M[i] >= M[ip] && M[i] > 0);
      if (margin) {
        if (M[i] == 0) {
          margin[i] = INFINITY;
        } else {
          double sp = sqrt((double)M[i]);
          double a = fabs((double)gx[i]), c = fabs((double)gy[i]);
          double m1 = fabs(sp - sqrt((double)M[im])), m2 = fabs(sp - sqrt((double)M[ip]));
          double m3 = fabs(c - t * a), m4 = fabs(a - t * c);
          double mm = m1 < m2 ? m1 : m2;
          if (m3 < mm) mm = m3;
          if (m4 < mm) mm = m4;
          margin[i] = mm / sp;
        }
      }
    }
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/*
 * Median normalisation (Sec. 2.1, paragraph after the steps). Readings: the
 * median is taken over the surviving pixels of one view (about two thirds of
 * all pixels are zero after suppression, so a median over every pixel would
 * be zero), as the lower median, the floor((n-1)/2)-th smallest (0-based),
 * so it is one existing value; no clamp afterwards. The surviving magnitude
 * is m = sqrt(M) / 256000 in DN per pixel of an unnormalised Sobel.
 * Ordering by M is ordering by m, so the median is selected on the exact M.
 * E(p) = m(p) / med for survivors, 0 elsewhere; E = 0 everywhere if no pixel
 * survives. Returns the survivor count n; *med and *Mmed get the median
 * magnitude and its squared-integer form (0 if n = 0).
 */
int64_t orc_normalise(const int64_t* M, const uint8_t* keep, int32_t W, int32_t H, double* m_out, double* E,
                      double* med_out, int64_t* Mmed_out) {
  int64_t npx = (int64_t)W * H, n = 0;
  for (int64_t i = 0; i < npx; ++i) n += keep[i] != 0;
  int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t j = 0;
  for (int64_t i = 0; i < npx; ++i)
    if (keep[i]) s[j++] = M[i];
  qsort(s, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t Mmed = n > 0 ? s[(n - 1) / 2] : 0;
  double med = sqrt((double)Mmed) / 256000.0;
  for (int64_t i = 0; i < npx; ++i) {
    double m = keep[i] ? sqrt((double)M[i]) / 256000.0 : 0.0;
    if (m_out) m_out[i] = m;
    E[i] = (keep[i] && n > 0) ? m / med : 0.0;
  }
  if (med_out) *med_out = med;
  if (Mmed_out) *Mmed_out = Mmed;
  free(s);
  return n;
}

/*
 * Whole pipeline for one view. Any stage output pointer may be NULL.
 * Returns the survivor count, or -1 if W or H < 3.
 */
int64_t orc_edge_view(const uint8_t* rgb, int32_t W, int32_t H, int64_t* gray_o, int64_t* b_o, int64_t* gx_o,
                      int64_t* gy_o, int64_t* M_o, uint8_t* bin_o, uint8_t* keep_o, double* m_o, double* E,
                      double* margin_o, double* med_o, int64_t* Mmed_o) {
  if (W < 3 || H < 3) return -1;
  size_t npx = (size_t)W * H;
  int64_t* gray = gray_o ? gray_o : (int64_t*)malloc(sizeof(int64_t) * npx);
  int64_t* b = b_o ? b_o : (int64_t*)malloc(sizeof(int64_t) * npx);
  int64_t* gx = gx_o ? gx_o : (int64_t*)malloc(sizeof(int64_t) * npx);
  int64_t* gy = gy_o ? gy_o : (int64_t*)malloc(sizeof(int64_t) * npx);
  int64_t* M = M_o ? M_o : (int64_t*)malloc(sizeof(int64_t) * npx);
  uint8_t* keep = keep_o ? keep_o : (uint8_t*)malloc(npx);
  orc_gray(rgb, W, H, gray);
  orc_blur(gray, W, H, b);
  orc_sobel(b, W, H, gx, gy);
  orc_nms(gx, gy, W, H, M, bin_o, keep, margin_o);
  int64_t n = orc_normalise(M, keep, W, H, m_o, E, med_o, Mmed_o);
  if (!gray_o) free(gray);
  if (!b_o) free(b);
  if (!gx_o) free(gx);
  if (!gy_o) free(gy);
  if (!M_o) free(M);
  if (!keep_o) free(keep);
  return n;
}

/*
 * Many views in one packed buffer: view v is W[v] x H[v] bytes*3 at
 * rgb + in_off[v]; its map goes to E + out_off[v]. Views are independent;
 * they are spread over up to `threads` OpenMP threads (<= 0: runtime
 * default). keep_out (optional) follows the out_off layout.
 */
void orc_edge_batch(const uint8_t* rgb, int32_t n, const int32_t* W, const int32_t* H, const int64_t* in_off,
                    const int64_t* out_off, double* E, uint8_t* keep_out, double* med_out, int64_t* nsurv_out,
                    int32_t threads) {
  if (threads > 0) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
    for (int v = 0; v < n; ++v) {
      double med = 0.0;
      int64_t ns = orc_edge_view(rgb + in_off[v], W[v], H[v], NULL, NULL, NULL, NULL, NULL, NULL,
                                 keep_out ? keep_out + out_off[v] : NULL, NULL, E + out_off[v], NULL, &med, NULL);
      if (med_out) med_out[v] = med;
      if (nsurv_out) nsurv_out[v] = ns;
    }
  } else {
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < n; ++v) {
      double med = 0.0;
      int64_t ns = orc_edge_view(rgb + in_off[v], W[v], H[v], NULL, NULL, NULL, NULL, NULL, NULL,
                                 keep_out ? keep_out + out_off[v] : NULL, NULL, E + out_off[v], NULL, &med, NULL);
      if (med_out) med_out[v] = med;
      if (nsurv_out) nsurv_out[v] = ns;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Part 2: Long-Axis-Split                                                    */
/* ------------------------------------------------------------------------- */

/*
 * Rotation matrix of a unit quaternion (w, x, y, z), the convention of 3D
 * Gaussian Splatting; a zero quaternion is read as the identity rotation,
 * any other one is normalised first (Algorithm 1 takes R as given).
 * Returned flat, row-major: R[3*row + col].
 */
void orc_quat_to_R(const double q_in[4], double R[9]) {
  double n2 = q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3];
  double w = 1.0, x = 0.0, y = 0.0, z = 0.0;
  if (n2 > 0.0) {
    double n = sqrt(n2);
    w = q_in[0] / n; x = q_in[1] / n; y = q_in[2] / n; z = q_in[3] / n;
  }
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/*
 * Opacity update of Algorithm 1: the stored logit o is activated with the
 * sigmoid, scaled by beta in activated space, and mapped back with the
 * logit. Written in the algebraically equal form
 *   logit(beta * sigmoid(o)) = log(beta) - log(1 - beta + exp(-o)),
 * evaluated without overflow on either sign of o.
 */
double orc_opacity(double o, double beta) {
  if (o >= 0.0) return log(beta) - log(1.0 - beta + exp(-o));
  return o + log(beta) - log1p((1.0 - beta) * exp(o));
}

/*
 * Long-Axis-Split in place (Sec. 2.2, Algorithm 1 with Algorithm 2).
 * Inputs are FP32 arrays of `capacity` rows (rows [0, N) are live):
 *   means[3], log_scales[3], quats[4] (w,x,y,z), opacity logits, feats[F].
 * For each row i < N with mask[i] != 0, taken in ascending i, with r its
 * rank among the selected rows:
 *   l      = index of the largest log-scale (reading: lowest index on ties)
 *   offset = alpha * exp(s_l)                     (physical long-axis scale)
 *   s'_l   = s_l + log(alpha); s'_j = s_j + log(gamma) for j != l
 *   o'     = logit(beta * sigmoid(o))
 *   d      = offset * (column l of R)             (Algorithm 2: the three
 *            entries R[l], R[l+3], R[l+6] of the flat row-major matrix)
 *   row i      <- (p + d, s', q, o', f)           (first child, in place)
 *   row N + r  <- (p - d, s', q, o', f)           (second child, appended)
 * (readings: the second child goes to the first free row after the live
 * ones, in rank order; the quaternion and features are copied.)
 * All-or-nothing: if N + K > capacity nothing is split and -6 is returned.
 * Outputs are FP64 arrays of `capacity` rows (rows not written are the
 * inputs widened), split_idx[r] = i, axis[r] = l, *K_out = K,
 * *count_out = new live count. Returns 0 on success.
 */
int32_t orc_las(int64_t N, int64_t capacity, const float* means, const float* log_scales, const float* quats,
                const float* opac, const float* feats, int32_t F, const uint8_t* mask, double alpha, double gamma,
                double beta, double* means_o, double* ls_o, double* quats_o, double* opac_o, double* feats_o,
                int32_t* split_idx, int32_t* axis, int64_t* K_out, int64_t* count_out) {
  for (int64_t i = 0; i < capacity; ++i) {
    for (int k = 0; k < 3; ++k) means_o[i * 3 + k] = means[i * 3 + k];
    for (int k = 0; k < 3; ++k) ls_o[i * 3 + k] = log_scales[i * 3 + k];
    for (int k = 0; k < 4; ++k) quats_o[i * 4 + k] = quats[i * 4 + k];
    opac_o[i] = opac[i];
    for (int k = 0; k < F; ++k) feats_o[i * F + k] = feats[i * F + k];
  }
  int64_t K = 0;
  for (int64_t i = 0; i < N; ++i) K += mask[i] != 0;
  *K_out = K;
  if (N + K > capacity) {
    *count_out = N;
    return -6;
  }
  int64_t r = 0;
  for (int64_t i = 0; i < N; ++i) {
    if (!mask[i]) continue;
    double s[3] = {log_scales[i * 3 + 0], log_scales[i * 3 + 1], log_scales[i * 3 + 2]};
    int l = 0;
    if (s[1] > s[l]) l = 1;
    if (s[2] > s[l]) l = 2;
    double offset = exp(s[l]) * alpha;
    double sn[3];
    for (int k = 0; k < 3; ++k) sn[k] = s[k] + (k == l ? log(alpha) : log(gamma));
    double on = orc_opacity((double)opac[i], beta);
    double q[4] = {quats[i * 4 + 0], quats[i * 4 + 1], quats[i * 4 + 2], quats[i * 4 + 3]};
    double R[9];
    orc_quat_to_R(q, R);
    double d[3] = {R[l] * offset, R[l + 3] * offset, R[l + 6] * offset};
    int64_t j = N + r;
    for (int k = 0; k < 3; ++k) {
      double p = means[i * 3 + k];
      means_o[i * 3 + k] = p + d[k];
      means_o[j * 3 + k] = p - d[k];
      ls_o[i * 3 + k] = sn[k];
      ls_o[j * 3 + k] = sn[k];
    }
    for (int k = 0; k < 4; ++k) quats_o[j * 4 + k] = quats[i * 4 + k];
    opac_o[i] = on;
    opac_o[j] = on;
    for (int k = 0; k < F; ++k) feats_o[j * F + k] = feats[i * F + k];
    split_idx[r] = (int32_t)i;
    axis[r] = l;
    ++r;
  }
  *count_out = N + K;
  return 0;
}
