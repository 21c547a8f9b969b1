/*
 * igsp.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of the ImprovedGS+ densification strategy (arXiv 2603.08661):
 *
 *   edge_importance  -- per-view edge-score importance maps (Sec. 2.1):
 *                       grayscale, 5x5 Gaussian blur, Sobel magnitude and
 *                       orientation, non-maximum suppression along the
 *                       gradient, median normalisation;
 *   long_axis_split  -- Long-Axis-Split of selected Gaussians (Sec. 2.2,
 *                       Algorithm 1 with the column-extraction transform of
 *                       Algorithm 2); long_axis_split_full also carries
 *                       features of any width and the children's optimiser
 *                       state;
 *   split_mask       -- which Gaussians to split: edge scores moved onto the
 *                       Gaussians, gradient threshold with warm-up, budget;
 * plus the tile/form autotuner (igsp_edge_autotune, igsp_edge_resolve), one
 * densification step as a HIP graph (igsp_step_*) and the exponential
 * learning-rate schedule (igsp_lr_exponential, host only).
 *
 * Conventions for every entry point:
 *   - Pointers marked (device) are HIP device memory on the current device;
 *     pointers marked (host) are host memory read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls return without waiting for the GPU.
 *   - The caller owns every buffer passed in. The library owns only its
 *     plans (device view tables, work lists, histograms, intermediate maps,
 *     split workspaces), created on the first call with a given geometry and
 *     reused afterwards; igsp_release_plans() frees them.
 *   - A call that creates a plan allocates device memory and synchronises
 *     the device, so it is not capturable into a HIP graph; when more than
 *     eight edge (or split-mask) geometries are cached, creating another one
 *     frees the least recently used plan, which also waits for the device.
 *     Repeated calls with a cached geometry allocate nothing, never wait,
 *     never read device memory back to the host, and can be captured (see
 *     igsp_step_*; a step keeps its plans alive until it is destroyed).
 *   - Errors detectable on the host return a negative status and enqueue
 *     nothing. No C++ exception crosses this boundary.
 *   - Calls on one device that share a plan must be ordered (one stream, or
 *     synchronised): the plan's intermediate buffers are reused.
 */
#ifndef IGSP_H
#define IGSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IGSP_OK = 0,
  IGSP_ERR_NULL = -1,        /* a required pointer is NULL                       */
  IGSP_ERR_DIMS = -2,        /* a view below 3x3, W*H >= 2^31, n_views < 0,
                                negative offsets or counts                       */
  IGSP_ERR_ALIGN = -3,       /* `images` not 16-byte aligned                     */
  IGSP_ERR_OVERLAP = -4,     /* input and output byte ranges overlap             */
  IGSP_ERR_PARAM = -5,       /* unknown precision, bad tile option, feat_dim < 0,
                                alpha/gamma/beta outside (0, 1]                  */
  IGSP_ERR_CAPACITY = -6,    /* (device status) N + K > capacity: nothing split  */
  IGSP_ERR_HIP = -7,         /* a HIP runtime call failed (no device, OOM, ...)  */
  IGSP_ERR_UNSUPPORTED = -8, /* the current device is not gfx950                 */
  IGSP_ERR_TIMEOUT = -9,     /* (device status) a wait inside the persistent
                                launch gave up: its maps are not valid          */
  IGSP_ERR_TOO_LARGE = -10   /* capacity beyond the fixed workspace of
                                long_axis_split_noalloc                         */
} igsp_status;

/* ------------------------------------------------------------------------ */
/* Edge-score importance maps (Sec. 2.1)                                     */
/* ------------------------------------------------------------------------ */

/*
 * One view. Its pixels are packed 8-bit R,G,B bytes, row-major, row pitch
 * 3*width bytes, starting `in_offset` bytes after `images` (any byte
 * offset). Its map is width*height float32 values, row-major, row pitch
 * `width`, starting `out_offset` floats after `out_maps`.
 * Requires width >= 3, height >= 3, width*height < 2^31.
 */
typedef struct {
  int32_t width;
  int32_t height;
  int64_t in_offset;
  int64_t out_offset;
} igsp_view;

/* Storage type of the one intermediate that reaches HBM: the thinned
   (suppressed) gradient magnitude kept between the stencil pass and the
   normalisation. Arithmetic is integer-exact through the gradient and FP32
   after it in every mode; maps are float32 in every mode. */
typedef enum { IGSP_FP32 = 0, IGSP_FP16 = 1, IGSP_BF16 = 2 } igsp_precision;

/* Launch form of edge_importance. All forms compute identical maps. */
typedef enum {
  IGSP_PLAIN = 0,               /* each view by its own sequence of launches  */
  IGSP_BATCHED = 1,             /* every view together; the library picks the
                                   form below (tuned, else staged)            */
  IGSP_BATCHED_STAGED = 2,      /* every view in one launch per stage         */
  IGSP_BATCHED_PERSISTENT = 3,  /* every view and stage in one persistent
                                   launch; later stages of earlier views run
                                   beside the stencil pass of later ones      */
  IGSP_UNFUSED = 4              /* the paper's layout, for comparison: gray,
                                   blur, Sobel and suppression as separate
                                   launches over every view, each step's
                                   result in HBM (16 B/px of extra plan
                                   memory); never chosen by IGSP_BATCHED     */
} igsp_form;

typedef struct {
  int32_t precision;     /* igsp_precision                                    */
  int32_t batched;       /* igsp_form                                         */
  int32_t seg_rows;      /* output rows per wavefront segment; 0 = tuned      */
  int32_t wg_waves;      /* wavefronts per work-group (1, 2, 4, 8); 0 = tuned */
  float* medians;        /* (device, optional) [n_views]: the median surviving
                            magnitude of each view, in DN per pixel of an
                            unnormalised Sobel, as stored (0 if none survive) */
  int32_t* survivors;    /* (device, optional) [n_views]: surviving pixels    */
  void** stage_events;   /* (host, optional) 4 hipEvent_t recorded on `stream`
                            before the stencil pass, after it, after the median
                            selection and after the normalisation (staged
                            form; the plain and persistent forms record the
                            last three after their final launch). Profiling
                            only: no work changes. Ignored by
                            igsp_step_create.                                  */
  int32_t* status;       /* (device, optional) [1]: set by the call's kernels to
                            IGSP_OK, or by the persistent form to
                            IGSP_ERR_TIMEOUT if one of its bounded waits gave
                            up (then the maps are not valid; the next call
                            starts clean). Untouched when n_views = 0.        */
} igsp_edge_opts;

/*
 * Edge-score importance map of every view (Sec. 2.1). For each view:
 *   gray  = 299 R + 587 G + 114 B (BT.601 luma x 1000, exact);
 *   blur  = binomial 5x5 Gaussian, taps (1,4,6,4,1)/16 per axis;
 *   gx,gy = unnormalised Sobel; M = gx^2 + gy^2;
 *   orientation quantised to the nearest of 0/45/90/135 degrees;
 *   a pixel survives iff M(p) > M(p-d) and M(p) >= M(p+d) and M(p) > 0, d the
 *   unit step along its gradient (ties: strict toward -d);
 *   map = sqrt(M) / (lower median of sqrt(M) over the view's survivors) at
 *   survivors, 0 elsewhere (0 everywhere if none survive).
 * Borders mirror without repeating the edge pixel (reflect-101).
 *
 * images   (device) the packed views; must be 16-byte aligned.
 * views    (host)   [n_views] geometry, see igsp_view.
 * n_views  number of views; 0 is a no-op returning IGSP_OK.
 * out_maps (device) float32 output, see igsp_view. May not overlap images.
 * opts     (host, optional) NULL = batched, FP32, tuned tiles.
 * stream   hipStream_t or NULL.
 */
igsp_status edge_importance(const uint8_t* images, const igsp_view* views, int32_t n_views,
                            float* out_maps, const igsp_edge_opts* opts, void* stream);

/*
 * Autotune the tile shape (rows per wavefront segment x wavefronts per
 * work-group, i.e. waves per CU through the work-groups resident per CU) and,
 * for IGSP_BATCHED, the launch form, for these views and this storage
 * precision: every candidate is run on the given data (out_maps is
 * overwritten) and timed with HIP events on `stream`. The fastest is
 * remembered for calls with the same `batched` value whose opts leave
 * seg_rows and wg_waves at 0 and whose geometry falls in the same size class
 * (device, precision, total pixels and mean width rounded to powers of two).
 * If the environment variable IGSP_TUNE_CACHE names a file, tuned entries are
 * loaded from it on first use and the file is rewritten after tuning (one
 * JSON object per line).
 * batched  igsp_form requested by later calls.
 * best     (host, out, optional) receives the choice: seg_rows, wg_waves and
 *          in `batched` the concrete form.
 * Synchronises `stream`; allocates (it creates plans), so never capture it.
 */
igsp_status igsp_edge_autotune(const uint8_t* images, const igsp_view* views, int32_t n_views,
                               float* out_maps, int32_t precision, int32_t batched,
                               igsp_edge_opts* best, void* stream);

/*
 * The launch form and tile shape edge_importance would use for these views
 * and options: on return opts->batched holds the concrete igsp_form and
 * seg_rows / wg_waves are filled in (explicit values are kept; zeros become
 * the tuned entry of the size class, else 4 wavefronts per work-group and
 * the tallest of 64, 40, 28, 22, 16 rows that gives the stencil launch 16
 * wavefronts per CU, or 10 rows if none does; the plain form counts the
 * wavefronts of one view's launch, the batched forms those of all views).
 * Tuned entries
 * come from the file IGSP_TUNE_DEFAULTS names (the shipped table, read only)
 * and then IGSP_TUNE_CACHE (the autotuner's output), read once per process.
 * opts (host, in/out). Touches no device memory and enqueues nothing.
 */
igsp_status igsp_edge_resolve(const igsp_view* views, int32_t n_views, igsp_edge_opts* opts);

/* ------------------------------------------------------------------------ */
/* Long-Axis-Split (Sec. 2.2, Algorithms 1 and 2)                            */
/* ------------------------------------------------------------------------ */

/*
 * Gaussian parameters as structure-of-arrays, float32, `capacity` rows each
 * (device). Rows [0, N) are live, N = *count. Scales are stored as logs,
 * opacity as a logit, rotation as a quaternion (w, x, y, z), not necessarily
 * normalised (a zero quaternion is read as the identity).
 */
typedef struct {
  float* means;            /* (device) [capacity][3]                          */
  float* log_scales;       /* (device) [capacity][3]                          */
  float* quats;            /* (device) [capacity][4]                          */
  float* opacity_logits;   /* (device) [capacity]                             */
  float* features;         /* (device) [capacity][feat_dim], NULL if 0        */
  int32_t feat_dim;        /* >= 0                                            */
  int64_t* count;          /* (device) scalar N; becomes N + K on success     */
  int64_t capacity;        /* rows allocated, >= 0                            */
} igsp_gaussians;

/* Shrink factor of the longest axis (also scales the child offset), shrink
   factor of the other axes, opacity factor; NULL = 0.5, 0.85, 0.6, the
   values the paper uses (Sec. 2.2). Each must lie in (0, 1]. */
typedef struct {
  float alpha;
  float gamma;
  float beta;
} igsp_las_params;

typedef struct {
  int32_t* split_idx;      /* (device) [capacity]: the first K entries become
                              the split rows in ascending order               */
  int32_t* status;         /* (device) scalar: IGSP_OK or IGSP_ERR_CAPACITY   */
  int64_t* n_split;        /* (device, optional) scalar K                     */
} igsp_las_out;

/*
 * Split every live row i with mask[i] != 0, in place (Sec. 2.2, Alg. 1):
 * l = index of the largest log-scale (lowest index on ties);
 * log-scales: s_l += log(alpha), the others += log(gamma);
 * opacity: o = logit(beta * sigmoid(o));
 * d = alpha * exp(s_l) * (column l of R(q)), read as the three entries
 * R[l], R[l+3], R[l+6] of the flat row-major matrix (Alg. 2);
 * row i becomes the first child (mean + d), row N + r the second child
 * (mean - d, same scales, opacity, quaternion and features), r = rank of i
 * among the selected rows.
 * All or nothing: if N + K > capacity, nothing is written except
 * *status = IGSP_ERR_CAPACITY (and *n_split = K); *count stays N.
 * mask (device) uint8 [capacity], entries [0, N) read.
 * Calling twice splits twice (the operation is not idempotent).
 */
igsp_status long_axis_split(const igsp_gaussians* g, const uint8_t* mask, const igsp_las_out* out,
                            const igsp_las_params* params, void* stream);

/*
 * long_axis_split for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and result as long_axis_split (features included),
 * but its workspace (per-tile counts and offsets, the split's scalars) is a
 * fixed device array of the library, about 1.5 MiB per GPU, held from the
 * first call on a device until the process ends. Calls no hipMalloc or
 * hipFree, never synchronises, and builds no plan.
 * Limit: capacity <= 2^28 rows, else IGSP_ERR_TOO_LARGE and nothing enqueued.
 * Every call on one GPU shares that GPU's workspace: calls that overlap on a
 * GPU (different streams without ordering, several host threads) race and
 * must be serialised by the caller; consecutive calls on one stream are safe.
 */
igsp_status long_axis_split_noalloc(const igsp_gaussians* g, const uint8_t* mask, const igsp_las_out* out,
                                    const igsp_las_params* params, void* stream);

/*
 * Adam moments kept by the caller's optimiser for each parameter group, in
 * the same row layout as the parameters (device, float32, `capacity` rows).
 * [0] = first moment, [1] = second moment; any pointer may be NULL (that
 * state is not kept).
 */
typedef struct {
  float* means[2];            /* [capacity][3]        */
  float* log_scales[2];       /* [capacity][3]        */
  float* quats[2];            /* [capacity][4]        */
  float* opacity_logits[2];   /* [capacity]           */
  float* features[2];         /* [capacity][feat_dim] */
} igsp_adam_moments;

/*
 * The full-record split a trainer calls: long_axis_split (same arguments and
 * result, features of any width copied to the second child) plus the
 * optimiser state of both children. The paper does not say what happens to
 * optimiser state; the reading taken here is the usual one for a split that
 * replaces a parent by two new Gaussians: every given moment row of both
 * children (rows i and N + r) is set to 0, all other rows are untouched.
 * adam (host, optional) NULL = no optimiser state, i.e. long_axis_split.
 * Same all-or-nothing rule: on IGSP_ERR_CAPACITY no moment row changes.
 */
igsp_status long_axis_split_full(const igsp_gaussians* g, const igsp_adam_moments* adam, const uint8_t* mask,
                                 const igsp_las_out* out, const igsp_las_params* params, void* stream);

/* ------------------------------------------------------------------------ */
/* Which Gaussians to split (the selection that feeds Long-Axis-Split)      */
/* ------------------------------------------------------------------------ */

/*
 * Pixel contributions of Gaussians, as a rasteriser's backward pass knows
 * them: entry c says Gaussian gauss[c] covers pixel pixel[c] (y * width + x)
 * of view view[c] with blending weight weight[c]. Any order. (device)
 */
typedef struct {
  const int32_t* gauss;
  const int32_t* view;
  const int32_t* pixel;
  const float* weight;
  int64_t n;               /* entries, >= 0 */
} igsp_contributions;

typedef struct {
  float grad_threshold;    /* candidate iff grad[g] >= grad_threshold ...     */
  int32_t warmup;          /* ... unless warmup != 0: every live Gaussian     */
  int64_t budget;          /* Gaussians allowed after the split               */
} igsp_select_params;

/*
 * Split mask from edge scores (Sec. 2.1's maps moved onto the Gaussians,
 * Sec. 3's gradient threshold and warm-up, and a Gaussian budget). The paper
 * names these parts without giving formulas; the readings taken are:
 *   score[g] = sum over g's contributions of E_view[pixel] * weight, each
 *              product in float32, accumulated exactly in int64 units of
 *              2^-32 (floor of each product x 2^32; non-positive products
 *              add nothing), so the sum does not depend on order;
 *   candidates: live g (g < N = *count) with warmup or grad[g] >= threshold;
 *   K = min(candidates, max(0, budget - N)) candidates with the largest
 *   scores are selected, ties by lower index.
 * maps     (device) float32 edge maps as edge_importance writes them, laid
 *          out by `views` (only out_offset, width and height are read).
 * views    (host) [n_views].
 * contrib  (host struct, device arrays); entries naming a Gaussian >= N, a
 *          view outside [0, n_views) or a pixel outside its view are ignored.
 * grad     (device) float32 [capacity], rows [0, N) read.
 * count    (device) int64 scalar N (not changed).
 * mask     (device, out) uint8 [capacity]: rows [0, N) get 1 (selected) or 0.
 * scores   (device, out) int64 [capacity]: rows [0, N) get the scores.
 * n_selected (device, out, optional) int64 scalar K.
 * Captures as kernel launches only (after a first call has built the plan).
 */
igsp_status split_mask(const float* maps, const igsp_view* views, int32_t n_views,
                       const igsp_contributions* contrib, const float* grad, const int64_t* count,
                       int64_t capacity, const igsp_select_params* params, uint8_t* mask, int64_t* scores,
                       int64_t* n_selected, void* stream);

/* ------------------------------------------------------------------------ */
/* Learning-rate schedules (Sec. 3)                                          */
/* ------------------------------------------------------------------------ */

/*
 * Exponential schedule: lr(t) = lr_init * (lr_final / lr_init)^(s / t_max)
 * with s = t clamped to [0, t_max]. The paper decays the scale learning rate
 * from 0.020 to 0.002 (gamma = 0.1) and the position learning rate from
 * 0.000128 to 0.0000128; the iteration span it decays over is not stated, the
 * caller passes it (t_max). Host function, no GPU work.
 * Returns NaN if lr_init or lr_final is not positive or t_max < 1.
 */
double igsp_lr_exponential(int64_t t, double lr_init, double lr_final, int64_t t_max);

/* ------------------------------------------------------------------------ */
/* One densification step as a HIP graph                                    */
/* ------------------------------------------------------------------------ */

typedef struct igsp_step igsp_step;

/*
 * Record one densification step -- edge_importance over the given views
 * followed by long_axis_split -- into a HIP graph and instantiate it. The
 * plans are created first (outside the capture), so the graph holds only
 * kernel launches. Arguments as for the two calls; every pointer is baked
 * into the graph, so the buffers must outlive it. The live count stays on
 * the device: the graph remains valid as N grows.
 * step (host, out) receives the handle.
 */
igsp_status igsp_step_create(const uint8_t* images, const igsp_view* views, int32_t n_views,
                             float* out_maps, const igsp_edge_opts* opts, const igsp_gaussians* g,
                             const uint8_t* mask, const igsp_las_out* out, const igsp_las_params* params,
                             void* stream, igsp_step** step);
/* Launch the recorded step on `stream`. */
igsp_status igsp_step_launch(igsp_step* step, void* stream);
/* Destroy the graph (after the launches that use it have finished). */
void igsp_step_destroy(igsp_step* step);

/* ------------------------------------------------------------------------ */
/* Utilities                                                                 */
/* ------------------------------------------------------------------------ */

/* Static English text for a status code. */
const char* igsp_status_string(int32_t status);

/* Free every plan and workspace on every device (the caller must ensure no
   enqueued work still uses them). */
void igsp_release_plans(void);

/* Library version, for the binding's load check. */
int32_t igsp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IGSP_H */
