// Host-side argument validation of the C ABI. Pure C++ with no HIP calls, so
// every error path can be exercised on a machine without a GPU; a call that
// fails here enqueues nothing.
#include "validate.h"

#include <cmath>

namespace igsp {

static bool unit_interval(float v) { return v > 0.0f && v <= 1.0f; }  // NaN fails both

igsp_status validate_edge(const uint8_t* images, const igsp_view* views, int32_t n_views, const float* out,
                          const igsp_edge_opts* opts, EdgeExtent* ext) {
  if (n_views < 0) return IGSP_ERR_DIMS;
  if (n_views == 0) return IGSP_OK;
  if (!images || !views || !out) return IGSP_ERR_NULL;
  if ((reinterpret_cast<uintptr_t>(images) & 15u) != 0) return IGSP_ERR_ALIGN;
  if (opts) {
    if (opts->precision < IGSP_FP32 || opts->precision > IGSP_BF16) return IGSP_ERR_PARAM;
    if (opts->batched < IGSP_PLAIN || opts->batched > IGSP_UNFUSED) return IGSP_ERR_PARAM;
    if (opts->seg_rows != 0 && (opts->seg_rows < 8 || opts->seg_rows > 4096)) return IGSP_ERR_PARAM;
    const int w = opts->wg_waves;
    if (w != 0 && w != 1 && w != 2 && w != 4 && w != 8) return IGSP_ERR_PARAM;
    if (opts->stage_events)
      for (int k = 0; k < 4; ++k)
        if (!opts->stage_events[k]) return IGSP_ERR_NULL;
  }
  int64_t in_end = 0, out_end = 0, px = 0;
  for (int32_t v = 0; v < n_views; ++v) {
    const igsp_view& d = views[v];
    if (d.width < 3 || d.height < 3) return IGSP_ERR_DIMS;
    const int64_t npx = (int64_t)d.width * d.height;
    if (npx >= (int64_t(1) << 31)) return IGSP_ERR_DIMS;
    if (d.in_offset < 0 || d.out_offset < 0) return IGSP_ERR_DIMS;
    if (d.in_offset > (int64_t(1) << 60) || d.out_offset > (int64_t(1) << 60)) return IGSP_ERR_DIMS;
    const int64_t ie = d.in_offset + 3 * npx, oe = d.out_offset + npx;
    if (ie > in_end) in_end = ie;
    if (oe > out_end) out_end = oe;
    px += npx;
  }
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(images), a1 = a0 + (uintptr_t)in_end;
  const uintptr_t b0 = reinterpret_cast<uintptr_t>(out), b1 = b0 + (uintptr_t)out_end * sizeof(float);
  if (a0 < b1 && b0 < a1) return IGSP_ERR_OVERLAP;
  if (ext) {
    ext->img_end = in_end;
    ext->out_end = out_end;
    ext->pixels = px;
  }
  return IGSP_OK;
}

igsp_status validate_las(const igsp_gaussians* g, const uint8_t* mask, const igsp_las_out* out,
                         const igsp_las_params* p) {
  if (!g || !mask || !out) return IGSP_ERR_NULL;
  if (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->count) return IGSP_ERR_NULL;
  if (!out->split_idx || !out->status) return IGSP_ERR_NULL;
  if (g->feat_dim < 0) return IGSP_ERR_PARAM;
  if (g->feat_dim > 0 && !g->features) return IGSP_ERR_NULL;
  if (g->capacity < 0 || g->capacity >= (int64_t(1) << 31)) return IGSP_ERR_DIMS;
  if (p && (!unit_interval(p->alpha) || !unit_interval(p->gamma) || !unit_interval(p->beta)))
    return IGSP_ERR_PARAM;
  return IGSP_OK;
}

igsp_status validate_select(const float* maps, const igsp_view* views, int32_t n_views,
                            const igsp_contributions* c, const float* grad, const int64_t* count,
                            int64_t capacity, const igsp_select_params* p, const uint8_t* mask,
                            const int64_t* scores) {
  if (!c || !grad || !count || !p || !mask || !scores) return IGSP_ERR_NULL;
  if (n_views < 0 || c->n < 0) return IGSP_ERR_DIMS;
  if (capacity < 0 || capacity >= (int64_t(1) << 31)) return IGSP_ERR_DIMS;
  if (c->n > 0 && (!c->gauss || !c->view || !c->pixel || !c->weight || !maps || (n_views > 0 && !views)))
    return IGSP_ERR_NULL;
  if (p->warmup != 0 && p->warmup != 1) return IGSP_ERR_PARAM;
  if (p->budget < 0) return IGSP_ERR_PARAM;
  if (std::isnan(p->grad_threshold)) return IGSP_ERR_PARAM;
  for (int32_t v = 0; v < n_views; ++v) {
    const igsp_view& d = views[v];
    if (d.width < 0 || d.height < 0 || d.out_offset < 0) return IGSP_ERR_DIMS;
    if ((int64_t)d.width * d.height >= (int64_t(1) << 31)) return IGSP_ERR_DIMS;
  }
  return IGSP_OK;
}

}  // namespace igsp

extern "C" double igsp_lr_exponential(int64_t t, double lr_init, double lr_final, int64_t t_max) {
  if (!(lr_init > 0.0) || !(lr_final > 0.0) || t_max < 1) return std::nan("");
  const double s = t < 0 ? 0.0 : (t > t_max ? 1.0 : (double)t / (double)t_max);
  return std::exp((1.0 - s) * std::log(lr_init) + s * std::log(lr_final));
}

extern "C" const char* igsp_status_string(int32_t status) {
  switch (status) {
    case IGSP_OK: return "ok";
    case IGSP_ERR_NULL: return "a required pointer is NULL";
    case IGSP_ERR_DIMS: return "invalid dimensions, offsets or counts";
    case IGSP_ERR_ALIGN: return "images must be 16-byte aligned";
    case IGSP_ERR_OVERLAP: return "input and output ranges overlap";
    case IGSP_ERR_PARAM: return "invalid parameter";
    case IGSP_ERR_CAPACITY: return "capacity exceeded: nothing was split";
    case IGSP_ERR_HIP: return "HIP runtime error";
    case IGSP_ERR_UNSUPPORTED: return "unsupported device (gfx950 required)";
    case IGSP_ERR_TIMEOUT: return "a wait inside the persistent launch gave up: its maps are not valid";
    case IGSP_ERR_TOO_LARGE: return "capacity above the fixed workspace of the allocation-free split (2^28 rows)";
    default: return "unknown status";
  }
}
