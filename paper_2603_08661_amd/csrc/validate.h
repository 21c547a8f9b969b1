// Host-side validation of the C ABI (no HIP dependency).
#pragma once

#include <stdint.h>

#include "../../include/igsp.h"

namespace igsp {

struct EdgeExtent {
  int64_t img_end;   // bytes of `images` covered by the views
  int64_t out_end;   // floats of `out_maps` covered by the views
  int64_t pixels;    // total pixels
};

igsp_status validate_edge(const uint8_t* images, const igsp_view* views, int32_t n_views, const float* out,
                          const igsp_edge_opts* opts, EdgeExtent* ext);
igsp_status validate_select(const float* maps, const igsp_view* views, int32_t n_views,
                            const igsp_contributions* c, const float* grad, const int64_t* count,
                            int64_t capacity, const igsp_select_params* p, const uint8_t* mask,
                            const int64_t* scores);
igsp_status validate_las(const igsp_gaussians* g, const uint8_t* mask, const igsp_las_out* out,
                         const igsp_las_params* p);

}  // namespace igsp
