"""MI355X-native (gfx950) hot path of the ImprovedGS+ densification strategy.

Two operations, both hand-written HIP behind the C ABI of include/igsp.h:

* ``edge_importance`` -- per-view edge-score importance maps (Sec. 2.1 of
  arXiv 2603.08661: grayscale, 5x5 Gaussian blur, Sobel, non-maximum
  suppression, median normalisation), in a plain per-view form and a
  batched form with FP32, FP16 or BF16 intermediate storage;
* ``long_axis_split`` -- Long-Axis-Split of selected Gaussians (Sec. 2.2,
  Algorithms 1 and 2), in place into pre-allocated capacity;

plus ``Step``, one densification step recorded as a HIP graph.
"""
from ._binding import (  # noqa: F401
    BATCHED, BATCHED_PERSISTENT, BATCHED_STAGED, BF16, EXPORTS, FORMS, FP16, FP32, LIB_PATH, PLAIN, PRECISIONS,
    IgspError, Step, edge_autotune, edge_importance, edge_resolve, form_code, lib, long_axis_split, long_axis_split_full, lr_exponential, release_plans, split_mask, status_string,
    view_table,
)
