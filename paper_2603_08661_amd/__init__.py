"""MI355X-native (gfx950) hot path of the ImprovedGS+ densification strategy.

Hand-written HIP behind the C ABI of include/igsp.h (arXiv 2603.08661):

* ``edge_importance`` -- per-view edge-score importance maps (Sec. 2.1:
  grayscale, 5x5 Gaussian blur, Sobel, non-maximum suppression, median
  normalisation), plain per view or batched over every view (staged,
  persistent or the unfused layout), with FP32, FP16 or BF16 storage of the
  one intermediate; ``edge_autotune`` / ``edge_resolve`` pick and report the
  form and tile shape;
* ``long_axis_split`` -- Long-Axis-Split of selected Gaussians (Sec. 2.2,
  Algorithms 1 and 2), in place into pre-allocated capacity;
  ``long_axis_split_full`` adds feature rows and the optimiser's moments;
  ``long_axis_split_noalloc`` is the split for callers that cannot allocate
  (a fixed workspace of the library, capacity up to 2^28 rows);
* ``split_mask`` -- which Gaussians to split: edge scores moved onto the
  Gaussians through pixel contributions, the gradient threshold with its
  warm-up, and a budget;
* ``lr_exponential`` -- the exponential learning-rate schedule (host);

plus ``Step``, one densification step (edge maps and split) recorded as a
HIP graph.
"""
from ._binding import (  # noqa: F401
    BATCHED, BATCHED_PERSISTENT, BATCHED_STAGED, BF16, EXPORTS, FORMS, FP16, FP32, LIB_PATH, PLAIN, PRECISIONS,
    IgspError, Step, edge_autotune, edge_importance, edge_resolve, form_code, lib, long_axis_split, long_axis_split_full,
    long_axis_split_noalloc,
    lr_exponential, release_plans, split_mask, status_string, view_table,
)
