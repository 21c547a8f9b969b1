// Internal declarations of libigsp: device-side tables, plan workspaces and
// the launch wrappers each kernel file provides to the host layer.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/igsp.h"

namespace igsp {

// ---------------------------------------------------------------- edge path

// Strip geometry of the fused stencil kernel: a wavefront owns 64 lanes x 4
// adjacent columns = 256 input columns, of which the 4 outermost on each
// side are halo (2 blur + 1 Sobel + 1 suppression), leaving 248 outputs.
constexpr int kLanePx = 4;
constexpr int kWaveCols = 64 * kLanePx;       // 256
constexpr int kHalo = 4;
constexpr int kStripCols = kWaveCols - 2 * kHalo;  // 248
constexpr int kStageBytes = 1024;              // per-wave LDS row staging

// Survivor magnitudes are stored as sqrt(M) * 2^-13 (M the exact squared
// unnormalised Sobel magnitude, 1 <= M < 2^57 for 8-bit input): the scale
// keeps every value inside the normal range of FP16 and cancels in the
// normalisation. The median is found by radix selection on the bit pattern
// of the stored value widened to float32: the first histogram resolves the
// top 16 bits, whose possible range for survivors is [kKeyLo, kKeyLo+kBins).
constexpr float kStoreScale = 1.0f / 8192.0f;
constexpr uint32_t kKeyLo = 114u * 128u;  // float32 exponent 114 = 2^-13
constexpr int kBins = 30 * 128;           // 30 binades x 7 mantissa bits
constexpr int kRefineBins = 256;          // radix digit of the refine passes

struct ViewDesc {
  int32_t W, H;
  int64_t in_off;    // bytes from `images`
  int64_t out_off;   // floats from `out_maps`
  int64_t map_off;   // elements from the plan's map buffer (pitch W)
};

struct EdgeItem {    // one work-group of the fused stencil kernel
  int32_t view;
  int32_t x0;        // first output column of the strip
  int32_t y0;        // first output row of the band
  int32_t rows;      // output rows in the band
};

struct FlatItem {    // one work-group of an element-wise pass
  int32_t view;
  int32_t pad;
  int64_t p0, p1;    // flat pixel range [p0, p1) of the view
};

struct MedState {    // radix-select state of one view's median
  uint32_t prefix;   // resolved high bits of the float32 key
  int32_t shift;     // low bits still unresolved
  uint32_t rank;     // rank of the median inside the resolved bucket
  uint32_t n;        // survivors
  float med;         // median, stored units (valid once shift == final)
  uint32_t pad[3];
};

struct EdgeLaunch {
  const uint8_t* images;
  int64_t img_end;           // bytes of `images` that may be read
  float* out;
  const ViewDesc* views;
  const EdgeItem* items;
  const FlatItem* flat;
  void* map;
  uint32_t* hist;            // [n_views][kBins]
  uint32_t* rhist;           // [n_views][kRefineBins]
  MedState* state;           // [n_views]
  float* medians_dn;         // optional outputs
  int32_t* survivors;
  hipEvent_t* stage_events;  // optional, 4 events
  int precision;
  int wg_waves;
  int seg_rows;
};

// Enqueue each stage over the given ranges (item ranges index the plan's
// tables; view ranges are [v0, v1)).
hipError_t launch_edge_fused(const EdgeLaunch& L, int item0, int n_items, hipStream_t s);
hipError_t launch_median_select(const EdgeLaunch& L, int v0, int nv, hipStream_t s);
hipError_t launch_median_refine(const EdgeLaunch& L, int flat0, int n_flat, int digit_bits, hipStream_t s);
hipError_t launch_refine_select(const EdgeLaunch& L, int v0, int nv, int digit_bits, int final_shift,
                                hipStream_t s);
hipError_t launch_normalise(const EdgeLaunch& L, int flat0, int n_flat, hipStream_t s);

// ---------------------------------------------------------------- LAS

constexpr int kLasThreads = 256;
constexpr int kLasRounds = 8;
constexpr int kLasRows = kLasThreads * kLasRounds;  // rows per block

struct LasScalars {
  int64_t n_live;    // N read before the split
  int64_t k;         // rows selected
  int32_t ok;        // 1 if the split proceeds
  int32_t pad;
};

struct LasLaunch {
  igsp_gaussians g;
  const uint8_t* mask;
  int32_t* split_idx;
  int32_t* status;
  int64_t* n_split;
  float alpha, ln_alpha, ln_gamma, ln_beta, one_minus_beta;
  int32_t* block_counts;     // [n_blocks]
  int64_t* block_offsets;    // [n_blocks]
  LasScalars* scalars;
  int n_blocks;
};

hipError_t launch_las(const LasLaunch& L, hipStream_t s);

}  // namespace igsp
