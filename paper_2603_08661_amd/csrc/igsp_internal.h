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

// What the stencil pass stores for a surviving pixel, from the exact squared
// unnormalised Sobel magnitude M (1 <= M < 2^57 for 8-bit input):
//   FP16 storage : q = sqrt(M) * 2^-13, inside FP16's normal range;
//   FP32 / BF16  : q = M itself (no root in the stencil; the normalisation
//                  takes sqrt(q / median), which also halves BF16's rounding).
// Both are monotone in M, so the lower median of q is the q of the median
// magnitude. The median is found by radix selection on the bit pattern of
// q widened to float32; the first histogram resolves the top 16 bits
// (exponent + 7 mantissa bits), whose possible range for survivors is
// [key_lo, key_lo + bins).
constexpr float kStoreScaleRoot = 1.0f / 8192.0f;          // 2^-13
constexpr uint32_t kKeyLoRoot = 114u * 128u;               // float32 exponent of 2^-13
constexpr int kBinsRoot = 30 * 128;                        // 2^-13 .. 2^17
constexpr uint32_t kKeyLoSquare = 127u * 128u;             // float32 exponent of 1
constexpr int kBinsSquare = 58 * 128;                      // 1 .. 2^58
constexpr int kBinsMax = kBinsSquare;
constexpr int kRefineBins = 256;          // radix digit of the refine passes
constexpr int kRefineChunkSlots = 64;     // slots per work-group of a refinement pass

// The stored intermediate of a view is kept strip by strip: strip s (output
// columns 248 s .. 248 s + 247) holds its rows one after another in slots of
// 256 values (its 248 outputs and 8 unused values: one aligned 512-byte or
// 1 KiB store per wavefront and row, whole cache lines only). Row c of strip
// s starts at element map_off + (s * strip_rows + c) * 256, strip_rows = H.
// Every stencil wavefront thus writes one contiguous stream and no cache line
// is shared between two slots.
constexpr int kStripGroups = kStripCols / kLanePx;  // 62 groups of 4 pixels
constexpr int kSlotPitch = kWaveCols;               // 256 values per stored row

struct ViewDesc {
  int32_t W, H;
  int64_t in_off;      // bytes from `images`
  int64_t out_off;     // floats from `out_maps`
  int64_t map_off;     // elements from the plan's map buffer
  int32_t strip_rows;  // rows per strip of the stored map (H)
  int32_t cand_cap;    // FP32: room for the view's median candidates (0: none)
  int64_t cand_off;    // first candidate of the view in the candidate buffer
};

struct EdgeItem {    // one work-group of the fused stencil kernel
  int32_t view;
  int32_t x0;        // first output column of the strip
  int32_t y0;        // first output row of the band
  int32_t rows;      // output rows in the band
};

// One work-group of an element-wise pass (median refinement, normalisation):
// slots [u0, u1) of a view, in row-major order over (row c, strip s), slot
// u = c * strips + s. Consecutive slots cover consecutive pixels of the map,
// so a chunk's output is one contiguous range.
struct RowChunk {
  int32_t view;
  int32_t u0, u1;
  int32_t pad;
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
  const RowChunk* chunks;
  void* map;
  uint32_t* hist;            // [n_views][kBinsMax]
  uint32_t* rhist;           // [2][n_views][kRefineBins]: refinement pass p's digit histograms
  MedState* state;           // [3][n_views]: the selection state after p refinement steps
  uint32_t* cand;            // FP32: survivors in the first histogram's median bucket, per view
  uint32_t* cand_n;          // [n_views]: candidates found (more than the room: list not used)
  int use_cand;              // the refinement passes of this launch use the candidate lists
  float* medians_dn;         // optional outputs
  int32_t* survivors;
  hipEvent_t* stage_events;  // optional, 4 events
  int32_t* status;           // optional device status word
  int precision;
  int wg_waves;
  int seg_rows;
  int n_views;               // views of the plan (the stride of state and rhist)
};

// Work list of the single persistent launch of the batched form. Phases of
// a view: 0 = stencil items, 1..levels = refinement passes of the median's
// radix selection, levels + 1 = normalisation; each later phase waits for
// the selection step that closes the phase before it.
enum : int32_t { kTaskStencil = 0, kTaskRefine = 1, kTaskNorm = 2 };

struct PTask {
  int32_t type;
  int32_t view;
  int32_t idx;       // stencil: index into items; refine / norm: into chunks
  int32_t phase;     // 0 .. levels + 1
};

struct PViewSync {   // per view, in device memory
  uint32_t left[4];  // tasks of each phase still running; the last one
                     // restores the count for the next launch
  uint32_t ready;    // selection steps completed (reset to 0 at the end)
  uint32_t n_items;  // restore values: stencil items, row chunks
  uint32_t n_chunks;
  uint32_t pad;
};

struct PCtl {        // whole launch, in device memory
  uint32_t queue;    // next task to hand out
  uint32_t exited;   // work-groups that found the queue empty
  uint32_t error;    // bit 0: a wait exceeded its spin limit
  uint32_t pad;
};

struct PersistLaunch {
  const PTask* tasks;
  PViewSync* sync;
  PCtl* ctl;
  int32_t n_tasks;
  int32_t levels;      // refinement passes: BF16 0, FP16 1, FP32 2
  int32_t n_views;
  uint32_t spin_limit; // polls before a wait gives up (>= 1)
  uint32_t wait_bias;  // added to every awaited level: 0, or (host-forced
                       // timeouts, for tests) a level no view ever reaches
};

// Polls of one wait of the persistent form before it gives up (about half a
// second); the host can shorten it to force the timeout path in tests.
constexpr uint32_t kSpinLimit = 1u << 19;

// The unfused form (the paper's layout, kept as an ablation): one kernel per
// step over tiles of 256 columns x kUfRows rows, each step's result in HBM.
constexpr int kUfCols = 256;
constexpr int kUfRows = 32;

struct UfItem {
  int32_t view, x0, y0, pad;
};

struct UfLaunch {
  const UfItem* items;
  int32_t n_items;
  int32_t* gray;     // 299 R + 587 G + 114 B, per pixel (plan map layout)
  int32_t* blur;     // 5x5 binomial blur x 256000
  float* mag;        // squared Sobel magnitude
  uint8_t* code;     // orientation: bit 0 cH, bit 1 cV, bit 2 c45, bit 3 gradient along -e
};

// Enqueue each stage over the given ranges (item ranges index the plan's
// tables; view ranges are [v0, v1)).
hipError_t launch_edge_fused(const EdgeLaunch& L, int item0, int n_items, hipStream_t s);
hipError_t launch_median_select(const EdgeLaunch& L, int v0, int nv, hipStream_t s);
hipError_t launch_median_refine(const EdgeLaunch& L, int chunk0, int n_chunks, int pass, hipStream_t s);
// the last selection step where the normalisation does not take it (no-op otherwise)
hipError_t launch_median_step(const EdgeLaunch& L, int v0, int nv, hipStream_t s);
hipError_t launch_normalise(const EdgeLaunch& L, int chunk0, int n_chunks, hipStream_t s);
// The stencil steps of the unfused form: gray, blur, Sobel, suppression
// (+ histogram), four launches; the median and normalisation follow as in the
// staged form.
hipError_t launch_edge_unfused(const EdgeLaunch& L, const UfLaunch& U, hipStream_t s);
// The whole batched pipeline as one launch of `grid` persistent work-groups.
hipError_t launch_edge_persistent(const EdgeLaunch& L, const PersistLaunch& P, int grid, hipStream_t s);
// Work-groups of the persistent kernel resident per compute unit.
int persistent_blocks_per_cu(int precision, int wg_waves);

// ---------------------------------------------------------------- LAS

constexpr int kLasThreads = 256;
constexpr int kLasRounds = 8;
constexpr int kLasRows = kLasThreads * kLasRounds;  // rows per tile (8 per thread)
constexpr int kLasGrid = 1024;                      // work-groups of the count and split kernels

struct LasScalars {
  int64_t n_live;    // N read before the split
  int64_t k;         // rows selected
  int32_t ok;        // 1 if the split proceeds
  int32_t pad;
};

struct LasLaunch {
  igsp_gaussians g;
  igsp_adam_moments adam;    // all NULL for the plain split
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

// ---------------------------------------------------------------- split mask

constexpr int kSelThreads = 256;
constexpr int kSelTile = 2048;         // rows per tile of the count / mask kernels
constexpr int kSelGrid = 1024;         // work-groups of the grid-stride kernels
constexpr int kSelScatterGrid = 2048;  // work-groups of the contribution scatter (8 waves per SIMD)

struct SelView {
  int64_t out_offset;  // floats from `maps`
  int64_t pixels;      // width * height
};

struct SelState {      // device scalars of one selection
  uint64_t prefix;     // resolved high bits of the K-th largest key
  uint64_t kth;        // the K-th largest key (valid once shift == 0)
  int64_t rank;        // rank inside the prefix group, from the top; at the
                       // end: the ties at kth still to take
  int64_t k;           // Gaussians to select
  int64_t candidates;
  int64_t ties;
  uint64_t top;        // bitwise OR of the candidates' keys
  int32_t shift;       // low bits still unresolved
  int32_t pad;
};

struct SelRadix {      // the selection after one radix pass
  uint64_t prefix;
  int64_t rank;
  int32_t shift;
  int32_t pad;
};

constexpr int kSelPasses = 8;  // 8-bit digits of a 64-bit key

struct SelLaunch {
  const float* maps;
  const SelView* views;
  int32_t n_views;
  const int32_t* gauss;
  const int32_t* view;
  const int32_t* pixel;
  const float* weight;
  int64_t n_contrib;
  const float* grad;
  const int64_t* count;
  int64_t capacity;
  float grad_threshold;
  int32_t warmup;
  int64_t budget;
  uint8_t* mask;
  int64_t* scores;
  int64_t* n_selected;
  uint32_t* hist;           // [3][256]: pass p adds into slot p % 3, reads p - 1's
  SelRadix* ring;           // [2]: the selection after pass p in slot p % 2
  uint64_t* ckeys;          // [capacity]: the candidates' keys, in row order
  uint32_t* tile_counts;    // [tiles]
  int64_t* tile_offsets;    // [tiles]
  SelState* state;
  int grid;
};

hipError_t launch_select(const SelLaunch& S, hipStream_t s);

}  // namespace igsp
