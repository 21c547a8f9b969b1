// Long-Axis-Split on gfx950 (Sec. 2.2 of arXiv 2603.08661, Algorithm 1 with
// the column-extraction transform of Algorithm 2).
//
// Three launches, so the split is all-or-nothing and the live count N can
// stay on the device (a captured graph stays valid as N grows); a small plain
// split (capacity <= 65536 rows) runs the same steps in one work-group and
// one launch (las_small_kernel):
//   las_count : per tile of 2048 live rows, the number of selected rows
//               (8 mask bytes per lane, a byte-wise non-zero test, popcount);
//   las_scan  : one work-group: exclusive scan of the live tiles' counts, K,
//               the capacity decision, status, and the new count N + K;
//   las_split : per tile, the selected rows compacted in ascending order in
//               LDS, then split with every lane busy: child A in place at row
//               i, child B appended at row N + rank (consecutive lanes write
//               consecutive rows), split_idx[rank] = i.
// Count and split work-groups stride over the live tiles with a grid fixed
// by the capacity, so a captured graph stays valid as N grows.
// All split arithmetic is FP32 in registers; the paper's transform reads
// only column l of R, computed straight from the normalised quaternion.

#include "igsp_internal.h"

namespace igsp {
namespace {

__device__ __forceinline__ int64_t live_rows(const LasLaunch& L) {
  const int64_t n = *L.g.count;
  return n < 0 ? 0 : (n > L.g.capacity ? L.g.capacity : n);
}

__device__ __forceinline__ int tiles_of(int64_t n) { return (int)((n + kLasRows - 1) / kLasRows); }

// The 8 mask bytes of rows [i0, i0 + 8); bytes of rows >= N read as 0. A
// full group is one unaligned 8-byte load; the group holding row N - 1 (if
// partial) reads its valid bytes one by one.
__device__ __forceinline__ uint64_t mask8(const LasLaunch& L, int64_t i0, int64_t N) {
  const int64_t valid = N - i0;
  if (valid >= 8) {
    uint64_t x;
    __builtin_memcpy(&x, L.mask + i0, 8);
    return x;
  }
  uint64_t x = 0;
  for (int k = 0; k < valid; ++k) x |= (uint64_t)L.mask[i0 + k] << (8 * k);
  return x;
}

// Bit 8k set iff byte k of x is non-zero.
__device__ __forceinline__ uint64_t nonzero_bytes(uint64_t x) {
  x |= x >> 4;
  x |= x >> 2;
  x |= x >> 1;
  return x & 0x0101010101010101ull;
}

// Exclusive scan of one value per thread over a work-group of NT threads.
template <int NT>
__device__ __forceinline__ int wg_scan(int v, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const int t = wsum[k];
    if (k < w) before += t;
    tot += t;
  }
  total = tot;
  __syncthreads();
  return before + x - v;
}

// Selected rows per tile of 2048 live rows (grid-stride over the live tiles).
__global__ __launch_bounds__(kLasThreads) void las_count_kernel(LasLaunch L) {
  __shared__ int wsum[kLasThreads / 64];
  const int64_t N = live_rows(L);
  const int nt = tiles_of(N);
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int64_t i0 = (int64_t)t * kLasRows + 8 * threadIdx.x;
    const int c = __popcll(nonzero_bytes(mask8(L, i0, N)));
    int total = 0;
    (void)wg_scan<kLasThreads>(c, wsum, total);
    if (threadIdx.x == 0) L.block_counts[t] = total;
  }
}

// One work-group: exclusive scan of the live tiles' counts, K, the capacity
// decision, status, and the new count N + K.
__global__ __launch_bounds__(1024) void las_scan_kernel(LasLaunch L) {
  __shared__ int64_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t N = live_rows(L);
  const int nt = tiles_of(N);
  const int per = (nt + 1023) / 1024;   // consecutive tiles per thread
  const int t0 = tid * per;
  int64_t v = 0;
  for (int k = 0; k < per; ++k)
    if (t0 + k < nt) v += L.block_counts[t0 + k];
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int64_t run = 0, K = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) run += wsum[k];
    K += wsum[k];
  }
  run += x - v;
  for (int k = 0; k < per; ++k)
    if (t0 + k < nt) {
      L.block_offsets[t0 + k] = run;
      run += L.block_counts[t0 + k];
    }
  if (tid == 0) {
    const int64_t n_raw = *L.g.count;
    const bool valid = n_raw >= 0 && n_raw <= L.g.capacity;
    const bool ok = valid && n_raw + K <= L.g.capacity;
    L.scalars->n_live = n_raw;
    L.scalars->k = K;
    L.scalars->ok = ok ? 1 : 0;
    *L.status = ok ? IGSP_OK : IGSP_ERR_CAPACITY;
    if (L.n_split) *L.n_split = K;
    if (ok) *L.g.count = n_raw + K;
  }
}

// The split of selected row i into child A (row i) and child B (row j).
__device__ __forceinline__ void split_row(const LasLaunch& L, int64_t i, int64_t j, int64_t rank) {
  // ---- Algorithm 1: longest axis (lowest index on ties)
  const float s0 = L.g.log_scales[3 * i], s1 = L.g.log_scales[3 * i + 1], s2 = L.g.log_scales[3 * i + 2];
  int l = 0;
  float sl = s0;
  if (s1 > sl) { l = 1; sl = s1; }
  if (s2 > sl) { l = 2; sl = s2; }
  const float offset = expf(sl) * L.alpha;
  const float n0 = s0 + (l == 0 ? L.ln_alpha : L.ln_gamma);
  const float n1 = s1 + (l == 1 ? L.ln_alpha : L.ln_gamma);
  const float n2 = s2 + (l == 2 ? L.ln_alpha : L.ln_gamma);
  // opacity: logit(beta * sigmoid(o)) = log(beta) - log(1 - beta + exp(-o))
  const float o = L.g.opacity_logits[i];
  const float on = o >= 0.0f ? L.ln_beta - logf(L.one_minus_beta + expf(-o))
                             : o + L.ln_beta - log1pf(L.one_minus_beta * expf(o));
  // ---- Algorithm 2: column l of R from the normalised quaternion
  const float qw = L.g.quats[4 * i], qx = L.g.quats[4 * i + 1], qy = L.g.quats[4 * i + 2],
              qz = L.g.quats[4 * i + 3];
  const float nq = qw * qw + qx * qx + qy * qy + qz * qz;
  float w_ = 1.0f, x_ = 0.0f, y_ = 0.0f, z_ = 0.0f;
  if (nq > 0.0f) {
    const float inv = 1.0f / sqrtf(nq);
    w_ = qw * inv; x_ = qx * inv; y_ = qy * inv; z_ = qz * inv;
  }
  float c0, c1, c2;
  if (l == 0) {
    c0 = 1.0f - 2.0f * (y_ * y_ + z_ * z_); c1 = 2.0f * (x_ * y_ + w_ * z_); c2 = 2.0f * (x_ * z_ - w_ * y_);
  } else if (l == 1) {
    c0 = 2.0f * (x_ * y_ - w_ * z_); c1 = 1.0f - 2.0f * (x_ * x_ + z_ * z_); c2 = 2.0f * (y_ * z_ + w_ * x_);
  } else {
    c0 = 2.0f * (x_ * z_ + w_ * y_); c1 = 2.0f * (y_ * z_ - w_ * x_); c2 = 1.0f - 2.0f * (x_ * x_ + y_ * y_);
  }
  const float d0 = c0 * offset, d1 = c1 * offset, d2 = c2 * offset;
  const float p0 = L.g.means[3 * i], p1 = L.g.means[3 * i + 1], p2 = L.g.means[3 * i + 2];
  // ---- children
  L.g.means[3 * i] = p0 + d0; L.g.means[3 * i + 1] = p1 + d1; L.g.means[3 * i + 2] = p2 + d2;
  L.g.means[3 * j] = p0 - d0; L.g.means[3 * j + 1] = p1 - d1; L.g.means[3 * j + 2] = p2 - d2;
  L.g.log_scales[3 * i] = n0; L.g.log_scales[3 * i + 1] = n1; L.g.log_scales[3 * i + 2] = n2;
  L.g.log_scales[3 * j] = n0; L.g.log_scales[3 * j + 1] = n1; L.g.log_scales[3 * j + 2] = n2;
  L.g.opacity_logits[i] = on;
  L.g.opacity_logits[j] = on;
  L.g.quats[4 * j] = qw; L.g.quats[4 * j + 1] = qx; L.g.quats[4 * j + 2] = qy; L.g.quats[4 * j + 3] = qz;
  L.split_idx[rank] = (int32_t)i;
}

// Row-wide work for the `total` selected rows of a tile: the second
// children's feature rows copied from the parents, and the given moment rows
// of both children cleared. The second children of a tile are consecutive
// rows, so their moment rows form one contiguous span, cleared with 16-byte
// stores. A parent's moment row of at most 4 floats is cleared by one lane;
// a wider row (features, their moments) by consecutive lanes, 64 / w rows per
// wavefront step (the lane's row and element come from divisions done once),
// each lane moving one float, or one float4 when the row width is a
// multiple of 4 and the array 16-byte aligned.

// Zero n floats from p (p 4-byte aligned): 16-byte stores in the aligned middle.
__device__ __forceinline__ void zero_span(float* p, int64_t n) {
  const int head = (int)min<int64_t>(n, ((16 - (int)(reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 4);
  if (threadIdx.x < head) p[threadIdx.x] = 0.0f;
  float* q = p + head;
  const int64_t m = n - head, m4 = m / 4;
  for (int64_t k = threadIdx.x; k < m4; k += kLasThreads)
    reinterpret_cast<float4*>(q)[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int64_t k = 4 * m4 + threadIdx.x; k < m; k += kLasThreads) q[k] = 0.0f;
}

// Lane layout for rows of width w (1 <= w): rows per wavefront step and this
// lane's (row, element), or a whole row per step split over 64-lane chunks.
struct RowLanes {
  int rpw;    // rows per wavefront step (0: one row, elements strided by 64)
  int lr, le; // this lane's row within the step and element
};

__device__ __forceinline__ RowLanes row_lanes(int w) {
  const int lane = threadIdx.x & 63;
  RowLanes r;
  if (w <= 64) {
    r.rpw = 64 / w;
    r.lr = lane / w;
    r.le = lane - r.lr * w;
    if (r.lr >= r.rpw) r.lr = -1;  // lanes past the last whole row idle
  } else {
    r.rpw = 0;
    r.lr = 0;
    r.le = lane;
  }
  return r;
}

// a[parent row] = 0 for the tile's selected rows.
__device__ __forceinline__ void zero_parents(float* a, int w, const RowLanes& rl, const int32_t* rows, int64_t base,
                                             int total) {
  const int wv = threadIdx.x >> 6;
  constexpr int NWV = kLasThreads / 64;
  if (rl.rpw > 0) {
    if (rl.lr < 0) return;
    for (int r = wv * rl.rpw + rl.lr; r < total; r += NWV * rl.rpw) a[(base + rows[r]) * w + rl.le] = 0.0f;
  } else {
    for (int r = wv; r < total; r += NWV)
      for (int e = rl.le; e < w; e += 64) a[(base + rows[r]) * w + e] = 0.0f;
  }
}

// Wide rows (width a multiple of 4 floats, 16-byte aligned array): a lane
// moves 16 bytes, and each wavefront keeps kWideInFlight rows' loads in
// flight before their stores (a row-by-row copy waits a full memory latency
// per row).
constexpr int kWideInFlight = 4;

__device__ __forceinline__ bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// dst row N + first + r = src row base + rows[r] for the tile's r < total
// (w4 = row width in float4).
__device__ __forceinline__ void copy_rows4(float4* a, int w4, const int32_t* rows, int64_t base, int64_t dst0,
                                           int total) {
  const RowLanes rl = row_lanes(w4);
  const int wv = threadIdx.x >> 6;
  constexpr int NWV = kLasThreads / 64;
  if (rl.rpw > 0) {
    if (rl.lr < 0) return;
    const int step = NWV * rl.rpw;
    for (int r0 = wv * rl.rpw + rl.lr; r0 < total; r0 += step * kWideInFlight) {
      // no lane branches around its loads or stores (a lane past the tile's
      // last row copies that row again: the same bytes to the same place),
      // so the rows stay in registers, all in flight before the stores
      static_assert(kWideInFlight == 4, "four named rows in flight");
      const int ra = min(r0, total - 1), rb = min(r0 + step, total - 1), rc = min(r0 + 2 * step, total - 1),
                rd = min(r0 + 3 * step, total - 1);
      const float4 va = a[(base + rows[ra]) * w4 + rl.le], vb = a[(base + rows[rb]) * w4 + rl.le],
                   vc = a[(base + rows[rc]) * w4 + rl.le], vd = a[(base + rows[rd]) * w4 + rl.le];
      a[(dst0 + ra) * w4 + rl.le] = va;
      a[(dst0 + rb) * w4 + rl.le] = vb;
      a[(dst0 + rc) * w4 + rl.le] = vc;
      a[(dst0 + rd) * w4 + rl.le] = vd;
    }
  } else {
    for (int r = wv; r < total; r += NWV)
      for (int e = rl.le; e < w4; e += 64) a[(dst0 + r) * w4 + e] = a[(base + rows[r]) * w4 + e];
  }
}

// The tile's parent rows of a wide array cleared with 16-byte stores.
__device__ __forceinline__ void zero_parents4(float4* a, int w4, const int32_t* rows, int64_t base, int total) {
  const RowLanes rl = row_lanes(w4);
  const int wv = threadIdx.x >> 6;
  constexpr int NWV = kLasThreads / 64;
  const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (rl.rpw > 0) {
    if (rl.lr < 0) return;
    for (int r = wv * rl.rpw + rl.lr; r < total; r += NWV * rl.rpw) a[(base + rows[r]) * w4 + rl.le] = z;
  } else {
    for (int r = wv; r < total; r += NWV)
      for (int e = rl.le; e < w4; e += 64) a[(base + rows[r]) * w4 + e] = z;
  }
}

// Narrow parent rows (W <= 4 floats) cleared one row per lane.
template <int W>
__device__ __forceinline__ void zero_parents_rows(float* a, const int32_t* rows, int64_t base, int total) {
  for (int r = threadIdx.x; r < total; r += kLasThreads) {
    float* p = a + (base + rows[r]) * W;
#pragma unroll
    for (int j = 0; j < W; ++j) p[j] = 0.0f;
  }
}

__device__ __forceinline__ void row_work(const LasLaunch& L, const int32_t* rows, int64_t base, int64_t N,
                                         int64_t first, int total) {
  const int F = L.g.feat_dim;
  const int wv = threadIdx.x >> 6;
  constexpr int NWV = kLasThreads / 64;
  const bool wideF = F > 0 && (F & 3) == 0;
  if (F > 0) {  // second children's features from the parents
    float* f = L.g.features;
    if (wideF && aligned16(f)) {
      copy_rows4(reinterpret_cast<float4*>(f), F / 4, rows, base, N + first, total);
    } else {
      const RowLanes rl = row_lanes(F);
      if (rl.rpw > 0) {
        if (rl.lr >= 0)
          for (int r = wv * rl.rpw + rl.lr; r < total; r += NWV * rl.rpw)
            f[(N + first + r) * F + rl.le] = f[(base + rows[r]) * F + rl.le];
      } else {
        for (int r = wv; r < total; r += NWV)
          for (int e = rl.le; e < F; e += 64) f[(N + first + r) * F + e] = f[(base + rows[r]) * F + e];
      }
    }
  }
  const igsp_adam_moments& A = L.adam;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    float* const narrow[4] = {A.means[m], A.log_scales[m], A.quats[m], A.opacity_logits[m]};
    const int width[4] = {3, 3, 4, 1};
    if (narrow[0]) zero_parents_rows<3>(narrow[0], rows, base, total);
    if (narrow[1]) zero_parents_rows<3>(narrow[1], rows, base, total);
    if (narrow[2]) zero_parents_rows<4>(narrow[2], rows, base, total);
    if (narrow[3]) zero_parents_rows<1>(narrow[3], rows, base, total);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (narrow[k]) zero_span(narrow[k] + (N + first) * width[k], (int64_t)total * width[k]);
    float* const fm = F > 0 ? A.features[m] : nullptr;
    if (fm) {
      if (wideF && aligned16(fm)) zero_parents4(reinterpret_cast<float4*>(fm), F / 4, rows, base, total);
      else zero_parents(fm, F, row_lanes(F), rows, base, total);
      zero_span(fm + (N + first) * F, (int64_t)total * F);
    }
  }
}

// Per live tile: the selected rows, compacted in ascending order into LDS
// (each thread owns 8 consecutive rows; a work-group scan places them), then
// split with every lane busy: consecutive lanes take consecutive ranks, so
// the appended children of a wavefront are contiguous rows. FULL adds the
// row-wide work (feature rows, optimiser moments); the plain split (no
// features, no moments) is compiled without it, so it keeps its registers
// for the split itself.
template <bool FULL>
__device__ __forceinline__ void split_tiles(const LasLaunch& L) {
  __shared__ int32_t rows[kLasRows];
  __shared__ int wsum[kLasThreads / 64];
  if (!L.scalars->ok) return;  // uniform across the grid
  const int64_t N = L.scalars->n_live;
  const int nt = tiles_of(N);
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int64_t base = (int64_t)t * kLasRows;
    const uint64_t nz = nonzero_bytes(mask8(L, base + 8 * threadIdx.x, N));
    int total = 0;
    int pos = wg_scan<kLasThreads>(__popcll(nz), wsum, total);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((nz >> (8 * k)) & 1ull) rows[pos++] = 8 * threadIdx.x + k;
    __syncthreads();
    const int64_t first = L.block_offsets[t];
    for (int k = threadIdx.x; k < total; k += kLasThreads) {
      const int64_t rank = first + k;
      split_row(L, base + rows[k], N + rank, rank);
    }
    if constexpr (FULL) row_work(L, rows, base, N, first, total);
    __syncthreads();  // rows[] is rewritten by the next tile
  }
}

// The plain split fits 64 registers: eight waves per SIMD.
__global__ __launch_bounds__(kLasThreads) __attribute__((amdgpu_waves_per_eu(8))) void las_split_kernel(LasLaunch L) {
  split_tiles<false>(L);
}

__global__ __launch_bounds__(kLasThreads) __attribute__((amdgpu_waves_per_eu(4))) void las_split_full_kernel(LasLaunch L) {
  split_tiles<true>(L);
}

// A small plain split (capacity <= kLasSmallCapacity rows) in one launch by
// one work-group: it counts the selected rows, takes the capacity decision,
// then compacts and splits them round by round (8 rows per thread and
// round). Same rows, same order, same all-or-nothing rule as the three
// launches; a call then costs one launch instead of three.
constexpr int kSmallThreads = 1024;
constexpr int kSmallRows = 8 * kSmallThreads;
constexpr int64_t kLasSmallCapacity = 8 * kSmallRows;

__global__ __launch_bounds__(kSmallThreads) void las_small_kernel(LasLaunch L) {
  __shared__ int32_t rows[kSmallRows];
  __shared__ int wsum[kSmallThreads / 64];
  __shared__ int s_ok;
  const int64_t N = live_rows(L);
  const int rounds = (int)((N + kSmallRows - 1) / kSmallRows);
  int64_t K = 0;  // the same in every thread (a work-group total)
  for (int r = 0; r < rounds; ++r) {
    int total = 0;
    (void)wg_scan<kSmallThreads>(__popcll(nonzero_bytes(mask8(L, (int64_t)r * kSmallRows + 8 * threadIdx.x, N))),
                                 wsum, total);
    K += total;
  }
  if (threadIdx.x == 0) {
    const int64_t n_raw = *L.g.count;
    const bool valid = n_raw >= 0 && n_raw <= L.g.capacity;
    const bool ok = valid && n_raw + K <= L.g.capacity;
    L.scalars->n_live = n_raw;
    L.scalars->k = K;
    L.scalars->ok = ok ? 1 : 0;
    *L.status = ok ? IGSP_OK : IGSP_ERR_CAPACITY;
    if (L.n_split) *L.n_split = K;
    if (ok) *L.g.count = n_raw + K;
    s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  if (!s_ok) return;  // uniform
  int64_t first = 0;
  for (int r = 0; r < rounds; ++r) {
    const int64_t base = (int64_t)r * kSmallRows;
    const uint64_t nz = nonzero_bytes(mask8(L, base + 8 * threadIdx.x, N));
    int total = 0;
    int pos = wg_scan<kSmallThreads>(__popcll(nz), wsum, total);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((nz >> (8 * k)) & 1ull) rows[pos++] = 8 * threadIdx.x + k;
    __syncthreads();
    for (int k = threadIdx.x; k < total; k += kSmallThreads) split_row(L, base + rows[k], N + first + k, first + k);
    first += total;
    __syncthreads();  // rows[] is rewritten by the next round
  }
}

}  // namespace

hipError_t launch_las(const LasLaunch& L, hipStream_t s) {
  const igsp_adam_moments& A = L.adam;
  bool full = L.g.feat_dim > 0;
  for (int m = 0; m < 2; ++m)
    full = full || A.means[m] || A.log_scales[m] || A.quats[m] || A.opacity_logits[m] || A.features[m];
  if (!full && L.g.capacity <= kLasSmallCapacity) {
    hipLaunchKernelGGL(las_small_kernel, dim3(1), dim3(kSmallThreads), 0, s, L);
    return hipGetLastError();
  }
  // grids are fixed by the capacity (the live count is only known on the
  // device); work-groups stride over the live tiles
  const int grid = L.n_blocks < kLasGrid ? L.n_blocks : kLasGrid;
  hipLaunchKernelGGL(las_count_kernel, dim3(grid), dim3(kLasThreads), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(las_scan_kernel, dim3(1), dim3(1024), 0, s, L);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (full) hipLaunchKernelGGL(las_split_full_kernel, dim3(grid), dim3(kLasThreads), 0, s, L);
  else hipLaunchKernelGGL(las_split_kernel, dim3(grid), dim3(kLasThreads), 0, s, L);
  return hipGetLastError();
}

}  // namespace igsp
