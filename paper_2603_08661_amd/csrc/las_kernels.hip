// Long-Axis-Split on gfx950 (Sec. 2.2 of arXiv 2603.08661, Algorithm 1 with
// the column-extraction transform of Algorithm 2).
//
// Three launches, so the split is all-or-nothing and the live count N can
// stay on the device (a captured graph stays valid as N grows):
//   las_count : per block of 2048 rows, the number of selected live rows
//               (wave ballots + popcount);
//   las_scan  : one work-group: exclusive scan of the block counts, K, the
//               capacity decision, status, and the new count N + K;
//   las_split : per block, the rank of each selected row (wave ballot +
//               mbcnt + block offset), then the split of that row: child A
//               in place at row i, child B appended at row N + rank (the
//               appended rows of one wavefront are contiguous, so those
//               writes coalesce), split_idx[rank] = i.
// All split arithmetic is FP32 in registers; the paper's transform reads
// only column l of R, computed straight from the normalised quaternion.

#include "igsp_internal.h"

namespace igsp {
namespace {

__device__ __forceinline__ int64_t live_rows(const LasLaunch& L) {
  const int64_t n = *L.g.count;
  return n < 0 ? 0 : (n > L.g.capacity ? L.g.capacity : n);
}

__global__ __launch_bounds__(kLasThreads) void las_count_kernel(LasLaunch L) {
  __shared__ int32_t wsum[kLasThreads / 64];
  const int64_t N = live_rows(L);
  const int64_t base = (int64_t)blockIdx.x * kLasRows;
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < kLasRounds; ++r) {
    const int64_t i = base + r * kLasThreads + threadIdx.x;
    const bool sel = i < N && L.mask[i] != 0;
    cnt += __popcll(__ballot(sel));
  }
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kLasThreads / 64; ++w) s += wsum[w];
    L.block_counts[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(1024) void las_scan_kernel(LasLaunch L) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < L.n_blocks; c0 += 1024) {
    const int b = c0 + tid;
    const int64_t v = b < L.n_blocks ? L.block_counts[b] : 0;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int64_t before = carry;
    for (int k = 0; k < w; ++k) before += wsum[k];
    if (b < L.n_blocks) L.block_offsets[b] = before + x - v;
    __syncthreads();
    if (tid == 0) {
      int64_t t = 0;
      for (int k = 0; k < 16; ++k) t += wsum[k];
      carry += t;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t n_raw = *L.g.count;
    const int64_t K = carry;
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

__global__ __launch_bounds__(kLasThreads) void las_split_kernel(LasLaunch L) {
  __shared__ int32_t wcnt[kLasThreads / 64];
  if (!L.scalars->ok) return;  // uniform across the grid
  const int64_t N = L.scalars->n_live;
  const int64_t base = (int64_t)blockIdx.x * kLasRows;
  int64_t running = L.block_offsets[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int F = L.g.feat_dim;
  for (int r = 0; r < kLasRounds; ++r) {
    const int64_t i = base + r * kLasThreads + threadIdx.x;
    const bool sel = i < N && L.mask[i] != 0;
    const uint64_t bal = __ballot(sel);
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int64_t woff = running;
    int total = 0;
    for (int k = 0; k < kLasThreads / 64; ++k) {
      if (k < w) woff += wcnt[k];
      total += wcnt[k];
    }
    __syncthreads();
    running += total;
    if (!sel) continue;

    const int64_t rank = woff + below;
    const int64_t j = N + rank;
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
    for (int f = 0; f < F; ++f) L.g.features[j * F + f] = L.g.features[i * F + f];
    L.split_idx[rank] = (int32_t)i;
  }
}

}  // namespace

hipError_t launch_las(const LasLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL(las_count_kernel, dim3(L.n_blocks), dim3(kLasThreads), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(las_scan_kernel, dim3(1), dim3(1024), 0, s, L);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(las_split_kernel, dim3(L.n_blocks), dim3(kLasThreads), 0, s, L);
  return hipGetLastError();
}

}  // namespace igsp
