// Split-mask generation on gfx950: which Gaussians the next Long-Axis-Split
// takes (the selection that feeds it; Sec. 2.1's edge scores moved to the
// Gaussians, Sec. 3's gradient threshold and warm-up, and a budget).
//
//   sel_clear   : scores[0, N) = 0, the radix histograms and the key OR = 0
//                 (fill kernels, so the call can be captured)
//   sel_scatter : per contribution (Gaussian g, view v, pixel p, weight w):
//                 scores[g] += floor(fl32(E_v[p] * w) * 2^32); each
//                 work-group sums a chunk of the contributions per Gaussian
//                 (runs on consecutive lanes, then an LDS hash table) and
//                 adds each sum with one 64-bit atomic; fixed
//                 point makes the sum exact and independent of the order
//                 the additions land in
//   sel_count<0> / sel_scan<0> : candidates (warm-up, or grad[g] >=
//                 threshold) per tile, their offsets, and
//                 K = min(candidates, max(0, budget - N))
//   sel_compact : the candidates' keys (score + 1) packed in row order, and
//                 the OR of them (the highest digit any of them uses)
//   sel_hist    : exact radix selection, 8 bits at a time from the highest
//                 used digit, of the K-th largest key among the packed keys;
//                 each pass first resolves the previous pass's digit from
//                 that pass's histogram (every work-group alike), so no
//                 separate launch picks the digit
//   sel_count<1> / sel_scan<1> / sel_mask : the last digit, then ties at the
//                 K-th key taken in ascending index order (per-tile counts,
//                 one scan, write)
#include "igsp_internal.h"

namespace igsp {
namespace {

__device__ __forceinline__ int64_t live_count(const SelLaunch& S) {
  const int64_t n = *S.count;
  return n < 0 ? 0 : (n > S.capacity ? S.capacity : n);
}

__device__ __forceinline__ bool candidate(const SelLaunch& S, int64_t g) {
  return S.warmup || S.grad[g] >= S.grad_threshold;
}

__device__ __forceinline__ uint64_t key_of(const SelLaunch& S, int64_t g) {
  return candidate(S, g) ? (uint64_t)S.scores[g] + 1ull : 0ull;
}

__global__ __launch_bounds__(kSelThreads) void sel_clear_kernel(SelLaunch S) {
  const int64_t N = live_count(S);
  for (int64_t g = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; g < N; g += (int64_t)gridDim.x * kSelThreads)
    S.scores[g] = 0;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < 3 * 256; i += kSelThreads) S.hist[i] = 0;
    if (threadIdx.x == 0) S.state->top = 0;
  }
}

// Contributions arrive in image order, so neighbouring entries often name the
// same Gaussian, and a Gaussian's entries recur a few image rows later. The
// grid sweeps the list in order, one chunk of kScatterRounds x kSelThreads
// contributions per work-group at a time (so the map reads of neighbouring
// chunks stay close). Each wavefront first sums the runs of equal Gaussian
// index on consecutive lanes (a segmented suffix sum over the lanes); a run's
// first lane then adds the run's sum into the work-group's LDS hash table
// (open addressing, kScatterProbes linear probes; a run that finds no slot
// goes straight to its global atomic); at the end of the chunk every used
// slot issues one 64-bit atomic and is cleared.
constexpr int kScatterRounds = 16;
constexpr int kScatterSlots = 1024;  // 12 KB of LDS: keys and 64-bit sums
constexpr int kScatterProbes = 16;
static_assert(kScatterSlots == 1 << 10, "the slot hash keeps the top 10 bits");

// LDS_VIEWS: the view table is copied into (dynamic) LDS first, so each
// contribution's map read waits on one global load fewer.
constexpr int kSelLdsViews = 512;  // at most this many views go to LDS (8 KB)

template <bool LDS_VIEWS>
__global__ __launch_bounds__(kSelThreads) void sel_scatter_kernel(SelLaunch S) {
  __shared__ int32_t keys[kScatterSlots];
  __shared__ unsigned long long sums[kScatterSlots];
  extern __shared__ SelView lviews[];
  constexpr int64_t kChunk = (int64_t)kScatterRounds * kSelThreads;
  const int64_t N = live_count(S);
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < kScatterSlots; i += kSelThreads) {
    keys[i] = -1;
    sums[i] = 0ull;
  }
  if constexpr (LDS_VIEWS)
    for (int i = threadIdx.x; i < S.n_views; i += kSelThreads) lviews[i] = S.views[i];
  __syncthreads();
  for (int64_t b0 = (int64_t)blockIdx.x * kChunk; b0 < S.n_contrib; b0 += (int64_t)gridDim.x * kChunk) {
    const int64_t b1 = b0 + kChunk < S.n_contrib ? b0 + kChunk : S.n_contrib;
    // software pipeline over the chunk's rounds: while round r's values are
    // scattered, round r + 1's map value and round r + 2's entries are in
    // flight (entries past the chunk read as ignored)
    auto load_entry = [&](int64_t c, int32_t& gi, int32_t& v, int32_t& p, float& w) {
      gi = -1;
      if (c < b1) {
        gi = S.gauss[c]; v = S.view[c]; p = S.pixel[c]; w = S.weight[c];
      }
    };
    // the contribution's map value (0 for an ignored entry) and its Gaussian (-1)
    auto map_value = [&](int32_t gi, int32_t v, int32_t p, float w, int32_t& g) -> float {
      g = -1;
      if (gi >= 0 && gi < N && v >= 0 && v < S.n_views) {                 // else outside the live set: ignored
        const SelView sv = LDS_VIEWS ? lviews[v] : S.views[v];
        if (p >= 0 && (int64_t)p < sv.pixels) {
          g = gi;
          return S.maps[sv.out_offset + p] * w;                            // one FP32 product
        }
      }
      return 0.0f;
    };
    int32_t gi1 = -1, v1 = 0, p1 = 0, gi2 = -1, v2 = 0, p2 = 0, g1 = -1;
    float w1 = 0.0f, w2 = 0.0f;
    load_entry(b0 + threadIdx.x, gi1, v1, p1, w1);
    load_entry(b0 + kSelThreads + threadIdx.x, gi2, v2, p2, w2);
    float e1 = map_value(gi1, v1, p1, w1, g1);
    for (int64_t c0 = b0; c0 < b1; c0 += kSelThreads) {
      const int32_t g = g1;
      const float e = e1;
      e1 = map_value(gi2, v2, p2, w2, g1);                                 // round r + 1
      load_entry(c0 + 2 * kSelThreads + threadIdx.x, gi2, v2, p2, w2);    // round r + 2
      uint64_t q = 0;
      if (e > 0.0f) q = (uint64_t)floorf(e * 4294967296.0f);               // exact: a power-of-two scale
      const int32_t gp = __shfl_up(g, 1, 64);
      const bool head = lane == 0 || gp != g;
      const uint64_t heads = __ballot(head);
      const int rid = __popcll(heads & ((2ull << lane) - 1ull));        // run of this lane
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint64_t qo = __shfl_down(q, o, 64);
        const int ro = __shfl_down(rid, o, 64);
        if (lane + o < 64 && ro == rid) q += qo;
      }
      if (head && g >= 0 && q != 0) {
        uint32_t h = ((uint32_t)g * 2654435761u) >> (32 - 10);         // 10 bits: kScatterSlots
        bool placed = false;
        for (int k = 0; k < kScatterProbes && !placed; ++k) {
          const int32_t prev = atomicCAS(&keys[h], -1, g);
          if (prev == -1 || prev == g) {
            atomicAdd(&sums[h], (unsigned long long)q);
            placed = true;
          }
          h = (h + 1) & (kScatterSlots - 1);
        }
        if (!placed) atomicAdd(reinterpret_cast<unsigned long long*>(S.scores + g), (unsigned long long)q);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kScatterSlots; i += kSelThreads) {
      const int32_t g = keys[i];
      if (g >= 0) {
        const unsigned long long q = sums[i];
        if (q != 0ull) atomicAdd(reinterpret_cast<unsigned long long*>(S.scores + g), q);
        keys[i] = -1;
        sums[i] = 0ull;
      }
    }
    __syncthreads();
  }
}

// Exclusive scan over the work-group (kSelThreads threads).
__device__ __forceinline__ uint32_t sel_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kSelThreads / 64; ++k) {
    const uint32_t t = wsum[k];
    if (k < w) before += t;
    tot += t;
  }
  total = tot;
  __syncthreads();
  return before + x - v;
}

__device__ __forceinline__ void radix_pick(const uint32_t* cnt, SelRadix& r, uint32_t* wsum, int64_t* pick);

// Per tile of kSelTile rows: candidates (mode 0) or keys equal to the
// selected K-th key (mode 1, which first resolves the last digit from the
// last radix pass's histogram; work-group 0 records the result).
template <int MODE>
__global__ __launch_bounds__(kSelThreads) void sel_count_kernel(SelLaunch S) {
  __shared__ uint32_t wsum[kSelThreads / 64];
  __shared__ int64_t pick[2];
  const int64_t N = live_count(S);
  const int nt = (int)((N + kSelTile - 1) / kSelTile);
  uint64_t T = 0;
  if (MODE == 1) {
    SelRadix r = S.ring[(kSelPasses - 1) & 1];
    if (r.shift > 0) radix_pick(S.hist + ((kSelPasses - 1) % 3) * 256, r, wsum, pick);
    T = r.prefix;  // every digit resolved: the K-th largest key (0 when K = 0)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      S.state->prefix = r.prefix;
      S.state->kth = r.prefix;
      S.state->rank = r.rank;
      S.state->shift = r.shift;
    }
  }
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    uint32_t c = 0;
    for (int k = 0; k < kSelTile / kSelThreads; ++k) {
      const int64_t g = (int64_t)t * kSelTile + k * kSelThreads + threadIdx.x;
      if (g < N) c += MODE == 0 ? (candidate(S, g) ? 1u : 0u) : (key_of(S, g) == T ? 1u : 0u);
    }
    uint32_t total = 0;
    (void)sel_scan(c, wsum, total);
    if (threadIdx.x == 0) S.tile_counts[t] = total;
  }
}

// One work-group: exclusive scan of the tile counts; mode 0 derives K and
// starts the selection, mode 1 turns the tie counts into tie ranks.
template <int MODE>
__global__ __launch_bounds__(1024) void sel_scan_kernel(SelLaunch S) {
  __shared__ int64_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t N = live_count(S);
  const int nt = (int)((N + kSelTile - 1) / kSelTile);
  const int per = (nt + 1023) / 1024;
  const int t0 = tid * per;
  int64_t v = 0;
  for (int k = 0; k < per; ++k)
    if (t0 + k < nt) v += S.tile_counts[t0 + k];
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int64_t run = 0, total = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) run += wsum[k];
    total += wsum[k];
  }
  run += x - v;
  for (int k = 0; k < per; ++k)
    if (t0 + k < nt) {
      S.tile_offsets[t0 + k] = run;
      run += S.tile_counts[t0 + k];
    }
  if (tid == 0) {
    SelState* st = S.state;
    if (MODE == 0) {
      const int64_t room = S.budget > N ? S.budget - N : 0;
      const int64_t K = total < room ? total : room;
      st->candidates = total;
      st->k = K;
      st->prefix = 0;
      st->rank = K;          // the K-th largest key: K - 1 keys above it
      st->shift = 64;
      st->kth = 0;           // (the radix passes keep their progress in the ring)
      if (S.n_selected) *S.n_selected = K;
    } else {
      st->ties = total;
    }
  }
}

// Packs the candidates' keys in row order (tile offsets from sel_scan<0>)
// and ORs them into the state: the highest set bit of the OR bounds every
// candidate key, so the radix passes start at the highest digit in use.
__global__ __launch_bounds__(kSelThreads) void sel_compact_kernel(SelLaunch S) {
  __shared__ uint32_t wsum[kSelThreads / 64];
  __shared__ uint64_t wor[kSelThreads / 64];
  const int64_t N = live_count(S);
  const int nt = (int)((N + kSelTile - 1) / kSelTile);
  uint64_t acc = 0;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int64_t before = S.tile_offsets[t];
    for (int k = 0; k < kSelTile / kSelThreads; ++k) {
      const int64_t g = (int64_t)t * kSelTile + k * kSelThreads + threadIdx.x;
      const bool cand = g < N && candidate(S, g);
      const uint64_t key = cand ? (uint64_t)S.scores[g] + 1ull : 0ull;
      uint32_t total = 0;
      const uint32_t r = sel_scan(cand ? 1u : 0u, wsum, total);
      if (cand) S.ckeys[before + r] = key;
      acc |= key;
      before += total;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc |= __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) wor[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) a |= wor[w];
    if (a) atomicOr(reinterpret_cast<unsigned long long*>(&S.state->top), (unsigned long long)a);
  }
}

// Resolves the digit of a radix pass from its histogram cnt[256] (all
// threads of the work-group take part): the largest digit d whose keys and
// those of all higher digits number at least the rank; the rank becomes the
// rank inside digit d. Suffix sums come from a scan over the digits in
// descending order (thread t holds digit 255 - t).
__device__ __forceinline__ void radix_pick(const uint32_t* cnt, SelRadix& r, uint32_t* wsum, int64_t* pick) {
  const int t = threadIdx.x, d = 255 - t;
  const uint32_t c = cnt[d];
  uint32_t total = 0;
  const uint64_t above = sel_scan(c, wsum, total);   // keys of digits > d
  const uint64_t upto = above + c;                   // keys of digits >= d
  if ((int64_t)above < r.rank && ((int64_t)upto >= r.rank || d == 0)) {
    pick[0] = d;
    pick[1] = r.rank - (int64_t)above;
  }
  __syncthreads();
  r.prefix = (r.prefix << 8) | (uint64_t)pick[0];
  r.rank = pick[1];
  r.shift -= 8;
  __syncthreads();
}

// Radix pass `pass`: resolve the previous pass's digit (pass 0: the highest
// digit in use), then count the next digit of the packed keys whose
// resolved high bits equal the prefix. Work-group 0 records the selection
// for the next pass and clears the histogram slot the pass after next
// adds into (last read by the pass before this one).
__global__ __launch_bounds__(kSelThreads) void sel_hist_kernel(SelLaunch S, int pass) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t wsum[kSelThreads / 64];
  __shared__ int64_t pick[2];
  SelRadix r;
  if (pass == 0) {
    const SelState st = *S.state;
    const int bits = st.top ? 64 - __clzll((long long)st.top) : 0;
    r = SelRadix{0ull, st.k, st.k > 0 ? (bits + 7) / 8 * 8 : 0, 0};
  } else {
    r = S.ring[(pass - 1) & 1];
    if (r.shift > 0) radix_pick(S.hist + ((pass - 1) % 3) * 256, r, wsum, pick);
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) S.ring[pass & 1] = r;
    if (pass >= 2) S.hist[((pass + 1) % 3) * 256 + threadIdx.x] = 0;
  }
  if (r.shift == 0) return;  // nothing to select, or resolved
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = S.state->candidates;
  const int shift = r.shift - 8;
  for (int64_t c = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; c < n; c += (int64_t)gridDim.x * kSelThreads) {
    const uint64_t key = S.ckeys[c];
    if (r.shift == 64 || (key >> r.shift) == r.prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t cnt = h[threadIdx.x];
  if (cnt) atomicAdd(&S.hist[(pass % 3) * 256 + threadIdx.x], cnt);
}

__global__ __launch_bounds__(kSelThreads) void sel_mask_kernel(SelLaunch S) {
  __shared__ uint32_t wsum[kSelThreads / 64];
  const SelState st = *S.state;
  const int64_t N = live_count(S);
  const int nt = (int)((N + kSelTile - 1) / kSelTile);
  // keys above the K-th key: K - rank of them; the remaining `need` come
  // from the ties at the K-th key, lowest index first
  const int64_t need = st.rank;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int64_t before = st.k > 0 ? S.tile_offsets[t] : 0;
    for (int k = 0; k < kSelTile / kSelThreads; ++k) {
      const int64_t g = (int64_t)t * kSelTile + k * kSelThreads + threadIdx.x;
      const uint64_t key = g < N ? key_of(S, g) : 0;
      const bool tie = st.k > 0 && g < N && key == st.kth;
      uint32_t total = 0;
      const uint32_t r = sel_scan(tie ? 1u : 0u, wsum, total);
      if (g < N) S.mask[g] = (uint8_t)(st.k > 0 && (key > st.kth || (tie && before + r < need)));
      before += total;
    }
  }
}

}  // namespace

hipError_t launch_select(const SelLaunch& S, hipStream_t s) {
  const int grid = S.grid;
  hipLaunchKernelGGL(sel_clear_kernel, dim3(grid), dim3(kSelThreads), 0, s, S);
  if (S.n_contrib > 0) {
    const int64_t chunks = (S.n_contrib + kScatterRounds * kSelThreads - 1) / (kScatterRounds * kSelThreads);
    const dim3 g((unsigned)(chunks < kSelScatterGrid ? chunks : kSelScatterGrid));
    if (S.n_views <= kSelLdsViews)
      hipLaunchKernelGGL(sel_scatter_kernel<true>, g, dim3(kSelThreads), (size_t)S.n_views * sizeof(SelView), s, S);
    else
      hipLaunchKernelGGL(sel_scatter_kernel<false>, g, dim3(kSelThreads), 0, s, S);
  }
  hipLaunchKernelGGL(sel_count_kernel<0>, dim3(grid), dim3(kSelThreads), 0, s, S);
  hipLaunchKernelGGL(sel_scan_kernel<0>, dim3(1), dim3(1024), 0, s, S);
  hipLaunchKernelGGL(sel_compact_kernel, dim3(grid), dim3(kSelThreads), 0, s, S);
  for (int pass = 0; pass < kSelPasses; ++pass)
    hipLaunchKernelGGL(sel_hist_kernel, dim3(grid), dim3(kSelThreads), 0, s, S, pass);
  hipLaunchKernelGGL(sel_count_kernel<1>, dim3(grid), dim3(kSelThreads), 0, s, S);
  hipLaunchKernelGGL(sel_scan_kernel<1>, dim3(1), dim3(1024), 0, s, S);
  hipLaunchKernelGGL(sel_mask_kernel, dim3(grid), dim3(kSelThreads), 0, s, S);
  return hipGetLastError();
}

}  // namespace igsp
