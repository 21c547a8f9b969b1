// Edge-score importance maps on gfx950 (Sec. 2.1 of arXiv 2603.08661).
//
// Stage 1, edge_fused: one pass over the 8-bit RGB input computes grayscale,
// the binomial 5x5 blur, the Sobel gradient, the orientation bin and the
// non-maximum suppression, writes the surviving magnitudes (FP32, FP16 or
// BF16 storage) and accumulates a per-view histogram of their top 16 bits.
// The paper runs these as separate kernels with HBM intermediates and names
// a shared-memory fusion as future work; here nothing between the bytes and
// the suppressed magnitude leaves the register file.
//
//   - A wavefront owns a vertical strip of 256 input columns (64 lanes x 4
//     adjacent pixels) and marches down its rows. Vertical taps live in
//     register sliding windows; horizontal neighbours cross lanes with DPP
//     wave shifts (one VALU modifier per value), never through LDS.
//   - Rows are not 4-byte aligned (pitch 3*W), so each row span is fetched as
//     aligned 16-byte chunks into a per-wave LDS buffer, prefetched one row
//     ahead, and every lane extracts its 12 bytes with byte-align shifts.
//   - Gray, blur and Sobel run in exact 32-bit integers (|gx|,|gy| < 2^28).
//     The magnitude, its orientation test and the suppression comparisons
//     are FP32.
//
// Stage 2, median_select / median_refine / refine_select: exact radix
// selection of the lower median of each view's stored survivor values; BF16
// needs no refinement, FP16 one 3-bit pass, FP32 two 8-bit passes.
// Stage 3, normalise: map = stored / median at survivors, 0 elsewhere.

#include <hip/hip_fp16.h>

#include "igsp_internal.h"

namespace igsp {
namespace {

// ------------------------------------------------------------- cross-lane

// DPP wave shifts: lane i receives lane i-1 (from_left) or i+1 (from_right);
// lanes at the wave ends receive 0 (only halo columns depend on them).
// The moves are kept opaque to the compiler: folding them into the
// consuming ALU instruction (a combined VOP2 DPP op with a wave shift) gave
// wrong values at run time on gfx950 in this toolchain, while the plain
// v_mov_b32_dpp form is exact.
__device__ __forceinline__ int from_left(int v) {
  int r = __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
  asm volatile("" : "+v"(r));
  return r;
}
__device__ __forceinline__ int from_right(int v) {
  int r = __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
  asm volatile("" : "+v"(r));
  return r;
}
__device__ __forceinline__ float from_left(float v) { return __int_as_float(from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(from_right(__float_as_int(v))); }

// Reflect-101 as an even periodic extension of period 2(n-1): the same map as
// mirroring each stage at the border, because the blur is symmetric and the
// Sobel difference odd (so the squared magnitude is again even).
__device__ __forceinline__ int fold(int i, int n) {
  const int P = 2 * (n - 1);
  i %= P;
  if (i < 0) i += P;
  return i < n ? i : P - i;
}

// ------------------------------------------------------------- storage

template <int PREC> struct Store;
template <> struct Store<IGSP_FP32> {
  using T = float;
  __device__ static float round(float v) { return v; }
  __device__ static float widen(float v) { return v; }
};
template <> struct Store<IGSP_FP16> {
  using T = uint16_t;
  __device__ static float round(float v) { return __half2float(__float2half_rn(v)); }
  __device__ static uint16_t pack(float v) { return __half_as_ushort(__float2half_rn(v)); }
  __device__ static float widen(uint16_t b) { return __half2float(__ushort_as_half(b)); }
};
template <> struct Store<IGSP_BF16> {
  using T = uint16_t;
  // round to nearest even on the top 16 bits (finite, non-negative inputs)
  __device__ static uint16_t pack(float v) {
    const uint32_t u = __float_as_uint(v);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
  __device__ static float round(float v) { return __uint_as_float((uint32_t)pack(v) << 16); }
  __device__ static float widen(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
};

__device__ __forceinline__ int hist_bin(float stored) {
  int b = (int)(__float_as_uint(stored) >> 16) - (int)kKeyLo;
  return b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
}

// Launch order of work-groups is round-robin over the 8 XCDs; map
// consecutive blocks of one XCD onto consecutive items so that vertically
// adjacent bands (which share halo rows) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// ------------------------------------------------------------- row staging

struct RowFetch {
  uint4 v;     // this lane's 16-byte chunk
  int delta;   // offset of the span start inside the first chunk
};

__device__ __forceinline__ RowFetch fetch_row(const uint8_t* images, int64_t img_end, const uint8_t* span,
                                              int span_bytes, int lane) {
  RowFetch f;
  const uintptr_t s = reinterpret_cast<uintptr_t>(span);
  const uintptr_t a = s & ~uintptr_t(15);
  f.delta = (int)(s - a);
  const int nchunk = (span_bytes + f.delta + 15) >> 4;
  f.v = make_uint4(0, 0, 0, 0);
  if (lane < nchunk) {
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a) + 16 * lane;
    const int64_t rel = (int64_t)(src - images);
    if (rel + 16 <= img_end) {
      f.v = *reinterpret_cast<const uint4*>(src);
    } else {  // last chunk of the buffer: never read past the caller's bytes
      uint32_t w[4] = {0, 0, 0, 0};
      for (int k = 0; k < 16; ++k)
        if (rel + k < img_end) w[k >> 2] |= (uint32_t)src[k] << (8 * (k & 3));
      f.v = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
  return f;
}

// BT.601 luma x 1000 of 4 packed pixels (12 bytes in d0..d2) with byte dot
// products: 299 = 256 + 43, 587 = 2*256 + 75, 114 = 114.
__device__ __forceinline__ void gray4(uint32_t d0, uint32_t d1, uint32_t d2, int g[4]) {
  const uint32_t lo0 = __builtin_amdgcn_udot4(d0, 0x00724B2Bu, 0u, false);               // R0 G0 B0
  const uint32_t hi0 = __builtin_amdgcn_udot4(d0, 0x00000201u, 0u, false);
  const uint32_t lo1 = __builtin_amdgcn_udot4(d1, 0x0000724Bu, __builtin_amdgcn_udot4(d0, 0x2B000000u, 0u, false), false);
  const uint32_t hi1 = __builtin_amdgcn_udot4(d1, 0x00000002u, __builtin_amdgcn_udot4(d0, 0x01000000u, 0u, false), false);
  const uint32_t lo2 = __builtin_amdgcn_udot4(d2, 0x00000072u, __builtin_amdgcn_udot4(d1, 0x4B2B0000u, 0u, false), false);
  const uint32_t hi2 = __builtin_amdgcn_udot4(d1, 0x02010000u, 0u, false);
  const uint32_t lo3 = __builtin_amdgcn_udot4(d2, 0x724B2B00u, 0u, false);               // R3 G3 B3
  const uint32_t hi3 = __builtin_amdgcn_udot4(d2, 0x00020100u, 0u, false);
  g[0] = (int)(lo0 + (hi0 << 8));
  g[1] = (int)(lo1 + (hi1 << 8));
  g[2] = (int)(lo2 + (hi2 << 8));
  g[3] = (int)(lo3 + (hi3 << 8));
}

// ------------------------------------------------------------- stage 1

template <int PREC>
__device__ __forceinline__ void wave_strip(const EdgeLaunch& L, const ViewDesc& vd, int x0, int ys, int ye,
                                           uint8_t* stage, uint32_t* hist) {
  using S = Store<PREC>;
  const int lane = threadIdx.x & 63;
  const int W = vd.W, H = vd.H;
  const int cx0 = x0 - kHalo + kLanePx * lane;            // first input column of the lane
  const bool interior = (x0 - kHalo >= 0) && (x0 - kHalo + kWaveCols <= W);
  const int clo = max(0, x0 - kHalo), chi = min(W, x0 - kHalo + kWaveCols);
  const int span_bytes = 3 * (chi - clo);
  const uint8_t* img = L.images + vd.in_off;
  const bool out_lane = lane >= 1 && lane <= 62;
  const bool row_aligned = (W & 3) == 0;

  int soff[4];  // byte offsets of this lane's pixels inside the staged span
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int sc = fold(cx0 + i, W);
    sc = sc < clo ? clo : (sc >= chi ? chi - 1 : sc);
    soff[i] = 3 * (sc - clo);
  }

  int hp[4] = {}, s1p[4] = {}, s2p[4] = {}, s3p[4] = {};
  int bp[4] = {}, bpp[4] = {};
  int sxp[4] = {}, u1p[4] = {};
  float Mp[4] = {}, Mpp[4] = {};
  int codep[4] = {};

  const float kTan = 0.41421356237309503f;  // tan(22.5 deg) = sqrt(2) - 1
  const int T = (ye - ys) + 2 * kHalo;

  RowFetch nxt = fetch_row(L.images, L.img_end, img + (int64_t)fold(ys - kHalo, H) * 3 * W + 3 * clo,
                           span_bytes, lane);
  for (int t = 0; t < T; ++t) {
    // ---- stage this row's bytes, prefetch the next row
    *reinterpret_cast<uint4*>(stage + 16 * lane) = nxt.v;
    const int delta = nxt.delta;
    if (t + 1 < T)
      nxt = fetch_row(L.images, L.img_end, img + (int64_t)fold(ys - kHalo + t + 1, H) * 3 * W + 3 * clo,
                      span_bytes, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // ---- 1. grayscale
    int g[4];
    if (interior) {
      const int off = 12 * lane + delta;
      const uint32_t* s32 = reinterpret_cast<const uint32_t*>(stage + (off & ~3));
      const uint32_t w0 = s32[0], w1 = s32[1], w2 = s32[2], w3 = s32[3];
      const int sh = off & 3;
      gray4(__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh),
            __builtin_amdgcn_alignbyte(w3, w2, sh), g);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint8_t* p = stage + soff[i] + delta;
        g[i] = 299 * (int)p[0] + 587 * (int)p[1] + 114 * (int)p[2];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();

    // ---- 2. horizontal binomial taps (1 4 6 4 1)
    const int gL2 = from_left(g[2]), gL3 = from_left(g[3]);
    const int gR0 = from_right(g[0]), gR1 = from_right(g[1]);
    int h[4];
    h[0] = (gL2 + g[2]) + 4 * (gL3 + g[1]) + 6 * g[0];
    h[1] = (gL3 + g[3]) + 4 * (g[0] + g[2]) + 6 * g[1];
    h[2] = (g[0] + gR0) + 4 * (g[1] + g[3]) + 6 * g[2];
    h[3] = (g[1] + gR1) + 4 * (g[2] + gR0) + 6 * g[3];

    // ---- 3. vertical taps as four (1 1) sums: b = blur of row yy-2
    int b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s1 = h[i] + hp[i], s2 = s1 + s1p[i], s3 = s2 + s2p[i];
      b[i] = s3 + s3p[i];
      hp[i] = h[i]; s1p[i] = s1; s2p[i] = s2; s3p[i] = s3;
    }

    // ---- 4. Sobel: gx(yy-3) = (1 2 1)^T on the horizontal difference
    const int bL = from_left(b[3]), bR = from_right(b[0]);
    int sx[4] = {b[1] - bL, b[2] - b[0], b[3] - b[1], bR - b[2]};
    int gx[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u1 = sx[i] + sxp[i];
      gx[i] = u1 + u1p[i];
      sxp[i] = sx[i]; u1p[i] = u1;
    }
    //      gy(yy-3) = (1 2 1) along x on the vertical difference
    int sy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sy[i] = b[i] - bpp[i];
      bpp[i] = bp[i]; bp[i] = b[i];
    }
    const int syL = from_left(sy[3]), syR = from_right(sy[0]);
    int gy[4] = {syL + 2 * sy[0] + sy[1], sy[0] + 2 * sy[1] + sy[2], sy[1] + 2 * sy[2] + sy[3],
                 sy[2] + 2 * sy[3] + syR};

    // ---- 5. magnitude and orientation of row yy-3
    float M[4];
    int code[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float fx = (float)gx[i], fy = (float)gy[i];
      M[i] = __builtin_fmaf(fx, fx, fy * fy);
      const float ax = __builtin_fabsf(fx), ay = __builtin_fabsf(fy);
      const bool isH = ay < kTan * ax;
      const bool isV = ax < kTan * ay;
      const int sel = isH ? 0 : (isV ? 1 : (((gx[i] ^ gy[i]) >= 0) ? 2 : 3));
      const bool neg = isV ? (gy[i] < 0) : (gx[i] < 0);
      code[i] = sel | (neg ? 4 : 0);
    }

    // ---- 6. suppression of row yy-4 (up = Mpp, centre = Mp, down = M)
    if (t >= 2 * kHalo) {
      const int c = ys - 2 * kHalo + t;
      const float uL = from_left(Mpp[3]), uR = from_right(Mpp[0]);
      const float cL = from_left(Mp[3]), cR = from_right(Mp[0]);
      const float dL = from_left(M[3]), dR = from_right(M[0]);
      float val[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float Ul = i > 0 ? Mpp[i - 1] : uL, Uc = Mpp[i], Ur = i < 3 ? Mpp[i + 1] : uR;
        const float Cl = i > 0 ? Mp[i - 1] : cL, Cr = i < 3 ? Mp[i + 1] : cR;
        const float Dl = i > 0 ? M[i - 1] : dL, Dc = M[i], Dr = i < 3 ? M[i + 1] : dR;
        const int sel = codep[i] & 3;
        // A = p - e, B = p + e for the axis e of the bin: x, y, (1,1), (1,-1)
        const float A = sel == 0 ? Cl : (sel == 1 ? Uc : (sel == 2 ? Ul : Dl));
        const float B = sel == 0 ? Cr : (sel == 1 ? Dc : (sel == 2 ? Dr : Ur));
        const bool neg = (codep[i] & 4) != 0;
        const float lo = neg ? B : A, hi = neg ? A : B;   // M(p - d), M(p + d)
        const float m = Mp[i];
        const bool keep = (m > lo) && (m >= hi) && (m > 0.0f);
        val[i] = keep ? S::round(__builtin_amdgcn_sqrtf(m) * kStoreScale) : 0.0f;
      }
      if (out_lane && cx0 < W) {
        typename S::T* mrow = reinterpret_cast<typename S::T*>(L.map) + vd.map_off + (int64_t)c * W + cx0;
        if (row_aligned) {
          if constexpr (PREC == IGSP_FP32) {
            *reinterpret_cast<float4*>(mrow) = make_float4(val[0], val[1], val[2], val[3]);
          } else {
            const uint32_t lo2 = (uint32_t)S::pack(val[0]) | ((uint32_t)S::pack(val[1]) << 16);
            const uint32_t hi2 = (uint32_t)S::pack(val[2]) | ((uint32_t)S::pack(val[3]) << 16);
            *reinterpret_cast<uint2*>(mrow) = make_uint2(lo2, hi2);
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (cx0 + i < W) {
              if constexpr (PREC == IGSP_FP32) mrow[i] = val[i];
              else mrow[i] = S::pack(val[i]);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (val[i] > 0.0f && cx0 + i < W) atomicAdd(&hist[hist_bin(val[i])], 1u);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Mpp[i] = Mp[i]; Mp[i] = M[i]; codep[i] = code[i];
    }
  }
}

template <int PREC, int NW>
__global__ __launch_bounds__(NW * 64) void edge_fused_kernel(EdgeLaunch L, int item0, int n_items) {
  __shared__ uint32_t hist[kBins];
  __shared__ __align__(16) uint8_t stage[NW][kStageBytes];
  const int item = item0 + xcd_remap((int)blockIdx.x, n_items);
  const EdgeItem it = L.items[item];
  const ViewDesc vd = L.views[it.view];
  for (int i = threadIdx.x; i < kBins; i += NW * 64) hist[i] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int ys = it.y0 + w * L.seg_rows;
  const int ye = min(ys + L.seg_rows, it.y0 + it.rows);
  if (ys < ye) wave_strip<PREC>(L, vd, it.x0, ys, ye, stage[w], hist);
  __syncthreads();
  uint32_t* gh = L.hist + (int64_t)it.view * kBins;
  for (int i = threadIdx.x; i < kBins; i += NW * 64) {
    const uint32_t c = hist[i];
    if (c) atomicAdd(&gh[i], c);
  }
}

// ------------------------------------------------------------- stage 2

// Final shift of the radix selection: the stored format's own resolution.
__device__ __forceinline__ int final_shift(int prec) {
  return prec == IGSP_BF16 ? 16 : (prec == IGSP_FP16 ? 13 : 0);
}

__device__ __forceinline__ void finish_view(const EdgeLaunch& L, int v, MedState& st) {
  st.med = st.n ? __uint_as_float(st.prefix << st.shift) : 0.0f;
  if (L.medians_dn) L.medians_dn[v] = st.med * (8192.0f / 256000.0f);
  if (L.survivors) L.survivors[v] = (int32_t)st.n;
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t& total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[w] = x;
  __syncthreads();
  uint32_t before = 0;
  for (int k = 0; k < w; ++k) before += tmp[k];
  total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
  __syncthreads();
  return before + x - v;
}

__global__ __launch_bounds__(256) void median_select_kernel(EdgeLaunch L, int v0) {
  __shared__ uint32_t tmp[4];
  const int v = v0 + blockIdx.x;
  uint32_t* h = L.hist + (int64_t)v * kBins;
  constexpr int PER = kBins / 256;
  static_assert(kBins % 256 == 0, "bins per thread");
  const int b0 = threadIdx.x * PER;
  uint32_t c[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) { c[k] = h[b0 + k]; sum += c[k]; }
  uint32_t n = 0;
  const uint32_t excl = block_excl_scan(sum, tmp, n);
  const uint32_t k = n ? (n - 1) / 2 : 0;
  if (n == 0) {
    if (threadIdx.x == 0) {
      MedState st = {0u, 0, 0u, 0u, 0.0f, {0u, 0u, 0u}};
      finish_view(L, v, st);
      L.state[v] = st;
    }
  } else if (excl <= k && k < excl + sum) {
    uint32_t cum = excl;
    int b = b0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (cum + c[j] > k) { b = b0 + j; break; }
      cum += c[j];
    }
    MedState st = {kKeyLo + (uint32_t)b, 16, k - cum, n, 0.0f, {0u, 0u, 0u}};
    if (16 == final_shift(L.precision)) finish_view(L, v, st);
    L.state[v] = st;
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) h[b0 + j] = 0;  // ready for the next call
}

template <int PREC>
__global__ __launch_bounds__(256) void median_refine_kernel(EdgeLaunch L, int flat0, int digit_bits) {
  using S = Store<PREC>;
  __shared__ uint32_t hs[kRefineBins];
  const FlatItem it = L.flat[flat0 + blockIdx.x];
  const MedState st = L.state[it.view];
  const ViewDesc vd = L.views[it.view];
  hs[threadIdx.x] = 0;
  __syncthreads();
  if (st.n > 0 && st.shift > final_shift(PREC)) {
    const int dshift = st.shift - digit_bits;
    const uint32_t dmask = (1u << digit_bits) - 1u;
    const typename S::T* m = reinterpret_cast<const typename S::T*>(L.map) + vd.map_off;
    for (int64_t p = it.p0 + 4 * threadIdx.x; p < it.p1; p += 4 * 256) {
      float v[4];
      if constexpr (PREC == IGSP_FP32) {
        const float4 q = *reinterpret_cast<const float4*>(m + p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
        const uint2 q = *reinterpret_cast<const uint2*>(m + p);
        v[0] = S::widen((uint16_t)(q.x & 0xFFFF)); v[1] = S::widen((uint16_t)(q.x >> 16));
        v[2] = S::widen((uint16_t)(q.y & 0xFFFF)); v[3] = S::widen((uint16_t)(q.y >> 16));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t bits = __float_as_uint(v[i]);
        if (p + i < it.p1 && v[i] > 0.0f && (bits >> st.shift) == st.prefix)
          atomicAdd(&hs[(bits >> dshift) & dmask], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t c = hs[threadIdx.x];
  if (c) atomicAdd(&L.rhist[(int64_t)it.view * kRefineBins + threadIdx.x], c);
}

__global__ __launch_bounds__(256) void refine_select_kernel(EdgeLaunch L, int v0, int digit_bits) {
  __shared__ uint32_t tmp[4];
  const int v = v0 + blockIdx.x;
  uint32_t* h = L.rhist + (int64_t)v * kRefineBins;
  const uint32_t c = h[threadIdx.x];
  MedState st = L.state[v];
  const int fin = final_shift(L.precision);
  uint32_t tot = 0;
  const uint32_t excl = block_excl_scan(c, tmp, tot);
  if (st.n > 0 && st.shift > fin && excl <= st.rank && st.rank < excl + c) {
    st.prefix = (st.prefix << digit_bits) | (uint32_t)threadIdx.x;
    st.shift -= digit_bits;
    st.rank -= excl;
    if (st.shift == fin) finish_view(L, v, st);
    L.state[v] = st;
  }
  h[threadIdx.x] = 0;
}

// ------------------------------------------------------------- stage 3

template <int PREC>
__global__ __launch_bounds__(256) void normalise_kernel(EdgeLaunch L, int flat0) {
  using S = Store<PREC>;
  const FlatItem it = L.flat[flat0 + blockIdx.x];
  const ViewDesc vd = L.views[it.view];
  const float med = L.state[it.view].med;
  const typename S::T* m = reinterpret_cast<const typename S::T*>(L.map) + vd.map_off;
  float* out = L.out + vd.out_off;
  const bool aligned = (vd.out_off & 3) == 0;
  for (int64_t p = it.p0 + 4 * threadIdx.x; p < it.p1; p += 4 * 256) {
    float v[4];
    if constexpr (PREC == IGSP_FP32) {
      const float4 q = *reinterpret_cast<const float4*>(m + p);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      const uint2 q = *reinterpret_cast<const uint2*>(m + p);
      v[0] = S::widen((uint16_t)(q.x & 0xFFFF)); v[1] = S::widen((uint16_t)(q.x >> 16));
      v[2] = S::widen((uint16_t)(q.y & 0xFFFF)); v[3] = S::widen((uint16_t)(q.y >> 16));
    }
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = v[i] > 0.0f ? v[i] / med : 0.0f;
    if (aligned && p + 4 <= it.p1) {
      *reinterpret_cast<float4*>(out + p) = make_float4(e[0], e[1], e[2], e[3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (p + i < it.p1) out[p + i] = e[i];
    }
  }
}

template <int PREC>
hipError_t fused_for_prec(const EdgeLaunch& L, int item0, int n_items, hipStream_t s) {
  switch (L.wg_waves) {
    case 1: hipLaunchKernelGGL((edge_fused_kernel<PREC, 1>), dim3(n_items), dim3(64), 0, s, L, item0, n_items); break;
    case 2: hipLaunchKernelGGL((edge_fused_kernel<PREC, 2>), dim3(n_items), dim3(128), 0, s, L, item0, n_items); break;
    case 8: hipLaunchKernelGGL((edge_fused_kernel<PREC, 8>), dim3(n_items), dim3(512), 0, s, L, item0, n_items); break;
    default: hipLaunchKernelGGL((edge_fused_kernel<PREC, 4>), dim3(n_items), dim3(256), 0, s, L, item0, n_items); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_edge_fused(const EdgeLaunch& L, int item0, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16: return fused_for_prec<IGSP_FP16>(L, item0, n_items, s);
    case IGSP_BF16: return fused_for_prec<IGSP_BF16>(L, item0, n_items, s);
    default: return fused_for_prec<IGSP_FP32>(L, item0, n_items, s);
  }
}

hipError_t launch_median_select(const EdgeLaunch& L, int v0, int nv, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(median_select_kernel, dim3(nv), dim3(256), 0, s, L, v0);
  return hipGetLastError();
}

hipError_t launch_median_refine(const EdgeLaunch& L, int flat0, int n_flat, int digit_bits, hipStream_t s) {
  if (n_flat <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16:
      hipLaunchKernelGGL(median_refine_kernel<IGSP_FP16>, dim3(n_flat), dim3(256), 0, s, L, flat0, digit_bits);
      break;
    case IGSP_BF16:
      hipLaunchKernelGGL(median_refine_kernel<IGSP_BF16>, dim3(n_flat), dim3(256), 0, s, L, flat0, digit_bits);
      break;
    default:
      hipLaunchKernelGGL(median_refine_kernel<IGSP_FP32>, dim3(n_flat), dim3(256), 0, s, L, flat0, digit_bits);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_refine_select(const EdgeLaunch& L, int v0, int nv, int digit_bits, int /*final_shift*/,
                                hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_select_kernel, dim3(nv), dim3(256), 0, s, L, v0, digit_bits);
  return hipGetLastError();
}

hipError_t launch_normalise(const EdgeLaunch& L, int flat0, int n_flat, hipStream_t s) {
  if (n_flat <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16: hipLaunchKernelGGL(normalise_kernel<IGSP_FP16>, dim3(n_flat), dim3(256), 0, s, L, flat0); break;
    case IGSP_BF16: hipLaunchKernelGGL(normalise_kernel<IGSP_BF16>, dim3(n_flat), dim3(256), 0, s, L, flat0); break;
    default: hipLaunchKernelGGL(normalise_kernel<IGSP_FP32>, dim3(n_flat), dim3(256), 0, s, L, flat0); break;
  }
  return hipGetLastError();
}

}  // namespace igsp
