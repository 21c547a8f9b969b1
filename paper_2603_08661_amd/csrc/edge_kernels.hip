// Edge-score importance maps on gfx950 (Sec. 2.1 of arXiv 2603.08661).
//
// Stage 1, edge_fused: one pass over the 8-bit RGB input computes grayscale,
// the binomial 5x5 blur, the Sobel gradient, the orientation bin and the
// non-maximum suppression, writes one stored value per pixel (the thinned
// magnitude at survivors, 0 elsewhere; FP32, FP16 or BF16) into the view's
// strip-major slots and accumulates a per-view histogram of its top 16
// bits. The paper runs these steps as separate kernels with HBM
// intermediates and names a shared-memory fusion as future work; here
// nothing between the input bytes and the suppressed magnitude leaves the
// register file.
//
//   - A wavefront owns a vertical strip of 256 input columns (64 lanes x 4
//     adjacent pixels) and marches down its rows. Vertical taps live in
//     register sliding windows; horizontal neighbours cross lanes with DPP
//     wave shifts, never through LDS.
//   - Each lane reads its 12 bytes of a row with one unaligned 96-bit buffer
//     load, one row ahead of its use; a wave's loads cover 768 contiguous
//     bytes. Row indices, descriptors and bounds are wave-uniform scalar
//     work, and the loop body issues the same memory operations on every
//     lane (a wavefront's store of one row fills one 256-value slot of its
//     strip with one aligned store per lane; rows that are not outputs get
//     an empty descriptor and are dropped), so waits never drain the
//     prefetch.
//   - Gray, blur and Sobel run in exact 32-bit integers (|gx|,|gy| < 2^28).
//     The magnitude, its orientation test and the suppression comparisons
//     are FP32.
//
// Stage 2, median_select / median_refine: exact radix selection of the
// lower median of each view's stored survivor values; BF16 needs no
// refinement, FP16 one 3-bit pass, FP32 two 8-bit passes. A refinement
// pass's selection step is taken by every work-group of the launch after it
// (the next pass, or the normalisation), so no launch of its own is needed.
// Stage 3, normalise: map = q / median (FP16) or sqrt(q / median) (FP32,
// BF16) at survivors, 0 elsewhere. Stages 2 and 3 walk the slots, one per
// wavefront at a time, and stage 3 writes each chunk's row-major map range
// with 16-byte stores.

#include <hip/hip_fp16.h>

#include "igsp_internal.h"

// Waves per SIMD the register allocation is held to (128 VGPRs at 4; the
// stencil needs about 110). Five waves fit its hot loop in 96 VGPRs but gain
// nothing measurable: the loop is bound by vector-ALU issue, not latency.
#ifndef IGSP_FUSED_WAVES_PER_EU
#define IGSP_FUSED_WAVES_PER_EU 4
#endif
#ifndef IGSP_PERSIST_WAVES_PER_EU
#define IGSP_PERSIST_WAVES_PER_EU 4
#endif

namespace igsp {
namespace {

template <class T>
using gptr = __attribute__((address_space(1))) T*;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}
template <class T>
__device__ __forceinline__ gptr<const T> as_global(const T* p) {
  return (gptr<const T>)p;
}

// ------------------------------------------------------------- cross-lane

// DPP wave shifts: lane i receives lane i-1 (from_left) or i+1 (from_right);
// lanes at the wave ends receive 0 (only halo columns depend on them).
// The moves are kept opaque to the compiler: folding them into the
// consuming ALU instruction (a combined VOP2 DPP op with a wave shift) gave
// wrong values at run time on gfx950 in this toolchain, while the plain
// v_mov_b32_dpp form is exact.
__device__ __forceinline__ int from_left(int v) {
  int r = __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
  asm volatile("" : "+v"(r));
  return r;
}
__device__ __forceinline__ int from_right(int v) {
  int r = __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
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
// The same map for an overshoot of at most 4 and n >= 3 (row indices).
__device__ __forceinline__ int fold_near(int i, int n) {
  if (i < 0) i = -i;
  if (i >= n) i = 2 * (n - 1) - i;
  if (i < 0) i = -i;
  return i;
}

// 6 a + c in one instruction (a < 2^24): kept opaque so that the sum c is
// formed first (two instructions) and not re-associated around a separate
// multiply (three).
__device__ __forceinline__ int mad6(int a, int c) {
  int r;
  asm("v_mad_u32_u24 %0, %1, 6, %2" : "=v"(r) : "v"(a), "v"(c));
  return r;
}

// 4 k + c for the 16-bit half k of w (HI: bits 16..31), one instruction:
// the byte offset of histogram bin k - lo from the histogram's start when
// c = -4 lo (mod 2^32).
template <bool HI>
__device__ __forceinline__ uint32_t half_x4_plus(uint32_t w, uint32_t c) {
  uint32_t r;
  if constexpr (HI) asm("v_mad_u32_u16 %0, %1, 4, %2 op_sel:[1,0,0,0]" : "=v"(r) : "v"(w), "s"(c));
  else asm("v_mad_u32_u16 %0, %1, 4, %2" : "=v"(r) : "v"(w), "s"(c));
  return r;
}

// ------------------------------------------------------------- storage

template <int PREC> struct Store;
template <> struct Store<IGSP_FP32> {
  using T = float;
  static constexpr bool kSquare = true;
  __device__ static float widen(float v) { return v; }
};
template <> struct Store<IGSP_FP16> {
  using T = uint16_t;
  static constexpr bool kSquare = false;
  __device__ static uint16_t pack(float v) { return __half_as_ushort(__float2half_rn(v)); }
  __device__ static uint32_t pack2(float a, float b) { return (uint32_t)pack(a) | ((uint32_t)pack(b) << 16); }
  __device__ static float widen(uint16_t b) { return __half2float(__ushort_as_half(b)); }
};
template <> struct Store<IGSP_BF16> {
  using T = uint16_t;
  static constexpr bool kSquare = true;
  // round to nearest even, two values per instruction (v_cvt_pk_bf16_f32)
  __device__ static uint32_t pack2(float a, float b) {
    const bf16x2 v = __builtin_convertvector(f32x2{a, b}, bf16x2);
    uint32_t r;
    __builtin_memcpy(&r, &v, 4);
    return r;
  }
  __device__ static float widen(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
};

template <int PREC> struct Keys {
  static constexpr uint32_t lo = Store<PREC>::kSquare ? kKeyLoSquare : kKeyLoRoot;
  static constexpr int bins = Store<PREC>::kSquare ? kBinsSquare : kBinsRoot;
};

// Launch order of work-groups is round-robin over the 8 XCDs; map
// consecutive blocks of one XCD onto consecutive items so that vertically
// adjacent bands (which share halo rows) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// ------------------------------------------------------------- row input

typedef unsigned u32x3 __attribute__((ext_vector_type(3)));

// Raw buffer descriptor over [base, base + bytes): the base lives in SGPRs,
// lanes pass 32-bit offsets, and the hardware drops accesses past `bytes`.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

// The 12 bytes (4 RGB pixels) of one lane, straight from HBM. Rows have pitch
// 3*W, so the offset is only byte aligned; gfx950 under the HSA ABI runs
// buffer loads in unaligned mode, and a wave's 64 lanes read 768 contiguous
// bytes. Every lane issues exactly one load per row (so the wait for a row
// never has to drain the prefetch of the next one): a lane whose columns
// cross a view border loads the 4-pixel window that holds their mirror
// images and puts them in order after the gray conversion.
struct Lane12 {
  u32x3 v;
};

__device__ __forceinline__ Lane12 load_lane(__amdgpu_buffer_rsrc_t row, int off) {
  return Lane12{__builtin_amdgcn_raw_buffer_load_b96(row, off, 0, 0)};
}

// Views narrower than 4 pixels have no 4-pixel window: gather byte by byte.
__device__ __forceinline__ Lane12 load_lane_bytes(__amdgpu_buffer_rsrc_t row, const int soff[4]) {
  uint32_t w[3] = {0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      w[k >> 2] |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(row, soff[i] + c, 0, 0) << (8 * (k & 3));
    }
  return Lane12{u32x3{w[0], w[1], w[2]}};
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

// ------------------------------------------------------------- suppression

// Orientation of a gradient: within 22.5 degrees of the x axis (cH), of the
// y axis (cV), else diagonal, (1,1) if gx and gy have equal signs (c45),
// else (1,-1); tan 22.5 = sqrt 2 - 1. sgn = -1 if the gradient points along
// -e for the bin's axis e, else 0.
struct Dir {
  bool cH, cV, c45;
  int sgn;
};

constexpr float kTan = 0.41421356237309503f;

__device__ __forceinline__ Dir direction(float fx, float fy) {
  const float ax = __builtin_fabsf(fx), ay = __builtin_fabsf(fy);
  Dir d;
  d.cH = ay < kTan * ax;
  d.cV = ax < kTan * ay;
  d.c45 = (__float_as_int(fx) ^ __float_as_int(fy)) >= 0;
  d.sgn = (d.cV ? __float_as_int(fy) : __float_as_int(fx)) >> 31;
  return d;
}

// keep iff M(p) > M(p - d) and M(p) >= M(p + d) and M(p) > 0, d = +e or -e.
// Magnitudes are non-negative floats, so they order as their bit patterns,
// and "m > x" is "m >= the next float after x" = bits(x) + 1: one unsigned
// compare against a maximum decides the pixel. U*, C*, D* are the
// magnitudes of the row above, this row and the row below (l, c, r columns).
__device__ __forceinline__ bool keep_of(const Dir& d, float m, float Ul, float Uc, float Ur, float Cl, float Cr,
                                        float Dl, float Dc, float Dr) {
  // A = p - e, B = p + e for the axis e of the bin: x, y, (1,1), (1,-1)
  const float A = d.cH ? Cl : (d.cV ? Uc : (d.c45 ? Ul : Dl));
  const float B = d.cH ? Cr : (d.cV ? Dc : (d.c45 ? Dr : Ur));
  const uint32_t bA = __float_as_uint(A) + 1u + (uint32_t)d.sgn;  // strict unless d = -e
  const uint32_t bB = __float_as_uint(B) - (uint32_t)d.sgn;       // strict if d = -e
  return __float_as_uint(m) >= max(max(bA, bB), 1u);
}

// ------------------------------------------------------------- stage 1

// Loop-carried state of one wavefront's march down its strip. Depth-one
// windows are kept twice and addressed by the parity of the row, the
// magnitude rows three times and addressed by the row modulo 3, so after
// unrolling the loop by six every value stays in its register (no copies).
struct StripState {
  Lane12 rows[2];                  // raw bytes: this row / next row
  // rows r-1 (other parity slot) and r-2 (same parity slot) of:
  int h[2][4];                     // the horizontal blur
  int e[2][4];                     // e(r) = h(r) + h(r-2)
  int sx[2][4];                    // the horizontal difference of the blur
  int hs[2][4];                    // the horizontal (1 2 1) smoothing of the blur
  float M[3][4];                   // squared magnitude of the last three rows
  float ML[3], MR[3];              // and the lanes' outer neighbours of each
  float fx[2][4], fy[2][4];        // gradient of the last two rows (exact in float for |g| < 2^24,
                                   // else rounded; only its orientation is read back)
};

struct StripCtx {
  const uint8_t* img;
  int64_t pitch;                   // 3 * W
  int W, H, ys, ye, T;
  bool remap;                      // some lane reorders its window (wave-uniform)
  int win_off;                     // byte offset of the lane's 4-pixel window
  uint32_t permA[3], permB[3];     // byte selectors that put the window's mirrored
                                   // pixels in lane order (edge strips)
  int soff[4];                     // byte offsets of the lane's mirrored columns
  int store_off;                   // byte offset of the lane's 4 values in a stored row of
                                   // the strip, or past its end (dropped): halo lanes
  bool out_px[4];                  // pixel i is an output of this strip
  uint8_t* map;                    // this strip's rows of the stored map
};


// Cache policy of buffer accesses: 0 = default; kCpolAgent = device-coherent
// (the SC1 scope bit, the same encoding the compiler gives agent-scope
// relaxed atomic loads and stores): such stores are visible device-wide once
// they complete, and such loads never return a stale line from another XCD's
// L2, with no cache write-back or invalidation around them.
constexpr int kCpolAgent = 16;

template <bool NARROW>
__device__ __forceinline__ Lane12 fetch_row(const StripCtx& C, int yy) {
  const __amdgpu_buffer_rsrc_t row = buffer_rsrc(C.img + fold_near(yy, C.H) * C.pitch, 3 * C.W);
  if constexpr (NARROW) return load_lane_bytes(row, C.soff);
  else return load_lane(row, C.win_off);
}

template <int PREC, bool NARROW, int P, int MS, int CPOL>
__device__ __forceinline__ void strip_row(const StripCtx& C, StripState& S, int t, uint32_t* hist) {
  using St = Store<PREC>;
  constexpr int Q = P ^ 1;             // previous row's parity slot
  constexpr int MD = MS;               // magnitude slots: new (down) row,
  constexpr int MC = (MS + 2) % 3;     // the row before it (centre),
  constexpr int MU = (MS + 1) % 3;     // and the one before that (up)
  constexpr int ES = sizeof(typename St::T);
  // ---- prefetch the next row (the last step re-reads a row: one load per
  //      step keeps the wait for this row from draining the prefetch)
  S.rows[Q] = fetch_row<NARROW>(C, min(C.ys - kHalo + t + 1, C.ye + kHalo - 1));

  // ---- 1. grayscale of row yy = ys - 4 + t (edge strips first put the
  //      mirrored pixels of the window in lane order: two byte permutes per
  //      output word, the first over window bytes 0-7, the second adding
  //      bytes 8-11)
  int g[4];
  uint32_t d0 = S.rows[P].v.x, d1 = S.rows[P].v.y, d2 = S.rows[P].v.z;
  if (!NARROW && C.remap) {
    asm volatile("");  // keeps this a branch that interior strips skip, not selects every strip pays for
    const uint32_t o0 = __builtin_amdgcn_perm(d2, __builtin_amdgcn_perm(d1, d0, C.permA[0]), C.permB[0]);
    const uint32_t o1 = __builtin_amdgcn_perm(d2, __builtin_amdgcn_perm(d1, d0, C.permA[1]), C.permB[1]);
    const uint32_t o2 = __builtin_amdgcn_perm(d2, __builtin_amdgcn_perm(d1, d0, C.permA[2]), C.permB[2]);
    d0 = o0;
    d1 = o1;
    d2 = o2;
  }
  gray4(d0, d1, d2, g);

  // ---- 2. horizontal binomial taps (1 4 6 4 1)
  const int gL2 = from_left(g[2]), gL3 = from_left(g[3]);
  const int gR0 = from_right(g[0]), gR1 = from_right(g[1]);
  int h[4];
  h[0] = mad6(g[0], (gL2 + g[2]) + 4 * (gL3 + g[1]));
  h[1] = mad6(g[1], (gL3 + g[3]) + 4 * (g[0] + g[2]));
  h[2] = mad6(g[2], (g[0] + gR0) + 4 * (g[1] + g[3]));
  h[3] = mad6(g[3], (g[1] + gR1) + 4 * (g[2] + gR0));

  // ---- 3. vertical taps (1 4 6 4 1): b = blur of row yy-2, three
  //      instructions per pixel from the pair sums e(r) = h(r) + h(r-2):
  //      h(r) + 4 h(r-1) + 6 h(r-2) + 4 h(r-3) + h(r-4)
  //        = e(r) + e(r-2) + 4 (e(r-1) + h(r-2))
  //      (slot P holds rows r-2, slot Q rows r-1, before the update)
  int b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int en = h[i] + S.h[P][i];
    const int t4 = (S.e[Q][i] + S.h[P][i]) << 2;
    b[i] = en + S.e[P][i] + t4;
    S.h[P][i] = h[i];
    S.e[P][i] = en;
  }

  // ---- 4. Sobel of row yy-3: gx = (1 2 1)^T on the horizontal difference,
  //      gy = the vertical difference hs(r+1) - hs(r-1) of the horizontal
  //      (1 2 1) smoothing (equal to smoothing the difference: the taps are
  //      linear), so both use the same two lane-edge neighbours of b
  const int bL = from_left(b[3]), bR = from_right(b[0]);
  const int sxn[4] = {b[1] - bL, b[2] - b[0], b[3] - b[1], bR - b[2]};
  const int hsn[4] = {bL + 2 * b[0] + b[1], b[0] + 2 * b[1] + b[2], b[1] + 2 * b[2] + b[3], b[2] + 2 * b[3] + bR};
  int gx[4], gy[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gx[i] = S.sx[P][i] + 2 * S.sx[Q][i] + sxn[i];          // (1 2 1) down the column
    S.sx[P][i] = sxn[i];
    gy[i] = hsn[i] - S.hs[P][i];       // the same parity slot still holds hs(r-2)
    S.hs[P][i] = hsn[i];
  }

  // ---- 5. squared magnitude of row yy-3, and its lane-edge neighbours
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    S.fx[P][i] = (float)gx[i];
    S.fy[P][i] = (float)gy[i];
    S.M[MD][i] = __builtin_fmaf(S.fx[P][i], S.fx[P][i], S.fy[P][i] * S.fy[P][i]);
  }
  S.ML[MD] = from_left(S.M[MD][3]);
  S.MR[MD] = from_right(S.M[MD][0]);

  // ---- 6. suppression of row c = yy-4: up = M[MU], centre = M[MC], down = M[MD]
  // (rows before the strip's first output are computed too and their stores
  // dropped, so the loop body has no branch around memory operations)
  const int c = C.ys - 2 * kHalo + t;
  const bool row_out = t >= 2 * kHalo && t < C.T;
  const float* Mu = S.M[MU];
  const float* Mc = S.M[MC];
  const float* Md = S.M[MD];
  float q[4];
  bool kept[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float Ul = i > 0 ? Mu[i - 1] : S.ML[MU], Uc = Mu[i], Ur = i < 3 ? Mu[i + 1] : S.MR[MU];
    const float Cl = i > 0 ? Mc[i - 1] : S.ML[MC], Cr = i < 3 ? Mc[i + 1] : S.MR[MC];
    const float Dl = i > 0 ? Md[i - 1] : S.ML[MD], Dc = Md[i], Dr = i < 3 ? Md[i + 1] : S.MR[MD];
    const float m = Mc[i];
    kept[i] = keep_of(direction(S.fx[Q][i], S.fy[Q][i]), m, Ul, Uc, Ur, Cl, Cr, Dl, Dc, Dr);
    const float v = St::kSquare ? m : __builtin_amdgcn_sqrtf(m) * kStoreScaleRoot;
    q[i] = kept[i] ? v : 0.0f;
  }
  // one aligned store per lane and row into the strip's stored row c, which
  // the wavefront's 64 lanes fill whole (rows outside the strip's outputs get
  // an empty descriptor: dropped)
  const __amdgpu_buffer_rsrc_t mrow =
      buffer_rsrc(C.map + (int64_t)max(c, 0) * (kSlotPitch * ES), row_out ? kSlotPitch * ES : 0);
  uint32_t bits[4];  // words whose high halves are the histogram keys
  if constexpr (PREC == IGSP_FP32) {
#pragma unroll
    for (int i = 0; i < 4; ++i) bits[i] = __float_as_uint(q[i]);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{bits[0], bits[1], bits[2], bits[3]}, mrow, C.store_off, 0, CPOL);
  } else {
    const uint32_t w0 = St::pack2(q[0], q[1]), w1 = St::pack2(q[2], q[3]);
    bits[0] = w0 << 16;
    bits[1] = w0;
    bits[2] = w1 << 16;
    bits[3] = w1;
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{w0, w1}, mrow, C.store_off, 0, CPOL);
    if constexpr (PREC == IGSP_FP16) {
#pragma unroll
      for (int i = 0; i < 4; ++i) bits[i] = __float_as_uint(St::widen((uint16_t)(bits[i] >> 16)));
    }
  }
  // A survivor's stored value is never 0 and its key lies in [lo, lo + bins),
  // so the keep decision selects the counted pixels and no clamp is needed:
  // M is integer-valued in [1, 2^57) (|gx|, |gy| < 2^28), its float32 and
  // BF16 patterns run from the exponent of 1 to below 2^58, and the FP16
  // root sqrt(M) 2^-13 lies in [2^-13, 2^17) (normal, never rounded to 0).
  // BF16 takes the keys of pixels 0 and 2 from the low halves of the stored
  // words, everything else from high halves.
  constexpr uint32_t kBase = 0u - 4u * Keys<PREC>::lo;
  char* const hbytes = reinterpret_cast<char*>(hist);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (row_out && kept[i] && C.out_px[i]) {
      uint32_t off;
      if constexpr (PREC == IGSP_BF16) {
        const uint32_t w = i < 2 ? bits[1] : bits[3];
        off = (i & 1) ? half_x4_plus<true>(w, kBase) : half_x4_plus<false>(w, kBase);
      } else {
        off = half_x4_plus<true>(bits[i], kBase);
      }
      atomicAdd(reinterpret_cast<uint32_t*>(hbytes + off), 1u);
    }
}

template <int PREC, bool NARROW, int CPOL>
__device__ __forceinline__ void march(const StripCtx& C, uint32_t* hist) {
  StripState S = {};
  S.rows[0] = fetch_row<NARROW>(C, C.ys - kHalo);
  // six rows per iteration (parity slot t % 2, magnitude slot t % 3), with no
  // exit inside the body: rows past the strip's last one (up to five) are
  // computed and neither stored nor counted
  for (int t = 0; t < C.T; t += 6) {
    strip_row<PREC, NARROW, 0, 0, CPOL>(C, S, t, hist);
    strip_row<PREC, NARROW, 1, 1, CPOL>(C, S, t + 1, hist);
    strip_row<PREC, NARROW, 0, 2, CPOL>(C, S, t + 2, hist);
    strip_row<PREC, NARROW, 1, 0, CPOL>(C, S, t + 3, hist);
    strip_row<PREC, NARROW, 0, 1, CPOL>(C, S, t + 4, hist);
    strip_row<PREC, NARROW, 1, 2, CPOL>(C, S, t + 5, hist);
  }
}

template <int PREC, int CPOL = 0>
__device__ __forceinline__ void wave_strip(const EdgeLaunch& L, const ViewDesc& vd, int x0, int ys, int ye,
                                           uint32_t* hist) {
  using St = Store<PREC>;
  constexpr int ES = sizeof(typename St::T);
  const int lane = __lane_id();
  StripCtx C;
  C.W = vd.W;
  C.H = vd.H;
  C.ys = ys;
  C.ye = ye;
  C.T = (ye - ys) + 2 * kHalo;
  C.img = L.images + vd.in_off;
  C.pitch = 3 * (int64_t)vd.W;
  C.map = reinterpret_cast<uint8_t*>(reinterpret_cast<typename St::T*>(L.map) + vd.map_off +
                                     (int64_t)(x0 / kStripCols) * vd.strip_rows * kSlotPitch);
  const int cx0 = x0 - kHalo + kLanePx * lane;            // first input column of the lane
  int sc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sc[i] = fold(cx0 + i, C.W);
    C.soff[i] = 3 * sc[i];
  }
  // 4-pixel window holding the lane's (possibly mirrored) columns: its own
  // columns inside the view, else the smallest in-bounds window that covers
  // the mirror images (lanes wholly past the border only feed halo columns)
  int ws = cx0;
  if (cx0 < 0 || cx0 + 3 >= C.W) {
    ws = min(min(sc[0], sc[1]), min(sc[2], sc[3]));
    ws = min(ws, C.W - 4);
  }
  ws = max(ws, 0);
  C.win_off = 3 * ws;
  // Output byte q (pixel q / 3, channel q % 3) is window byte b = 3 k + q % 3
  // for the window pixel k that holds that pixel's column. A byte permute
  // picks bytes of {S0, S1} by selector: 0-3 = S1's bytes, 4-7 = S0's, 12 =
  // zero. Stage A permutes (d1, d0), i.e. window bytes 0-7 at selector b;
  // stage B permutes (d2, A) and keeps A's byte j (selector j) or takes
  // window byte b >= 8 from d2 (selector 4 + b - 8).
  bool ident = true;
  int kwin[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    kwin[i] = min(max(sc[i] - ws, 0), 3);
    ident = ident && kwin[i] == i;
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    uint32_t a = 0, b = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * m + j, src = 3 * kwin[q / 3] + q % 3;
      a |= (uint32_t)(src < 8 ? src : 12) << (8 * j);
      b |= (uint32_t)(src < 8 ? j : 4 + src - 8) << (8 * j);
    }
    C.permA[m] = a;
    C.permB[m] = b;
  }
  const bool narrow = C.W < 4;
  C.remap = !narrow && __builtin_amdgcn_ballot_w64(!ident) != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) C.out_px[i] = lane >= 1 && lane <= 62 && cx0 + i < C.W;
  // lanes 1..62 store the strip's 248 columns at slot positions 0..247 (also
  // past the view's right edge, where the values are never read); the halo
  // lanes 63 and 0 fill positions 248..255, which nothing reads
  C.store_off = ((lane + 63) & 63) * kLanePx * ES;
  if (narrow) march<PREC, true, CPOL>(C, hist);
  else march<PREC, false, CPOL>(C, hist);
}

template <int PREC, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(IGSP_FUSED_WAVES_PER_EU))) void edge_fused_kernel(EdgeLaunch L, int item0, int n_items) {
  constexpr int NB = Keys<PREC>::bins;
  __shared__ uint32_t hist[NB];
  const int item = item0 + xcd_remap((int)blockIdx.x, n_items);
  const EdgeItem it = L.items[item];
  const ViewDesc vd = L.views[it.view];
  for (int i = threadIdx.x; i < NB; i += NW * 64) hist[i] = 0;
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ys = it.y0 + w * L.seg_rows;
  const int ye = min(ys + L.seg_rows, it.y0 + it.rows);
  if (ys < ye) wave_strip<PREC>(L, vd, it.x0, ys, ye, hist);
  __syncthreads();
  gptr<uint32_t> gh = as_global(L.hist) + (int64_t)it.view * kBinsMax;
  for (int i = threadIdx.x; i < NB; i += NW * 64) {
    const uint32_t c = hist[i];
    if (c) atomicAdd((uint32_t*)(gh + i), c);
  }
}

// ------------------------------------------------------------- stage 2

// Final shift of the radix selection: the stored format's own resolution.
__device__ __forceinline__ int final_shift(int prec) {
  return prec == IGSP_BF16 ? 16 : (prec == IGSP_FP16 ? 13 : 0);
}
// Refinement passes after the first histogram, and the digit bits of each.
__host__ __device__ constexpr int refine_passes(int prec) {
  return prec == IGSP_BF16 ? 0 : (prec == IGSP_FP16 ? 1 : 2);
}
__host__ __device__ constexpr int refine_digit_bits(int prec) { return prec == IGSP_FP16 ? 3 : 8; }
// Whether the normalisation takes the last selection step itself (every
// work-group from the last pass's histogram) instead of a launch of its own
// before it. Measured on the same box: FP32 (300 views) 2.78 -> 2.67-2.68 ms
// for the edge maps; FP16 (200 views) 0.69 -> 0.72-0.73 ms, so FP16 keeps
// the separate step.
__host__ __device__ constexpr bool fold_last_step(int prec) { return prec == IGSP_FP32; }

__device__ __forceinline__ void finish_view(const EdgeLaunch& L, int v, MedState& st, bool outputs = true) {
  st.med = st.n ? __uint_as_float(st.prefix << st.shift) : 0.0f;
  if (!outputs) return;
  if (L.medians_dn) {
    // back to DN per pixel of an unnormalised Sobel: sqrt(M) / 256000
    const float m = L.precision == IGSP_FP16 ? st.med * 8192.0f : sqrtf(st.med);
    L.medians_dn[v] = m * (1.0f / 256000.0f);
  }
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

template <int PREC>
__global__ __launch_bounds__(256) void median_select_kernel(EdgeLaunch L, int v0) {
  constexpr int NB = Keys<PREC>::bins;
  constexpr int PER = NB / 256;
  static_assert(NB % 256 == 0, "bins per thread");
  __shared__ uint32_t tmp[4];
  const int v = v0 + blockIdx.x;
  if (L.status && blockIdx.x == 0 && threadIdx.x == 0) *L.status = IGSP_OK;  // the staged stages cannot fail
  uint32_t* h = L.hist + (int64_t)v * kBinsMax;
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
    MedState st = {Keys<PREC>::lo + (uint32_t)b, 16, k - cum, n, 0.0f, {0u, 0u, 0u}};
    if (16 == final_shift(PREC)) finish_view(L, v, st);
    L.state[v] = st;
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) h[b0 + j] = 0;  // ready for the next call
  // the digit histograms of this view's refinement passes and its
  // candidate count start from zero
  for (int p = 0; p < refine_passes(PREC); ++p)
    L.rhist[((int64_t)p * L.n_views + v) * kRefineBins + threadIdx.x] = 0;
  if (L.cand_n && threadIdx.x == 0) L.cand_n[v] = 0;
}

// One refinement step of view v's radix selection, taken by a 256-thread
// work-group from the digit histogram h of the pass that resolved the next
// `digit_bits` bits: the bucket holding the median's rank becomes the new
// prefix. Every thread gets the new state (the median is set once the
// stored format's resolution is reached; no output is written here).
__device__ MedState refine_step(const EdgeLaunch& L, const MedState& st, const uint32_t* h, int digit_bits,
                                uint32_t* tmp, MedState* s_st) {
  const int fin = final_shift(L.precision);
  const uint32_t c = h[threadIdx.x];
  uint32_t tot = 0;
  const uint32_t excl = block_excl_scan(c, tmp, tot);
  if (threadIdx.x == 0) *s_st = st;
  __syncthreads();
  if (st.n > 0 && st.shift > fin && excl <= st.rank && st.rank < excl + c) {
    MedState r = st;
    r.prefix = (st.prefix << digit_bits) | (uint32_t)threadIdx.x;
    r.shift = st.shift - digit_bits;
    r.rank = st.rank - excl;
    if (r.shift == fin) finish_view(L, 0, r, false);
    *s_st = r;
  }
  __syncthreads();
  return *s_st;
}

// ------------------------------------------------------------- element-wise walk
//
// The refinement and normalisation passes walk a chunk slot by slot: a
// slot is one strip's stored row (248 values used). A wavefront takes whole slots,
// lane l the 4 pixels at columns 248 s + 4 l .. + 3 (lanes 62 and 63 idle),
// so the slot's index arithmetic is wave-uniform, a wavefront reads 496
// contiguous bytes (BF16 / FP16) and writes 992 contiguous bytes of the map.
struct SlotAt {
  int64_t stored;  // element of the lane's first stored value in the plan's map
  int64_t pixel;   // flat index of the lane's first pixel in the view
  int valid;       // pixels of the lane inside the view (<= 0: none)
};

// The strips of a view (248 columns each).
__device__ __forceinline__ int strips_of(const ViewDesc& vd) { return (vd.W + kStripCols - 1) / kStripCols; }

// Slot u of a view (row u / strips, strip u % strips), lane `lane`.
__device__ __forceinline__ SlotAt view_slot(const ViewDesc& vd, int ns, int u, int lane) {
  const int c = __builtin_amdgcn_readfirstlane(u / ns);
  const int s = u - c * ns;
  // lanes with no pixel in the view (62, 63, and those past its right edge)
  // read the last lane's values again: no cache line beyond the view's part
  // of the slot is fetched
  const int last = min(kStripGroups, (vd.W - kStripCols * s + kLanePx - 1) / kLanePx) - 1;
  const int l = min(lane, last);
  SlotAt a;
  a.stored = vd.map_off + ((int64_t)s * vd.strip_rows + c) * kSlotPitch + kLanePx * l;
  a.pixel = (int64_t)c * vd.W + kStripCols * s + kLanePx * lane;
  a.valid = lane < kStripGroups ? vd.W - (kStripCols * s + kLanePx * lane) : 0;
  return a;
}

// The 4 stored values at element e, widened to float32. COHERENT reads them
// device-coherently (agent-scope relaxed loads, i.e. with the SC1 bit): the
// persistent form reads values other work-groups of the same launch wrote.
template <int PREC, bool COHERENT>
__device__ __forceinline__ void load4(const EdgeLaunch& L, int64_t e, float v[4]) {
  using S = Store<PREC>;
  if constexpr (PREC == IGSP_FP32) {
    uint64_t* p = reinterpret_cast<uint64_t*>(reinterpret_cast<float*>(L.map) + e);
    uint64_t x, y;
    if constexpr (COHERENT) {
      x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      y = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const u32x4 q = *as_global(reinterpret_cast<const u32x4*>(p));
      x = q.x | ((uint64_t)q.y << 32);
      y = q.z | ((uint64_t)q.w << 32);
    }
    v[0] = __uint_as_float((uint32_t)x);
    v[1] = __uint_as_float((uint32_t)(x >> 32));
    v[2] = __uint_as_float((uint32_t)y);
    v[3] = __uint_as_float((uint32_t)(y >> 32));
  } else {
    uint64_t* p = reinterpret_cast<uint64_t*>(reinterpret_cast<uint16_t*>(L.map) + e);
    uint64_t x;
    if constexpr (COHERENT) x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else x = *as_global(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = S::widen((uint16_t)(x >> (16 * i)));
  }
}

// Slots' loads in flight per wavefront in the element-wise walks: 4 in their
// own launches (lean kernels at eight waves per SIMD), 12 inside the
// persistent kernel, whose register budget is the stencil's and whose four
// waves per SIMD need more loads each to keep HBM busy.
constexpr int kWalkUnroll = 4;
constexpr int kPersistWalkUnroll = 12;

// Digit histogram (into LDS) of a chunk's survivors inside the resolved
// bucket of the radix selection, by the NW wavefronts of a work-group.
// APPEND also gathers each of them in the work-group's LDS list lds_cand
// (count in *lds_n; the first FP32 pass: the second then reads the view's
// list instead of the map).
constexpr int kLdsCand = 2048;  // candidates a work-group gathers before it flushes them

template <int PREC, int NW, bool COHERENT, bool APPEND = false>
__device__ __forceinline__ void refine_slots(const EdgeLaunch& L, const ViewDesc& vd, const RowChunk& ck,
                                             const MedState& st, int digit_bits, uint32_t* hs, int lane, int wave,
                                             uint32_t* lds_cand = nullptr, uint32_t* lds_n = nullptr) {
  constexpr int kRefineUnroll = COHERENT ? kPersistWalkUnroll : kWalkUnroll;
  const int ns = strips_of(vd);
  const int dshift = st.shift - digit_bits;
  const uint32_t dmask = (1u << digit_bits) - 1u;
  // kRefineUnroll slots' loads in flight per wavefront (slots past the
  // chunk's end load the last slot again and count nothing)
  for (int u0 = ck.u0 + wave; u0 < ck.u1; u0 += kRefineUnroll * NW) {
    SlotAt a[kRefineUnroll];
    float v[kRefineUnroll][4];
#pragma unroll
    for (int k = 0; k < kRefineUnroll; ++k) {
      a[k] = view_slot(vd, ns, min(u0 + k * NW, ck.u1 - 1), lane);
      load4<PREC, COHERENT>(L, a[k].stored, v[k]);
    }
    uint32_t hit = 0;  // bit 4k + i: value i of slot k is counted
#pragma unroll
    for (int k = 0; k < kRefineUnroll; ++k) {
      if (u0 + k * NW >= ck.u1) break;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t bits = __float_as_uint(v[k][i]);
        if (i < a[k].valid && v[k][i] > 0.0f && (bits >> st.shift) == st.prefix) {
          atomicAdd(&hs[(bits >> dshift) & dmask], 1u);
          hit |= 1u << (4 * k + i);
        }
      }
    }
    if constexpr (APPEND) {
      // the counted values go to the work-group's LDS list (flushed to the
      // view's list once per work-group by the caller)
#pragma unroll
      for (int k = 0; k < kRefineUnroll; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if ((hit >> (4 * k + i)) & 1u) {
            const uint32_t at = atomicAdd(lds_n, 1u);
            if (at < (uint32_t)kLdsCand) lds_cand[at] = __float_as_uint(v[k][i]);
          }
    }
  }
}

// Refinement pass `pass` over a row chunk: the state after `pass` steps
// comes from the previous pass's histogram (each work-group takes that
// step itself; the view's first chunk stores it for the next launch), then
// the chunk's survivors inside the resolved bucket are counted by their
// next digit, in LDS, and added to this pass's histogram.
template <int PREC>
__global__ __launch_bounds__(256) void median_refine_kernel(EdgeLaunch L, int chunk0, int pass) {
  __shared__ uint32_t hs[kRefineBins];
  __shared__ uint32_t tmp[4];
  __shared__ MedState s_st;
  constexpr int DB = refine_digit_bits(PREC);
  const RowChunk ck = L.chunks[chunk0 + blockIdx.x];
  const int v = ck.view;
  const int64_t n = L.n_views;
  MedState st = L.state[v];
  if (pass > 0) {
    st = refine_step(L, L.state[(pass - 1) * n + v], L.rhist + ((pass - 1) * n + v) * kRefineBins, DB, tmp, &s_st);
    if (ck.u0 == 0 && threadIdx.x == 0) L.state[pass * n + v] = st;
  }
  const ViewDesc vd = L.views[v];
  hs[threadIdx.x] = 0;
  __syncthreads();
  const int lane = __lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (st.n > 0 && st.shift > final_shift(PREC)) {
    if (PREC == IGSP_FP32 && pass == 0 && L.use_cand && vd.cand_cap > 0) {
      __shared__ uint32_t cand[kLdsCand];
      __shared__ uint32_t cn, cbase;
      if (threadIdx.x == 0) cn = 0;
      __syncthreads();
      refine_slots<PREC, 4, false, true>(L, vd, ck, st, DB, hs, lane, wave, cand, &cn);
      __syncthreads();
      // one reservation per work-group; a work-group that found more than
      // its LDS list holds marks the view's list as overflowed instead (bit
      // 31: the counts themselves stay below 2^31, a view's pixel count)
      if (threadIdx.x == 0) {
        if (cn <= (uint32_t)kLdsCand) cbase = atomicAdd(&L.cand_n[v], cn);
        else atomicOr(&L.cand_n[v], 0x80000000u);
      }
      __syncthreads();
      if (cn <= (uint32_t)kLdsCand)
        for (uint32_t k = threadIdx.x; k < cn; k += 256)
          if (cbase + k < (uint32_t)vd.cand_cap) L.cand[vd.cand_off + cbase + k] = cand[k];
    } else if (PREC == IGSP_FP32 && pass == 1 && L.use_cand && vd.cand_cap > 0 &&
               L.cand_n[v] <= (uint32_t)vd.cand_cap) {
      // the second FP32 pass counts the first pass's candidates, not the
      // map: every survivor of the new bucket is one of them. The view's
      // chunks share the list evenly, in chunk order.
      const uint32_t nc = L.cand_n[v];
      const uint32_t chunks = (uint32_t)((strips_of(vd) * (int64_t)vd.H + kRefineChunkSlots - 1) / kRefineChunkSlots);
      const uint32_t j = (uint32_t)(ck.u0 / kRefineChunkSlots), per = (nc + chunks - 1) / chunks;
      const uint32_t c0 = min(nc, j * per), c1 = min(nc, c0 + per);
      const int dshift = st.shift - DB;
      for (uint32_t k = c0 + threadIdx.x; k < c1; k += 256) {
        const uint32_t bits = L.cand[vd.cand_off + k];
        if ((bits >> st.shift) == st.prefix) atomicAdd(&hs[(bits >> dshift) & ((1u << DB) - 1u)], 1u);
      }
    } else {
      refine_slots<PREC, 4, false>(L, vd, ck, st, DB, hs, lane, wave);
    }
  }
  __syncthreads();
  const uint32_t c = hs[threadIdx.x];
  if (c) atomicAdd(&L.rhist[(pass * n + v) * kRefineBins + threadIdx.x], c);
}

// The last selection step of views [v0, v0 + gridDim.x) as a launch of its
// own (one work-group per view), where the normalisation does not take it.
__global__ __launch_bounds__(256) void median_step_kernel(EdgeLaunch L, int v0, int pass) {
  __shared__ uint32_t tmp[4];
  __shared__ MedState s_st;
  const int v = v0 + blockIdx.x;
  const int64_t n = L.n_views;
  MedState st = refine_step(L, L.state[(pass - 1) * n + v], L.rhist + ((pass - 1) * n + v) * kRefineBins,
                            refine_digit_bits(L.precision), tmp, &s_st);
  if (threadIdx.x == 0) {
    if (st.shift == final_shift(L.precision)) finish_view(L, v, st);
    L.state[pass * n + v] = st;
  }
}

// ------------------------------------------------------------- stage 3

template <int PREC>
__device__ __forceinline__ void normalise4(const float v[4], float med, float inv, float e[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // the stored median itself maps to exactly 1
    const float r = v[i] == med ? 1.0f : v[i] * inv;
    e[i] = v[i] > 0.0f ? (Store<PREC>::kSquare ? __builtin_amdgcn_sqrtf(r) : r) : 0.0f;
  }
}

// Normalisation of one row chunk by NW wavefronts. Each wavefront keeps
// kNormUnroll slots' loads in flight (slots past the chunk's end load the
// last slot again and store nothing). The chunk's output pixels are one
// contiguous range of the map; a buffer descriptor over it takes a lane's
// four values in one 16-byte store, and the last lane of a row whose width is
// not a multiple of 4 stores its pixels one by one (a fourth value would land
// on the next row).
template <int PREC, int NW, bool COHERENT>
__device__ __forceinline__ void norm_slots(const EdgeLaunch& L, const ViewDesc& vd, const RowChunk& ck, float med,
                                           int lane, int wave) {
  constexpr int kNormUnroll = COHERENT ? kPersistWalkUnroll : kWalkUnroll;
  const int ns = strips_of(vd);
  const float inv = med > 0.0f ? 1.0f / med : 0.0f;
  // the chunk's output pixels: from its first slot's first pixel to its last
  // slot's last
  const int cb = ck.u0 / ns, ce = (ck.u1 - 1) / ns;
  const int64_t p_begin = (int64_t)cb * vd.W + kStripCols * (ck.u0 - cb * ns);
  const int64_t p_end = (int64_t)ce * vd.W + min(vd.W, kStripCols * (ck.u1 - ce * ns));
  const __amdgpu_buffer_rsrc_t out = buffer_rsrc(L.out + vd.out_off + p_begin, (int)(4 * (p_end - p_begin)));
  for (int u0 = ck.u0 + wave; u0 < ck.u1; u0 += kNormUnroll * NW) {
    SlotAt a[kNormUnroll];
    float v[kNormUnroll][4];
#pragma unroll
    for (int k = 0; k < kNormUnroll; ++k) {
      a[k] = view_slot(vd, ns, min(u0 + k * NW, ck.u1 - 1), lane);
      load4<PREC, COHERENT>(L, a[k].stored, v[k]);
    }
#pragma unroll
    for (int k = 0; k < kNormUnroll; ++k) {
      if (u0 + k * NW >= ck.u1) break;
      float e[4];
      normalise4<PREC>(v[k], med, inv, e);
      const int off = 4 * (int)(a[k].pixel - p_begin);
      if (a[k].valid >= kLanePx) {
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{__float_as_uint(e[0]), __float_as_uint(e[1]),
                                                     __float_as_uint(e[2]), __float_as_uint(e[3])},
                                               out, off, 0, 0);
      } else {
        for (int i = 0; i < a[k].valid; ++i)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(e[i]), out, off + 4 * i, 0, 0);
      }
    }
  }
}

// Normalisation of a row chunk. Where the last selection step is folded in
// (FP32), each work-group takes it itself from the last pass's histogram and
// the view's first chunk stores the final state and writes the view's
// outputs; otherwise the final state is read.
template <int PREC>
__global__ __launch_bounds__(256) void normalise_kernel(EdgeLaunch L, int chunk0) {
  __shared__ uint32_t tmp[4];
  __shared__ MedState s_st;
  constexpr int P = refine_passes(PREC);
  const RowChunk ck = L.chunks[chunk0 + blockIdx.x];
  const int v = ck.view;
  MedState st;
  if constexpr (!fold_last_step(PREC)) {
    st = L.state[(int64_t)P * L.n_views + v];
  } else {
    const int64_t n = L.n_views;
    st = refine_step(L, L.state[(P - 1) * n + v], L.rhist + ((P - 1) * n + v) * kRefineBins,
                     refine_digit_bits(PREC), tmp, &s_st);
    if (ck.u0 == 0 && threadIdx.x == 0) {
      finish_view(L, v, st);
      L.state[P * n + v] = st;
    }
  }
  const ViewDesc vd = L.views[v];
  norm_slots<PREC, 4, false>(L, vd, ck, st.med, __lane_id(), __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
}

// ------------------------------------------------------------- unfused form
//
// The paper's kernel layout on this GPU, kept as an ablation of the fusion:
// gray, the 5x5 blur (direct 25-tap sum), Sobel magnitude and orientation,
// and suppression are separate launches, each reading the previous step's
// result from HBM. Same integer and FP32 arithmetic as the fused stencil
// (shared direction and decision functions), so the maps agree bit for bit.

__device__ __forceinline__ int refl(int i, int n) { return fold_near(i, n); }

__global__ __launch_bounds__(kUfCols) void uf_gray_kernel(EdgeLaunch L, UfLaunch U) {
  const UfItem it = U.items[blockIdx.x];
  const ViewDesc vd = L.views[it.view];
  const int x = it.x0 + threadIdx.x;
  if (x >= vd.W) return;
  const int y1 = min(it.y0 + kUfRows, vd.H);
  for (int y = it.y0; y < y1; ++y) {
    const int64_t p = (int64_t)y * vd.W + x;
    const uint8_t* px = L.images + vd.in_off + 3 * p;
    U.gray[vd.map_off + p] = 299 * (int)px[0] + 587 * (int)px[1] + 114 * (int)px[2];
  }
}

__global__ __launch_bounds__(kUfCols) void uf_blur_kernel(EdgeLaunch L, UfLaunch U) {
  const UfItem it = U.items[blockIdx.x];
  const ViewDesc vd = L.views[it.view];
  const int x = it.x0 + threadIdx.x;
  if (x >= vd.W) return;
  const int w[5] = {1, 4, 6, 4, 1};
  int xs[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) xs[k] = refl(x + k - 2, vd.W);
  const int32_t* g = U.gray + vd.map_off;
  const int y1 = min(it.y0 + kUfRows, vd.H);
  for (int y = it.y0; y < y1; ++y) {
    int acc = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int32_t* row = g + (int64_t)refl(y + j - 2, vd.H) * vd.W;
      int h = 0;
#pragma unroll
      for (int k = 0; k < 5; ++k) h += w[k] * row[xs[k]];
      acc += w[j] * h;
    }
    U.blur[vd.map_off + (int64_t)y * vd.W + x] = acc;
  }
}

__global__ __launch_bounds__(kUfCols) void uf_sobel_kernel(EdgeLaunch L, UfLaunch U) {
  const UfItem it = U.items[blockIdx.x];
  const ViewDesc vd = L.views[it.view];
  const int x = it.x0 + threadIdx.x;
  if (x >= vd.W) return;
  const int xl = refl(x - 1, vd.W), xr = refl(x + 1, vd.W);
  const int32_t* b = U.blur + vd.map_off;
  const int y1 = min(it.y0 + kUfRows, vd.H);
  for (int y = it.y0; y < y1; ++y) {
    const int32_t* ru = b + (int64_t)refl(y - 1, vd.H) * vd.W;
    const int32_t* rc = b + (int64_t)y * vd.W;
    const int32_t* rd = b + (int64_t)refl(y + 1, vd.H) * vd.W;
    const int gx = (ru[xr] - ru[xl]) + 2 * (rc[xr] - rc[xl]) + (rd[xr] - rd[xl]);
    const int gy = (rd[xl] - ru[xl]) + 2 * (rd[x] - ru[x]) + (rd[xr] - ru[xr]);
    const float fx = (float)gx, fy = (float)gy;
    const int64_t p = vd.map_off + (int64_t)y * vd.W + x;
    U.mag[p] = __builtin_fmaf(fx, fx, fy * fy);
    const Dir d = direction(fx, fy);
    U.code[p] = (uint8_t)((d.cH ? 1 : 0) | (d.cV ? 2 : 0) | (d.c45 ? 4 : 0) | (d.sgn ? 8 : 0));
  }
}

template <int PREC>
__global__ __launch_bounds__(kUfCols) void uf_nms_kernel(EdgeLaunch L, UfLaunch U) {
  using St = Store<PREC>;
  constexpr int NB = Keys<PREC>::bins;
  __shared__ uint32_t hist[NB];
  for (int i = threadIdx.x; i < NB; i += kUfCols) hist[i] = 0;
  __syncthreads();
  const UfItem it = U.items[blockIdx.x];
  const ViewDesc vd = L.views[it.view];
  const int x = it.x0 + threadIdx.x;
  if (x < vd.W) {
    const int xl = refl(x - 1, vd.W), xr = refl(x + 1, vd.W);
    const float* M = U.mag + vd.map_off;
    // this column's place in the stored map: strip x / 248, offset x % 248
    const int sx = x / kStripCols;
    typename St::T* out = reinterpret_cast<typename St::T*>(L.map) + vd.map_off +
                          (int64_t)sx * vd.strip_rows * kSlotPitch + (x - kStripCols * sx);
    const int y1 = min(it.y0 + kUfRows, vd.H);
    for (int y = it.y0; y < y1; ++y) {
      const float* ru = M + (int64_t)refl(y - 1, vd.H) * vd.W;
      const float* rc = M + (int64_t)y * vd.W;
      const float* rd = M + (int64_t)refl(y + 1, vd.H) * vd.W;
      const uint8_t c = U.code[vd.map_off + (int64_t)y * vd.W + x];
      Dir d;
      d.cH = c & 1;
      d.cV = (c >> 1) & 1;
      d.c45 = (c >> 2) & 1;
      d.sgn = (c & 8) ? -1 : 0;
      const float m = rc[x];
      const bool keep = keep_of(d, m, ru[xl], ru[x], ru[xr], rc[xl], rc[xr], rd[xl], rd[x], rd[xr]);
      const float v = St::kSquare ? m : __builtin_amdgcn_sqrtf(m) * kStoreScaleRoot;
      const float q = keep ? v : 0.0f;
      uint32_t bits;
      if constexpr (PREC == IGSP_FP32) {
        out[(int64_t)y * kSlotPitch] = q;
        bits = __float_as_uint(q);
      } else {
        const uint16_t h = (uint16_t)(St::pack2(q, 0.0f) & 0xFFFFu);
        out[(int64_t)y * kSlotPitch] = h;
        bits = __float_as_uint(St::widen(h));
      }
      if (bits != 0u)
        atomicAdd(&hist[min(max((int)(bits >> 16) - (int)Keys<PREC>::lo, 0), NB - 1)], 1u);
    }
  }
  __syncthreads();
  uint32_t* gh = L.hist + (int64_t)it.view * kBinsMax;
  for (int i = threadIdx.x; i < NB; i += kUfCols) {
    const uint32_t c = hist[i];
    if (c) atomicAdd(gh + i, c);
  }
}

// ------------------------------------------------------------- persistent form
//
// The batched pipeline as one launch: resident work-groups take tasks from a
// queue in list order. A view's stencil items come first; each later phase
// (refinement passes, normalisation) of the view sits a window of other
// views' work behind it, so memory-bound normalisation of earlier views runs
// beside the ALU-bound stencil of later ones. The work-group that finishes a
// phase's last task runs that view's selection step and publishes it; tasks
// of the next phase wait for it. Every task waited on was handed out
// earlier, to a work-group that is already running, so the waits end.

// Every wait is bounded (P.spin_limit polls, about half a second by default);
// the bound is never reached when the waited-on work is running. If it were,
// the launch records an error bit, finishes instead of hanging, and reports
// IGSP_ERR_TIMEOUT through the caller's status word.

__device__ __forceinline__ uint32_t ld_agent(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// MedState through device-coherent accesses (it is written by other
// work-groups of the same launch).
__device__ __forceinline__ MedState load_state(MedState* s) {
  uint32_t* p = reinterpret_cast<uint32_t*>(s);
  MedState r;
  r.prefix = ld_agent(p);
  r.shift = (int32_t)ld_agent(p + 1);
  r.rank = ld_agent(p + 2);
  r.n = ld_agent(p + 3);
  r.med = __uint_as_float(ld_agent(p + 4));
  r.pad[0] = r.pad[1] = r.pad[2] = 0u;
  return r;
}
__device__ __forceinline__ void store_state(MedState* s, const MedState& r) {
  uint32_t* p = reinterpret_cast<uint32_t*>(s);
  st_agent(p, r.prefix);
  st_agent(p + 1, (uint32_t)r.shift);
  st_agent(p + 2, r.rank);
  st_agent(p + 3, r.n);
  st_agent(p + 4, __float_as_uint(r.med));
}

// Exclusive scan over a work-group of NW waves; `total` gets the sum.
template <int NW>
__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t v, uint32_t* tmp, uint32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[w] = x;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t t = tmp[k];
    if (k < w) before += t;
    tot += t;
  }
  total = tot;
  __syncthreads();
  return before + x - v;
}

// Data crosses work-groups of this launch only through device-coherent
// accesses: the stored survivor values (buffer stores and loads with the SC1
// scope bit, kCpolAgent, which write through to and read from the
// device-coherent level instead of an XCD's L2), histograms (device-scope
// atomics, read back with SC1 loads), the selection state and the counters
// (relaxed agent-scope atomics, which are SC1 accesses too). There is no
// acquire or release fence anywhere: ordering comes from the hardware alone.
// Each wave waits for its own memory operations to complete (s_waitcnt 0)
// before the work-group barrier that precedes the counter update, and a
// reader issues its data loads only after the flag load it waited for has
// returned. A fence would instead write back or invalidate a whole XCD's L2
// per task.
__device__ __forceinline__ void drain() { __builtin_amdgcn_s_waitcnt(0); }

// The end of one task: count it off its phase and tell every thread whether
// it was the phase's last (then the count is restored for the next launch).
template <int NW>
__device__ __forceinline__ bool arrive(uint32_t* left, uint32_t restore, uint32_t* s_flag) {
  drain();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = __hip_atomic_fetch_add(left, 0xFFFFFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool last = old == 1u;
    if (last) st_agent(left, restore);
    *s_flag = last ? 1u : 0u;
  }
  __syncthreads();
  return *s_flag != 0u;
}

// Publish a view's selection step `level` (all threads call it).
__device__ __forceinline__ void publish(uint32_t* ready, uint32_t level) {
  drain();
  __syncthreads();
  if (threadIdx.x == 0) st_agent(ready, level);
}

// Wait until a view's selection has reached `level` (all threads call it),
// for at most `limit` (>= 1) polls; past that, record the error and go on.
__device__ __forceinline__ void await(uint32_t* ready, uint32_t level, uint32_t limit, uint32_t* error) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (ld_agent(ready) < level) {
      __builtin_amdgcn_s_sleep(8);
      if (++spins >= limit) {
        atomicOr(error, 1u);
        break;
      }
    }
  }
  __syncthreads();
}

// The thread index as a value the compiler cannot prove loop-invariant, for
// the task functions of the persistent kernel: addresses built from it are
// then recomputed inside each task instead of being held in registers across
// the whole task loop (where the stencil's register demand made them spill).
__device__ __forceinline__ int task_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// First selection step of view v from its global histogram (then cleared).
template <int PREC, int NW>
__device__ void select_hist(const EdgeLaunch& L, int v, uint32_t* tmp) {
  constexpr int NT = NW * 64, NB = Keys<PREC>::bins, PER = (NB + NT - 1) / NT;
  uint32_t* h = L.hist + (int64_t)v * kBinsMax;
  const int b0 = task_tid() * PER;
  uint32_t sum = 0;
  for (int k = 0; k < PER; ++k)
    if (b0 + k < NB) sum += ld_agent(h + b0 + k);
  uint32_t n = 0;
  const uint32_t excl = wg_excl_scan<NW>(sum, tmp, n);
  const uint32_t k = n ? (n - 1) / 2 : 0;
  if (n == 0) {
    if (threadIdx.x == 0) {
      MedState st = {0u, 0, 0u, 0u, 0.0f, {0u, 0u, 0u}};
      finish_view(L, v, st);
      store_state(L.state + v, st);
    }
  } else if (excl <= k && k < excl + sum) {
    uint32_t cum = excl;
    int b = b0;
    for (int j = 0; j < PER && b0 + j < NB; ++j) {
      const uint32_t c = ld_agent(h + b0 + j);
      if (cum + c > k) {
        b = b0 + j;
        break;
      }
      cum += c;
    }
    MedState st = {Keys<PREC>::lo + (uint32_t)b, 16, k - cum, n, 0.0f, {0u, 0u, 0u}};
    if (16 == final_shift(PREC)) finish_view(L, v, st);
    store_state(L.state + v, st);
  }
  for (int j = 0; j < PER; ++j)
    if (b0 + j < NB) st_agent(h + b0 + j, 0u);
  // the view's digit histogram starts from zero (the staged form's passes
  // leave theirs for the next call's median_select to clear); no refinement
  // task of the view runs before this step is published
  if (refine_passes(PREC) > 0)
    for (int i = task_tid(); i < kRefineBins; i += NT) st_agent(L.rhist + (int64_t)v * kRefineBins + i, 0u);
}

// A refinement selection step of view v from its digit histogram (then cleared).
template <int NW>
__device__ void select_refine(const EdgeLaunch& L, int v, int digit_bits, uint32_t* tmp) {
  constexpr int NT = NW * 64, PER = (kRefineBins + NT - 1) / NT;
  uint32_t* h = L.rhist + (int64_t)v * kRefineBins;
  MedState st = load_state(L.state + v);
  const int fin = final_shift(L.precision);
  const int b0 = task_tid() * PER;
  uint32_t sum = 0;
  for (int j = 0; j < PER; ++j)
    if (b0 + j < kRefineBins) sum += ld_agent(h + b0 + j);
  uint32_t tot = 0;
  const uint32_t excl = wg_excl_scan<NW>(sum, tmp, tot);
  if (st.n > 0 && st.shift > fin && excl <= st.rank && st.rank < excl + sum) {
    uint32_t cum = excl;
    int b = b0;
    for (int j = 0; j < PER && b0 + j < kRefineBins; ++j) {
      const uint32_t c = ld_agent(h + b0 + j);
      if (cum + c > st.rank) {
        b = b0 + j;
        break;
      }
      cum += c;
    }
    st.prefix = (st.prefix << digit_bits) | (uint32_t)b;
    st.shift -= digit_bits;
    st.rank -= cum;
    if (st.shift == fin) finish_view(L, v, st);
    store_state(L.state + v, st);
  }
  for (int j = 0; j < PER; ++j)
    if (b0 + j < kRefineBins) st_agent(h + b0 + j, 0u);
}

// Digit histogram of one row chunk for refinement pass `digit_bits`.
template <int PREC, int NW>
__device__ void refine_chunk(const EdgeLaunch& L, const RowChunk& ck, const MedState& st, int digit_bits,
                             uint32_t* hs) {
  constexpr int NT = NW * 64;
  const int tid = task_tid();
  for (int i = tid; i < kRefineBins; i += NT) hs[i] = 0;
  __syncthreads();
  if (st.n > 0 && st.shift > final_shift(PREC)) {
    const ViewDesc vd = L.views[ck.view];
    refine_slots<PREC, NW, true>(L, vd, ck, st, digit_bits, hs, tid & 63, __builtin_amdgcn_readfirstlane(tid >> 6));
  }
  __syncthreads();
  for (int i = tid; i < kRefineBins; i += NT) {
    const uint32_t c = hs[i];
    if (c) atomicAdd(&L.rhist[(int64_t)ck.view * kRefineBins + i], c);
  }
}

// Normalisation of one row chunk.
template <int PREC, int NW>
__device__ void norm_chunk(const EdgeLaunch& L, const RowChunk& ck, float med) {
  const ViewDesc vd = L.views[ck.view];
  const int tid = task_tid();
  norm_slots<PREC, NW, true>(L, vd, ck, med, tid & 63, __builtin_amdgcn_readfirstlane(tid >> 6));
}


template <int PREC, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(IGSP_PERSIST_WAVES_PER_EU))) void
edge_persistent_kernel(EdgeLaunch L, PersistLaunch P) {
  constexpr int NT = NW * 64;
  constexpr int NB = Keys<PREC>::bins;
  __shared__ uint32_t lds[NB];
  __shared__ uint32_t tmp[NW];
  __shared__ uint32_t s_task, s_flag;
  int acq_view = -1;   // readiness this work-group has already acquired
  uint32_t acq_level = 0;
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(&P.ctl->queue, 1u);
    __syncthreads();
    // re-read per task: values derived from the task index or the thread
    // index are recomputed inside each task instead of living across all
    const uint32_t t = __builtin_amdgcn_readfirstlane(*(volatile uint32_t*)&s_task);
    if (t >= (uint32_t)P.n_tasks) break;
    const PTask tk = P.tasks[t];
    const int v = tk.view;
    PViewSync* sy = P.sync + v;
    if (tk.type == kTaskStencil) {
      const EdgeItem it = L.items[tk.idx];
      const ViewDesc vd = L.views[v];
      const int tid = task_tid();
      for (int i = tid; i < NB; i += NT) lds[i] = 0;
      __syncthreads();
      const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int ys = it.y0 + w * L.seg_rows;
      const int ye = min(ys + L.seg_rows, it.y0 + it.rows);
      if (ys < ye) wave_strip<PREC, kCpolAgent>(L, vd, it.x0, ys, ye, lds);
      __syncthreads();
      uint32_t* gh = L.hist + (int64_t)v * kBinsMax;
      for (int i = tid; i < NB; i += NT) {
        const uint32_t c = lds[i];
        if (c) atomicAdd(gh + i, c);
      }
      if (arrive<NW>(&sy->left[0], sy->n_items, &s_flag)) {
        select_hist<PREC, NW>(L, v, tmp);
        publish(&sy->ready, 1u);
      }
    } else {
      const uint32_t need = (uint32_t)tk.phase;
      if (acq_view != v || acq_level < need) {
        await(&sy->ready, need + P.wait_bias, P.spin_limit, &P.ctl->error);
        acq_view = v;
        acq_level = need;
      }
      const RowChunk ck = L.chunks[tk.idx];
      const MedState st = load_state(L.state + v);
      if (tk.type == kTaskRefine) {
        const int db = refine_digit_bits(PREC);
        refine_chunk<PREC, NW>(L, ck, st, db, lds);
        if (arrive<NW>(&sy->left[tk.phase], sy->n_chunks, &s_flag)) {
          select_refine<NW>(L, v, db, tmp);
          publish(&sy->ready, need + 1u);
        }
      } else {
        norm_chunk<PREC, NW>(L, ck, st.med);
        // Nothing in this launch reads the output maps, so this count-off
        // does not wait for the task's stores: it only lets the view's last
        // normalisation task restore the counter and reset the readiness
        // level for the next launch, and every task that reads that level
        // has passed its wait before it counts itself off.
        if (threadIdx.x == 0) {
          uint32_t* left = &sy->left[tk.phase];
          if (__hip_atomic_fetch_add(left, 0xFFFFFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1u) {
            st_agent(left, sy->n_chunks);
            st_agent(&sy->ready, 0u);
          }
        }
      }
    }
    __syncthreads();
  }
  // The last work-group to leave reports the launch's status and restores
  // the queue. After a timeout a view's readiness level may be left behind
  // (a phase that went on without its predecessor), so every level is reset:
  // the next launch starts clean. (The phase counters are restored by their
  // last task in any case, and the histograms by the selection steps.)
  if (threadIdx.x == 0) s_flag = atomicAdd(&P.ctl->exited, 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (s_flag) {
    const uint32_t err = ld_agent(&P.ctl->error);
    if (err)
      for (int v = threadIdx.x; v < P.n_views; v += NT) st_agent(&P.sync[v].ready, 0u);
    drain();
    __syncthreads();
    if (threadIdx.x == 0) {
      if (L.status) *L.status = err ? IGSP_ERR_TIMEOUT : IGSP_OK;
      st_agent(&P.ctl->error, 0u);
      st_agent(&P.ctl->queue, 0u);
      st_agent(&P.ctl->exited, 0u);
    }
  }
}

template <int PREC>
hipError_t persistent_for_prec(const EdgeLaunch& L, const PersistLaunch& P, int grid, hipStream_t s) {
  switch (L.wg_waves) {
    case 1: hipLaunchKernelGGL((edge_persistent_kernel<PREC, 1>), dim3(grid), dim3(64), 0, s, L, P); break;
    case 2: hipLaunchKernelGGL((edge_persistent_kernel<PREC, 2>), dim3(grid), dim3(128), 0, s, L, P); break;
    case 8: hipLaunchKernelGGL((edge_persistent_kernel<PREC, 8>), dim3(grid), dim3(512), 0, s, L, P); break;
    default: hipLaunchKernelGGL((edge_persistent_kernel<PREC, 4>), dim3(grid), dim3(256), 0, s, L, P); break;
  }
  return hipGetLastError();
}

template <int PREC>
int blocks_per_cu_for_prec(int wg_waves) {
  int nb = 0;
  hipError_t e;
  switch (wg_waves) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_persistent_kernel<PREC, 1>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_persistent_kernel<PREC, 2>, 128, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_persistent_kernel<PREC, 8>, 512, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_persistent_kernel<PREC, 4>, 256, 0); break;
  }
  return e == hipSuccess ? nb : 0;
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

hipError_t launch_edge_persistent(const EdgeLaunch& L, const PersistLaunch& P, int grid, hipStream_t s) {
  if (grid <= 0 || P.n_tasks <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16: return persistent_for_prec<IGSP_FP16>(L, P, grid, s);
    case IGSP_BF16: return persistent_for_prec<IGSP_BF16>(L, P, grid, s);
    default: return persistent_for_prec<IGSP_FP32>(L, P, grid, s);
  }
}

int persistent_blocks_per_cu(int precision, int wg_waves) {
  switch (precision) {
    case IGSP_FP16: return blocks_per_cu_for_prec<IGSP_FP16>(wg_waves);
    case IGSP_BF16: return blocks_per_cu_for_prec<IGSP_BF16>(wg_waves);
    default: return blocks_per_cu_for_prec<IGSP_FP32>(wg_waves);
  }
}

hipError_t launch_edge_unfused(const EdgeLaunch& L, const UfLaunch& U, hipStream_t s) {
  if (U.n_items <= 0) return hipSuccess;
  const dim3 g(U.n_items), b(kUfCols);
  hipLaunchKernelGGL(uf_gray_kernel, g, b, 0, s, L, U);
  hipLaunchKernelGGL(uf_blur_kernel, g, b, 0, s, L, U);
  hipLaunchKernelGGL(uf_sobel_kernel, g, b, 0, s, L, U);
  switch (L.precision) {
    case IGSP_FP16: hipLaunchKernelGGL(uf_nms_kernel<IGSP_FP16>, g, b, 0, s, L, U); break;
    case IGSP_BF16: hipLaunchKernelGGL(uf_nms_kernel<IGSP_BF16>, g, b, 0, s, L, U); break;
    default: hipLaunchKernelGGL(uf_nms_kernel<IGSP_FP32>, g, b, 0, s, L, U); break;
  }
  return hipGetLastError();
}

hipError_t launch_median_select(const EdgeLaunch& L, int v0, int nv, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16: hipLaunchKernelGGL(median_select_kernel<IGSP_FP16>, dim3(nv), dim3(256), 0, s, L, v0); break;
    case IGSP_BF16: hipLaunchKernelGGL(median_select_kernel<IGSP_BF16>, dim3(nv), dim3(256), 0, s, L, v0); break;
    default: hipLaunchKernelGGL(median_select_kernel<IGSP_FP32>, dim3(nv), dim3(256), 0, s, L, v0); break;
  }
  return hipGetLastError();
}

hipError_t launch_median_refine(const EdgeLaunch& L, int chunk0, int n_chunks, int pass, hipStream_t s) {
  if (n_chunks <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16:
      hipLaunchKernelGGL(median_refine_kernel<IGSP_FP16>, dim3(n_chunks), dim3(256), 0, s, L, chunk0, pass);
      break;
    case IGSP_BF16:
      return hipSuccess;  // resolved by the first histogram
    default:
      hipLaunchKernelGGL(median_refine_kernel<IGSP_FP32>, dim3(n_chunks), dim3(256), 0, s, L, chunk0, pass);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_median_step(const EdgeLaunch& L, int v0, int nv, hipStream_t s) {
  const int passes = refine_passes(L.precision);
  if (nv <= 0 || passes == 0 || fold_last_step(L.precision)) return hipSuccess;
  hipLaunchKernelGGL(median_step_kernel, dim3(nv), dim3(256), 0, s, L, v0, passes);
  return hipGetLastError();
}

hipError_t launch_normalise(const EdgeLaunch& L, int chunk0, int n_chunks, hipStream_t s) {
  if (n_chunks <= 0) return hipSuccess;
  switch (L.precision) {
    case IGSP_FP16: hipLaunchKernelGGL(normalise_kernel<IGSP_FP16>, dim3(n_chunks), dim3(256), 0, s, L, chunk0); break;
    case IGSP_BF16: hipLaunchKernelGGL(normalise_kernel<IGSP_BF16>, dim3(n_chunks), dim3(256), 0, s, L, chunk0); break;
    default: hipLaunchKernelGGL(normalise_kernel<IGSP_FP32>, dim3(n_chunks), dim3(256), 0, s, L, chunk0); break;
  }
  return hipGetLastError();
}

}  // namespace igsp
