// common.h -- shared device types and helpers of libdsi (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef unsigned char u8;

#define DSI_INLINE __device__ __forceinline__

// ---------------------------------------------------------------- conversions
template <typename T> DSI_INLINE T from_f32(float v);
template <> DSI_INLINE float from_f32<float>(float v) { return v; }
template <> DSI_INLINE double from_f32<double>(float v) { return (double)v; }
template <> DSI_INLINE bf16 from_f32<bf16>(float v) { return (bf16)v; }  // RNE (v_cvt_pk_bf16_f32)

DSI_INLINE float to_f32(float v) { return v; }
DSI_INLINE float to_f32(double v) { return (float)v; }
DSI_INLINE float to_f32(bf16 v) { return (float)v; }

// OCP FP8 e4m3 ("fn": bias 7, no infinities, max 448, 0x7f/0xff are NaN).
// Round to nearest even with saturation to +-448; NaN maps to 0x7f.
DSI_INLINE u8 f32_to_e4m3(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t sign = (u >> 24) & 0x80u;
  float a = fabsf(f);
  if (!(a == a)) return 0x7f;
  if (a >= 448.0f) return (u8)(sign | 0x7e);
  if (a < 0.0009765625f) {  // below 2^-10: rounds to 0 or the smallest subnormal 2^-9
    return (u8)(sign | (a > 0.0009765625f ? 1u : 0u));
  }
  int e;
  float m = frexpf(a, &e);  // a = m * 2^e, m in [0.5, 1)
  int E = e - 1;            // a = (2m) * 2^E, 2m in [1, 2)
  float q;
  if (E < -6) {             // subnormal: multiples of 2^-9
    q = rintf(a * 512.0f);  // rintf rounds half to even
    uint32_t code = (uint32_t)q;  // 0..8 (8 == 2^-6, the smallest normal)
    return (u8)(sign | code);
  }
  q = rintf(ldexpf(a, 3 - E));  // 8..16 mantissa steps
  if (q >= 16.0f) { q = 8.0f; E += 1; }
  if (E > 8) return (u8)(sign | 0x7e);
  uint32_t code = ((uint32_t)(E + 7) << 3) | ((uint32_t)q - 8u);
  if (code > 0x7e) code = 0x7e;
  return (u8)(sign | code);
}

DSI_INLINE float e4m3_to_f32(u8 c) {
  uint32_t s = c & 0x80u, e = (c >> 3) & 0xfu, m = c & 7u;
  float v = e == 0 ? ldexpf((float)m, -9) : ldexpf((float)(8u + m), (int)e - 10);
  return s ? -v : v;
}

// f(std::integral_constant<int, I>{}) for I = 0 .. N-1, in order: a loop whose index
// is a compile-time constant in the body (fully unrolled straight-line code)
template <typename F, int... I> DSI_INLINE void static_for_seq(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F> DSI_INLINE void static_for(F &&f) { static_for_seq(f, std::make_integer_sequence<int, N>{}); }

// ------------------------------------------------------------------ XCDs
// The workgroups of a launch go to the 8 XCDs in turn (block i to XCD i % 8), and each
// XCD has its own L2.  xcd_logical(i, n) renumbers the n blocks of a grid so that
// every XCD runs one contiguous range of logical indices: blocks that read the same
// data, given neighbouring logical indices, then run side by side on one L2.
DSI_INLINE int xcd_logical(int i, int n) {
  const int x = i & 7, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

// ------------------------------------------------------------------ MFMA
// 32x32 result tile, lane l holds D[8*(r/4) + 4*(l/32) + r%4][l%32] in acc[r].
DSI_INLINE int mfma_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

DSI_INLINE f32x16 mfma_bf16(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
DSI_INLINE f32x16 mfma_f32(float a, float b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// FP8 e4m3 x e4m3 with unit block scales (E8M0 exponent 127 = 2^0).
DSI_INLINE f32x16 mfma_fp8(const i32x8 &a, const i32x8 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// 8 consecutive K elements per lane ("fragment slice").  For bf16 one MFMA
// consumes them; for fp32, eight 32x32x2 MFMAs consume element e of both
// operands at step e.  The K order inside a 16-wide step is irrelevant as
// long as both operands use the same one.
template <typename T> struct Frag8;
template <> struct Frag8<bf16> {
  bf16x8 v;
  DSI_INLINE void mma(const Frag8 &b, f32x16 &acc) const { acc = mfma_bf16(v, b.v, acc); }
};
template <> struct Frag8<float> {
  f32x4 lo, hi;
  DSI_INLINE void mma(const Frag8 &b, f32x16 &acc) const {
    acc = mfma_f32(lo[0], b.lo[0], acc);
    acc = mfma_f32(lo[1], b.lo[1], acc);
    acc = mfma_f32(lo[2], b.lo[2], acc);
    acc = mfma_f32(lo[3], b.lo[3], acc);
    acc = mfma_f32(hi[0], b.hi[0], acc);
    acc = mfma_f32(hi[1], b.hi[1], acc);
    acc = mfma_f32(hi[2], b.hi[2], acc);
    acc = mfma_f32(hi[3], b.hi[3], acc);
  }
};

// FP8 e4m3 (stored as bytes): 32 consecutive K elements per lane, one
// 32x32x64 MFMA per fragment pair.
template <> struct Frag8<u8> {
  i32x8 v;
  DSI_INLINE void mma(const Frag8 &b, f32x16 &acc) const { acc = mfma_fp8(v, b.v, acc); }
};

template <typename T> DSI_INLINE Frag8<T> frag_load(const T *p);  // p 16-byte aligned
template <> DSI_INLINE Frag8<bf16> frag_load<bf16>(const bf16 *p) {
  Frag8<bf16> f;
  f.v = *reinterpret_cast<const bf16x8 *>(p);
  return f;
}
template <> DSI_INLINE Frag8<float> frag_load<float>(const float *p) {
  Frag8<float> f;
  f.lo = *reinterpret_cast<const f32x4 *>(p);
  f.hi = *reinterpret_cast<const f32x4 *>(p + 4);
  return f;
}
template <> DSI_INLINE Frag8<u8> frag_load<u8>(const u8 *p) {
  Frag8<u8> f;
  const i32x4 lo = *reinterpret_cast<const i32x4 *>(p), hi = *reinterpret_cast<const i32x4 *>(p + 16);
  f.v = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return f;
}
template <typename T> DSI_INLINE Frag8<T> frag_zero() {
  Frag8<T> f;
  if constexpr (sizeof(T) == 2) {
    for (int e = 0; e < 8; ++e) f.v[e] = (bf16)0.0f;
  } else {
    f.lo = f32x4{0, 0, 0, 0};
    f.hi = f32x4{0, 0, 0, 0};
  }
  return f;
}
// element-wise build from 8 floats (converted to T)
template <typename T> DSI_INLINE Frag8<T> frag_from(const float *x) {
  Frag8<T> f;
  if constexpr (sizeof(T) == 2) {
    for (int e = 0; e < 8; ++e) f.v[e] = (bf16)x[e];
  } else {
    f.lo = f32x4{x[0], x[1], x[2], x[3]};
    f.hi = f32x4{x[4], x[5], x[6], x[7]};
  }
  return f;
}

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
