// Device-side building blocks shared by the emulation kernels: FP64 bit-field
// exponent extraction, exact fixed-point conversion, balanced base-256
// digits, the one-rounding conversion of a scaled 128-bit integer to FP64,
// and the gfx950 INT8 MFMA operand types.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ozk.h"

namespace ozk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __int128 i128;
typedef unsigned __int128 u128;

// v_mfma_i32_32x32x32_i8 lane layout (gfx950, checked on the device):
//   A operand: lane l holds A[l % 32][16 (l / 32) + j], j < 16 (16 int8);
//   B operand: lane l holds B[16 (l / 32) + j][l % 32];
//   accumulator register v of lane l is C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
__device__ __forceinline__ v16i mfma_i8_32x32x32(const v4i& a, const v4i& b, const v16i& c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Exponent e with 2^(e-1) <= |x| < 2^e for a finite nonzero x; OZK_EXP_ZERO
// for zero and OZK_EXP_NONFINITE for NaN/inf, so that max() over a row gives
// the row exponent or the right sentinel.
__device__ __forceinline__ int expo_of(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int ef = (int)((b >> 52) & 0x7ff);
  const uint64_t man = b & 0xfffffffffffffull;
  // branch-free selects, so that unrolled loads are not serialised behind branches
  const int sub = man == 0 ? OZK_EXP_ZERO : (64 - __clzll(man)) - 1074;  // subnormal: man 2^-1074
  const int e = ef == 0 ? sub : ef - 1022;
  return ef == 0x7ff ? OZK_EXP_NONFINITE : e;
}

// |x| = m 2^q with m an integer below 2^53 (signed result in m); x finite.
__device__ __forceinline__ void split_fp64(double x, int64_t& m, int& q) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int ef = (int)((b >> 52) & 0x7ff);
  uint64_t man = b & 0xfffffffffffffull;
  if (ef == 0) {
    q = -1074;
  } else {
    man |= 1ull << 52;
    q = ef - 1075;
  }
  m = (b >> 63) ? -(int64_t)man : (int64_t)man;
}

// X = floor(x 2^sh + 1/2) as an int64, exactly, for a finite x whose value
// times 2^sh is below 2^62 in magnitude; branch-free in FP64.  y = x 2^sh is
// exact unless it underflows, and then |y| < 2^-1022 gives X = 0 either way.
// f = floor(y) is exact, y - f is exact or (y in (-1/2, 0) with f = -1)
// rounds within [1/2, 1], so the test y - f >= 1/2 is decided correctly and
// X = f + [y - f >= 1/2] is an exact double (53 significant bits at most).
// It is split as hi 2^32 + lo with lo in [0, 2^32), both exact.
__device__ __forceinline__ int64_t round_half_up_scaled(double x, int sh) {
  const double y = ldexp(x, sh);
  const double f = floor(y);
  const double X = f + (y - f >= 0.5 ? 1.0 : 0.0);
  const double hi = floor(X * 0x1p-32);
  const double lo = __fma_rn(-hi, 0x1p32, X);
  return (int64_t)(((uint64_t)(uint32_t)(int32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Round-to-nearest-even of +-mag 2^E as one rounding (gradual underflow and
// overflow included); round_scaled takes a signed Z.
__device__ __forceinline__ double round_mag(u128 mag, bool neg, int E) {
  if (mag == 0) return 0.0;
  const uint64_t hi = (uint64_t)(mag >> 64), lo = (uint64_t)mag;
  const int n = hi ? 128 - __clzll(hi) : 64 - __clzll(lo);
  if (n + E >= -1021) {
    // Normal (or overflowing) result: the top 64 bits of mag with the bits
    // below folded into the lowest one (sticky; the 53-bit rounding never
    // keeps it), one RN-even conversion to double, then an exact scaling.
    const int sh = n > 64 ? n - 64 : 0;
    const uint64_t w = sh ? (uint64_t)(mag >> sh) | (uint64_t)((lo << (64 - sh)) != 0) : lo;
    const double r = ldexp((double)w, E + sh);
    return neg ? -r : r;
  }
  // Subnormal result: round at the fixed position 2^-1074 directly.
  int drop = n - 53;
  if (-1074 - E > drop) drop = -1074 - E;
  uint64_t q;
  if (drop <= 0) {
    q = lo;  // n <= 53
    drop = 0;
  } else if (drop >= 128) {
    if (drop > 128) return neg ? -0.0 : 0.0;
    q = (mag > ((u128)1 << 127)) ? 1 : 0;
  } else {
    const u128 qq = mag >> drop;
    const u128 rem = mag & (((u128)1 << drop) - 1);
    const u128 half = (u128)1 << (drop - 1);
    q = (uint64_t)qq;
    if (rem > half || (rem == half && (q & 1))) q += 1;
  }
  const long long Eq = (long long)E + drop;
  const double r = (Eq > 2100) ? __builtin_inf() : ldexp((double)q, (int)Eq);
  return neg ? -r : r;
}

// The same single rounding to binary32 (24 significant bits, gradual
// underflow at 2^-149, overflow to infinity).
__device__ __forceinline__ float round_mag_f32(u128 mag, bool neg, int E) {
  if (mag == 0) return 0.0f;
  const uint64_t hi = (uint64_t)(mag >> 64), lo = (uint64_t)mag;
  const int n = hi ? 128 - __clzll(hi) : 64 - __clzll(lo);
  if (n + E >= -125) {
    // normal or overflowing: top 64 bits with a sticky bit, one RN-even
    // conversion to binary32, an exact scaling
    const int sh = n > 64 ? n - 64 : 0;
    const uint64_t w = sh ? (uint64_t)(mag >> sh) | (uint64_t)((lo << (64 - sh)) != 0) : lo;
    const float r = ldexpf((float)w, E + sh);
    return neg ? -r : r;
  }
  // subnormal: round at the fixed position 2^-149
  int drop = n - 24;
  if (-149 - E > drop) drop = -149 - E;
  uint64_t q;
  if (drop <= 0) {
    q = lo;  // n <= 24
    drop = 0;
  } else if (drop >= 128) {
    if (drop > 128) return neg ? -0.0f : 0.0f;
    q = (mag > ((u128)1 << 127)) ? 1 : 0;
  } else {
    const u128 qq = mag >> drop;
    const u128 rem = mag & (((u128)1 << drop) - 1);
    const u128 half = (u128)1 << (drop - 1);
    q = (uint64_t)qq;
    if (rem > half || (rem == half && (q & 1))) q += 1;
  }
  const float r = ldexpf((float)q, E + drop);
  return neg ? -r : r;
}

__device__ __forceinline__ float round_scaled_f32(i128 Z, int E) {
  const bool neg = Z < 0;
  return round_mag_f32(neg ? (u128)0 - (u128)Z : (u128)Z, neg, E);
}

__device__ __forceinline__ double round_scaled(i128 Z, int E) {
  const bool neg = Z < 0;
  return round_mag(neg ? (u128)0 - (u128)Z : (u128)Z, neg, E);
}

// BLAS-style update: alpha*h when beta == 0 (c not read), else
// fma(alpha, h, beta*c).
__device__ __forceinline__ double axpby(double alpha, double h, double beta, const double* c) {
  if (beta == 0.0) return alpha * h;
  const double bc = beta * (*c);
  return __fma_rn(alpha, h, bc);
}

__device__ __forceinline__ float axpby_f32(float alpha, float h, float beta, const float* c) {
  if (beta == 0.0f) return alpha * h;
  const float bc = beta * (*c);
  return __fmaf_rn(alpha, h, bc);
}

// Fused multiply-add in the precision of the operands.
__device__ __forceinline__ double fma_any(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fma_any(float a, float b, float c) { return __fmaf_rn(a, b, c); }

// Maximum / sum over each aligned group of 16 lanes.
__device__ __forceinline__ int group16_max(int v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) {
    const int o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  return v;
}

__device__ __forceinline__ int64_t group16_sum64(int64_t v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  return v;
}

}  // namespace ozk
