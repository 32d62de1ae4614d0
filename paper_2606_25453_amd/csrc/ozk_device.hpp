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
  if (ef == 0x7ff) return OZK_EXP_NONFINITE;
  if (ef != 0) return ef - 1022;
  if (man == 0) return OZK_EXP_ZERO;
  return (64 - __clzll(man)) - 1074;  // subnormal: man 2^-1074
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

// X = floor(x 2^sh + 1/2) exactly for a finite x whose value times 2^sh is
// below 2^62 in magnitude.
__device__ __forceinline__ int64_t round_half_up_scaled(double x, int sh_extra) {
  int64_t m;
  int q;
  split_fp64(x, m, q);
  const int sh = q + sh_extra;
  if (m == 0) return 0;
  if (sh >= 0) return (int64_t)((uint64_t)m << sh);
  if (sh <= -62) return 0;  // |m 2^sh| < 2^-9
  return (m + ((int64_t)1 << (-sh - 1))) >> (-sh);  // arithmetic shift = floor
}

// Round-to-nearest-even of Z 2^E as one rounding (gradual underflow and
// overflow included).
__device__ __forceinline__ double round_scaled(i128 Z, int E) {
  if (Z == 0) return 0.0;
  const bool neg = Z < 0;
  const u128 mag = neg ? (u128)0 - (u128)Z : (u128)Z;
  const uint64_t hi = (uint64_t)(mag >> 64), lo = (uint64_t)mag;
  const int n = hi ? 128 - __clzll(hi) : 64 - __clzll(lo);
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

// BLAS-style update: alpha*h when beta == 0 (c not read), else
// fma(alpha, h, beta*c).
__device__ __forceinline__ double axpby(double alpha, double h, double beta, const double* c) {
  if (beta == 0.0) return alpha * h;
  const double bc = beta * (*c);
  return __fma_rn(alpha, h, bc);
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
