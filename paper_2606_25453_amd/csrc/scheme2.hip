// Ozaki Scheme II on gfx950 INT8 MFMA (paper Sec. II-C.2 and Sec. IV), real
// and 3M complex.
//
//   k_s2_split_rows     row scale sigma_i from an exact bound on the row's
//                       2-norm, then the s symmetric residue planes (Eq. 5)
//   k_s2_col_scales     the same for the columns of B (LDS reductions of
//                       integers, so the result does not depend on the order)
//   k_s2_gemm_mod       one INT8 GEMM per modulus with smod in the epilogue
//                       (Eqs. 6-7); 3M: three products per modulus and the
//                       combination T1-T2, T3-T1-T2 before the reduction
//   k_s2_crt            CRT recombination in multiword integers (Eq. 8) with
//                       the symmetric lift, then one rounding of Z 2^-(sigma+tau)
#include <type_traits>

#include "mfma_gemm.hpp"
#include "ozk_device.hpp"
#include "ozk_internal.hpp"

namespace ozk {

// ------------------------------------------------------------- moduli table

struct S2Tables {
  int m[OZK_MAX_S];
  double md[OZK_MAX_S];     // m_l as a double
  double inv_m[OZK_MAX_S];  // 1 / m_l rounded
  double p26[OZK_MAX_S];    // 2^26 mod m_l
  double p52[OZK_MAX_S];    // 2^52 mod m_l
};

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Greedy descending pairwise-coprime moduli from 256 (256, 255, 253, ...).
constexpr S2Tables make_s2_tables() {
  S2Tables t{};
  int n = 0;
  for (int c = 256; n < OZK_MAX_S; --c) {
    bool ok = true;
    for (int i = 0; i < n; ++i)
      if (gcd_c(c, t.m[i]) != 1) ok = false;
    if (ok) t.m[n++] = c;
  }
  for (int i = 0; i < OZK_MAX_S; ++i) {
    t.md[i] = t.m[i];
    t.inv_m[i] = 1.0 / t.m[i];
    const int64_t r26 = ((int64_t)1 << 26) % t.m[i];
    t.p26[i] = (double)r26;
    t.p52[i] = (double)((r26 * r26) % t.m[i]);
  }
  return t;
}

constexpr S2Tables kS2 = make_s2_tables();
__constant__ S2Tables c_s2 = kS2;

int s2_modulus(int l) { return kS2.m[l]; }

// smod(t, m_l) for an integer-valued double |t| < 2^40: with
// q = floor(t / m + 1/2) the remainder t - q m lies in [-floor(m/2),
// ceil(m/2) - 1].  For odd m, t / m is at least 1/(2m) >= 2^-9 away from a
// half-integer while the computed t / m + 1/2 is within 2^-19 of its exact
// value, so q is the nearest integer; for m = 256 everything is exact.  The
// final fma is exact as well.
__device__ __forceinline__ int smod_exact(double t, int l) {
  const double q = floor(__fma_rn(t, c_s2.inv_m[l], 0.5));
  return (int)__fma_rn(-q, c_s2.md[l], t);
}

// smod of an INT32 accumulator.
__device__ __forceinline__ int smod_i32(int x, int l) { return smod_exact((double)x, l); }

// The low byte of smod(x, m_l) for |x| < 2^30, in two binary64 operations
// and a 24-bit multiply: fma(x, 1/m, 1.5 * 2^52) rounds x / m to the nearest
// integer q, which the low 32 bits of that double hold (its unit in the last
// place is 1 and 2^51 + q is its fraction); the product's error is below
// 2^-29 while an odd m keeps x / m at least 1/(2m) from a half-integer, so q
// is exact and x - q m is the symmetric residue.  Only its byte is kept, which
// needs q m mod 256 alone (from the low byte of q), and for m = 256 (the only
// even modulus) any integer q leaves the low byte of x, the byte of the
// symmetric residue.  The upper bytes of the result are not defined.
__device__ __forceinline__ uint32_t smod_small_byte(int x, int l) {
  const double y = __fma_rn((double)x, c_s2.inv_m[l], 6755399441055744.0);
  const uint32_t q = (uint32_t)(uint64_t)__double_as_longlong(y);
  // both factors visibly below 2^24 (m <= 256), so that the product is one
  // 24-bit multiply
  return (uint32_t)x - (q & 0xFFu) * ((uint32_t)c_s2.m[l] & 0x1FFu);
}

// smod(a + b, m_l) for a, b already symmetric residues of m_l.
__device__ __forceinline__ int smod_sum(int a, int b, int l) {
  const int m = c_s2.m[l];
  int r = a + b;
  r -= r > (m - 1) / 2 ? m : 0;
  r += r < -(m / 2) ? m : 0;
  return r;
}

// a' = trunc(a 2^sigma) as three 26-bit limbs, exact doubles carrying the
// sign of a: a' = x2 2^52 + x1 2^26 + x0.  The row (column) norm bound gives
// |a'| < 2^T <= 2^77, so three limbs hold it; t = x2 (2^52 mod m) +
// x1 (2^26 mod m) + x0 is then an exact double (|t| < 2^35) congruent to a'.
// Branch-free in FP64: a 2^sigma is exact unless it underflows (then its
// truncation is 0 either way), truncation is exact, and each limb split is an
// exact scaling, truncation and fma (the remainders keep the sign of a').
struct Limbs3 {
  double x0, x1, x2;
};

__device__ __forceinline__ Limbs3 scaled_limbs(double a, int sigma) {
  const double y = trunc(ldexp(a, sigma));
  const double x2 = trunc(y * 0x1p-52);
  const double r1 = __fma_rn(-x2, 0x1p52, y);
  const double x1 = trunc(r1 * 0x1p-26);
  const double x0 = __fma_rn(-x1, 0x1p26, r1);
  return Limbs3{x0, x1, x2};
}

__device__ __forceinline__ int residue_of(const Limbs3& v, int l) {
  return smod_exact(__fma_rn(v.x2, c_s2.p52[l], __fma_rn(v.x1, c_s2.p26[l], v.x0)), l);
}

// Per-entry exponent for the scale bound: |entry| < 2^ex.  Complex entries
// bound |re| + |im| < 2^(max(expo re, expo im) + 1).
template <bool CPLX, typename T>
__device__ __forceinline__ int entry_expo(const T* x) {
  if (!CPLX) return expo_of((double)x[0]);
  const int a = expo_of((double)x[0]), b = expo_of((double)x[1]);
  const int e = a > b ? a : b;  // the non-finite sentinel is the largest value
  return (e == OZK_EXP_NONFINITE || e == OZK_EXP_ZERO) ? e : e + 1;
}

// ceil(2^40 4^(ex - emax)) for an entry with exponent ex <= emax; 0 for zero.
__device__ __forceinline__ int64_t norm_term(int ex, int emax) {
  if (ex == OZK_EXP_ZERO) return 0;
  const int d = ex - emax;
  return d >= -20 ? ((int64_t)1 << (40 + 2 * d)) : 1;
}

// sigma = T - nb with nb = emax + ceil((ceil(log2 S) - 40) / 2).
__device__ __forceinline__ int scale_from(int emax, int64_t S, int T) {
  if (emax == OZK_EXP_NONFINITE) return OZK_EXP_NONFINITE;
  if (emax == OZK_EXP_ZERO || S <= 0) return 0;
  const int clog = S == 1 ? 0 : 64 - __clzll((uint64_t)(S - 1));
  const int c = clog - 40;
  const int half = c >= 0 ? (c + 1) / 2 : -((-c) / 2);
  return T - (emax + half);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct S2Args {
  int s;
  int T;  // T_A for rows, T_B for columns
};

// Residues of 4 consecutive entries of a line with scale sigma for every
// modulus, stored as one dword per plane at dst (plane stride `plane`; the
// complex planes re, im, sum of one chunk are `slab` bytes apart).
template <bool CPLX>
__device__ __forceinline__ void s2_store_residues(const double (&re)[4], const double (&im)[4], int sigma, int s,
                                                  int8_t* __restrict__ dst, int64_t plane, int64_t slab) {
  Limbs3 vr[4], vi[CPLX ? 4 : 1];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    vr[j] = scaled_limbs(re[j], sigma);
    if (CPLX) vi[CPLX ? j : 0] = scaled_limbs(im[j], sigma);
  }
  for (int l = 0; l < s; ++l, dst += plane) {
    uint32_t w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = residue_of(vr[j], l);
      w0 |= (uint32_t)(uint8_t)a << (8 * j);
      if (CPLX) {
        const int b = residue_of(vi[CPLX ? j : 0], l);
        w1 |= (uint32_t)(uint8_t)b << (8 * j);
        w2 |= (uint32_t)(uint8_t)smod_sum(a, b, l) << (8 * j);
      }
    }
    *reinterpret_cast<uint32_t*>(dst) = w0;
    if (CPLX) {
      *reinterpret_cast<uint32_t*>(dst + slab) = w1;
      *reinterpret_cast<uint32_t*>(dst + 2 * slab) = w2;
    }
  }
}

// Four packed rows per wave, 16 lanes per row: exponent max and norm-bound
// sum by 16-lane reductions, then residues of 4 consecutive k per lane (one
// dword per plane).  The four rows of one chunk are adjacent in the packed
// layout, so every store instruction writes whole 128-byte lines.  Every
// modulus plane is a packed operand of the shared GEMM core: real
// packed[l][c][r][32], complex packed[l][c][q][r][32] (q = re, im, sum).
// Non-finite rows and k past K get zero residues, and so do the padding rows
// when zero_pad is set (an operand whose padding rows feed only outputs that
// are never stored may leave them as they are); the main loop has no
// condition between its loads (only the 4-k group straddling K takes the
// guarded path).  Rows past `rows` load row 0 and discard it, so that every
// lane takes part in the reductions.
constexpr int S2_ROWS_PER_BLOCK = 16;

// The entry exponents of a row block kept in LDS between the maximum and the
// norm-bound pass (one read of the operand instead of two): int16 per entry,
// rows (K + 2) entries apart (a row per bank offset), zero entries as
// INT16_MIN.  The batched pre-pass caches rows up to this K.
constexpr int S2_ECACHE_BATCH_K = 1024;
// The row-scale launch caches rows up to this K (128 KB of LDS).
constexpr int S2_ECACHE_MAX_K = 4096;

__host__ __device__ constexpr int s2_ecache_bytes(int64_t kc) {
  return kc > 0 ? (int)(S2_ROWS_PER_BLOCK * (kc + 2) * 2) : 0;
}

template <bool CPLX, typename T = double>
// kb0, kb1 (multiples of 64): the K range whose residues this block writes
// (kb1 < 0: to Kp); sigma_in: the row scales already computed (the residue
// pass split over K), else this block computes and stores them; ecache: LDS
// for the exponents of rows with K <= kc (null: read the row twice).
__device__ __forceinline__ void s2_split_rows_block(const T* __restrict__ X, int64_t ldx, int64_t rows,
                                                    int64_t K, int64_t Kp, int64_t rows_packed, S2Args sa,
                                                    int32_t* __restrict__ sigma_out, int8_t* __restrict__ packed,
                                                    int64_t blk, int64_t kb0 = 0, int64_t kb1 = -1,
                                                    const int32_t* __restrict__ sigma_in = nullptr,
                                                    bool zero_pad = true, int16_t* ecache = nullptr,
                                                    int64_t kc = 0) {
  constexpr int W = CPLX ? 2 : 1, NP = CPLX ? 3 : 1;
  const int lane = threadIdx.x & 63, q = lane & 15;
  const int64_t r = (blk * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
  if (r >= rows_packed) return;  // whole waves only (rows_packed is a multiple of 16)
  const bool in = r < rows;
  if (!in && !zero_pad) return;  // a whole row's 16 lanes: the reductions stay within rows
  const T* xr = X + (in ? r : 0) * ldx * W;
  int sigma = 0;
  if (sigma_in) {
    sigma = in ? sigma_in[r] : 0;
  } else {
    const bool cached = ecache != nullptr && K <= kc;  // uniform
    int16_t* er = cached ? ecache + (threadIdx.x >> 4) * (kc + 2) : nullptr;
    int e = OZK_EXP_ZERO;
    if (cached) {
#pragma unroll 8
      for (int64_t k = q; k < K; k += 16) {
        const int ek = entry_expo<CPLX>(xr + k * W);
        // finite exponents lie in [-1074, 1025]; a non-finite entry makes the
        // row's scale non-finite, so its cached value is never read
        er[k] = (int16_t)(ek == OZK_EXP_ZERO ? -32768 : ek > 32767 ? 32767 : ek);
        e = ek > e ? ek : e;
      }
    } else {
#pragma unroll 8
      for (int64_t k = q; k < K; k += 16) {
        const int ek = entry_expo<CPLX>(xr + k * W);
        e = ek > e ? ek : e;
      }
    }
    e = group16_max(in ? e : OZK_EXP_ZERO);
    int64_t S = 0;
    if (e != OZK_EXP_NONFINITE && e != OZK_EXP_ZERO) {
      if (cached) {  // each lane reads back the entries it wrote
#pragma unroll 8
        for (int64_t k = q; k < K; k += 16) {
          const int c = er[k];
          S += norm_term(c == -32768 ? OZK_EXP_ZERO : c, e);
        }
      } else {
#pragma unroll 8
        for (int64_t k = q; k < K; k += 16) S += norm_term(entry_expo<CPLX>(xr + k * W), e);
      }
    }
    S = group16_sum64(S);
    sigma = in ? scale_from(e, S, sa.T) : 0;
    if (in && q == 0) sigma_out[r] = sigma;
  }
  const int64_t kend = kb1 < 0 || kb1 > Kp ? Kp : kb1, kfull = K < kend ? K : kend;
  const int64_t plane = rows_packed * Kp * NP, slab = rows_packed * OZK_K_CHUNK;
  auto dst_of = [&](int64_t k0) { return packed + (k0 / OZK_K_CHUNK) * NP * slab + r * OZK_K_CHUNK + k0 % OZK_K_CHUNK; };
  int64_t k0 = kb0 + (int64_t)q * 4;
  if (in && sigma != OZK_EXP_NONFINITE) {
    for (; k0 + 4 <= kfull; k0 += 64) {
      double re[4], im[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        re[j] = xr[(k0 + j) * W];
        im[j] = CPLX ? xr[(k0 + j) * W + 1] : 0.0;
      }
      s2_store_residues<CPLX>(re, im, sigma, sa.s, dst_of(k0), plane, slab);
    }
    for (; k0 < kend; k0 += 64) {
      double re[4], im[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool kin = k0 + j < K;
        re[j] = kin ? xr[(k0 + j) * W] : 0.0;
        im[j] = CPLX && kin ? xr[(k0 + j) * W + 1] : 0.0;
      }
      s2_store_residues<CPLX>(re, im, sigma, sa.s, dst_of(k0), plane, slab);
    }
  } else {
    for (; k0 < kend; k0 += 64) {
      int8_t* dst = dst_of(k0);
      for (int l = 0; l < sa.s; ++l, dst += plane)
#pragma unroll
        for (int qq = 0; qq < NP; ++qq) *reinterpret_cast<uint32_t*>(dst + qq * slab) = 0u;
    }
  }
}

// kc > 0: the exponents cached in s2_ecache_bytes(kc) bytes of dynamic LDS.
template <bool CPLX, typename T = double>
__global__ __launch_bounds__(256) void k_s2_split_rows(const T* __restrict__ X, int64_t ldx, int64_t rows,
                                                       int64_t K, int64_t Kp, int64_t rows_packed, S2Args sa,
                                                       int32_t* __restrict__ sigma_out,
                                                       int8_t* __restrict__ packed, int64_t kc) {
  extern __shared__ int16_t ecache[];
  s2_split_rows_block<CPLX, T>(X, ldx, rows, K, Kp, rows_packed, sa, sigma_out, packed, blockIdx.x, 0, -1, nullptr,
                               true, kc > 0 ? ecache : nullptr, kc);
}

// The residues of a row block over one K range per grid y (the row scales
// computed beforehand): enough workgroups to fill the GPU when the rows are
// few and long.
constexpr int64_t S2_ROW_KR = 512;

template <bool CPLX, typename T = double>
__global__ __launch_bounds__(256) void k_s2_row_residues(const T* __restrict__ X, int64_t ldx, int64_t rows,
                                                         int64_t K, int64_t Kp, int64_t rows_packed, S2Args sa,
                                                         const int32_t* __restrict__ sigma,
                                                         int8_t* __restrict__ packed) {
  const int64_t kb0 = (int64_t)blockIdx.y * S2_ROW_KR;
  s2_split_rows_block<CPLX, T>(X, ldx, rows, K, Kp, rows_packed, sa, nullptr, packed, blockIdx.x, kb0, kb0 + S2_ROW_KR,
                               sigma);
}

// Column scales: a block of 256 threads covers 32 consecutive columns with 8
// k-groups per column (coalesced 32-column row segments); the max exponent
// and then the norm-bound sum are reduced through LDS, so no atomics and no
// scratch memory are needed and the result does not depend on the order.
template <bool CPLX, typename TX = double>
__device__ __forceinline__ void s2_col_scales_block(const TX* __restrict__ X, int64_t ldx, int64_t K,
                                                    int64_t cols, int T, int32_t* __restrict__ tau, int64_t blk) {
  constexpr int W = CPLX ? 2 : 1;
  __shared__ int red_e[8][32];
  __shared__ int64_t red_s[8][32];
  const int cl = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t j = blk * 32 + cl;
  const bool in = j < cols;
  int e = OZK_EXP_ZERO;
  if (in)
#pragma unroll 8
    for (int64_t k = g; k < K; k += 8) {
      const int ek = entry_expo<CPLX>(X + (k * ldx + j) * W);
      e = ek > e ? ek : e;
    }
  red_e[g][cl] = e;
  __syncthreads();
  int emax = red_e[0][cl];
#pragma unroll
  for (int i = 1; i < 8; ++i) emax = red_e[i][cl] > emax ? red_e[i][cl] : emax;
  int64_t S = 0;
  if (in && emax != OZK_EXP_ZERO && emax != OZK_EXP_NONFINITE)
#pragma unroll 8
    for (int64_t k = g; k < K; k += 8) S += norm_term(entry_expo<CPLX>(X + (k * ldx + j) * W), emax);
  red_s[g][cl] = S;
  __syncthreads();
  if (g == 0 && in) {
    int64_t tot = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) tot += red_s[i][cl];
    tau[j] = scale_from(emax, tot, T);
  }
}

template <bool CPLX, typename TX = double>
__global__ __launch_bounds__(256) void k_s2_col_scales(const TX* __restrict__ X, int64_t ldx, int64_t K,
                                                       int64_t cols, int T, int32_t* __restrict__ tau) {
  s2_col_scales_block<CPLX, TX>(X, ldx, K, cols, T, tau, blockIdx.x);
}

// Column scales with one read of the operand: a block covers CC columns
// (16 real, 8 complex: 128 bytes of a row) over all of K in 256 / CC k-groups
// of CC lanes, keeping each entry's exponent in LDS (int16, k-major, zero
// entries as INT16_MIN) for the norm-bound pass; the maximum and the sum are
// reduced through LDS, in a fixed order.  Used when the cache of every block
// of the launch fits the GPU at once (K <= S2_ECACHE_MAX_K).
template <bool CPLX>
struct S2CCols {
  static constexpr int CC = CPLX ? 8 : 16;  // columns per block
  static constexpr int G = 256 / CC;        // k-groups
};

__host__ __device__ constexpr int s2_ccache_bytes(bool cplx, int64_t K) {
  return (int)((cplx ? S2CCols<true>::CC : S2CCols<false>::CC) * 2 * K);
}

template <bool CPLX, typename TX = double>
__device__ __forceinline__ void s2_col_scales_cached_block(const TX* __restrict__ X, int64_t ldx, int64_t K,
                                                           int64_t cols, int T, int32_t* __restrict__ tau,
                                                           int64_t blk, int16_t* ecache) {
  constexpr int W = CPLX ? 2 : 1, CC = S2CCols<CPLX>::CC, G = S2CCols<CPLX>::G;
  __shared__ int red_e[G][CC];
  __shared__ int64_t red_s[G][CC];
  const int cl = threadIdx.x & (CC - 1), g = threadIdx.x / CC;
  const int64_t j = blk * CC + cl;
  const bool in = j < cols;
  const TX* xc = X + (in ? j : 0) * W;
  int e = OZK_EXP_ZERO;
#pragma unroll 8
  for (int64_t k = g; k < K; k += G) {
    const int ek = entry_expo<CPLX>(xc + k * ldx * W);
    // finite exponents lie in [-1074, 1025]; a non-finite entry makes the
    // column's scale non-finite, so its cached value is never read
    ecache[k * CC + cl] = (int16_t)(ek == OZK_EXP_ZERO ? -32768 : ek > 32767 ? 32767 : ek);
    e = ek > e ? ek : e;
  }
  red_e[g][cl] = in ? e : OZK_EXP_ZERO;
  __syncthreads();
  int emax = red_e[0][cl];
#pragma unroll
  for (int i = 1; i < G; ++i) emax = red_e[i][cl] > emax ? red_e[i][cl] : emax;
  int64_t S = 0;
  if (in && emax != OZK_EXP_ZERO && emax != OZK_EXP_NONFINITE)
#pragma unroll 8
    for (int64_t k = g; k < K; k += G) {
      const int c = ecache[k * CC + cl];
      S += norm_term(c == -32768 ? OZK_EXP_ZERO : c, emax);
    }
  red_s[g][cl] = S;
  __syncthreads();
  if (g == 0 && in) {
    int64_t tot = 0;
#pragma unroll
    for (int i = 0; i < G; ++i) tot += red_s[i][cl];
    tau[j] = scale_from(emax, tot, T);
  }
}

template <bool CPLX, typename TX = double>
__global__ __launch_bounds__(256) void k_s2_col_scales_cached(const TX* __restrict__ X, int64_t ldx, int64_t K,
                                                              int64_t cols, int T, int32_t* __restrict__ tau) {
  extern __shared__ int16_t ecache[];
  s2_col_scales_cached_block<CPLX, TX>(X, ldx, K, cols, T, tau, blockIdx.x, ecache);
}

// The batched column-scale pass caches the exponents of problems up to this K
// (16 KB of LDS per block: eight blocks still share a CU).
template <bool CPLX>
constexpr int64_t s2_batch_ccache_k() {
  return 8192 / S2CCols<CPLX>::CC;
}

int64_t s2_batch_col_blocks(bool cplx, int64_t K, int64_t cols) {
  const int64_t kc = cplx ? s2_batch_ccache_k<true>() : s2_batch_ccache_k<false>();
  const int cc = cplx ? S2CCols<true>::CC : S2CCols<false>::CC;
  return K <= kc ? (cols + cc - 1) / cc : (cols + 31) / 32;
}

// Column scales for long K, split over K so that every CU has work: pass 1
// the exponent maximum per column (integer atomic max), pass 2 the
// norm-bound sum relative to it (integer atomic add), then the scale.  Both
// reductions are exact integer operations, so the result equals that of
// k_s2_col_scales whatever the order.  A block covers 64 columns x
// S2_COLS_KB rows (4 row groups of 64 lanes, each lane one column).
constexpr int S2_COLS_KB = 128;

__global__ __launch_bounds__(256) void k_s2_col_stats_init(int64_t cols, int32_t* __restrict__ emax,
                                                           unsigned long long* __restrict__ S) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  emax[j] = OZK_EXP_ZERO;
  S[j] = 0ull;
}

template <bool CPLX, typename T = double>
__global__ __launch_bounds__(256) void k_s2_col_emax(const T* __restrict__ X, int64_t ldx, int64_t K,
                                                     int64_t cols, int32_t* __restrict__ emax) {
  constexpr int W = CPLX ? 2 : 1;
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (j >= cols) return;
  const int64_t k0 = (int64_t)blockIdx.y * S2_COLS_KB, k1 = k0 + S2_COLS_KB < K ? k0 + S2_COLS_KB : K;
  int e = OZK_EXP_ZERO;
#pragma unroll 8
  for (int64_t k = k0 + (threadIdx.x >> 6); k < k1; k += 4) {
    const int ek = entry_expo<CPLX>(X + (k * ldx + j) * W);
    e = ek > e ? ek : e;
  }
  if (e != OZK_EXP_ZERO) atomicMax(&emax[j], e);
}

template <bool CPLX, typename T = double>
__global__ __launch_bounds__(256) void k_s2_col_norm(const T* __restrict__ X, int64_t ldx, int64_t K,
                                                     int64_t cols, const int32_t* __restrict__ emax,
                                                     unsigned long long* __restrict__ S) {
  constexpr int W = CPLX ? 2 : 1;
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (j >= cols) return;
  const int em = emax[j];
  if (em == OZK_EXP_NONFINITE || em == OZK_EXP_ZERO) return;
  const int64_t k0 = (int64_t)blockIdx.y * S2_COLS_KB, k1 = k0 + S2_COLS_KB < K ? k0 + S2_COLS_KB : K;
  int64_t acc = 0;
#pragma unroll 8
  for (int64_t k = k0 + (threadIdx.x >> 6); k < k1; k += 4) acc += norm_term(entry_expo<CPLX>(X + (k * ldx + j) * W), em);
  if (acc) atomicAdd(&S[j], (unsigned long long)acc);
}

__global__ __launch_bounds__(256) void k_s2_col_finish(int64_t cols, int T, const int32_t* __restrict__ emax,
                                                       const unsigned long long* __restrict__ S,
                                                       int32_t* __restrict__ tau) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  tau[j] = scale_from(emax[j], (int64_t)S[j], T);
}

// A block covers 64 columns of one K chunk.  Thread (column j, quarter q)
// takes the 8 k of quarter q of the chunk in column j and writes one 8-byte
// piece per plane: the four quarters of 16 consecutive columns are 512
// contiguous bytes of a plane (16 packed rows of 32 bytes), and every load
// reads 16 consecutive columns in 4 rows of B.  Padding columns get zero
// residues when zero_pad is set, else they are left as they are.
constexpr int S2_COL_BLOCK = 64;
constexpr int S2_COL_K = OZK_K_CHUNK / 4;

int64_t s2_split_rows_blocks(int64_t rows_packed) { return rows_packed / S2_ROWS_PER_BLOCK; }

int64_t s2_split_cols_blocks(int64_t cols_packed, int64_t Kp) {
  return (cols_packed / S2_COL_BLOCK) * (Kp / OZK_K_CHUNK);
}

template <bool CPLX, typename T = double>
__device__ __forceinline__ void s2_split_cols_block(const T* __restrict__ X, int64_t ldx, int64_t K,
                                                    int64_t cols, int64_t Kp, int64_t cols_packed, int s,
                                                    const int32_t* __restrict__ tau, int8_t* __restrict__ packed,
                                                    int64_t jb, int64_t c, bool zero_pad = true) {
  constexpr int W = CPLX ? 2 : 1, NP = CPLX ? 3 : 1;
  const int lane = threadIdx.x & 63, qk = lane & 3;
  const int64_t j = jb * S2_COL_BLOCK + (threadIdx.x >> 6) * 16 + (lane >> 2);
  const int64_t k0 = c * OZK_K_CHUNK + qk * S2_COL_K;
  if (j >= cols && !zero_pad) return;  // no cross-lane work below
  const int t = j < cols ? tau[j] : 0;
  const bool live = j < cols && t != OZK_EXP_NONFINITE;
  double re[S2_COL_K], im[S2_COL_K];
  if (live && k0 + S2_COL_K <= K) {  // all loads first, no condition between them
#pragma unroll
    for (int kk = 0; kk < S2_COL_K; ++kk) {
      const T* src = X + ((k0 + kk) * ldx + j) * W;
      re[kk] = src[0];
      im[kk] = CPLX ? src[1] : 0.0;
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < S2_COL_K; ++kk) {
      const bool in = live && k0 + kk < K;
      re[kk] = in ? X[((k0 + kk) * ldx + j) * W] : 0.0;
      im[kk] = CPLX && in ? X[((k0 + kk) * ldx + j) * W + 1] : 0.0;
    }
  }
  Limbs3 vr[S2_COL_K], vi[CPLX ? S2_COL_K : 1];
#pragma unroll
  for (int kk = 0; kk < S2_COL_K; ++kk) {
    vr[kk] = scaled_limbs(re[kk], t);
    if (CPLX) vi[CPLX ? kk : 0] = scaled_limbs(im[kk], t);
  }
  const int64_t plane = cols_packed * Kp * NP, slab = cols_packed * OZK_K_CHUNK;
  int8_t* dst = packed + c * NP * slab + j * OZK_K_CHUNK + qk * S2_COL_K;
  for (int l = 0; l < s; ++l, dst += plane) {
    uint32_t w0[2] = {0, 0}, w1[2] = {0, 0}, w2[2] = {0, 0};
#pragma unroll
    for (int kk = 0; kk < S2_COL_K; ++kk) {
      const int a = residue_of(vr[kk], l);
      w0[kk / 4] |= (uint32_t)(uint8_t)a << (8 * (kk % 4));
      if (CPLX) {
        const int b = residue_of(vi[CPLX ? kk : 0], l);
        w1[kk / 4] |= (uint32_t)(uint8_t)b << (8 * (kk % 4));
        w2[kk / 4] |= (uint32_t)(uint8_t)smod_sum(a, b, l) << (8 * (kk % 4));
      }
    }
    *reinterpret_cast<uint2*>(dst) = make_uint2(w0[0], w0[1]);
    if (CPLX) {
      *reinterpret_cast<uint2*>(dst + slab) = make_uint2(w1[0], w1[1]);
      *reinterpret_cast<uint2*>(dst + 2 * slab) = make_uint2(w2[0], w2[1]);
    }
  }
}

template <bool CPLX, typename T = double>
__global__ __launch_bounds__(256) void k_s2_split_cols(const T* __restrict__ X, int64_t ldx, int64_t K,
                                                       int64_t cols, int64_t Kp, int64_t cols_packed, int s,
                                                       const int32_t* __restrict__ tau,
                                                       int8_t* __restrict__ packed) {
  s2_split_cols_block<CPLX, T>(X, ldx, K, cols, Kp, cols_packed, s, tau, packed, blockIdx.x, blockIdx.y);
}

// ----------------------------------------------------------- modular GEMM

// Steps per INT32-safe run: |acc| <= 32 * steps * 128^2 must stay below 2^31,
// so the accumulators are reduced mod m every 4095 steps (K = 131040); the
// reduction is exact because only the residue is kept.
constexpr int64_t S2_RUN_STEPS = 4095;
// K chunks up to which a tile's sums stay within 2^28 (|T| <= 32 * 128^2 per
// chunk), so that the epilogue can use the short reduction.
constexpr int64_t S2_SMALL_STEPS = 512;

// Tiling of the per-modulus GEMM.  Base tile: real 128 x 128, 3M 128 x 64;
// large tile: real 256 x 128 (4 x 2 MFMA tiles per wave; variant 3: 256 x 256,
// 4 x 4, all 256 matrix registers), 3M 128 x 128.  An LDS stage holds G
// consecutive K chunks (a stage of G P planes; one barrier per G chunks):
//   V0 base,  G = 2, 4 stages     V1 base,  G = 1, 4 stages
//   V2 large, G = 1, 4 stages     V3 large, G = 2, 3 stages
// The real base tile and the real V2 (192 registers, 48 KB of LDS) run two
// workgroups per CU, so that one's tile epilogue and pipeline ramp overlap the
// other's MFMAs (V2 pays off at short K); the others run one.  The large tile reuses each operand
// fragment read from LDS over more MFMAs; it holds one INT32-safe run only
// (no mid-run reduction, which would push its accumulators out of the matrix
// registers), so the launcher takes the base tile (variant - 2) when K is
// longer.
// Variant 4 (the batch GEMM only): the small tile, 64 x 64 with one MFMA
// tile per wave, one chunk per stage, two stages; it needs few registers and
// little LDS, so four workgroups share a CU and hide each other's per-item
// latency.
// Variants 5 and 6: the large tiles with other stagings (real: 256 x 128
// with G = 4 over 2 stages, 256 x 256 with G = 3 over 2 stages -- one barrier
// per more MFMAs; 3M: 128 x 128 with G = 2 over 3 stages, G = 1 over 6
// stages -- more chunks in flight), within the registers that two sets of
// step fragments and the accumulators leave.
template <bool CPLX, int V = 0>
struct S2Cfg {
  static constexpr int P = CPLX ? 3 : 1;
  static constexpr bool LARGE = V == 2 || V == 3 || V == 5 || V == 6;
  static constexpr bool SMALL = V == 4;
  static constexpr int TM = SMALL ? 1 : LARGE && !CPLX ? 4 : 2;
  static constexpr int TN = SMALL ? 1 : ((V == 3 || V == 6) && !CPLX) ? 4 : CPLX && !LARGE ? 1 : 2;
  static constexpr int NS = V == 3 ? 3 : V == 4 ? 2 : V == 5 ? (CPLX ? 3 : 2) : V == 6 ? (CPLX ? 6 : 2) : 4;
  static constexpr int G = V == 0 ? 2 : V == 1 || V == 4 ? 1 : V == 2 ? 1 : V == 5 ? (CPLX ? 2 : 4)
                                       : V == 6 ? (CPLX ? 1 : 3) : 2;
  static constexpr int LDS_BYTES = GemmTile<G * P, TM, TN, NS>::LDS_BYTES;
  static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
  static constexpr int MINB = V == 2 && !CPLX ? 2 : 1;  // workgroups per CU the registers must allow
};

// One output tile of one modulus: the per-modulus products, then smod (3M:
// the combination first) and the int8 output residues.
// Keep the accumulators small by subtracting a multiple of m_l (exact mod m_l).
template <int P, int TM, int TN>
__device__ __forceinline__ void s2_reduce_acc(v16i (&acc)[P][TM][TN], int l) {
  const int m = c_s2.m[l];
  const float inv = 1.0f / (float)m;
#pragma unroll
  for (int d = 0; d < P; ++d)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int x = acc[d][a][b][v];
          acc[d][a][b][v] = x - m * (int)rintf((float)x * inv);
        }
}

// Bytes of two words by a selector (v_perm_b32): selector byte i picks byte
// i of the result, 0-3 from lo, 4-7 from hi, 12 a zero byte.
__device__ __forceinline__ uint32_t perm_bytes(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Byte 0 of four values as one word (byte k from r[k]).
__device__ __forceinline__ uint32_t pack_bytes(const uint32_t (&r)[4]) {
  const uint32_t lo = perm_bytes(r[1], r[0], 0x0C0C0400u), hi = perm_bytes(r[3], r[2], 0x0C0C0400u);
  return lo | (hi << 16);
}

// A lane's four residues of rows r0..r0+3 of its column, one byte each
// (byte k: row r0 + k), transposed across its quad of lanes (columns c0..c0+3):
// afterwards lane q holds row r0 + q, byte j being column c0 + j.  Two
// exchanges with the quad neighbours (DPP quad permutations lane ^ 1, lane ^ 2),
// each followed by one byte selection whose selector depends on the lane:
// sel1 / sel2 from quad_selectors.
__device__ __forceinline__ void quad_selectors(int q, uint32_t& sel1, uint32_t& sel2) {
  // exchange with lane ^ 1: even lanes keep bytes 0, 2 and take the
  // neighbour's 0, 2 into 1, 3; odd lanes keep 1, 3 and take its 1, 3 into 0, 2
  sel1 = (q & 1) ? 0x03070105u : 0x06020400u;
  // exchange with lane ^ 2: lanes 0, 1 keep bytes 0, 1 and take the
  // neighbour's 0, 1 into 2, 3; lanes 2, 3 keep 2, 3 and take its 2, 3 into 0, 1
  sel2 = (q & 2) ? 0x03020706u : 0x05040100u;
}

__device__ __forceinline__ uint32_t quad_transpose4(uint32_t w, uint32_t sel1, uint32_t sel2) {
  // every lane of a quad permutation has a source lane
  uint32_t p = (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0xB1, 0xF, 0xF, true);
  w = perm_bytes(p, w, sel1);
  p = (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0x4E, 0xF, 0xF, true);
  return perm_bytes(p, w, sel2);
}

// The residues mod m_l of a finished tile (Eq. 7); for 3M the real and
// imaginary parts from the three products (Eq. 16), into planes of M rows
// of ldr >= N bytes.  `small`: the tile summed at most 512 K chunks in this
// run (|T| <= 512 * 32 * 128^2 = 2^28, so the 3M combinations stay below
// 2^30 in INT32), and the short reduction applies.  When ldr is a multiple of
// 4 (and `out` 4-byte aligned) each group of four rows of a lane is
// transposed across its quad so that every lane writes 4 bytes of one row:
// a quarter of the store instructions.
// The output positions are derived from a lane index the compiler cannot see
// through: inside a K loop (the batched tiles store every modulus there) it
// would otherwise keep all of them live across the loop.
template <bool CPLX, int P, int TM, int TN, bool SMALL>
__device__ __forceinline__ void s2_store_tile_as(const v16i (&acc)[P][TM][TN], int64_t m0, int64_t n0, int64_t M,
                                                 int64_t N, int8_t* __restrict__ out, int l, int64_t ldr) {
  const int64_t mn = (int64_t)M * ldr;  // a plane: M rows of ldr >= N bytes
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // residue byte(s) of value v of MFMA tile (a, b) (byte 0; the upper bytes
  // are not defined): real -> r[0]; 3M -> re, im
  auto residues = [&](int a, int b, int v, uint32_t (&r)[2]) {
    if constexpr (SMALL) {  // |T| <= 2^28: the differences in INT32, the short reduction
      if (!CPLX) {
        r[0] = smod_small_byte(acc[0][a][b][v], l);
        r[1] = 0;
      } else {
        const int t1 = acc[0][a][b][v], t2 = acc[CPLX ? 1 : 0][a][b][v], t3 = acc[CPLX ? 2 : 0][a][b][v];
        r[0] = smod_small_byte(t1 - t2, l);
        r[1] = smod_small_byte(t3 - t1 - t2, l);
      }
    } else if (!CPLX) {
      r[0] = (uint32_t)smod_i32(acc[0][a][b][v], l);
      r[1] = 0;
    } else {
      // T1 - T2 and T3 - T1 - T2 are exact in binary64 (|T| < 2^31): two
      // reductions instead of three and the residue sums
      const double t1 = (double)acc[0][a][b][v], t2 = (double)acc[CPLX ? 1 : 0][a][b][v],
                   t3 = (double)acc[CPLX ? 2 : 0][a][b][v];
      r[0] = (uint32_t)smod_exact(t1 - t2, l);
      r[1] = (uint32_t)smod_exact(t3 - t1 - t2, l);
    }
  };
  constexpr int NPL = CPLX ? 2 : 1;  // output planes per modulus
  if ((ldr & 3) == 0 && ((uintptr_t)out & 3) == 0) {
    const int q = lane & 3;
    uint32_t sel1, sel2;
    quad_selectors(q, sel1, sel2);
    // the lane's row and first column for a = b = g = 0; the others are
    // uniform offsets from there
    const int64_t row0 = m0 + wm * 32 * TM + 4 * (lane >> 5) + q;
    const int64_t col0 = n0 + wn * 32 * TN + ((lane & 31) & ~3);
    int8_t* const base = out + (int64_t)(NPL * l) * mn + row0 * ldr + col0;
    // rows and columns left from there (the whole workgroup tile inside the
    // output: no bound), so that each store's test is two 32-bit compares
    const bool full = m0 + 64 * TM <= M && n0 + 64 * TN <= N;
    const int64_t rl = M - row0, cl = N - col0;
    const int rlim = full || rl > 1024 ? 1024 : (int)rl, clim = full || cl > 1024 ? 1024 : (int)cl;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          uint32_t r4[2][4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            uint32_t r[2];
            residues(a, b, 4 * g + k, r);
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) r4[pl][k] = r[pl];
          }
          // columns col0 + 3 < ldr: past N only the plane's padding
          const bool in = a * 32 + 8 * g < rlim && b * 32 < clim;
#pragma unroll
          for (int pl = 0; pl < NPL; ++pl) {
            const uint32_t t = quad_transpose4(pack_bytes(r4[pl]), sel1, sel2);
            if (in)
              *reinterpret_cast<uint32_t*>(base + pl * mn + (int64_t)(a * 32 + 8 * g) * ldr + b * 32) = t;
          }
        }
    return;
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        // the layout of for_each_output
        const int64_t row = m0 + wm * 32 * TM + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        const int64_t col = n0 + wn * 32 * TN + b * 32 + (lane & 31);
        if (row >= M || col >= N) continue;
        uint32_t r[2];
        residues(a, b, v, r);
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) out[(NPL * l + pl) * mn + row * ldr + col] = (int8_t)r[pl];
      }
}

// The epilogue form chosen once per tile (each form keeps its values in
// straight-line code that the compiler interleaves).
template <bool CPLX, int P, int TM, int TN>
__device__ __forceinline__ void s2_store_tile(const v16i (&acc)[P][TM][TN], int64_t m0, int64_t n0, int64_t M,
                                              int64_t N, int8_t* __restrict__ out, int l, int64_t ldr, bool small) {
  if (small)
    s2_store_tile_as<CPLX, P, TM, TN, true>(acc, m0, n0, M, N, out, l, ldr);
  else
    s2_store_tile_as<CPLX, P, TM, TN, false>(acc, m0, n0, M, N, out, l, ldr);
}

template <bool CPLX, int V>
__device__ __forceinline__ void s2_gemm_tile(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                             int64_t plane_a, int64_t plane_b, int64_t rows_a, int64_t rows_b,
                                             int64_t nsteps, int64_t M, int64_t N, int8_t* __restrict__ out,
                                             int64_t tile, int l, int raster, int group, int8_t* lds) {
  using Cfg = S2Cfg<CPLX, V>;
  constexpr int P = Cfg::P, TM = Cfg::TM, TN = Cfg::TN, NS = Cfg::NS;
  using T = GemmTile<P, TM, TN, NS>;
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(tile, tiles_m, tiles_n, raster, group, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  constexpr int G = Cfg::G;
  v16i acc[P][TM][TN];
  zero_acc<P, TM, TN>(acc);
  // nsteps counts K chunks.  Runs of up to S2_RUN_STEPS chunks (a multiple of
  // G; the large tiles have one run, the launcher checks K): G-chunk steps,
  // then the chunks of the last run that do not fill one.
  const int64_t run = Cfg::LARGE ? nsteps : (S2_RUN_STEPS / G) * G;
  for (int64_t c0 = 0; c0 < nsteps || c0 == 0; c0 += run) {
    const int64_t n = nsteps - c0 < run ? nsteps - c0 : run;
    const int64_t full = n / G, rest = n - full * G;
    if (full > 0 || G == 1)
      gemm_tile_accumulate<G * P, TM, TN, NS, DIAGONAL, P>(Ap + l * plane_a, Bp + l * plane_b, rows_a, rows_b, m0,
                                                           n0, c0 / G, full, lds, acc);
    if (G > 1 && rest > 0)
      gemm_tile_accumulate<P, TM, TN, NS, DIAGONAL, P>(Ap + l * plane_a, Bp + l * plane_b, rows_a, rows_b, m0, n0,
                                                       c0 + full * G, rest, lds, acc);
    if (c0 + run >= nsteps) break;
    s2_reduce_acc<P, TM, TN>(acc, l);
  }
  s2_store_tile<CPLX, P, TM, TN>(acc, m0, n0, M, N, out, l, N, nsteps <= S2_SMALL_STEPS);
}

template <bool CPLX, int V>
__global__ __launch_bounds__(256, (S2Cfg<CPLX, V>::MINB)) void k_s2_gemm_mod(const int8_t* __restrict__ Ap,
                                                       const int8_t* __restrict__ Bp, int64_t plane_a,
                                                       int64_t plane_b, int64_t rows_a, int64_t rows_b,
                                                       int64_t nsteps, int M, int N, int raster, int group,
                                                       int8_t* __restrict__ out) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  s2_gemm_tile<CPLX, V>(Ap, Bp, plane_a, plane_b, rows_a, rows_b, nsteps, M, N, out, blockIdx.x, (int)blockIdx.z,
                        raster, group, lds);
}

// ------------------------------------------------------------------- CRT

constexpr int NL = 6;  // 32-bit limbs: P < 2^156 for s <= 20, sums < 2^170

struct CrtArgs {
  int s;
  uint32_t W[OZK_MAX_S][NL];  // (P/m_l) q_l
  uint32_t P[NL];
  double Pf;
  double Pinv;  // 1 / Pf rounded
};

// Z = smod(V, P) as a sign and magnitude limbs, for V = sum_l W_l c_l >= 0
// given as NL + 1 32-bit limbs; Z in [-P/2, P/2).
template <int U = NL>
__device__ __forceinline__ void crt_reduce(const CrtArgs& ca, const uint32_t (&v)[NL + 1], uint32_t (&mag)[NL],
                                           bool& neg) {
  static_assert(U >= 1 && U <= NL, "limbs used");
  // quotient estimate: V / P < s 2^8 <= 2^13 (W_l < P, c_l < 2^8) and the
  // estimate's relative error is below 2^-49 (U + 1 roundings of V, two of
  // 1 / P, one of the product), so its floor is floor(V / P) or one off
  double vf = 0.0;
#pragma unroll
  for (int i = U; i >= 0; --i) vf = vf * 4294967296.0 + (double)v[i];
  // Nearly always V / P + 1/2 lies well inside (q, q + 1) for an integer q:
  // the estimate, within 2^-35 of V / P + 1/2 (V / P < 2^13), then fixes
  // q = floor(V / P + 1/2) and Z = V - q P is the symmetric residue at once.
  // Otherwise (V near a half-multiple of P) the exact steps below decide.
  {
    const double h = __fma_rn(vf, ca.Pinv, 0.5);
    const double qh = floor(h), fr = h - qh;  // fr exact
    if (fr > 0x1p-30 && fr < 1.0 - 0x1p-30) {
      const uint32_t q = (uint32_t)qh;
      uint32_t r[NL + 1];
      uint64_t mc = 0;
      int64_t borrow = 0;
#pragma unroll
      for (int i = 0; i <= U; ++i) {
        const uint64_t prod = (uint64_t)(i < U ? ca.P[i] : 0u) * q + mc;
        mc = prod >> 32;
        const int64_t d = (int64_t)v[i] - (int64_t)(uint32_t)prod + borrow;
        r[i] = (uint32_t)d;
        borrow = d >> 32;
      }
      // |Z| <= P/2 < 2^(32U - 1): limb U is the sign extension
      neg = (int32_t)r[U] < 0;
      uint64_t c = neg ? 1u : 0u;
#pragma unroll
      for (int i = 0; i < U; ++i) {
        const uint64_t t = (uint64_t)(neg ? ~r[i] : r[i]) + c;
        mag[i] = (uint32_t)t;
        c = t >> 32;
      }
#pragma unroll
      for (int i = U; i < NL; ++i) mag[i] = 0;
      return;
    }
  }
  const double qd = floor(vf * ca.Pinv);
  const uint32_t q = qd > 0.0 ? (uint32_t)qd : 0u;
  // r = V - q P (U + 1 limbs, two's complement)
  uint32_t r[NL + 1];
  {
    uint64_t mc = 0;
    int64_t borrow = 0;
#pragma unroll
    for (int i = 0; i <= U; ++i) {
      const uint64_t prod = (uint64_t)(i < U ? ca.P[i] : 0u) * q + mc;
      mc = prod >> 32;
      const int64_t d = (int64_t)v[i] - (int64_t)(uint32_t)prod + borrow;
      r[i] = (uint32_t)d;
      borrow = d >> 32;  // 0 or -1
    }
  }
  // one step into [0, P): + P after an estimate one too high (rare), - P
  // after one too low
  if ((int32_t)r[U] < 0) {
    int64_t cy = 0;
#pragma unroll
    for (int i = 0; i <= U; ++i) {
      const int64_t d = (int64_t)r[i] + (int64_t)(i < U ? ca.P[i] : 0u) + cy;
      r[i] = (uint32_t)d;
      cy = d >> 32;
    }
  }
  {
    uint32_t d[NL + 1];
    int64_t b = 0;
#pragma unroll
    for (int i = 0; i <= U; ++i) {
      const int64_t t = (int64_t)r[i] - (int64_t)(i < U ? ca.P[i] : 0u) + b;
      d[i] = (uint32_t)t;
      b = t >> 32;
    }
    const bool ge = b == 0;  // r >= P
#pragma unroll
    for (int i = 0; i <= U; ++i) r[i] = ge ? d[i] : r[i];
  }
  // symmetric lift: Z = r - P when 2r >= P, i.e. r >= P - r
  uint32_t m2[NL];
  int64_t b = 0, b2 = 0;
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int64_t t = (int64_t)ca.P[i] - (int64_t)r[i] + b;
    m2[i] = (uint32_t)t;
    b = t >> 32;
  }
#pragma unroll
  for (int i = 0; i < U; ++i) b2 = ((int64_t)r[i] - (int64_t)m2[i] + b2) >> 32;
  neg = b2 == 0;
#pragma unroll
  for (int i = 0; i < U; ++i) mag[i] = neg ? m2[i] : r[i];
#pragma unroll
  for (int i = U; i < NL; ++i) mag[i] = 0;
}

// 32-bit limbs the CRT sums of the first s moduli need: sum_l W_l c_l <
// s 2^8 P < 2^(bits(P) + 13) for s <= 20 (the same count as the host's).
constexpr int crt_limbs_of(int s) {
  uint32_t p[NL + 1] = {1};
  for (int l = 0; l < s; ++l) {
    uint64_t c = 0;
    for (int i = 0; i <= NL; ++i) {
      const uint64_t t = (uint64_t)p[i] * (uint32_t)kS2.m[l] + c;
      p[i] = (uint32_t)t;
      c = t >> 32;
    }
  }
  int bits = 0;
  for (int i = NL; i >= 0 && bits == 0; --i)
    if (p[i]) {
      int b = 32;
      while (!((p[i] >> (b - 1)) & 1u)) --b;
      bits = 32 * i + b;
    }
  return (bits + 13 + 31) / 32;
}

// Z = smod(sum_l W_l c_l, P) from the S residue planes at res (stride apart),
// S known at compile time: straight-line code (a loop over a runtime count
// kept the residues in indexed registers and branched per modulus).
template <int S>
__device__ __forceinline__ void crt_combine_s(const CrtArgs& ca, const int8_t* res, int64_t stride,
                                              uint32_t (&mag)[NL], bool& neg) {
  constexpr int U = crt_limbs_of(S);
  static_assert(U >= 1 && U <= NL, "limbs");
  // all residues first (independent loads in flight together)
  int cv[S];
#pragma unroll
  for (int l = 0; l < S; ++l) cv[l] = (int)res[l * stride];
  // V = sum_l W_l u_l with the residues u_l in [0, m_l): 32 x 32-bit products
  // summed in 64 bits per limb of W (V < S 2^8 P fits U limbs)
  uint64_t acc[U] = {};
#pragma unroll
  for (int l = 0; l < S; ++l) {
    const int c = cv[l];
    const uint32_t u = (uint32_t)(c + (c < 0 ? kS2.m[l] : 0));
#pragma unroll
    for (int i = 0; i < U; ++i) acc[i] += (uint64_t)ca.W[l][i] * u;
  }
  uint32_t v[NL + 1] = {};
  uint64_t carry = 0;
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const uint64_t t = acc[i] + carry;
    v[i] = (uint32_t)t;
    carry = t >> 32;
  }
  v[U] = (uint32_t)carry;
  crt_reduce<U>(ca, v, mag, neg);
}

// Z = smod(sum_l W_l c_l, P) for the runtime s = ca.s, dispatched (a uniform
// branch) to the straight-line body of that s: among the s whose sums need
// U limbs, or every s when U = CRT_ANY_S.
constexpr int CRT_ANY_S = 0;

template <int U, int S = 1>
__device__ __forceinline__ void crt_combine(const CrtArgs& ca, const int8_t* res, int64_t stride, uint32_t (&mag)[NL],
                                            bool& neg) {
  if constexpr (S <= OZK_MAX_S) {
    if constexpr (U == CRT_ANY_S || crt_limbs_of(S) == U) {
      if (ca.s == S) {
        crt_combine_s<S>(ca, res, stride, mag, neg);
        return;
      }
    }
    crt_combine<U, S + 1>(ca, res, stride, mag, neg);
  } else {  // no such s (never launched so)
#pragma unroll
    for (int i = 0; i < NL; ++i) mag[i] = 0;
    neg = false;
  }
}

// The CRT sum of one output kept in registers while the moduli stream by
// (the fused variant): W_l in NZ 16-bit pieces (W_l < P <= 256^s, so NZ >=
// s / 2 pieces hold it) times the residue taken in [0, m_l) stays below 2^24,
// so the sums of s <= 20 such products fit 32 bits.

template <int NZ>
__device__ __forceinline__ void crt_add16(uint32_t (&z)[NZ], const CrtArgs& ca, int l, int c) {
  static_assert(NZ <= 2 * NL, "pieces of the NL limbs");
  const uint32_t u = (uint32_t)(c < 0 ? c + c_s2.m[l] : c);
#pragma unroll
  for (int i = 0; i < NZ; ++i) z[i] += __umul24((ca.W[l][i / 2] >> (16 * (i % 2))) & 0xFFFFu, u);
}

// The 16-bit-piece sums as NL + 1 32-bit limbs (exact carries).
template <int NZ>
__device__ __forceinline__ void crt_limbs16(const uint32_t (&z)[NZ], uint32_t (&v)[NL + 1]) {
  uint64_t carry = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const uint64_t lo = 2 * j < NZ ? z[2 * j] : 0, hi = 2 * j + 1 < NZ ? z[2 * j + 1] : 0;
    const uint64_t t = carry + lo + (hi << 16);
    v[j] = (uint32_t)t;
    carry = t >> 32;
  }
  v[NL] = (uint32_t)carry;
}

// RN-even of +-mag 2^E (one rounding, gradual underflow included).  A
// magnitude of 2^128 or more is cut to the 128 bits from its leading one down,
// with the bits below folded into the lowest of them (sticky): the rounding
// keeps at most 53 of the 128, so its round bit is bit 74 or higher, the
// sticky bit lies strictly below it and the result is the same.
// TO = float: the rounding to binary32 (round_mag_f32).
template <typename TO = double>
__device__ __forceinline__ TO round_limbs(const uint32_t (&mag)[NL], bool neg, int E) {
  static_assert(NL == 6, "three 64-bit words");
  auto rnd = [](u128 m, bool n, int e) -> TO {
    if constexpr (sizeof(TO) == 4) return round_mag_f32(m, n, e);
    else return round_mag(m, n, e);
  };
  const uint64_t w2 = ((uint64_t)mag[5] << 32) | mag[4], w1 = ((uint64_t)mag[3] << 32) | mag[2],
                 w0 = ((uint64_t)mag[1] << 32) | mag[0];
  if (w2 == 0) return rnd(((u128)w1 << 64) | w0, neg, E);
  const int lz = __clzll(w2);
  const int cut = 64 - lz;  // bits dropped
  u128 top = ((u128)w2 << 64) | w1;
  uint64_t rest = w0;
  if (lz) {
    top = (top << lz) | (w0 >> cut);
    rest = w0 << lz;
  }
  return rnd(top | (rest != 0), neg, E + cut);
}

// C = alpha h + beta C for one output (complex: the fixed FMA sequence), in
// the output's precision (TO = float: alpha, beta and h hold binary32 values).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __fmaf_rn(a, b, c); }

template <bool CPLX, typename TO = double>
__device__ __forceinline__ void s2_store_c(const TO (&h)[2], int64_t row, int64_t col, TO a_re, TO a_im, TO b_re,
                                           TO b_im, TO* __restrict__ C, int64_t ldc) {
  if (!CPLX) {
    TO* cp = C + row * ldc + col;
    if constexpr (sizeof(TO) == 4) *cp = axpby_f32(a_re, h[0], b_re, cp);
    else *cp = axpby(a_re, h[0], b_re, cp);
  } else {
    TO* cp = C + 2 * (row * ldc + col);
    TO bre = 0, bim = 0;
    if (!(b_re == 0 && b_im == 0)) {
      const TO cre = cp[0], cim = cp[1];
      bre = fma_t(b_re, cre, -(b_im * cim));
      bim = fma_t(b_re, cim, b_im * cre);
    }
    const TO ore = fma_t(a_re, h[0], fma_t(-a_im, h[1], bre));
    const TO oim = fma_t(a_re, h[1], fma_t(a_im, h[0], bim));
    cp[0] = ore;
    cp[1] = oim;
  }
}

// Residue planes of M rows of ldr >= N bytes (ldr < 0: N).
template <bool CPLX, typename TO = double, int U = NL>
__device__ __forceinline__ void s2_crt_block(const CrtArgs& ca, int64_t M, int64_t N, const int8_t* __restrict__ res,
                                             const int32_t* __restrict__ sigma, const int32_t* __restrict__ tau,
                                             TO a_re, TO a_im, TO b_re, TO b_im, TO* __restrict__ C, int64_t ldc,
                                             int64_t blk, int64_t ldr = -1) {
  // output blk * 256 + thread: the block's first row and column by one
  // uniform division, the thread's by a binary32 quotient estimate of the
  // few rows it lies past them (t / N < 256 / N + 2, estimate off by at most
  // one) and one correction
  if (N <= 0) return;
  const int64_t idx0 = blk * 256, row0 = idx0 / N, col0 = idx0 - row0 * N;
  const uint32_t t = (uint32_t)(col0 + (int64_t)threadIdx.x);  // < N + 256
  int64_t dq = (int64_t)(uint32_t)((float)t * __builtin_amdgcn_rcpf((float)N));
  int64_t col = (int64_t)t - dq * N;
  if (col < 0) {
    --dq;
    col += N;
  } else if (col >= N) {
    ++dq;
    col -= N;
  }
  const int64_t row = row0 + dq;
  if (row >= M) return;
  if (ldr < 0) ldr = N;
  const int64_t mn = (int64_t)M * ldr, at = row * ldr + col;
  const int si = sigma[row], tj = tau[col];
  const bool bad = si == OZK_EXP_NONFINITE || tj == OZK_EXP_NONFINITE;
  const int E = -si - tj;
  TO h[2];
#pragma unroll
  for (int q = 0; q < (CPLX ? 2 : 1); ++q) {
    if (bad) {
      h[q] = (TO)__builtin_nan("");
      continue;
    }
    uint32_t mag[NL];
    bool neg;
    crt_combine<U>(ca, res + (CPLX ? q * mn : 0) + at, CPLX ? 2 * mn : mn, mag, neg);
    h[q] = round_limbs<TO>(mag, neg, E);
  }
  s2_store_c<CPLX, TO>(h, row, col, a_re, a_im, b_re, b_im, C, ldc);
}

// U: the 32-bit limbs the sums of this call's s need (crt_limbs_of), or CRT_ANY_S.
template <bool CPLX, typename TO = double, int U = NL>
__global__ __launch_bounds__(256) void k_s2_crt(CrtArgs ca, int M, int N, const int8_t* __restrict__ res,
                                                const int32_t* __restrict__ sigma, const int32_t* __restrict__ tau,
                                                TO a_re, TO a_im, TO b_re, TO b_im, TO* __restrict__ C, int64_t ldc) {
  s2_crt_block<CPLX, TO, U>(ca, M, N, res, sigma, tau, a_re, a_im, b_re, b_im, C, ldc, blockIdx.x);
}

// ------------------------------------------------------------ host side

// Little host bignum in 32-bit limbs for the CRT constants.
static void big_mul_small(uint32_t* x, int n, uint32_t f) {
  uint64_t c = 0;
  for (int i = 0; i < n; ++i) {
    const uint64_t t = (uint64_t)x[i] * f + c;
    x[i] = (uint32_t)t;
    c = t >> 32;
  }
}
static uint32_t big_div_small(uint32_t* x, int n, uint32_t d) {
  uint64_t r = 0;
  for (int i = n - 1; i >= 0; --i) {
    const uint64_t cur = (r << 32) | x[i];
    x[i] = (uint32_t)(cur / d);
    r = cur % d;
  }
  return (uint32_t)r;
}
static int inv_mod(int a, int m) {
  int t = 0, nt = 1, r = m, nr = a % m;
  while (nr) {
    const int q = r / nr, tt = t - q * nt, rr = r - q * nr;
    t = nt;
    nt = tt;
    r = nr;
    nr = rr;
  }
  return t < 0 ? t + m : t;
}

static void crt_args(int s, CrtArgs& ca, int& ta, int& tb) {
  ca.s = s;
  uint32_t P[NL] = {1, 0, 0, 0, 0, 0};
  for (int l = 0; l < s; ++l) big_mul_small(P, NL, (uint32_t)kS2.m[l]);
  for (int i = 0; i < NL; ++i) ca.P[i] = P[i];
  double pf = 0.0;
  for (int i = NL - 1; i >= 0; --i) pf = pf * 4294967296.0 + (double)P[i];
  ca.Pf = pf;
  ca.Pinv = 1.0 / pf;
  for (int l = 0; l < OZK_MAX_S; ++l)
    for (int i = 0; i < NL; ++i) ca.W[l][i] = 0;
  for (int l = 0; l < s; ++l) {
    uint32_t Q[NL];
    for (int i = 0; i < NL; ++i) Q[i] = P[i];
    big_div_small(Q, NL, (uint32_t)kS2.m[l]);  // P / m_l
    uint32_t R[NL];
    for (int i = 0; i < NL; ++i) R[i] = Q[i];
    const int rem = (int)big_div_small(R, NL, (uint32_t)kS2.m[l]);  // (P/m_l) mod m_l
    const int q = kS2.m[l] == 1 ? 0 : inv_mod(rem, kS2.m[l]);
    big_mul_small(Q, NL, (uint32_t)q);
    for (int i = 0; i < NL; ++i) ca.W[l][i] = Q[i];
  }

  // ceil(log2 P) = bit length of P - 1
  uint32_t Pm1[NL];
  for (int i = 0; i < NL; ++i) Pm1[i] = P[i];
  for (int i = 0; i < NL; ++i) {
    if (Pm1[i]--) break;
  }
  int bl = 0;
  for (int i = NL - 1; i >= 0; --i)
    if (Pm1[i]) {
      bl = 32 * i + (32 - __builtin_clz(Pm1[i]));
      break;
    }
  const int L = bl - 2;
  ta = L / 2;
  tb = L - ta;
}

void s2_targets(int s, int& ta, int& tb) {
  CrtArgs ca;
  crt_args(s, ca, ta, tb);
}

template <typename T>
static hipError_t split_rows_t(int s, bool cplx, const T* X, int64_t ldx, int64_t rows, int64_t K, int32_t* sigma,
                         int8_t* packed, hipStream_t st, int budget) {
  int ta, tb;
  s2_targets(s, ta, tb);
  if (budget >= 0) ta = budget;
  const int64_t rp = round_up(rows, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (rp == 0) return hipSuccess;
  S2Args sa{s, ta};
  const int64_t blocks = rp / S2_ROWS_PER_BLOCK;
  if (blocks < 1024 && kp >= 2 * S2_ROW_KR) {
    // few long rows: the scales first (a launch that writes no residues),
    // then the residues over (row block, K range)
    const dim3 g2((unsigned)blocks, (unsigned)((kp + S2_ROW_KR - 1) / S2_ROW_KR));
    // the exponents cached in LDS when every block of the launch still fits
    // the GPU at once with them (the cache then costs no occupancy)
    int64_t kc = round_up(K, 16);
    const int bytes = s2_ecache_bytes(kc);
    if (K > S2_ECACHE_MAX_K || blocks > 256 * (int64_t)(160 * 1024 / bytes)) kc = 0;
    const int dyn = s2_ecache_bytes(kc);
    static std::atomic<uint64_t> lds_c{0}, lds_r{0};
    const hipError_t e_lds =
        kc ? lds_limit(cplx ? reinterpret_cast<const void*>(k_s2_split_rows<true, T>)
                            : reinterpret_cast<const void*>(k_s2_split_rows<false, T>),
                       s2_ecache_bytes(S2_ECACHE_MAX_K), cplx ? lds_c : lds_r)
           : hipSuccess;
    if (e_lds != hipSuccess) return e_lds;
    if (cplx) {
      hipLaunchKernelGGL((k_s2_split_rows<true, T>), dim3((unsigned)blocks), dim3(256), dyn, st, X, ldx, rows, K, 0,
                         rp, sa, sigma, packed, kc);
      hipLaunchKernelGGL((k_s2_row_residues<true, T>), g2, dim3(256), 0, st, X, ldx, rows, K, kp, rp, sa, sigma,
                         packed);
    } else {
      hipLaunchKernelGGL((k_s2_split_rows<false, T>), dim3((unsigned)blocks), dim3(256), dyn, st, X, ldx, rows, K, 0,
                         rp, sa, sigma, packed, kc);
      hipLaunchKernelGGL((k_s2_row_residues<false, T>), g2, dim3(256), 0, st, X, ldx, rows, K, kp, rp, sa, sigma,
                         packed);
    }
    return hipGetLastError();
  }
  if (cplx)
    hipLaunchKernelGGL((k_s2_split_rows<true, T>), dim3((unsigned)blocks), dim3(256), 0, st, X, ldx, rows, K, kp, rp,
                       sa, sigma, packed, (int64_t)0);
  else
    hipLaunchKernelGGL((k_s2_split_rows<false, T>), dim3((unsigned)blocks), dim3(256), 0, st, X, ldx, rows, K, kp,
                       rp, sa, sigma, packed, (int64_t)0);
  return hipGetLastError();
}

template <typename T>
static hipError_t split_cols_t(int s, bool cplx, const T* X, int64_t ldx, int64_t K, int64_t cols, int32_t* tau,
                         int8_t* packed, hipStream_t st, int budget) {
  int ta, tb;
  s2_targets(s, ta, tb);
  if (budget >= 0) tb = budget;
  const int64_t cp = round_up(cols, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  const int cc = cplx ? S2CCols<true>::CC : S2CCols<false>::CC;
  const int64_t cblocks = (cols + cc - 1) / cc;
  const int cbytes = s2_ccache_bytes(cplx, K);
  if (cols > 0 && K > 0 && K <= S2_ECACHE_MAX_K && cblocks <= 256 * (int64_t)(160 * 1024 / (cbytes + 3072))) {
    // one read of B: every block's exponent cache resident at once
    static std::atomic<uint64_t> lds_c{0}, lds_r{0};
    const hipError_t e_lds =
        lds_limit(cplx ? reinterpret_cast<const void*>(k_s2_col_scales_cached<true, T>)
                       : reinterpret_cast<const void*>(k_s2_col_scales_cached<false, T>),
                  s2_ccache_bytes(cplx, S2_ECACHE_MAX_K), cplx ? lds_c : lds_r);
    if (e_lds != hipSuccess) return e_lds;
    if (cplx)
      hipLaunchKernelGGL((k_s2_col_scales_cached<true, T>), dim3((unsigned)cblocks), dim3(256), cbytes, st, X, ldx, K,
                         cols, tb, tau);
    else
      hipLaunchKernelGGL((k_s2_col_scales_cached<false, T>), dim3((unsigned)cblocks), dim3(256), cbytes, st, X, ldx,
                         K, cols, tb, tau);
  } else if (cols > 0 && cp > 0 && kp >= 4 * S2_COLS_KB) {
    // long K: split over K; the statistics live at the start of `packed`
    // until the residues overwrite them (s Kp cp >= 12 cols bytes here)
    unsigned long long* S = reinterpret_cast<unsigned long long*>(packed);
    int32_t* emax = reinterpret_cast<int32_t*>(packed + 8 * cols);
    const unsigned g1 = (unsigned)((cols + 255) / 256);
    const dim3 g2((unsigned)((cols + 63) / 64), (unsigned)((K + S2_COLS_KB - 1) / S2_COLS_KB));
    hipLaunchKernelGGL(k_s2_col_stats_init, dim3(g1), dim3(256), 0, st, cols, emax, S);
    if (cplx) {
      hipLaunchKernelGGL((k_s2_col_emax<true, T>), g2, dim3(256), 0, st, X, ldx, K, cols, emax);
      hipLaunchKernelGGL((k_s2_col_norm<true, T>), g2, dim3(256), 0, st, X, ldx, K, cols, emax, S);
    } else {
      hipLaunchKernelGGL((k_s2_col_emax<false, T>), g2, dim3(256), 0, st, X, ldx, K, cols, emax);
      hipLaunchKernelGGL((k_s2_col_norm<false, T>), g2, dim3(256), 0, st, X, ldx, K, cols, emax, S);
    }
    hipLaunchKernelGGL(k_s2_col_finish, dim3(g1), dim3(256), 0, st, cols, tb, emax, S, tau);
  } else if (cols > 0) {
    const unsigned gx = (unsigned)((cols + 31) / 32);
    if (cplx)
      hipLaunchKernelGGL((k_s2_col_scales<true, T>), dim3(gx), dim3(256), 0, st, X, ldx, K, cols, tb, tau);
    else
      hipLaunchKernelGGL((k_s2_col_scales<false, T>), dim3(gx), dim3(256), 0, st, X, ldx, K, cols, tb, tau);
  }
  if (cp > 0 && kp > 0) {
    if (cplx)
      hipLaunchKernelGGL((k_s2_split_cols<true, T>), dim3((unsigned)(cp / S2_COL_BLOCK), (unsigned)(kp / OZK_K_CHUNK)),
                         dim3(256), 0, st, X, ldx, K, cols, kp, cp, s, tau, packed);
    else
      hipLaunchKernelGGL((k_s2_split_cols<false, T>), dim3((unsigned)(cp / S2_COL_BLOCK), (unsigned)(kp / OZK_K_CHUNK)),
                         dim3(256), 0, st, X, ldx, K, cols, kp, cp, s, tau, packed);
  }
  return hipGetLastError();
}

hipError_t s2_split_rows(int s, bool cplx, const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* sigma,
                         int8_t* packed, hipStream_t st, int budget) {
  return split_rows_t(s, cplx, X, ldx, rows, K, sigma, packed, st, budget);
}

hipError_t s2_split_rows(int s, bool cplx, const float* X, int64_t ldx, int64_t rows, int64_t K, int32_t* sigma,
                         int8_t* packed, hipStream_t st, int budget) {
  return split_rows_t(s, cplx, X, ldx, rows, K, sigma, packed, st, budget);
}

hipError_t s2_split_cols(int s, bool cplx, const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* tau,
                         int8_t* packed, hipStream_t st, int budget) {
  return split_cols_t(s, cplx, X, ldx, K, cols, tau, packed, st, budget);
}

hipError_t s2_split_cols(int s, bool cplx, const float* X, int64_t ldx, int64_t K, int64_t cols, int32_t* tau,
                         int8_t* packed, hipStream_t st, int budget) {
  return split_cols_t(s, cplx, X, ldx, K, cols, tau, packed, st, budget);
}

template <bool CPLX, int V>
static hipError_t launch_gemm_mod(int s, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                                  int8_t* out, int raster, int group, hipStream_t st) {
  using Cfg = S2Cfg<CPLX, V>;
  constexpr int P = Cfg::P;
  using T = GemmTile<P, Cfg::TM, Cfg::TN, Cfg::NS>;
  auto kern = k_s2_gemm_mod<CPLX, V>;
  static std::atomic<uint64_t> lds_done{0};
  const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(kern), Cfg::LDS_BYTES, lds_done);
  if (e_lds != hipSuccess) return e_lds;
  const int64_t kp = round_up(K, OZK_K_CHUNK);
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t plane_a = ra * kp * P, plane_b = rb * kp * P;
  const int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)s);
  hipLaunchKernelGGL(kern, grid, dim3(256), Cfg::LDS_BYTES, st, Ap, Bp, plane_a, plane_b, ra, rb, kp / OZK_K_CHUNK,
                     (int)M, (int)N, raster, group, out);
  return hipGetLastError();
}

hipError_t s2_gemm_mod(int s, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                       int8_t* out, hipStream_t st, int variant, int raster, int group) {
  if (M == 0 || N == 0) return hipSuccess;
  static_assert(OZK_S2_VARIANTS == 7 && OZK_S2_FUSED_CRT == 4, "the variant switch below covers six tile variants");
  if (variant == OZK_S2_FUSED_CRT) variant = 0;  // residue planes wanted: the separate-kernel form
  if (variant >= 2 && round_up(K, OZK_K_CHUNK) / OZK_K_CHUNK > S2_RUN_STEPS) variant &= 1;  // large tiles: one run
  switch (variant) {
    case 1:
      return cplx ? launch_gemm_mod<true, 1>(s, M, N, K, Ap, Bp, out, raster, group, st)
                  : launch_gemm_mod<false, 1>(s, M, N, K, Ap, Bp, out, raster, group, st);
    case 2:
      return cplx ? launch_gemm_mod<true, 2>(s, M, N, K, Ap, Bp, out, raster, group, st)
                  : launch_gemm_mod<false, 2>(s, M, N, K, Ap, Bp, out, raster, group, st);
    case 3:
      return cplx ? launch_gemm_mod<true, 3>(s, M, N, K, Ap, Bp, out, raster, group, st)
                  : launch_gemm_mod<false, 3>(s, M, N, K, Ap, Bp, out, raster, group, st);
    case 5:
      return cplx ? launch_gemm_mod<true, 5>(s, M, N, K, Ap, Bp, out, raster, group, st)
                  : launch_gemm_mod<false, 5>(s, M, N, K, Ap, Bp, out, raster, group, st);
    case 6:
      return cplx ? launch_gemm_mod<true, 6>(s, M, N, K, Ap, Bp, out, raster, group, st)
                  : launch_gemm_mod<false, 6>(s, M, N, K, Ap, Bp, out, raster, group, st);
  }
  return cplx ? launch_gemm_mod<true, 0>(s, M, N, K, Ap, Bp, out, raster, group, st)
              : launch_gemm_mod<false, 0>(s, M, N, K, Ap, Bp, out, raster, group, st);
}

// ------------------------------------------ unfused baselines (ablation)
//
// The naive Scheme II of the paper's traffic model (Sec. IV-A, Eq. 14) and
// its 3M form (Sec. IV-B, Eq. 17), kept as an ablation of the fused kernels:
// every modular product (3M: T1, T2, T3 of each modulus) is its own INT8
// GEMM whose INT32 result goes to HBM, and a second pass reads the planes
// back, reduces them mod m_l (3M: forms the combination) and writes the
// INT8 residues of the fused path, which the shared CRT kernel then reads.
// Same operands and result as the fused path; only the INT32 round trip
// (4 MN bytes per product written and read) differs.  |acc| <= K 2^14 stays
// exact in INT32 for K <= 131071.

constexpr int NAIVE_TM = 2, NAIVE_TN = 2, NAIVE_NS = 4;  // 128 x 128 tiles, four stages
using NaiveTile = GemmTile<1, NAIVE_TM, NAIVE_TN, NAIVE_NS>;

// Product z = l Q + q (Q = 1 real, 3 for 3M: q = 0 re x re, 1 im x im, 2 the
// sums): plane q of modulus l is every Q-th slab of that modulus's packed
// operand, from slab q.
__global__ __launch_bounds__(256, 1) void k_s2_plane_gemm(const int8_t* __restrict__ Ap,
                                                         const int8_t* __restrict__ Bp, int64_t rows_a,
                                                         int64_t rows_b, int Q, int64_t nchunk, int M, int N,
                                                         int32_t* __restrict__ planes) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  const int z = blockIdx.z, l = z / Q, q = z % Q;
  const int64_t tiles_m = (M + NaiveTile::BM - 1) / NaiveTile::BM, tiles_n = (N + NaiveTile::BN - 1) / NaiveTile::BN;
  int64_t tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, 0, 4, tm, tn);
  const int64_t m0 = tm * NaiveTile::BM, n0 = tn * NaiveTile::BN;
  const int64_t kp = nchunk * OZK_K_CHUNK;
  v16i acc[1][NAIVE_TM][NAIVE_TN];
  zero_acc<1, NAIVE_TM, NAIVE_TN>(acc);
  gemm_tile_accumulate<1, NAIVE_TM, NAIVE_TN, NAIVE_NS, DIAGONAL, 1>(
      Ap + (int64_t)l * Q * rows_a * kp + (int64_t)q * rows_a * OZK_K_CHUNK,
      Bp + (int64_t)l * Q * rows_b * kp + (int64_t)q * rows_b * OZK_K_CHUNK, Q * rows_a, Q * rows_b, m0, n0, 0,
      nchunk, lds, acc);
  int32_t* out = planes + (int64_t)z * M * N;
  for_each_output<1, NAIVE_TM, NAIVE_TN>(acc, m0, n0, M, N,
                                          [&](int64_t row, int64_t col, const int* vals) { out[row * N + col] = vals[0]; });
}

// The INT32 planes back from HBM, reduced to the residues the fused kernel
// writes: [l][M][N] (3M: [l][2][M][N], re = smod(T1 - T2), im = smod(T3 - T1 - T2)).
template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_planes_mod(const int32_t* __restrict__ planes, int s, int64_t mn,
                                                       int8_t* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= mn) return;
  for (int l = 0; l < s; ++l) {
    if (!CPLX) {
      out[l * mn + idx] = (int8_t)smod_i32(planes[l * mn + idx], l);
    } else {
      const int t1 = smod_i32(planes[(3 * l) * mn + idx], l), t2 = smod_i32(planes[(3 * l + 1) * mn + idx], l),
                t3 = smod_i32(planes[(3 * l + 2) * mn + idx], l);
      out[(2 * l) * mn + idx] = (int8_t)smod_sum(t1, -t2, l);
      out[(2 * l + 1) * mn + idx] = (int8_t)smod_sum(smod_sum(t3, -t1, l), -t2, l);
    }
  }
}

int64_t s2_unfused_planes_bytes(int s, bool cplx, int64_t M, int64_t N) { return (int64_t)s * (cplx ? 3 : 1) * M * N * 4; }

hipError_t s2_gemm_mod_unfused(int s, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                               int32_t* planes, int8_t* out, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  static std::atomic<uint64_t> lds_done{0};
  const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(k_s2_plane_gemm), NaiveTile::LDS_BYTES, lds_done);
  if (e_lds != hipSuccess) return e_lds;
  const int Q = cplx ? 3 : 1;
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t nchunk = round_up(K, OZK_K_CHUNK) / OZK_K_CHUNK;
  const int64_t tiles = ((M + NaiveTile::BM - 1) / NaiveTile::BM) * ((N + NaiveTile::BN - 1) / NaiveTile::BN);
  hipLaunchKernelGGL(k_s2_plane_gemm, dim3((unsigned)tiles, 1, (unsigned)(s * Q)), dim3(256), NaiveTile::LDS_BYTES,
                     st, Ap, Bp, ra, rb, Q, nchunk, (int)M, (int)N, planes);
  const int64_t mn = M * N;
  if (cplx)
    hipLaunchKernelGGL(k_s2_planes_mod<true>, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, planes, s, mn,
                       out);
  else
    hipLaunchKernelGGL(k_s2_planes_mod<false>, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, planes, s, mn,
                       out);
  return hipGetLastError();
}

// 32-bit limbs the CRT sums need: sum_l W_l c_l < s 2^8 P < 2^(bits(P) + 13) for s <= 20.
static int crt_limbs(const CrtArgs& ca) {
  int pbits = 0;
  for (int i = NL - 1; i >= 0 && !pbits; --i)
    if (ca.P[i]) pbits = 32 * i + (32 - __builtin_clz(ca.P[i]));
  return (pbits + 13 + 31) / 32;
}

template <typename TO>
static hipError_t crt_t(int s, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                       const int32_t* tau, const TO* alpha, const TO* beta, TO* C, int64_t ldc, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  CrtArgs ca;
  int ta, tb;
  crt_args(s, ca, ta, tb);
  const int64_t n = M * N;
  const TO ai = cplx ? alpha[1] : (TO)0, bi = cplx ? beta[1] : (TO)0;
  const int u = crt_limbs(ca);
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ca, (int)M, (int)N, res, sigma, tau,
                       alpha[0], ai, beta[0], bi, C, ldc);
    return hipGetLastError();
  };
  auto pick = [&](auto cplx_c) {
    constexpr bool CP = decltype(cplx_c)::value;
    switch (u) {
      case 1: return launch(k_s2_crt<CP, TO, 1>);
      case 2: return launch(k_s2_crt<CP, TO, 2>);
      case 3: return launch(k_s2_crt<CP, TO, 3>);
      case 4: return launch(k_s2_crt<CP, TO, 4>);
      case 5: return launch(k_s2_crt<CP, TO, 5>);
    }
    return launch(k_s2_crt<CP, TO, NL>);
  };
  return cplx ? pick(std::true_type{}) : pick(std::false_type{});
}

hipError_t s2_crt(int s, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                  const int32_t* tau, const double* alpha, const double* beta, double* C, int64_t ldc,
                  hipStream_t st) {
  return crt_t(s, cplx, M, N, res, sigma, tau, alpha, beta, C, ldc, st);
}

hipError_t s2_crt(int s, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                  const int32_t* tau, const float* alpha, const float* beta, float* C, int64_t ldc,
                  hipStream_t st) {
  return crt_t(s, cplx, M, N, res, sigma, tau, alpha, beta, C, ldc, st);
}

// ------------------------------------------------- fused CRT epilogue
//
// The real-GEMM variant that never writes residue planes: one workgroup per
// 64 x 64 output tile runs all s moduli in one K loop (the residue planes of
// consecutive moduli are consecutive K chunks of the packed operands), adds
// each modulus's residue times W_l into per-output CRT sums held in registers
// (crt_add16) as soon as its last chunk is in, and after the last modulus
// reduces, rounds and writes C like k_s2_crt.  Bit-identical to the separate
// kernels.  The register budget (up to ten 32-bit sums for each of the 16
// outputs a lane holds) allows only this small tile, which moves about four
// times the operand bytes per MFMA of the large tiles; for 3M (two sums per
// output) it does not fit without spilling, so complex products keep the
// separate kernels.
constexpr int S2_FUSED_V = 4;

template <int NZ>
__global__ __launch_bounds__(256, 1) void k_s2_gemm_crt(CrtArgs ca, const int8_t* __restrict__ Ap,
                                                       const int8_t* __restrict__ Bp, int64_t rows_a, int64_t rows_b,
                                                       int64_t nsteps, int M, int N, const int32_t* __restrict__ sigma,
                                                       const int32_t* __restrict__ tau, double alpha, double beta,
                                                       double* __restrict__ C, int64_t ldc, int raster, int group) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  using Cfg = S2Cfg<false, S2_FUSED_V>;
  static_assert(Cfg::P == 1 && Cfg::G == 1 && Cfg::TM == 1 && Cfg::TN == 1,
                "one plane, one 32 x 32 MFMA tile per wave, one chunk per stage");
  constexpr int NS = Cfg::NS;
  using T = GemmTile<1, 1, 1, NS>;
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, raster, group, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  v16i acc[1][1][1];
  zero_acc<1, 1, 1>(acc);
  uint32_t z[16][NZ];
#pragma unroll
  for (int v = 0; v < 16; ++v)
#pragma unroll
    for (int i = 0; i < NZ; ++i) z[v][i] = 0;
  int l = 0;
  int64_t in_mod = 0, in_run = 0;  // chunks of modulus l, of its current run
  // the short reduction in the small tile only: the large one keeps its
  // accumulators in registers around these stores only with one epilogue form
  const bool small = !Cfg::LARGE && Cfg::SMALL && nsteps <= S2_SMALL_STEPS;
  auto hook = [&](int64_t r) {
    if (r < 0) return;
    ++in_mod;
    ++in_run;
    if (in_mod == nsteps) {
#pragma unroll
      for (int v = 0; v < 16; ++v) crt_add16(z[v], ca, l, smod_i32(acc[0][0][0][v], l));
      zero_acc<1, 1, 1>(acc);
      ++l;
      in_mod = 0;
      in_run = 0;
    } else if (in_run == S2_RUN_STEPS) {
      s2_reduce_acc<1, 1, 1>(acc, l);
      in_run = 0;
    }
  };
  gemm_tile_accumulate<1, 1, 1, NS, DIAGONAL, 1>(Ap, Bp, rows_a, rows_b, m0, n0, 0, (int64_t)ca.s * nsteps, lds, acc,
                                                 hook);
  // K = 0 runs no step: every sum stays 0, as the residues would be.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    // the output layout of for_each_output
    const int64_t row = m0 + wm * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
    const int64_t col = n0 + wn * 32 + (lane & 31);
    if (row >= M || col >= N) continue;
    const int si = sigma[row], tj = tau[col];
    const bool bad = si == OZK_EXP_NONFINITE || tj == OZK_EXP_NONFINITE;
    uint32_t vl[NL + 1], mag[NL];
    bool neg;
    crt_limbs16(z[v], vl);
    crt_reduce(ca, vl, mag, neg);
    const double h[2] = {bad ? __builtin_nan("") : round_limbs(mag, neg, -si - tj), 0.0};
    s2_store_c<false>(h, row, col, alpha, 0.0, beta, 0.0, C, ldc);
  }
}

hipError_t s2_gemm_crt(int s, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                       const int32_t* sigma, const int32_t* tau, double alpha, double beta, double* C, int64_t ldc,
                       int raster, int group, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  CrtArgs ca;
  int ta, tb;
  crt_args(s, ca, ta, tb);
  using Cfg = S2Cfg<false, S2_FUSED_V>;
  using T = GemmTile<1, Cfg::TM, Cfg::TN, Cfg::NS>;
  const int64_t kp = round_up(K, OZK_K_CHUNK);
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
  auto launch = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       Cfg::LDS_BYTES);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(256), Cfg::LDS_BYTES, st, ca, Ap, Bp, ra, rb,
                       kp / OZK_K_CHUNK, (int)M, (int)N, sigma, tau, alpha, beta, C, ldc, raster, group);
    return hipGetLastError();
  };
  // 16-bit pieces of W_l < P <= 256^s
  if (s <= 12) return launch(k_s2_gemm_crt<6>);
  if (s <= 16) return launch(k_s2_gemm_crt<8>);
  return launch(k_s2_gemm_crt<10>);
}

// --------------------------------- modulus count chosen on the device

__constant__ CrtArgs c_crt_all[OZK_MAX_S];  // CRT constants of s = 1 .. OZK_MAX_S (index s - 1)

__device__ __forceinline__ bool s2_chosen(const int32_t* __restrict__ info, int& s) {
  if (info[4] != 2) return false;
  s = info[5];
  return s >= 1 && s <= OZK_MAX_S;
}

// The grids of these kernels are capped (AUTO_GRID workgroups, a multiple
// of 8) and each workgroup walks its blocks with the grid as stride: when
// Scheme I is chosen they dispatch a few workgroups that return at once
// instead of a full grid.
constexpr int64_t AUTO_GRID = 2048;

__host__ __device__ constexpr int64_t auto_grid(int64_t blocks) { return blocks < AUTO_GRID ? blocks : AUTO_GRID; }

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_split_rows_auto(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                            int64_t K, int64_t Kp, int64_t rows_packed, int64_t nblk,
                                                            const int32_t* __restrict__ info, S2Budgets bud,
                                                            int32_t* __restrict__ sigma_out,
                                                            int8_t* __restrict__ packed) {
  int s;
  if (!s2_chosen(info, s)) return;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x)
    s2_split_rows_block<CPLX>(X, ldx, rows, K, Kp, rows_packed, S2Args{s, bud.ta[s]}, sigma_out, packed, b);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_col_scales_auto(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                            int64_t cols, int64_t nblk,
                                                            const int32_t* __restrict__ info, S2Budgets bud,
                                                            int32_t* __restrict__ tau) {
  int s;
  if (!s2_chosen(info, s)) return;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) s2_col_scales_block<CPLX>(X, ldx, K, cols, bud.tb[s], tau, b);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_split_cols_auto(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                            int64_t cols, int64_t Kp, int64_t cols_packed,
                                                            int64_t jblocks, int64_t nblk,
                                                            const int32_t* __restrict__ info,
                                                            const int32_t* __restrict__ tau,
                                                            int8_t* __restrict__ packed) {
  int s;
  if (!s2_chosen(info, s)) return;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x)
    s2_split_cols_block<CPLX>(X, ldx, K, cols, Kp, cols_packed, s, tau, packed, b % jblocks, b / jblocks);
}

// Items (tile, modulus), modulus-major as the grid z of the fixed-s kernel;
// the items of moduli past the chosen s are not visited.
template <bool CPLX>
__global__ __launch_bounds__(256, 1) void k_s2_gemm_mod_auto(const int8_t* __restrict__ Ap,
                                                            const int8_t* __restrict__ Bp, int64_t plane_a,
                                                            int64_t plane_b, int64_t rows_a, int64_t rows_b,
                                                            int64_t nsteps, int M, int N, int64_t tiles,
                                                            const int32_t* __restrict__ info,
                                                            int8_t* __restrict__ out) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  int s;
  if (!s2_chosen(info, s)) return;
  for (int64_t it = blockIdx.x; it < tiles * s; it += gridDim.x)
    s2_gemm_tile<CPLX, 0>(Ap, Bp, plane_a, plane_b, rows_a, rows_b, nsteps, M, N, out, it % tiles, (int)(it / tiles),
                          0, 4, lds);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_crt_auto(int M, int N, int64_t nblk, const int8_t* __restrict__ res,
                                                     const int32_t* __restrict__ sigma,
                                                     const int32_t* __restrict__ tau,
                                                     const int32_t* __restrict__ info, double a_re, double a_im,
                                                     double b_re, double b_im, double* __restrict__ C, int64_t ldc) {
  int s;
  if (!s2_chosen(info, s)) return;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x)
    s2_crt_block<CPLX, double, CRT_ANY_S>(c_crt_all[s - 1], M, N, res, sigma, tau, a_re, a_im, b_re, b_im, C, ldc, b);
}

S2Budgets s2_budgets() {
  S2Budgets b;
  b.ta[0] = b.tb[0] = 0;
  for (int s = 1; s <= OZK_MAX_S; ++s) s2_targets(s, b.ta[s], b.tb[s]);
  return b;
}

hipError_t s2_upload_crt_tables() {
  static CrtArgs all[OZK_MAX_S];
  int ta, tb;
  for (int s = 1; s <= OZK_MAX_S; ++s) crt_args(s, all[s - 1], ta, tb);
  return hipMemcpyToSymbol(HIP_SYMBOL(c_crt_all), all, sizeof(all));
}

hipError_t s2_split_rows_auto(const int32_t* info, bool cplx, const double* X, int64_t ldx, int64_t rows, int64_t K,
                              int32_t* sigma, int8_t* packed, hipStream_t st) {
  const int64_t rp = round_up(rows, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (rp > 0) {
    const int64_t nblk = rp / S2_ROWS_PER_BLOCK;
    const dim3 grid((unsigned)auto_grid(nblk));
    if (cplx)
      hipLaunchKernelGGL(k_s2_split_rows_auto<true>, grid, dim3(256), 0, st, X, ldx, rows, K, kp, rp, nblk, info,
                         s2_budgets(), sigma, packed);
    else
      hipLaunchKernelGGL(k_s2_split_rows_auto<false>, grid, dim3(256), 0, st, X, ldx, rows, K, kp, rp, nblk, info,
                         s2_budgets(), sigma, packed);
  }
  return hipGetLastError();
}

hipError_t s2_split_cols_auto(const int32_t* info, bool cplx, const double* X, int64_t ldx, int64_t K, int64_t cols,
                              int32_t* tau, int8_t* packed, hipStream_t st) {
  const int64_t cp = round_up(cols, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (cols > 0) {
    const int64_t nblk = (cols + 31) / 32;
    const dim3 grid((unsigned)auto_grid(nblk));
    if (cplx)
      hipLaunchKernelGGL(k_s2_col_scales_auto<true>, grid, dim3(256), 0, st, X, ldx, K, cols, nblk, info,
                         s2_budgets(), tau);
    else
      hipLaunchKernelGGL(k_s2_col_scales_auto<false>, grid, dim3(256), 0, st, X, ldx, K, cols, nblk, info,
                         s2_budgets(), tau);
  }
  if (cp > 0 && kp > 0) {
    const int64_t jblocks = cp / S2_COL_BLOCK, nblk = jblocks * (kp / OZK_K_CHUNK);
    const dim3 grid((unsigned)auto_grid(nblk));
    if (cplx)
      hipLaunchKernelGGL(k_s2_split_cols_auto<true>, grid, dim3(256), 0, st, X, ldx, K, cols, kp, cp, jblocks, nblk,
                         info, tau, packed);
    else
      hipLaunchKernelGGL(k_s2_split_cols_auto<false>, grid, dim3(256), 0, st, X, ldx, K, cols, kp, cp, jblocks, nblk,
                         info, tau, packed);
  }
  return hipGetLastError();
}

template <bool CPLX>
static hipError_t launch_gemm_mod_auto(const int32_t* info, int64_t M, int64_t N, int64_t K, const int8_t* Ap,
                                       const int8_t* Bp, int8_t* out, hipStream_t st) {
  using Cfg = S2Cfg<CPLX, 0>;
  using T = GemmTile<Cfg::P, Cfg::TM, Cfg::TN, Cfg::NS>;
  static std::atomic<uint64_t> lds_done{0};
  const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(k_s2_gemm_mod_auto<CPLX>), Cfg::LDS_BYTES, lds_done);
  if (e_lds != hipSuccess) return e_lds;
  const int64_t kp = round_up(K, OZK_K_CHUNK);
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
  const dim3 grid((unsigned)auto_grid(tiles * OZK_MAX_S));
  hipLaunchKernelGGL(k_s2_gemm_mod_auto<CPLX>, grid, dim3(256), Cfg::LDS_BYTES, st, Ap, Bp, ra * kp * Cfg::P,
                     rb * kp * Cfg::P, ra, rb, kp / OZK_K_CHUNK, (int)M, (int)N, tiles, info, out);
  return hipGetLastError();
}

hipError_t s2_gemm_mod_auto(const int32_t* info, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap,
                            const int8_t* Bp, int8_t* out, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  return cplx ? launch_gemm_mod_auto<true>(info, M, N, K, Ap, Bp, out, st)
              : launch_gemm_mod_auto<false>(info, M, N, K, Ap, Bp, out, st);
}

hipError_t s2_crt_auto(const int32_t* info, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                       const int32_t* tau, const double* alpha, const double* beta, double* C, int64_t ldc,
                       hipStream_t st) {
  const int64_t n = M * N;
  if (n <= 0) return hipSuccess;
  const int64_t nblk = (n + 255) / 256;
  const dim3 grid((unsigned)auto_grid(nblk));
  if (cplx)
    hipLaunchKernelGGL(k_s2_crt_auto<true>, grid, dim3(256), 0, st, (int)M, (int)N, nblk, res, sigma, tau, info,
                       alpha[0], alpha[1], beta[0], beta[1], C, ldc);
  else
    hipLaunchKernelGGL(k_s2_crt_auto<false>, grid, dim3(256), 0, st, (int)M, (int)N, nblk, res, sigma, tau, info,
                       alpha[0], 0.0, beta[0], 0.0, C, ldc);
  return hipGetLastError();
}

// ------------------------------------------------------- batched problems
//
// Many uneven problems in one launch per step.  The plan uploads a problem
// table and, per step, the prefix sums of the work units of each problem;
// a workgroup finds its problem by binary search.  The GEMM step is one
// persistent launch per tile size over (problem, output tile) items, each
// running all s moduli in one K loop: the plan deals the items out to one
// queue per XCD in chunks of consecutive tiles of one problem (so that the
// operand panels a problem's tiles share are fetched into one L2, not eight),
// balancing the queues' INT8 work, longest items first within a queue, and
// the workgroups of an XCD walk its queue with a fixed stride, without atomics.

namespace {

__device__ __forceinline__ int find_problem(const BatchUnits& u, int64_t x) {
  const int64_t b = x >> OZK_BATCH_HINT_SHIFT;
  int lo = u.hint[b], hi = u.hint[b + 1];  // the largest i with start[i] <= x lies in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (u.start[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

// The batched pre-pass leaves the padding rows and columns of the packed
// operands as they are: they feed only outputs past M and N, which no later
// step reads.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_split_rows(BatchDev bd, int8_t* __restrict__ ws, S2Args sa) {
  __shared__ int16_t ecache[s2_ecache_bytes(S2_ECACHE_BATCH_K) / 2];
  const int p = find_problem(bd.rows, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  s2_split_rows_block<CPLX>(q.A, q.lda, q.M, q.K, q.Kp, q.ra, sa, reinterpret_cast<int32_t*>(ws + q.off_sig),
                            ws + q.off_a, blockIdx.x - bd.rows.start[p], 0, -1, nullptr, false, ecache,
                            S2_ECACHE_BATCH_K);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_col_scales(BatchDev bd, int8_t* __restrict__ ws, int T) {
  __shared__ int16_t ecache[S2CCols<CPLX>::CC * s2_batch_ccache_k<CPLX>()];
  const int p = find_problem(bd.cols, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  const int64_t blk = blockIdx.x - bd.cols.start[p];
  int32_t* tau = reinterpret_cast<int32_t*>(ws + q.off_tau);
  if (q.K <= s2_batch_ccache_k<CPLX>())  // uniform: the block count follows s2_batch_col_blocks
    s2_col_scales_cached_block<CPLX>(q.B, q.ldb, q.K, q.N, T, tau, blk, ecache);
  else
    s2_col_scales_block<CPLX>(q.B, q.ldb, q.K, q.N, T, tau, blk);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_split_cols(BatchDev bd, int8_t* __restrict__ ws, int s) {
  const int p = find_problem(bd.split, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  const int64_t local = blockIdx.x - bd.split.start[p];
  const int64_t jblocks = q.rb / S2_COL_BLOCK;
  s2_split_cols_block<CPLX>(q.B, q.ldb, q.K, q.N, q.Kp, q.rb, s, reinterpret_cast<const int32_t*>(ws + q.off_tau),
                            ws + q.off_b, local % jblocks, local / jblocks, false);
}

// Two batch GEMM tiles, chosen per problem by the plan (from the tuned
// table, see ozk_batch_plan_create): the small tile (variant 4, 64 x 64,
// several resident workgroups per CU overlapping the prologue and epilogue
// latency of short items) and the large one (128 x 128: variant 1 for real
// products, 2 for 3M), which reads half (real) or a quarter (3M) of the LDS
// bytes per MFMA and pays off on the larger problems.
constexpr int S2_BATCH_V = 4;
template <bool CPLX>
struct S2BatchLarge {
  static constexpr int V = CPLX ? 2 : 1;
};
template <bool CPLX, int V>
constexpr int batch_rows() {
  return GemmTile<S2Cfg<CPLX, V>::P, S2Cfg<CPLX, V>::TM, S2Cfg<CPLX, V>::TN, S2Cfg<CPLX, V>::NS>::BM;
}
template <bool CPLX, int V>
constexpr int batch_cols() {
  return GemmTile<S2Cfg<CPLX, V>::P, S2Cfg<CPLX, V>::TM, S2Cfg<CPLX, V>::TN, S2Cfg<CPLX, V>::NS>::BN;
}
static_assert(OZK_BATCH_ROW_ALIGN % batch_rows<false, S2_BATCH_V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_cols<false, S2_BATCH_V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_rows<true, S2_BATCH_V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_cols<true, S2_BATCH_V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_rows<false, S2BatchLarge<false>::V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_cols<false, S2BatchLarge<false>::V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_rows<true, S2BatchLarge<true>::V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % batch_cols<true, S2BatchLarge<true>::V>() == 0 &&
                  OZK_BATCH_ROW_ALIGN % S2_ROWS_PER_BLOCK == 0 && OZK_BATCH_ROW_ALIGN % S2_COL_BLOCK == 0,
              "batched packed rows cover whole tiles of both sizes and whole pre-pass blocks");

// One output tile of a batched problem for all s moduli.  The residue planes
// of consecutive moduli are consecutive K chunks of the packed operands, so
// when a modulus's sums fit one INT32 run (nsteps <= S2_RUN_STEPS) the s GEMMs
// run as one K loop of s nsteps chunks whose load pipeline never drains
// between moduli; the step hook stores a modulus's residues once its last
// chunk is in.  Longer K takes each modulus as its own sequence of runs.
template <bool CPLX, int V>
__device__ __forceinline__ void s2_gemm_tile_moduli(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                                    int64_t rows_a, int64_t rows_b, int64_t nsteps, int64_t M,
                                                    int64_t N, int8_t* __restrict__ out, int64_t ldr, int64_t tile,
                                                    int s, int8_t* lds) {
  using Cfg = S2Cfg<CPLX, V>;
  static_assert(Cfg::G == 1, "one K chunk per stage");
  constexpr int P = Cfg::P, TM = Cfg::TM, TN = Cfg::TN, NS = Cfg::NS;
  using T = GemmTile<P, TM, TN, NS>;
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(tile, tiles_m, tiles_n, 1, 4, tm, tn);  // a chunk's tiles run on one XCD: groups of 4 tile rows
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  v16i acc[P][TM][TN];
  zero_acc<P, TM, TN>(acc);
  if (nsteps == 0) {  // K = 0: every residue is 0
    for (int l = 0; l < s; ++l) s2_store_tile<CPLX, P, TM, TN>(acc, m0, n0, M, N, out, l, ldr, false);
    return;
  }
  if (nsteps > S2_RUN_STEPS) {
    for (int l = 0; l < s; ++l) {
      for (int64_t c0 = 0; c0 < nsteps; c0 += S2_RUN_STEPS) {
        const int64_t n = nsteps - c0 < S2_RUN_STEPS ? nsteps - c0 : S2_RUN_STEPS;
        gemm_tile_accumulate<P, TM, TN, NS, DIAGONAL, P>(Ap, Bp, rows_a, rows_b, m0, n0, l * nsteps + c0, n, lds,
                                                         acc);
        if (c0 + n < nsteps) s2_reduce_acc<P, TM, TN>(acc, l);
      }
      s2_store_tile<CPLX, P, TM, TN>(acc, m0, n0, M, N, out, l, ldr, false);
      zero_acc<P, TM, TN>(acc);
    }
    return;
  }
  int l = 0;
  int64_t in_mod = 0;  // chunks of modulus l done
  // the short reduction in the small tile only: the large one keeps its
  // accumulators in registers around these stores only with one epilogue form
  const bool small = !Cfg::LARGE && Cfg::SMALL && nsteps <= S2_SMALL_STEPS;
  // one rare branch that rewrites the accumulators in place (a second one,
  // for run reductions, made the compiler copy them on every step)
  auto hook = [&](int64_t r) {
    if (r < 0) return;
    if (++in_mod == nsteps) {
      s2_store_tile<CPLX, P, TM, TN>(acc, m0, n0, M, N, out, l, ldr, small);
      zero_acc<P, TM, TN>(acc);
      ++l;
      in_mod = 0;
    }
  };
  gemm_tile_accumulate<P, TM, TN, NS, DIAGONAL, P>(Ap, Bp, rows_a, rows_b, m0, n0, 0, (int64_t)s * nsteps, lds, acc,
                                                   hook);
}

// Persistent over the items of one tile size: with Q = OZK_BATCH_QUEUES
// (the grid a multiple of Q), workgroup w runs queue w % Q, taking its items
// w / Q, w / Q + G / Q, ...
template <bool CPLX, int V>
__global__ __launch_bounds__(256, V == S2_BATCH_V ? 3 : 1) void k_b_gemm_mod(BatchDev bd, BatchItems items,
                                                                            int8_t* __restrict__ ws, int s) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  const int x = blockIdx.x % OZK_BATCH_QUEUES;
  const int64_t stride = gridDim.x / OZK_BATCH_QUEUES, end = items.queue[x + 1];
  for (int64_t it = items.queue[x] + blockIdx.x / OZK_BATCH_QUEUES; it < end; it += stride) {
    const int c = find_problem(items.chunks, it);
    const BatchProb& q = bd.prob[items.prob[c]];
    s2_gemm_tile_moduli<CPLX, V>(ws + q.off_a, ws + q.off_b, q.ra, q.rb, q.Kp / OZK_K_CHUNK, q.M, q.N,
                                 ws + q.off_res, q.ldr, items.tile0[c] + (it - items.chunks.start[c]), s, lds);
  }
}

template <bool CPLX, int U = NL>
__global__ __launch_bounds__(256) void k_b_crt(CrtArgs ca, BatchDev bd, int8_t* __restrict__ ws) {
  const int p = find_problem(bd.crt, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  s2_crt_block<CPLX, double, U>(ca, q.M, q.N, ws + q.off_res, reinterpret_cast<const int32_t*>(ws + q.off_sig),
                                reinterpret_cast<const int32_t*>(ws + q.off_tau), q.a_re, q.a_im, q.b_re, q.b_im,
                                q.C, q.ldc, blockIdx.x - bd.crt.start[p], q.ldr);
}

int64_t s2_tile_count(bool cplx, bool large, int64_t M, int64_t N) {
  int bm, bn;
  if (large) {
    bm = cplx ? batch_rows<true, S2BatchLarge<true>::V>() : batch_rows<false, S2BatchLarge<false>::V>();
    bn = cplx ? batch_cols<true, S2BatchLarge<true>::V>() : batch_cols<false, S2BatchLarge<false>::V>();
  } else {
    bm = cplx ? batch_rows<true, S2_BATCH_V>() : batch_rows<false, S2_BATCH_V>();
    bn = cplx ? batch_cols<true, S2_BATCH_V>() : batch_cols<false, S2_BATCH_V>();
  }
  return ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
}

template <bool CPLX, int V>
static int batch_blocks_per_cu() {
  int n = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_b_gemm_mod<CPLX, V>, 256, S2Cfg<CPLX, V>::LDS_BYTES);
  return (e == hipSuccess && n > 0) ? n : 1;
}

int s2_batch_gemm_blocks_per_cu(bool cplx, bool large) {
  if (large) return cplx ? batch_blocks_per_cu<true, 2>() : batch_blocks_per_cu<false, 1>();
  return cplx ? batch_blocks_per_cu<true, S2_BATCH_V>() : batch_blocks_per_cu<false, S2_BATCH_V>();
}

template <bool CPLX, int V>
static hipError_t launch_batch_gemm(const BatchDev& bd, const BatchItems& items, int64_t n, int grid, int8_t* ws,
                                    int s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (grid < OZK_BATCH_QUEUES || grid % OZK_BATCH_QUEUES != 0) return hipErrorInvalidConfiguration;
  constexpr int lds = S2Cfg<CPLX, V>::LDS_BYTES;
  static std::atomic<uint64_t> lds_done{0};
  const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(k_b_gemm_mod<CPLX, V>), lds, lds_done);
  if (e_lds != hipSuccess) return e_lds;
  hipLaunchKernelGGL((k_b_gemm_mod<CPLX, V>), dim3((unsigned)grid), dim3(256), lds, st, bd, items, ws, s);
  return hipGetLastError();
}

// The GEMM step of a batch: the large-tile items, then the small-tile ones.
hipError_t s2_batched_gemm(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, int grid_small,
                           int grid_large, hipStream_t st) {
  hipError_t e = cplx ? launch_batch_gemm<true, 2>(bd, bd.items_l, tot.items_l, grid_large, ws, s, st)
                      : launch_batch_gemm<false, 1>(bd, bd.items_l, tot.items_l, grid_large, ws, s, st);
  if (e != hipSuccess) return e;
  return cplx ? launch_batch_gemm<true, S2_BATCH_V>(bd, bd.items, tot.items, grid_small, ws, s, st)
              : launch_batch_gemm<false, S2_BATCH_V>(bd, bd.items, tot.items, grid_small, ws, s, st);
}

hipError_t s2_batched_prepass(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws,
                              hipStream_t st) {
  int ta, tb;
  CrtArgs ca;
  crt_args(s, ca, ta, tb);
  if (tot.rows == 0) return hipSuccess;
  S2Args sa{s, ta};
  if (cplx) {
    hipLaunchKernelGGL(k_b_split_rows<true>, dim3((unsigned)tot.rows), dim3(256), 0, st, bd, ws, sa);
    hipLaunchKernelGGL(k_b_col_scales<true>, dim3((unsigned)tot.cols), dim3(256), 0, st, bd, ws, tb);
    if (tot.split) hipLaunchKernelGGL(k_b_split_cols<true>, dim3((unsigned)tot.split), dim3(256), 0, st, bd, ws, s);
  } else {
    hipLaunchKernelGGL(k_b_split_rows<false>, dim3((unsigned)tot.rows), dim3(256), 0, st, bd, ws, sa);
    hipLaunchKernelGGL(k_b_col_scales<false>, dim3((unsigned)tot.cols), dim3(256), 0, st, bd, ws, tb);
    if (tot.split) hipLaunchKernelGGL(k_b_split_cols<false>, dim3((unsigned)tot.split), dim3(256), 0, st, bd, ws, s);
  }
  return hipGetLastError();
}

hipError_t s2_batched_crt(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, hipStream_t st) {
  int ta, tb;
  CrtArgs ca;
  crt_args(s, ca, ta, tb);
  if (tot.crt == 0) return hipSuccess;
  const dim3 grid((unsigned)tot.crt);
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, ca, bd, ws);
    return hipGetLastError();
  };
  auto pick = [&](auto cplx_c) {
    constexpr bool CP = decltype(cplx_c)::value;
    switch (crt_limbs(ca)) {  // the kernel holding this s
      case 1: return launch(k_b_crt<CP, 1>);
      case 2: return launch(k_b_crt<CP, 2>);
      case 3: return launch(k_b_crt<CP, 3>);
      case 4: return launch(k_b_crt<CP, 4>);
      case 5: return launch(k_b_crt<CP, 5>);
    }
    return launch(k_b_crt<CP, NL>);
  };
  return cplx ? pick(std::true_type{}) : pick(std::false_type{});
}

hipError_t s2_batched(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, int grid_small,
                      int grid_large, hipStream_t st) {
  if (tot.rows == 0 || tot.crt == 0) return hipSuccess;
  hipError_t e = s2_batched_prepass(s, cplx, bd, tot, ws, st);
  if (e == hipSuccess) e = s2_batched_gemm(s, cplx, bd, tot, ws, grid_small, grid_large, st);
  if (e == hipSuccess) e = s2_batched_crt(s, cplx, bd, tot, ws, st);
  return e;
}

}  // namespace ozk
