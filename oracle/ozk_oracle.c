/*
 * Plain CPU oracle for FP64 GEMM emulated by the Ozaki schemes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header, table or constant with the HIP library.
 *
 * Everything here is deliberately slow and literal: triple loops, 64-bit and
 * 128-bit integers, one OpenMP pragma on the outermost row loop, and no
 * blocking or reordering beyond what the definitions state.
 *
 * Contents
 *   orc_gemm_naive      plain FP64 product, k ascending, one fma per term
 *   orc_gemm_dd         double-double dot products (error-free TwoProd/TwoSum)
 *   orc_zgemm_dd        complex double-double reference (four real dd dots)
 *   orc_expo            frexp exponent e with |x| < 2^e <= 2|x|
 *   orc_s1_*            Ozaki Scheme I with balanced signed 8-bit slices
 *                       (8p-2 bits in all):
 *                       Sec. II-C.1, Eq. (1) split, Eq. (2) diagonals,
 *                       Eq. (3) shift-reduce (made exact: integer sum, then a
 *                       single correctly rounded scaling)
 *   orc_round_scaled    round-to-nearest-even of Z * 2^E for a 128-bit Z
 *
 * Conventions: row-major, contiguous, element (i,k) of an MxK matrix at
 * i*K + k.  Exponent sentinels: a row/column with no nonzero entry gets
 * ORC_ZERO_EXP, one holding a NaN or infinity gets ORC_NONFINITE_EXP.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

#define ORC_ZERO_EXP (-100000)
#define ORC_NONFINITE_EXP (100000)

/* ------------------------------------------------------------------ */
/* References                                                          */
/* ------------------------------------------------------------------ */

/* C = A*B, every term added with one fma, k ascending. */
void orc_gemm_naive(int64_t M, int64_t N, int64_t K, const double* A,
                    const double* B, double* C) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < K; ++k) s = fma(A[i * K + k], B[k * N + j], s);
      C[i * N + j] = s;
    }
}

/* Error-free transformations (Knuth TwoSum; TwoProd through fma). */
static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  *s = x;
  *e = (a - av) + (b - bv);
}
static void two_prod(double a, double b, double* p, double* e) {
  double x = a * b;
  *p = x;
  *e = fma(a, b, -x);
}
/* (hi,lo) += (ph,pl), renormalised. */
static void dd_add(double* hi, double* lo, double ph, double pl) {
  double s, e;
  two_sum(*hi, ph, &s, &e);
  e += *lo + pl;
  double h = s + e;
  *lo = e - (h - s);
  *hi = h;
}

/* Double-double product: C = Chi + Clo to about 2^-104 relative per term. */
void orc_gemm_dd(int64_t M, int64_t N, int64_t K, const double* A,
                 const double* B, double* Chi, double* Clo) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double hi = 0.0, lo = 0.0;
      for (int64_t k = 0; k < K; ++k) {
        double p, e;
        two_prod(A[i * K + k], B[k * N + j], &p, &e);
        dd_add(&hi, &lo, p, e);
      }
      Chi[i * N + j] = hi;
      Clo[i * N + j] = lo;
    }
}

/* Complex double-double product; A, B, C interleaved (re, im). */
void orc_zgemm_dd(int64_t M, int64_t N, int64_t K, const double* A,
                  const double* B, double* Chi, double* Clo) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double rh = 0.0, rl = 0.0, ih = 0.0, il = 0.0;
      for (int64_t k = 0; k < K; ++k) {
        double ar = A[2 * (i * K + k)], ai = A[2 * (i * K + k) + 1];
        double br = B[2 * (k * N + j)], bi = B[2 * (k * N + j) + 1];
        double p, e;
        two_prod(ar, br, &p, &e);
        dd_add(&rh, &rl, p, e);
        two_prod(-ai, bi, &p, &e);
        dd_add(&rh, &rl, p, e);
        two_prod(ar, bi, &p, &e);
        dd_add(&ih, &il, p, e);
        two_prod(ai, br, &p, &e);
        dd_add(&ih, &il, p, e);
      }
      Chi[2 * (i * N + j)] = rh;
      Chi[2 * (i * N + j) + 1] = ih;
      Clo[2 * (i * N + j)] = rl;
      Clo[2 * (i * N + j) + 1] = il;
    }
}

/* ------------------------------------------------------------------ */
/* Exact scaled rounding                                               */
/* ------------------------------------------------------------------ */

/* Round-to-nearest-even of Z * 2^E, handled as one rounding: gradual
 * underflow and overflow to infinity included.  Z = 0 gives +0. */
double orc_round_scaled(i128 Z, int64_t E) {
  if (Z == 0) return 0.0;
  int neg = Z < 0;
  u128 mag = neg ? (u128)0 - (u128)Z : (u128)Z;
  int n = 0; /* bit length of mag */
  for (u128 t = mag; t != 0; t >>= 1) ++n;
  /* bits to drop: keep 53 significant bits, but never go below 2^-1074 */
  int64_t drop = n - 53;
  if (-1074 - E > drop) drop = -1074 - E;
  u128 q;
  int64_t Eq;
  if (drop <= 0) {
    q = mag;
    Eq = E;
  } else {
    u128 rem, half;
    if (drop >= 128) {
      q = 0;
      rem = mag;
      /* half = 2^(drop-1) > mag whenever drop >= 129; drop == 128 needs care */
      half = (drop == 128) ? ((u128)1 << 127) : 0;
      if (drop > 128) return neg ? -0.0 : 0.0;
      if (rem > half) q = 1;
    } else {
      q = mag >> drop;
      rem = mag & (((u128)1 << drop) - 1);
      half = (u128)1 << (drop - 1);
      if (rem > half || (rem == half && (q & 1))) q += 1;
    }
    Eq = E + drop;
  }
  /* q < 2^54 here and q * 2^Eq is representable (or overflows). */
  if (Eq > 2000) return neg ? -INFINITY : INFINITY;
  double r = ldexp((double)(uint64_t)q, (int)Eq);
  return neg ? -r : r;
}

/* ------------------------------------------------------------------ */
/* Scheme I                                                            */
/* ------------------------------------------------------------------ */
/* Slice format.  The paper cuts consecutive 8-bit segments of the scaled
 * mantissa into INT8 slices (Sec. II-C.1).  Here the segments are balanced
 * signed base-256 digits, the form a signed-only INT8 matrix unit takes
 * directly: with x = a 2^-e (|x| < 1) and the rounded fixed-point integer
 *   X = floor(x 2^(8p-2) + 1/2),   |X| <= 2^(8p-2),
 * the digits are  d_t = ((X_t + 128) mod 256) - 128  for t = p-1 .. 1 with
 * X_(t-1) = (X_t - d_t) / 256, and d_0 the last quotient (|d_0| <= 64), so that
 *   x = sum_t d_t 2^(-6-8t)  up to a rounding error of at most 2^-(8p-1). */

/* frexp exponent: x = f * 2^e with 0.5 <= |f| < 1.  Only for finite x != 0. */
int orc_expo(double x) {
  int e;
  frexp(x, &e);
  return e;
}

static int orc_exponent_of(const double* x, int64_t n, int64_t stride) {
  int e = ORC_ZERO_EXP;
  for (int64_t k = 0; k < n; ++k) {
    double v = x[k * stride];
    if (!isfinite(v)) return ORC_NONFINITE_EXP;
    if (v != 0.0) {
      int ek = orc_expo(v);
      if (ek > e) e = ek;
    }
  }
  return e;
}

/* Row scales of A (the power-of-two mu of Eq. 1 is 2^e[i]). */
void orc_s1_row_exponents(int64_t M, int64_t K, const double* A, int32_t* e) {
  for (int64_t i = 0; i < M; ++i) e[i] = orc_exponent_of(A + i * K, K, 1);
}
/* Column scales of B (nu of Eq. 1 is 2^f[j]). */
void orc_s1_col_exponents(int64_t K, int64_t N, const double* B, int32_t* f) {
  for (int64_t j = 0; j < N; ++j) f[j] = orc_exponent_of(B + j, K, N);
}

/* X = floor(a 2^(8p-2-e) + 1/2) exactly, from the integer significand of a. */
static int64_t orc_fixed_point(double a, int e, int p) {
  int ex;
  double fr = frexp(a, &ex);          /* a = fr 2^ex, 0.5 <= |fr| < 1 */
  int64_t m = (int64_t)ldexp(fr, 53); /* exact: a = m 2^(ex-53) */
  int sh = ex - 53 + 8 * p - 2 - e;   /* X = floor(m 2^sh + 1/2) */
  if (sh >= 0) return m * ((int64_t)1 << sh);
  if (sh <= -62) return 0;            /* |m 2^sh| < 2^-9 */
  int64_t d = (int64_t)1 << (-sh);
  int64_t n = m + d / 2;              /* floor(n / d) */
  int64_t q = n / d;
  if (n % d != 0 && n < 0) q -= 1;
  return q;
}

/* The p balanced digits of one entry a whose row/column exponent is e. */
static void orc_digits(double a, int e, int p, int8_t* D, int64_t dstride) {
  if (a == 0.0 || e == ORC_ZERO_EXP || e == ORC_NONFINITE_EXP || !isfinite(a)) {
    for (int t = 0; t < p; ++t) D[t * dstride] = 0;
    return;
  }
  int64_t X = orc_fixed_point(a, e, p);
  for (int t = p - 1; t >= 1; --t) {
    int64_t r = (X + 128) % 256;
    if (r < 0) r += 256;
    int64_t dt = r - 128;
    D[t * dstride] = (int8_t)dt;
    X = (X - dt) / 256; /* exact division */
  }
  D[0] = (int8_t)X;
}

/* Digits of A: V[t][i][k], t < p. */
void orc_s1_digits_a(int64_t M, int64_t K, const double* A, const int32_t* e,
                     int p, int8_t* V) {
  for (int64_t i = 0; i < M; ++i)
    for (int64_t k = 0; k < K; ++k)
      orc_digits(A[i * K + k], e[i], p, V + i * K + k, M * K);
}
/* Digits of B: W[t][k][j], t < p. */
void orc_s1_digits_b(int64_t K, int64_t N, const double* B, const int32_t* f,
                     int p, int8_t* W) {
  for (int64_t k = 0; k < K; ++k)
    for (int64_t j = 0; j < N; ++j)
      orc_digits(B[k * N + j], f[j], p, W + k * N + j, K * N);
}

/* Diagonal d = 0..p-1 of the triangular slice-pair sum (Eq. 2):
 * Cd[d][i][j] = sum_{t=0..d} sum_k V[t][i][k] * W[d-t][k][j]  (exact int64). */
void orc_s1_diagonals(int64_t M, int64_t N, int64_t K, int p, const int8_t* V,
                      const int8_t* W, int64_t* Cd) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j)
      for (int d = 0; d < p; ++d) {
        int64_t s = 0;
        for (int t = 0; t <= d; ++t) {
          const int8_t* Vt = V + (int64_t)t * M * K + i * K;
          const int8_t* Wu = W + (int64_t)(d - t) * K * N + j;
          for (int64_t k = 0; k < K; ++k) s += (int64_t)Vt[k] * (int64_t)Wu[k * N];
        }
        Cd[(int64_t)d * M * N + i * N + j] = s;
      }
}

/* BLAS-style update of one output: alpha*h if beta == 0 (C not read),
 * else fma(alpha, h, beta*c). */
static double orc_axpby(double alpha, double h, double beta, const double* c) {
  if (beta == 0.0) return alpha * h;
  double bc = beta * (*c);
  return fma(alpha, h, bc);
}

/* a b ~ 2^(e+f-12) sum_d 2^-8d C_d = 2^(e+f-12-8(p-1)) Z,
 * Z = sum_d 2^(8(p-1-d)) C_d. */
static int64_t orc_s1_scale(int e, int f, int p) {
  return (int64_t)e + f - 12 - 8 * (p - 1);
}

static double orc_s1_one(const int64_t* cd, int64_t stride, int p, int e, int f) {
  if (e == ORC_NONFINITE_EXP || f == ORC_NONFINITE_EXP) return NAN;
  if (e == ORC_ZERO_EXP || f == ORC_ZERO_EXP) return 0.0;
  i128 Z = 0;
  for (int d = 0; d < p; ++d)
    Z += (i128)cd[(int64_t)d * stride] * ((i128)1 << (8 * (p - 1 - d)));
  return orc_round_scaled(Z, orc_s1_scale(e, f, p));
}

/* Shift-reduce made exact (Eq. 3): Z = sum_d 2^(8(p-1-d)) Cd as a 128-bit
 * integer, then Chat = RN(Z 2^(e_i + f_j - 12 - 8(p-1))), then alpha/beta.
 * Non-finite rows of A or columns of B give NaN. */
void orc_s1_reconstruct(int64_t M, int64_t N, int p, const int64_t* Cd,
                        const int32_t* e, const int32_t* f, double alpha,
                        double beta, double* C) {
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double h = orc_s1_one(Cd + i * N + j, M * N, p, e[i], f[j]);
      C[i * N + j] = orc_axpby(alpha, h, beta, &C[i * N + j]);
    }
}

/* The 128-bit integer Z of every output (for checks), as two 64-bit words. */
void orc_s1_z(int64_t M, int64_t N, int p, const int64_t* Cd, int64_t* zlo,
              int64_t* zhi) {
  for (int64_t ij = 0; ij < M * N; ++ij) {
    i128 Z = 0;
    for (int d = 0; d < p; ++d)
      Z += (i128)Cd[(int64_t)d * M * N + ij] * ((i128)1 << (8 * (p - 1 - d)));
    zlo[ij] = (int64_t)(uint64_t)((u128)Z);
    zhi[ij] = (int64_t)(Z >> 64);
  }
}

/* Whole Scheme I DGEMM, C = alpha*A*B + beta*C, 1 <= p <= 8. */
int orc_s1_dgemm(int64_t M, int64_t N, int64_t K, int p, double alpha,
                 const double* A, const double* B, double beta, double* C) {
  if (p < 1 || p > 8) return -1;
  int32_t* e = (int32_t*)malloc(sizeof(int32_t) * (M > 0 ? M : 1));
  int32_t* f = (int32_t*)malloc(sizeof(int32_t) * (N > 0 ? N : 1));
  int8_t* V = (int8_t*)malloc((size_t)p * M * K + 1);
  int8_t* W = (int8_t*)malloc((size_t)p * K * N + 1);
  int64_t* Cd = (int64_t*)malloc(sizeof(int64_t) * ((size_t)p * M * N + 1));
  if (!e || !f || !V || !W || !Cd) {
    free(e); free(f); free(V); free(W); free(Cd);
    return -2;
  }
  orc_s1_row_exponents(M, K, A, e);
  orc_s1_col_exponents(K, N, B, f);
  orc_s1_digits_a(M, K, A, e, p, V);
  orc_s1_digits_b(K, N, B, f, p, W);
  orc_s1_diagonals(M, N, K, p, V, W, Cd);
  orc_s1_reconstruct(M, N, p, Cd, e, f, alpha, beta, C);
  free(e); free(f); free(V); free(W); free(Cd);
  return 0;
}

/* Scheme I on a sample of outputs (rows is[n], columns js[n]): the same
 * steps restricted to the entries asked for, so that large problems can be
 * checked entry by entry.  e, f are the full exponent vectors; cin holds the
 * old C values of the sampled entries (read only when beta != 0). */
void orc_s1_entries(int64_t M, int64_t N, int64_t K, int p, double alpha,
                    const double* A, const double* B, const int32_t* e,
                    const int32_t* f, int64_t n, const int64_t* is,
                    const int64_t* js, const double* cin, double beta,
                    double* out) {
  (void)M;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = is[s], j = js[s];
    int8_t va[8], wb[8];
    int64_t Cd[8] = {0};
    for (int64_t k = 0; k < K; ++k) {
      orc_digits(A[i * K + k], e[i], p, va, 1);
      orc_digits(B[k * N + j], f[j], p, wb, 1);
      for (int d = 0; d < p; ++d)
        for (int t = 0; t <= d; ++t) Cd[d] += (int64_t)va[t] * wb[d - t];
    }
    double h = orc_s1_one(Cd, 1, p, e[i], f[j]);
    out[s] = orc_axpby(alpha, h, beta, &cin[s]);
  }
}

/* Round-trip helper for tests: orc_round_scaled on Z = zhi*2^64 + zlo. */
double orc_round_scaled_parts(int64_t zlo, int64_t zhi, int64_t E) {
  i128 Z = ((i128)zhi << 64) | (i128)(uint64_t)zlo;
  return orc_round_scaled(Z, E);
}

/* ------------------------------------------------------------------ */
/* Scheme I with binary32 operands and result                          */
/* ------------------------------------------------------------------ */
/* The FP32-level operating points of Scheme I (the paper's low slice
 * counts, Sec. V-D) on binary32 matrices: every binary32 value is a binary64
 * value, so the operands are widened exactly and the exponents, slices,
 * diagonals and Z are those of the binary64 path; only the final rounding
 * differs: RN-even of Z 2^E to binary32 (24 significant bits, gradual
 * underflow at 2^-149, overflow to infinity), then alpha/beta in binary32. */

float orc_round_scaled_f32(i128 Z, int64_t E) {
  if (Z == 0) return 0.0f;
  int neg = Z < 0;
  u128 mag = neg ? (u128)0 - (u128)Z : (u128)Z;
  int n = 0;
  for (u128 t = mag; t != 0; t >>= 1) ++n;
  /* keep 24 significant bits, never below 2^-149 */
  int64_t drop = n - 24;
  if (-149 - E > drop) drop = -149 - E;
  u128 q;
  int64_t Eq = E;
  if (drop <= 0) {
    q = mag;
  } else if (drop > 128) {
    return neg ? -0.0f : 0.0f;
  } else if (drop == 128) {
    /* the kept part is 0; round up only above half = 2^127 */
    q = mag > ((u128)1 << 127) ? 1 : 0;
    Eq = E + drop;
  } else {
    u128 rem = mag & (((u128)1 << drop) - 1);
    u128 half = (u128)1 << (drop - 1);
    q = mag >> drop;
    if (rem > half || (rem == half && (q & 1))) q += 1;
    Eq = E + drop;
  }
  /* q <= 2^24 here; q 2^Eq is exact in binary32 unless it overflows */
  if (Eq > 300) return neg ? -INFINITY : INFINITY;
  float r = ldexpf((float)(uint64_t)q, (int)Eq);
  return neg ? -r : r;
}

float orc_round_scaled_f32_parts(int64_t zlo, int64_t zhi, int64_t E) {
  i128 Z = ((i128)zhi << 64) | (i128)(uint64_t)zlo;
  return orc_round_scaled_f32(Z, E);
}

static float orc_axpby_f32(float alpha, float h, float beta, const float* c) {
  if (beta == 0.0f) return alpha * h;
  float bc = beta * (*c);
  return fmaf(alpha, h, bc);
}

/* Whole Scheme I SGEMM, C = alpha*A*B + beta*C in binary32, 1 <= p <= 8. */
int orc_s1_sgemm(int64_t M, int64_t N, int64_t K, int p, float alpha,
                 const float* A, const float* B, float beta, float* C) {
  if (p < 1 || p > 8) return -1;
  double* Aw = (double*)malloc(sizeof(double) * ((size_t)M * K + 1));
  double* Bw = (double*)malloc(sizeof(double) * ((size_t)K * N + 1));
  int32_t* e = (int32_t*)malloc(sizeof(int32_t) * (M > 0 ? M : 1));
  int32_t* f = (int32_t*)malloc(sizeof(int32_t) * (N > 0 ? N : 1));
  int8_t* V = (int8_t*)malloc((size_t)p * M * K + 1);
  int8_t* W = (int8_t*)malloc((size_t)p * K * N + 1);
  int64_t* Cd = (int64_t*)malloc(sizeof(int64_t) * ((size_t)p * M * N + 1));
  if (!Aw || !Bw || !e || !f || !V || !W || !Cd) {
    free(Aw); free(Bw); free(e); free(f); free(V); free(W); free(Cd);
    return -2;
  }
  for (int64_t i = 0; i < M * K; ++i) Aw[i] = (double)A[i];
  for (int64_t i = 0; i < K * N; ++i) Bw[i] = (double)B[i];
  orc_s1_row_exponents(M, K, Aw, e);
  orc_s1_col_exponents(K, N, Bw, f);
  orc_s1_digits_a(M, K, Aw, e, p, V);
  orc_s1_digits_b(K, N, Bw, f, p, W);
  orc_s1_diagonals(M, N, K, p, V, W, Cd);
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      float h;
      if (e[i] == ORC_NONFINITE_EXP || f[j] == ORC_NONFINITE_EXP) {
        h = NAN;
      } else if (e[i] == ORC_ZERO_EXP || f[j] == ORC_ZERO_EXP) {
        h = 0.0f;
      } else {
        i128 Z = 0;
        for (int d = 0; d < p; ++d)
          Z += (i128)Cd[(int64_t)d * M * N + i * N + j] * ((i128)1 << (8 * (p - 1 - d)));
        h = orc_round_scaled_f32(Z, orc_s1_scale(e[i], f[j], p));
      }
      C[i * N + j] = orc_axpby_f32(alpha, h, beta, &C[i * N + j]);
    }
  free(Aw); free(Bw); free(e); free(f); free(V); free(W); free(Cd);
  return 0;
}
