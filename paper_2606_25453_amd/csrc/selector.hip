// Learned slice / modulus count selector and the tools it is trained with.
//
// The paper's implementation has no automatic precision selection (it names
// the runtime estimate of the slice count as missing, Sec. VI).  Here a small
// MLP predicts the smallest Scheme I slice count p and the smallest Scheme II
// modulus count s meeting a tolerance from exponent statistics gathered in
// the pre-pass, on the device, so that the emulated GEMM stays a
// stream-ordered, graph-capturable sequence:
//
//   k_sel_rows / k_sel_cols_*  row / column exponents (also the Scheme I scales)
//                            and histograms of the exponent deficits
//                            e_i - expo(a_ik) over 16 bins, plus the largest
//                            deficit (for the a-priori bound)
//   k_sel_infer              features -> MLP 34 -> 64 -> 64 -> 28 (ReLU) ->
//                            ordinal counts p_net = 1 + #{t : sigmoid(z_t) >
//                            thr_t} + margin over the 8 heads "p > t", s_net
//                            likewise over the 20 heads "s > t"; the a-priori
//                            bounds p_b, s_b; p = min(p_net, p_b) and s =
//                            min(s_net, s_b), or the bounds alone when the
//                            features are outside the training range; written
//                            to device memory
//   k_mlp_forward / k_mlp_grad / k_mlp_adam   training kernels (FP32)
//   k_ref_dd                 double-double dot products of chosen outputs
//                            (labels and accuracy measurement)
#include "ozk_device.hpp"
#include "ozk_internal.hpp"

namespace ozk {

constexpr int SEL_BINS = 16, SEL_FEAT = 34, SEL_H = 64, SEL_PH = 8, SEL_SH = 20, SEL_OUT = SEL_PH + SEL_SH;
static_assert(SEL_OUT == OZK_SELECTOR_HEADS, "head count");
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + SEL_FEAT * SEL_H, OFF_W2 = OFF_B1 + SEL_H,
              OFF_B2 = OFF_W2 + SEL_H * SEL_H, OFF_W3 = OFF_B2 + SEL_H, OFF_B3 = OFF_W3 + SEL_H * SEL_OUT,
              SEL_NPARAM = OFF_B3 + SEL_OUT;  // 8220
static_assert(SEL_NPARAM == OZK_SELECTOR_PARAMS, "parameter count");

// bins: [0] [1] [2] [3] [4,6) [6,8) [8,12) [12,16) [16,24) [24,32) [32,48)
// [48,64) [64,96) [96,128) [128,256) [256,inf)
__device__ __forceinline__ int deficit_bin(int d) {
  if (d < 4) return d;
  if (d < 8) return d < 6 ? 4 : 5;
  if (d < 16) return d < 12 ? 6 : 7;
  if (d < 32) return d < 24 ? 8 : 9;
  if (d < 64) return d < 48 ? 10 : 11;
  if (d < 128) return d < 96 ? 12 : 13;
  return d < 256 ? 14 : 15;
}

// counters: [0,16) A histogram, [16,32) B histogram, [32] max deficit of A,
// [33] max deficit of B.
__global__ void k_sel_zero(int32_t* __restrict__ cnt) {
  if (threadIdx.x < OZK_SELECTOR_COUNTERS) cnt[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_sel_fill(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Deficit histogram of one wave's 64 entries (valid lanes only), counted
// with one ballot per bin: the counts are wave-uniform and no lane waits on
// a shared counter (atomics on 16 bins serialise when most entries share a
// bin, as they do).
__device__ __forceinline__ void wave_bins(bool valid, int bin, int (&c)[SEL_BINS]) {
#pragma unroll
  for (int b = 0; b < SEL_BINS; ++b) c[b] += __popcll(__ballot(valid && bin == b));
}

// Per-wave counts into the block's shared bins, then one global add per bin.
__device__ __forceinline__ void flush_bins(const int (&c)[SEL_BINS], int dmax, int* h, int* md,
                                           int32_t* __restrict__ cnt_bins, int32_t* __restrict__ cnt_md) {
  const int lane = threadIdx.x & 63;
  if (lane < SEL_BINS) {
    int v = 0;
#pragma unroll
    for (int b = 0; b < SEL_BINS; ++b) v = lane == b ? c[b] : v;
    if (v) atomicAdd(&h[lane], v);
  }
  if (lane == 0 && dmax) atomicMax(md, dmax);
  __syncthreads();
  if (threadIdx.x < SEL_BINS && h[threadIdx.x]) atomicAdd(&cnt_bins[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 0 && *md) atomicMax(cnt_md, *md);
}

// One wave per row: the row exponent (written to e_out), then the deficit
// histogram of the row's nonzero entries.
// kc > 0: each wave keeps its row's entry exponents in kc int16 of dynamic
// LDS (K <= kc), so that the histogram pass reads them instead of the row.
__global__ __launch_bounds__(256) void k_sel_rows(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                  int64_t K, int32_t* __restrict__ e_out,
                                                  int32_t* __restrict__ cnt, int64_t kc) {
  extern __shared__ int16_t ecache[];
  __shared__ int h[SEL_BINS];
  __shared__ int md;
  if (threadIdx.x < SEL_BINS) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) md = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  int c[SEL_BINS] = {};
  int dmax = 0;
  if (r < rows) {  // wave-uniform
    const double* xr = X + r * ldx;
    const bool cached = kc > 0 && K <= kc;  // uniform
    int16_t* er = ecache + (cached ? (threadIdx.x >> 6) * kc : 0);
    int e = OZK_EXP_ZERO;
    if (cached) {
#pragma unroll 8
      for (int64_t k = lane; k < K; k += 64) {
        const int ek = expo_of(xr[k]);
        // finite exponents lie in [-1074, 1024]; a non-finite entry makes the
        // row's exponent non-finite, so its cached value is never read
        er[k] = (int16_t)(ek == OZK_EXP_ZERO ? -32768 : ek > 32767 ? 32767 : ek);
        e = ek > e ? ek : e;
      }
    } else {
#pragma unroll 8
      for (int64_t k = lane; k < K; k += 64) {
        const int ek = expo_of(xr[k]);
        e = ek > e ? ek : e;
      }
    }
    e = wave_max(e);
    if (lane == 0) e_out[r] = e;
    if (e != OZK_EXP_ZERO && e != OZK_EXP_NONFINITE) {
      for (int64_t k0 = 0; k0 < K; k0 += 256) {  // four loads in flight, then their bins
        int ek[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t k = k0 + 64 * u + lane;
          if (cached) {  // each lane reads back the entries it wrote
            const int c = k < K ? er[k] : -32768;
            ek[u] = c == -32768 ? OZK_EXP_ZERO : c;
          } else {
            ek[u] = k < K ? expo_of(xr[k < K ? k : 0]) : OZK_EXP_ZERO;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool valid = ek[u] != OZK_EXP_ZERO;
          const int d = e - ek[u];
          wave_bins(valid, deficit_bin(d), c);
          dmax = valid && d > dmax ? d : dmax;
        }
      }
    }
    dmax = wave_max(dmax);
  }
  flush_bins(c, dmax, h, &md, cnt, &cnt[32]);
}

// Columns, split over K so that every CU has work: pass 1 the column
// exponents (integer atomic max into f_out, filled with the zero sentinel
// first), pass 2 the deficit histogram against them.  A block covers 64
// columns x SEL_COL_KB rows (4 row groups, one column per lane).
constexpr int SEL_COL_KB = 128;

__global__ __launch_bounds__(256) void k_sel_cols_emax(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                       int64_t cols, int32_t* __restrict__ f_out) {
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (j >= cols) return;
  const int64_t k0 = (int64_t)blockIdx.y * SEL_COL_KB, k1 = k0 + SEL_COL_KB < K ? k0 + SEL_COL_KB : K;
  int e = OZK_EXP_ZERO;
#pragma unroll 8
  for (int64_t k = k0 + (threadIdx.x >> 6); k < k1; k += 4) {
    const int ek = expo_of(X[k * ldx + j]);
    e = ek > e ? ek : e;
  }
  if (e != OZK_EXP_ZERO) atomicMax(&f_out[j], e);
}

__global__ __launch_bounds__(256) void k_sel_cols_hist(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                       int64_t cols, const int32_t* __restrict__ f,
                                                       int32_t* __restrict__ cnt) {
  __shared__ int h[SEL_BINS];
  __shared__ int md;
  if (threadIdx.x < SEL_BINS) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) md = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int emax = j < cols ? f[j] : OZK_EXP_ZERO;
  const bool col_ok = j < cols && emax != OZK_EXP_ZERO && emax != OZK_EXP_NONFINITE;
  const int64_t k0 = (int64_t)blockIdx.y * SEL_COL_KB, k1 = k0 + SEL_COL_KB < K ? k0 + SEL_COL_KB : K;
  int c[SEL_BINS] = {};
  int dmax = 0;
  const int64_t jc = j < cols ? j : cols - 1;  // clamped: the loads need no condition
  for (int64_t kb = k0 + (threadIdx.x >> 6); kb < k1; kb += 16) {  // the same trip count in every lane of a wave
    int ek[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = kb + 4 * u;
      const int x = expo_of(X[(k < k1 ? k : k0) * ldx + jc]);
      ek[u] = col_ok && k < k1 ? x : OZK_EXP_ZERO;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool valid = ek[u] != OZK_EXP_ZERO;
      const int d = emax - ek[u];
      wave_bins(valid, deficit_bin(d), c);
      dmax = valid && d > dmax ? d : dmax;
    }
  }
  dmax = wave_max(dmax);
  flush_bins(c, dmax, h, &md, &cnt[SEL_BINS], &cnt[33]);
}

// A-priori componentwise error bound of Scheme I with p balanced slices for
// entries at most ra (rb) exponent steps below their row (column) maximum:
// rounding to 8p-2 bits (<= 2^-(8p-1) of the scale) on both operands, the
// dropped slice pairs (at most p-1 per diagonal d >= p, each below
// 128^2 2^(-12-8d)) and the final rounding 2^-53.
__device__ __forceinline__ double s1_bound(int p, int ra, int rb) {
  if (ra + rb + 2 > 1000) return __builtin_inf();
  double a = ldexp(1.0, -(8 * p - 1)) * (ldexp(1.0, ra + 1) + ldexp(1.0, rb + 1));
  a += ldexp(1.0, -2 * (8 * p - 1)) * ldexp(1.0, ra + rb + 2);
  a += (double)(p - 1) * 1.01 * ldexp(1.0, 2 - 8 * p) * ldexp(1.0, ra + rb + 2);
  return a + ldexp(1.0, -53);
}

// A-priori componentwise error bound of Scheme II with bit budgets ta, tb
// for entries at most ra (rb) steps below their row (column) maximum: the
// norm-bound scale exceeds the maximum by at most d = ceil(ceil(log2 K)/2),
// so truncation costs at most 2^(r+d+1-T) relative per operand; per product
// term the two relative errors and their product, plus the final rounding.
__device__ __forceinline__ double s2_bound(int ta, int tb, int ra, int rb, int64_t K) {
  int lk = 0;
  while (lk < 62 && ((int64_t)1 << lk) < K) ++lk;
  const int d = (lk + 1) / 2;
  const int ea = ra + d + 1 - ta, eb = rb + d + 1 - tb;
  if (ea > 1000 || eb > 1000 || ea + eb > 1000) return __builtin_inf();
  return ldexp(1.0, ea) + ldexp(1.0, eb) + ldexp(1.0, ea + eb) + ldexp(1.0, -53);
}

struct SelInfer {
  const float* w;  // device parameters, null = no network (bound only)
  float thr[SEL_OUT];  // per-head decision thresholds
  int margin;
  double tol;
  int64_t K;
  S2Budgets bud;   // Scheme II bit budgets per modulus count
};

// out[0] Scheme I slice count used (0 when Scheme II is chosen), [1] p from
// the network (0 if none), [2] p from the bound (9 = none up to 8), [3] 1 when
// the features were outside the training range, [4] scheme (1 or 2),
// [5] Scheme II modulus count used (0 with Scheme I), [6] s from the Scheme II
// bound (21 = none up to 20), [7] s from the network (0 if none).
__global__ __launch_bounds__(64) void k_sel_infer(const int32_t* __restrict__ cnt, SelInfer si,
                                                  int32_t* __restrict__ out, float* __restrict__ feat_out) {
  __shared__ float x[SEL_FEAT], h1[SEL_H], h2[SEL_H], z[SEL_OUT];
  __shared__ float tot[2];
  const int t = threadIdx.x;
  if (t < 2) {
    long long n = 0;
    for (int i = 0; i < SEL_BINS; ++i) n += cnt[t * SEL_BINS + i];
    tot[t] = (float)n;
  }
  __syncthreads();
  if (t < 2 * SEL_BINS) {
    const float n = tot[t / SEL_BINS];
    x[t] = n > 0.f ? (float)cnt[t] / n : 0.f;
  }
  if (t == 0) {
    x[32] = (float)(log2((double)(si.K > 0 ? si.K : 1)) / 14.0);
    x[33] = (float)(-log10(si.tol) / 16.0);
  }
  __syncthreads();
  if (feat_out && t < SEL_FEAT) feat_out[t] = x[t];
  int p_net = 0, s_net = 0;
  if (si.w) {
    float a = si.w[OFF_B1 + t];
    for (int i = 0; i < SEL_FEAT; ++i) a += si.w[OFF_W1 + i * SEL_H + t] * x[i];
    h1[t] = a > 0.f ? a : 0.f;
    __syncthreads();
    a = si.w[OFF_B2 + t];
    for (int i = 0; i < SEL_H; ++i) a += si.w[OFF_W2 + i * SEL_H + t] * h1[i];
    h2[t] = a > 0.f ? a : 0.f;
    __syncthreads();
    if (t < SEL_OUT) {
      a = si.w[OFF_B3 + t];
      for (int i = 0; i < SEL_H; ++i) a += si.w[OFF_W3 + i * SEL_OUT + t] * h2[i];
      z[t] = a;
    }
    __syncthreads();
    int cp = 0, cs = 0;
    for (int i = 0; i < SEL_PH; ++i) cp += (1.f / (1.f + expf(-z[i]))) > si.thr[i] ? 1 : 0;
    for (int i = SEL_PH; i < SEL_OUT; ++i) cs += (1.f / (1.f + expf(-z[i]))) > si.thr[i] ? 1 : 0;
    p_net = 1 + cp + si.margin;
    p_net = p_net > 9 ? 9 : p_net;
    s_net = 1 + cs + si.margin;
    s_net = s_net > OZK_MAX_S + 1 ? OZK_MAX_S + 1 : s_net;
  }
  if (t == 0) {
    int pb = 9;
    for (int p = 1; p <= 8; ++p)
      if (s1_bound(p, cnt[32], cnt[33]) <= si.tol) {
        pb = p;
        break;
      }
    // outside the training range: K beyond 2^14, tolerance outside
    // [1e-16, 1e-5], or mass in the last deficit bin
    const bool ood = si.K > 16384 || si.tol < 1e-16 || si.tol > 1e-5 || x[15] > 0.f || x[31] > 0.f;
    int p = pb;
    if (si.w && !ood) p = p_net < pb ? p_net : pb;
    int sb = OZK_MAX_S + 1;
    for (int q = 1; q <= OZK_MAX_S; ++q)
      if (s2_bound(si.bud.ta[q], si.bud.tb[q], cnt[32], cnt[33], si.K) <= si.tol) {
        sb = q;
        break;
      }
    int sc = sb;
    if (si.w && !ood) sc = s_net < sb ? s_net : sb;
    // Scheme I while p <= 8 meets the tolerance; otherwise Scheme II at
    // min(s_net, s_bound) (s = 20, the most accurate, when nothing is proven)
    const bool s1 = p <= OZK_MAX_P;
    p = p < 1 ? 1 : (p > OZK_MAX_P ? OZK_MAX_P : p);
    out[0] = s1 ? p : 0;
    out[1] = p_net;
    out[2] = pb;
    out[3] = ood ? 1 : 0;
    out[4] = s1 ? 1 : 2;
    out[5] = s1 ? 0 : (sc <= OZK_MAX_S ? (sc < 1 ? 1 : sc) : OZK_MAX_S);
    out[6] = sb;
    out[7] = s_net;
  }
}

// ----------------------------------------- automatic complex product (3M)
//
// The largest exponent deficit of a nonzero real or imaginary part below
// the largest part exponent of its row of A (column of B); rows and columns
// holding a non-finite part are skipped (their outputs are NaN whatever s).

// One wave per row of complex A (its 2K parts are contiguous).
__global__ __launch_bounds__(256) void k_zsel_rows(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                   int64_t K, int32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;  // wave-uniform
  const double* xr = X + 2 * r * ldx;
  const int64_t n = 2 * K;
  int e = OZK_EXP_ZERO;
  for (int64_t k = lane; k < n; k += 64) {
    const int ek = expo_of(xr[k]);
    e = ek > e ? ek : e;
  }
  e = wave_max(e);
  if (e == OZK_EXP_ZERO || e == OZK_EXP_NONFINITE) return;
  int dmax = 0;
  for (int64_t k = lane; k < n; k += 64) {
    const int ek = expo_of(xr[k]);
    if (ek != OZK_EXP_ZERO && e - ek > dmax) dmax = e - ek;
  }
  dmax = wave_max(dmax);
  if (lane == 0 && dmax) atomicMax(&cnt[32], dmax);
}

// Column maxima of the part exponents of complex B, split over K.
__global__ __launch_bounds__(256) void k_zsel_cols_emax(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                        int64_t cols, int32_t* __restrict__ f) {
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (j >= cols) return;
  const int64_t k0 = (int64_t)blockIdx.y * SEL_COL_KB, k1 = k0 + SEL_COL_KB < K ? k0 + SEL_COL_KB : K;
  int e = OZK_EXP_ZERO;
  for (int64_t k = k0 + (threadIdx.x >> 6); k < k1; k += 4) {
    const double* z = X + 2 * (k * ldx + j);
    const int a = expo_of(z[0]), b = expo_of(z[1]);
    e = a > e ? a : e;
    e = b > e ? b : e;
  }
  if (e != OZK_EXP_ZERO) atomicMax(&f[j], e);
}

__global__ __launch_bounds__(256) void k_zsel_cols_dmax(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                        int64_t cols, const int32_t* __restrict__ f,
                                                        int32_t* __restrict__ cnt) {
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int emax = j < cols ? f[j] : OZK_EXP_ZERO;
  int dmax = 0;
  if (j < cols && emax != OZK_EXP_ZERO && emax != OZK_EXP_NONFINITE) {
    const int64_t k0 = (int64_t)blockIdx.y * SEL_COL_KB, k1 = k0 + SEL_COL_KB < K ? k0 + SEL_COL_KB : K;
    for (int64_t k = k0 + (threadIdx.x >> 6); k < k1; k += 4) {
      const double* z = X + 2 * (k * ldx + j);
      const int a = expo_of(z[0]), b = expo_of(z[1]);
      if (a != OZK_EXP_ZERO && emax - a > dmax) dmax = emax - a;
      if (b != OZK_EXP_ZERO && emax - b > dmax) dmax = emax - b;
    }
  }
  dmax = wave_max(dmax);
  if ((threadIdx.x & 63) == 0 && dmax) atomicMax(&cnt[33], dmax);
}

// The decision of the automatic ZGEMM: Scheme II (3M) at the smallest s
// whose a-priori bound meets tol, with the deficits one more than the part
// deficits (the scales are taken from |re| + |im| < 2^(max(expo re, expo
// im) + 1)); s = 20 when none is proven.  info as k_sel_infer writes it,
// with no network: [1] 0, [2] 9, [7] 0.
__global__ void k_zsel_decide(const int32_t* __restrict__ cnt, double tol, int64_t K, S2Budgets bud,
                              int32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  int sb = OZK_MAX_S + 1;
  for (int q = 1; q <= OZK_MAX_S; ++q)
    if (s2_bound(bud.ta[q], bud.tb[q], cnt[32] + 1, cnt[33] + 1, K) <= tol) {
      sb = q;
      break;
    }
  out[0] = 0;
  out[1] = 0;
  out[2] = 9;
  out[3] = 0;
  out[4] = 2;
  out[5] = sb <= OZK_MAX_S ? sb : OZK_MAX_S;
  out[6] = sb;
  out[7] = 0;
}

// ------------------------------------------------------------- training

__device__ __forceinline__ void mlp_layers(const float* __restrict__ w, const float* __restrict__ xin, float* x,
                                           float* z1, float* h1, float* z2, float* h2, float* out) {
  const int t = threadIdx.x;
  if (t < SEL_FEAT) x[t] = xin[t];
  __syncthreads();
  float a = w[OFF_B1 + t];
  for (int i = 0; i < SEL_FEAT; ++i) a += w[OFF_W1 + i * SEL_H + t] * x[i];
  z1[t] = a;
  h1[t] = a > 0.f ? a : 0.f;
  __syncthreads();
  a = w[OFF_B2 + t];
  for (int i = 0; i < SEL_H; ++i) a += w[OFF_W2 + i * SEL_H + t] * h1[i];
  z2[t] = a;
  h2[t] = a > 0.f ? a : 0.f;
  __syncthreads();
  if (t < SEL_OUT) {
    a = w[OFF_B3 + t];
    for (int i = 0; i < SEL_H; ++i) a += w[OFF_W3 + i * SEL_OUT + t] * h2[i];
    out[t] = a;
  }
  __syncthreads();
}

// One block of 64 threads per sample.
__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ w, const float* __restrict__ X, int n,
                                                    float* __restrict__ logits) {
  __shared__ float x[SEL_FEAT], z1[SEL_H], h1[SEL_H], z2[SEL_H], h2[SEL_H], out[SEL_OUT];
  const int s = blockIdx.x;
  if (s >= n) return;
  mlp_layers(w, X + (int64_t)s * SEL_FEAT, x, z1, h1, z2, h2, out);
  if (threadIdx.x < SEL_OUT) logits[(int64_t)s * SEL_OUT + threadIdx.x] = out[threadIdx.x];
}

// Gradient of the mean binary cross-entropy over samples and the 28 ordinal
// heads, accumulated into grad (zeroed beforehand); loss sum into *loss.
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ w, const float* __restrict__ X,
                                                 const float* __restrict__ Y, int n, float* __restrict__ grad,
                                                 float* __restrict__ loss) {
  __shared__ float x[SEL_FEAT], z1[SEL_H], h1[SEL_H], z2[SEL_H], h2[SEL_H], out[SEL_OUT];
  __shared__ float go[SEL_OUT], gz2[SEL_H];
  const int s = blockIdx.x, t = threadIdx.x;
  if (s >= n) return;
  mlp_layers(w, X + (int64_t)s * SEL_FEAT, x, z1, h1, z2, h2, out);
  const float scale = 1.f / ((float)n * SEL_OUT);
  if (t < SEL_OUT) {
    const float y = Y[(int64_t)s * SEL_OUT + t], zz = out[t];
    const float sg = 1.f / (1.f + expf(-zz));
    go[t] = (sg - y) * scale;
    const float l = fmaxf(zz, 0.f) - zz * y + log1pf(expf(-fabsf(zz)));
    atomicAdd(loss, l * scale);
    atomicAdd(&grad[OFF_B3 + t], go[t]);
  }
  __syncthreads();
  // layer 3 weights and the gradient at z2 (thread t = hidden unit)
  float gh2 = 0.f;
  for (int o = 0; o < SEL_OUT; ++o) {
    atomicAdd(&grad[OFF_W3 + t * SEL_OUT + o], h2[t] * go[o]);
    gh2 += w[OFF_W3 + t * SEL_OUT + o] * go[o];
  }
  gz2[t] = z2[t] > 0.f ? gh2 : 0.f;
  __syncthreads();
  atomicAdd(&grad[OFF_B2 + t], gz2[t]);
  for (int i = 0; i < SEL_H; ++i) atomicAdd(&grad[OFF_W2 + i * SEL_H + t], h1[i] * gz2[t]);
  // gradient at z1 (thread t = layer-1 unit)
  float gh1 = 0.f;
  for (int j = 0; j < SEL_H; ++j) gh1 += w[OFF_W2 + t * SEL_H + j] * gz2[j];
  const float gz1 = z1[t] > 0.f ? gh1 : 0.f;
  atomicAdd(&grad[OFF_B1 + t], gz1);
  for (int i = 0; i < SEL_FEAT; ++i) atomicAdd(&grad[OFF_W1 + i * SEL_H + t], x[i] * gz1);
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Adam with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_mlp_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int n, float lr, float beta1, float beta2, float eps, float c1,
                           float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mi = beta1 * m[i] + (1.f - beta1) * g[i];
  const float vi = beta2 * v[i] + (1.f - beta2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------- double-double reference

__device__ __forceinline__ void dd_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Thread per chosen output (rows[i], cols[i]): hi + lo ~ sum_k a b with
// error-free products and sums, absab = sum_k |a||b|.
__global__ __launch_bounds__(256) void k_ref_dd(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                                int64_t lda, const double* __restrict__ B, int64_t ldb, int64_t n,
                                                const int64_t* __restrict__ rows, const int64_t* __restrict__ cols,
                                                double* __restrict__ hi, double* __restrict__ lo,
                                                double* __restrict__ absab) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int64_t i = rows[idx], j = cols[idx];
  if (i < 0 || i >= M || j < 0 || j >= N) {  // an index outside the matrix gives NaN
    hi[idx] = lo[idx] = absab[idx] = __builtin_nan("");
    return;
  }
  double h = 0.0, l = 0.0, ab = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double a = A[i * lda + k], b = B[k * ldb + j];
    const double p = a * b;
    const double pe = __fma_rn(a, b, -p);
    double s, e;
    dd_two_sum(h, p, s, e);
    e += l + pe;
    h = s + e;
    l = e - (h - s);
    ab += fabs(a) * fabs(b);
  }
  hi[idx] = h;
  lo[idx] = l;
  absab[idx] = ab;
}

// ------------------------------------------------------------ launchers

hipError_t sel_features(const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb, int64_t N, int64_t K,
                        int32_t* e, int32_t* f, int32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_sel_zero, dim3(1), dim3(64), 0, st, cnt);
  if (M > 0) {
    // the row exponents cached in LDS for K <= 4096 (32 KB per block of four rows)
    const int64_t kc = K > 0 && K <= 4096 ? K : 0;
    static std::atomic<uint64_t> lds_done{0};
    if (kc) {
      const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(k_sel_rows), 4 * 4096 * 2, lds_done);
      if (e_lds != hipSuccess) return e_lds;
    }
    hipLaunchKernelGGL(k_sel_rows, dim3((unsigned)((M + 3) / 4)), dim3(256), (unsigned)(4 * kc * 2), st, A, lda, M,
                       K, e, cnt, kc);
  }
  if (N > 0) {
    hipLaunchKernelGGL(k_sel_fill, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, f, N, (int32_t)OZK_EXP_ZERO);
    if (K > 0) {
      const dim3 g((unsigned)((N + 63) / 64), (unsigned)((K + SEL_COL_KB - 1) / SEL_COL_KB));
      hipLaunchKernelGGL(k_sel_cols_emax, g, dim3(256), 0, st, B, ldb, K, N, f);
      hipLaunchKernelGGL(k_sel_cols_hist, g, dim3(256), 0, st, B, ldb, K, N, f, cnt);
    }
  }
  return hipGetLastError();
}

hipError_t sel_infer(const int32_t* cnt, const float* w, const float* thresholds, int margin, double tol, int64_t K,
                     int32_t* info, float* feat, hipStream_t st) {
  SelInfer si;
  si.w = w;
  for (int i = 0; i < SEL_OUT; ++i) si.thr[i] = thresholds ? thresholds[i] : 0.5f;
  si.margin = margin;
  si.tol = tol;
  si.K = K;
  si.bud = s2_budgets();
  hipLaunchKernelGGL(k_sel_infer, dim3(1), dim3(64), 0, st, cnt, si, info, feat);
  return hipGetLastError();
}

hipError_t zsel_features(const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb, int64_t N, int64_t K,
                         int32_t* f_scratch, int32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_sel_zero, dim3(1), dim3(64), 0, st, cnt);
  if (M > 0 && K > 0) hipLaunchKernelGGL(k_zsel_rows, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, st, A, lda, M, K, cnt);
  if (N > 0 && K > 0) {
    hipLaunchKernelGGL(k_sel_fill, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, f_scratch, N,
                       (int32_t)OZK_EXP_ZERO);
    const dim3 g((unsigned)((N + 63) / 64), (unsigned)((K + SEL_COL_KB - 1) / SEL_COL_KB));
    hipLaunchKernelGGL(k_zsel_cols_emax, g, dim3(256), 0, st, B, ldb, K, N, f_scratch);
    hipLaunchKernelGGL(k_zsel_cols_dmax, g, dim3(256), 0, st, B, ldb, K, N, f_scratch, cnt);
  }
  return hipGetLastError();
}

hipError_t zsel_decide(const int32_t* cnt, double tol, int64_t K, int32_t* info, hipStream_t st) {
  hipLaunchKernelGGL(k_zsel_decide, dim3(1), dim3(64), 0, st, cnt, tol, K, s2_budgets(), info);
  return hipGetLastError();
}

hipError_t mlp_forward(const float* w, const float* X, int n, float* logits, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)n), dim3(64), 0, st, w, X, n, logits);
  return hipGetLastError();
}

hipError_t mlp_grad(const float* w, const float* X, const float* Y, int n, float* grad, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f32, dim3((SEL_NPARAM + 255) / 256), dim3(256), 0, st, grad, (int64_t)SEL_NPARAM, 0.f);
  hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, st, loss, (int64_t)1, 0.f);
  if (n > 0) hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)n), dim3(64), 0, st, w, X, Y, n, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, const float* g, float* m, float* v, int step, float lr, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((SEL_NPARAM + 255) / 256), dim3(256), 0, st, w, g, m, v, SEL_NPARAM, lr, b1,
                     b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t ref_dd(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb,
                  int64_t n, const int64_t* rows, const int64_t* cols, double* hi, double* lo, double* absab,
                  hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_ref_dd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, N, K, A, lda, B, ldb, n,
                       rows, cols, hi, lo, absab);
  return hipGetLastError();
}

}  // namespace ozk
