// Asynchronous condition flags of a context: kernels that OR condition bits
// into the context's device flag word after a call's pre-pass or decision,
// and the atomic read-and-clear behind ozk_get_flags.
//
//   k_flag_nonfinite   a row or column scale vector holds the non-finite
//                      sentinel (an input row of A or column of B with a NaN
//                      or an infinity)
//   k_flag_batch       the same over every problem of a batch
//   k_flag_decision    the conditions of an automatic decision (info vector)
//   k_flag_take        flags -> out, flags = 0, in one atomic exchange
#include <hip/hip_runtime.h>

#include "ozk_internal.hpp"

namespace ozk {

namespace {

constexpr int FLAG_BLOCK = 256;

__device__ __forceinline__ void or_if_any(bool hit, uint32_t bit, uint32_t* flags) {
  // one atomic per wave that saw the condition, from its first such lane
  const unsigned long long m = __ballot(hit);
  if (m != 0 && (int)(threadIdx.x & (warpSize - 1)) == __ffsll(m) - 1) atomicOr(flags, bit);
}

__global__ __launch_bounds__(FLAG_BLOCK) void k_flag_nonfinite(const int32_t* __restrict__ a, int64_t na,
                                                                const int32_t* __restrict__ b, int64_t nb,
                                                                uint32_t* __restrict__ flags) {
  bool hit = false;
  const int64_t stride = (int64_t)gridDim.x * FLAG_BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * FLAG_BLOCK + threadIdx.x; i < na + nb; i += stride)
    hit |= (i < na ? a[i] : b[i - na]) == OZK_EXP_NONFINITE;
  or_if_any(hit, OZK_FLAG_NONFINITE, flags);
}

// One workgroup per problem: its scale vectors sit at offsets of the workspace.
__global__ __launch_bounds__(FLAG_BLOCK) void k_flag_batch(const BatchProb* __restrict__ prob, int count,
                                                            const int8_t* __restrict__ ws, uint32_t* __restrict__ flags) {
  const int q = blockIdx.x;
  if (q >= count) return;
  const BatchProb& pr = prob[q];
  if (pr.M <= 0 || pr.N <= 0) return;
  const int32_t* sig = (const int32_t*)(ws + pr.off_sig);
  const int32_t* tau = (const int32_t*)(ws + pr.off_tau);
  bool hit = false;
  for (int64_t i = threadIdx.x; i < pr.M + pr.N; i += FLAG_BLOCK)
    hit |= (i < pr.M ? sig[i] : tau[i - pr.M]) == OZK_EXP_NONFINITE;
  or_if_any(hit, OZK_FLAG_NONFINITE, flags);
}

// info: [1] p_net (0 without a network), [3] out of range, [4] scheme,
// [6] s_bound (OZK_MAX_S + 1 when no modulus count is proven enough).
__global__ void k_flag_decision(const int32_t* __restrict__ info, uint32_t* __restrict__ flags) {
  if (threadIdx.x != 0) return;
  uint32_t f = 0;
  if (info[1] == 0 || info[3] != 0) f |= OZK_FLAG_SELECTOR_FALLBACK;
  if (info[4] == 2) f |= OZK_FLAG_SCHEME2_CHOSEN;
  if (info[4] == 2 && info[6] > OZK_MAX_S) f |= OZK_FLAG_S_UNPROVEN;
  if (f) atomicOr(flags, f);
}

__global__ void k_flag_take(uint32_t* __restrict__ flags, uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = atomicExch(flags, 0u);
}

}  // namespace

hipError_t flag_nonfinite(const int32_t* a, int64_t na, const int32_t* b, int64_t nb, uint32_t* flags,
                          hipStream_t st) {
  const int64_t n = na + nb;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + FLAG_BLOCK - 1) / FLAG_BLOCK;
  hipLaunchKernelGGL(k_flag_nonfinite, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(FLAG_BLOCK), 0, st, a,
                     na, b, nb, flags);
  return hipGetLastError();
}

hipError_t flag_batch(const BatchDev& bd, const int8_t* ws, uint32_t* flags, hipStream_t st) {
  if (bd.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flag_batch, dim3((unsigned)bd.count), dim3(FLAG_BLOCK), 0, st, bd.prob, bd.count, ws, flags);
  return hipGetLastError();
}

hipError_t flag_decision(const int32_t* info, uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_decision, dim3(1), dim3(64), 0, st, info, flags);
  return hipGetLastError();
}

hipError_t flag_take(uint32_t* flags, uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_take, dim3(1), dim3(64), 0, st, flags, out);
  return hipGetLastError();
}

}  // namespace ozk
