// Instantiations of the Scheme I GEMM launchers.  The build compiles this
// file once per slice count with -DOZK_S1_P=p so that the kernels of the
// eight slice counts compile in parallel; without the macro it instantiates
// all of them.
#include "s1_gemm.hpp"

namespace ozk {

#ifdef OZK_S1_P
template hipError_t s1_gemm_launch<OZK_S1_P>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
#else
template hipError_t s1_gemm_launch<1>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<2>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<3>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<4>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<5>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<6>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<7>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
template hipError_t s1_gemm_launch<8>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
#endif

}  // namespace ozk
