// Batched sweep launcher, MODE 0 (G^{-1} from Gsum): one item per instance, R =
// ceil(P / 16) <= 11 (P <= 161 with N <= 80).
#include "sweep.hpp"

namespace gnm {

hipError_t launch_batch_sweep_mode0(int R, const BatchInst* inst, const BatchLaunch& L,
                                     hipStream_t st) {
#define GNM_BS_CASE(RR)                                                                        \
  case RR:                                                                                     \
    hipLaunchKernelGGL((batch_sweep_kernel<RR, 0>), dim3(L.blocks), dim3(kSweepThreads), \
                       0, st, inst, L);                                                        \
    break;
  switch (R) {
    GNM_BS_CASE(1) GNM_BS_CASE(2) GNM_BS_CASE(3) GNM_BS_CASE(4) GNM_BS_CASE(5) GNM_BS_CASE(6)
    GNM_BS_CASE(7) GNM_BS_CASE(8) GNM_BS_CASE(9) GNM_BS_CASE(10) GNM_BS_CASE(11)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_BS_CASE
  return hipGetLastError();
}

}  // namespace gnm
