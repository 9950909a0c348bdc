// Single-instance sweep launcher, double output: one workgroup of kSweepWaves
// waves, R = ceil(P / 16) <= 13 for P <= 208.
#include "sweep.hpp"

namespace gnm {

hipError_t launch_sweep(int P, int npiv, int mode, const double* M, double* inv_out, int64_t ldo,
                        double* dir_out, int32_t* status, int fail_code, hipStream_t st,
                        const double* post, int64_t ldp) {
  const int R = (P + kSweepTD - 1) / kSweepTD;
#define GNM_SWEEP_CASE(RR)                                                                        \
  case RR:                                                                                        \
    hipLaunchKernelGGL((sweep_kernel<RR, double>), dim3(1), dim3(kSweepThreads), 0, st, M, P, \
                       npiv, mode, inv_out, ldo, dir_out, status, fail_code, post, ldp);          \
    break;
  switch (R) {
    GNM_SWEEP_CASE(1) GNM_SWEEP_CASE(2) GNM_SWEEP_CASE(3) GNM_SWEEP_CASE(4) GNM_SWEEP_CASE(5)
    GNM_SWEEP_CASE(6) GNM_SWEEP_CASE(7) GNM_SWEEP_CASE(8) GNM_SWEEP_CASE(9) GNM_SWEEP_CASE(10)
    GNM_SWEEP_CASE(11) GNM_SWEEP_CASE(12) GNM_SWEEP_CASE(13)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_SWEEP_CASE
  return hipGetLastError();
}

}  // namespace gnm
