// The plain-BF16 instantiations of the sample contraction (one bf16 product
// per term, the precision split) in a unit of their own, built with the MFMA
// accumulators in ordinary VGPRs; the BF16x3 ones stay in gemm.hip with
// theirs in AGPRs.  Everything else of gemm.hip is left out of this unit.
#define GNM_GEMM_PLAIN_UNIT
#include "gemm.hip"
