// k_mfma_full.hip -- matrix-core scan instantiations at both levels
// (first-level codes plus 8-bit residual codes, Sec. 2.3).
#include "k_mfma_impl.h"

namespace lvq {

MfmaKernelPtr mfma_kernel_full(int bits1, int kpos, int fp16, int *qb)
{
    if (bits1 == 8) return fp16 ? (MfmaKernelPtr)mfma_lookup<8, 8, true>(kpos, qb) : (MfmaKernelPtr)mfma_lookup<8, 8, false>(kpos, qb);
    if (bits1 == 4) return fp16 ? (MfmaKernelPtr)mfma_lookup<4, 8, true>(kpos, qb) : (MfmaKernelPtr)mfma_lookup<4, 8, false>(kpos, qb);
    return nullptr;
}

}  // namespace lvq
