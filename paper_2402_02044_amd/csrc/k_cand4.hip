// k_cand4.hip -- candidate-list similarity kernels for 4-bit first-level codes.
#include "k_cand_inst.h"

namespace lvq {

void *cand_kernel_b4(int bits2, int variant, int shape)
{
    CandKernel k = nullptr;
    if (bits2 == 0) k = cand_lookup<4, 0>(variant, shape);
    else if (bits2 == 4) k = cand_lookup<4, 4>(variant, shape);
    else if (bits2 == 8) k = cand_lookup<4, 8>(variant, shape);
    return reinterpret_cast<void *>(k);
}

}  // namespace lvq
