// k_cand8.hip -- candidate-list similarity kernels for 8-bit first-level codes.
#include "k_cand_inst.h"

namespace lvq {

void *cand_kernel_b8(int bits2, int variant, int shape)
{
    CandKernel k = nullptr;
    if (bits2 == 0) k = cand_lookup<8, 0>(variant, shape);
    else if (bits2 == 4) k = cand_lookup<8, 4>(variant, shape);
    else if (bits2 == 8) k = cand_lookup<8, 8>(variant, shape);
    return reinterpret_cast<void *>(k);
}

}  // namespace lvq
