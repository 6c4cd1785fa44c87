// k_scan4.hip -- exhaustive FP32 top-k scan kernels for 4-bit first-level codes.
#include "k_scan_inst.h"

namespace lvq {

void *scan_kernel_b4(int bits2, int variant, int shape)
{
    ScanKernel k = nullptr;
    if (bits2 == 0) k = scan_lookup<4, 0>(variant, shape);
    else if (bits2 == 4) k = scan_lookup<4, 4>(variant, shape);
    else if (bits2 == 8) k = scan_lookup<4, 8>(variant, shape);
    return reinterpret_cast<void *>(k);
}

}  // namespace lvq
