// k_scan8.hip -- exhaustive FP32 top-k scan kernels for 8-bit first-level codes.
#include "k_scan_inst.h"

namespace lvq {

void *scan_kernel_b8(int bits2, int variant, int shape)
{
    ScanKernel k = nullptr;
    if (bits2 == 0) k = scan_lookup<8, 0>(variant, shape);
    else if (bits2 == 4) k = scan_lookup<8, 4>(variant, shape);
    else if (bits2 == 8) k = scan_lookup<8, 8>(variant, shape);
    return reinterpret_cast<void *>(k);
}

}  // namespace lvq
