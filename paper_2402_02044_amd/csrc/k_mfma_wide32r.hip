// k_mfma_wide32r.hip -- FP32 instantiations of the queries-in-LDS matrix-core
// scan (k_mfma_wide_impl.h), both levels: FP32 queries times Delta c1 +
// Delta2 c2 (8-bit residual codes) decoded per lane, on v_mfma_f32_32x32x2_f32.
#include "k_mfma_wide_impl.h"

namespace lvq {

// 32-query blocks per workgroup: two, or one where the FP32 query fragments
// of two would not fit the LDS (at most 128 KB); more would not fit the
// registers.
WideKernel wide_kernel_f32r(int bits1, int kpos, int *qb, int *rb)
{
    *rb = 2;
    if (bits1 == 8) {
        switch (kpos) {
        case 96: *qb = 2; return k_scan_mfma_wide<8, 8, 96, 2, 2, LVQ_FP32>;
        case 128: *qb = 2; return k_scan_mfma_wide<8, 8, 128, 2, 2, LVQ_FP32>;
        case 256: *qb = 2; return k_scan_mfma_wide<8, 8, 256, 2, 2, LVQ_FP32>;
        case 384: *qb = 2; return k_scan_mfma_wide<8, 8, 384, 2, 2, LVQ_FP32>;
        case 512: *qb = 2; return k_scan_mfma_wide<8, 8, 512, 2, 2, LVQ_FP32>;
        case 768: *qb = 1; return k_scan_mfma_wide<8, 8, 768, 1, 2, LVQ_FP32>;
        case 1024: *qb = 1; return k_scan_mfma_wide<8, 8, 1024, 1, 2, LVQ_FP32>;
        default: return nullptr;
        }
    }
    if (bits1 == 4) {
        switch (kpos) {
        case 128: *qb = 2; return k_scan_mfma_wide<4, 8, 128, 2, 2, LVQ_FP32>;
        case 256: *qb = 2; return k_scan_mfma_wide<4, 8, 256, 2, 2, LVQ_FP32>;
        case 384: *qb = 2; return k_scan_mfma_wide<4, 8, 384, 2, 2, LVQ_FP32>;
        case 512: *qb = 2; return k_scan_mfma_wide<4, 8, 512, 2, 2, LVQ_FP32>;
        case 768: *qb = 1; return k_scan_mfma_wide<4, 8, 768, 1, 2, LVQ_FP32>;
        case 1024: *qb = 1; return k_scan_mfma_wide<4, 8, 1024, 1, 2, LVQ_FP32>;
        default: return nullptr;
        }
    }
    return nullptr;
}

}  // namespace lvq
