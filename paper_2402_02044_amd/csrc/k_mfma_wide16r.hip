// k_mfma_wide16r.hip -- bf16 / fp16 instantiations of the queries-in-LDS
// matrix-core scan (k_mfma_wide_impl.h) at both levels: the codes and the
// 8-bit residual codes each converted exactly to the query type, in two
// accumulator chains (v_mfma_f32_32x32x16), any mean count whose c_m table
// fits.
#include "k_mfma_wide_impl.h"

namespace lvq {
namespace {

// Two 32-query blocks per workgroup and one 32-row block per wave, so that
// both chains' accumulators fit a wave's registers.
template <int B1, int PREC>
WideKernel lookup_16r(int kpos, int *qb, int *rb)
{
    *qb = 2;
    *rb = 1;
    switch (kpos) {
    case 96: return B1 == 8 ? k_scan_mfma_wide<8, 8, 96, 2, 1, PREC> : nullptr;
    case 128: return k_scan_mfma_wide<B1, 8, 128, 2, 1, PREC>;
    case 256: return k_scan_mfma_wide<B1, 8, 256, 2, 1, PREC>;
    case 384: return k_scan_mfma_wide<B1, 8, 384, 2, 1, PREC>;
    case 512: return k_scan_mfma_wide<B1, 8, 512, 2, 1, PREC>;
    case 768: return k_scan_mfma_wide<B1, 8, 768, 2, 1, PREC>;
    case 1024: return k_scan_mfma_wide<B1, 8, 1024, 2, 1, PREC>;
    default: return nullptr;
    }
}

}  // namespace

WideKernel wide_kernel_16r(int bits1, int kpos, int prec, int *qb, int *rb)
{
    if (prec == LVQ_BF16) return bits1 == 8 ? lookup_16r<8, LVQ_BF16>(kpos, qb, rb) : lookup_16r<4, LVQ_BF16>(kpos, qb, rb);
    if (prec == LVQ_FP16) return bits1 == 8 ? lookup_16r<8, LVQ_FP16>(kpos, qb, rb) : lookup_16r<4, LVQ_FP16>(kpos, qb, rb);
    return nullptr;
}

}  // namespace lvq
