// k_cand_inst.h -- instantiation table of k_cand for one first-level width.
// Included by k_cand4.hip / k_cand8.hip with LVQ_CAND_B1 defined.
#pragma once

#include "k_cand_impl.h"

namespace lvq {

// (lanes per candidate, bytes per piece, pieces per lane and round)
using CandShape = TileShape;
constexpr CandShape kCandShapes[] = {
    {16, 16, 4},  // generic: 1024 code bytes per round
    {16, 8, 3},   // 384 bytes (4-bit d = 768)
    {8, 16, 3},   // 384 bytes
    {4, 8, 3},    // 96 bytes (8-bit d = 96)
    {16, 16, 2},  // 512 bytes (8-bit d = 512)
    {8, 16, 4},   // 512 bytes
    {2, 16, 3},   // 96 bytes
};
constexpr int kNumCandShapes = sizeof(kCandShapes) / sizeof(kCandShapes[0]);

using CandKernel = void (*)(CandArgs);

// variant: 0 = IP, 1 = L2 one mean, 2 = L2 several means, 3 = L2 masked,
//          4 = L2 masked several means
template <int B1, int B2, int S>
constexpr CandKernel cand_kernel_for(int variant)
{
    constexpr CandShape sh = kCandShapes[S];
    switch (variant) {
    case 0: return k_cand<B1, B2, LVQ_IP, false, false, sh.g, sh.ch, sh.nch>;
    case 1: return k_cand<B1, B2, LVQ_L2, false, false, sh.g, sh.ch, sh.nch>;
    case 2: return k_cand<B1, B2, LVQ_L2, true, false, sh.g, sh.ch, sh.nch>;
    default: break;
    }
    if constexpr (S == 0) {
        if (variant == 3) return k_cand<B1, B2, LVQ_L2, false, true, sh.g, sh.ch, sh.nch>;
        if (variant == 4) return k_cand<B1, B2, LVQ_L2, true, true, sh.g, sh.ch, sh.nch>;
    }
    return nullptr;
}

template <int B1, int B2>
inline CandKernel cand_lookup(int variant, int shape)
{
    switch (shape) {
    case 0: return cand_kernel_for<B1, B2, 0>(variant);
    case 1: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 1>(variant);
    case 2: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 2>(variant);
    case 3: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 3>(variant);
    case 4: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 4>(variant);
    case 5: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 5>(variant);
    case 6: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 6>(variant);
    default: return nullptr;
    }
}

}  // namespace lvq
