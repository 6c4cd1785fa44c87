// k_cand_inst.h -- instantiation table of k_cand for one first-level width.
// Included by k_cand4.hip / k_cand8.hip with LVQ_CAND_B1 defined.
#pragma once

#include "k_cand_impl.h"

namespace lvq {

// (lanes per candidate, bytes per piece, pieces per lane and round)
using CandShape = TileShape;
constexpr CandShape kCandShapes[] = {
    {16, 16, 4, 0},  // generic: 1024 code bytes per round
    {16, 8, 3, 0},   // 384 bytes (4-bit d = 768)
    {8, 16, 3, 0},   // 384 bytes
    {4, 8, 3, 0},    // 96 bytes (8-bit d = 96)
    {16, 16, 2, 0},  // 512 bytes (8-bit d = 512)
    {8, 16, 4, 0},   // 512 bytes
    {2, 16, 3, 0},   // 96 bytes
    // software-pipelined (next candidate's loads in flight), single round
    {16, 8, 3, 1},   // 384 bytes
    {8, 16, 3, 1},   // 384 bytes
    {4, 8, 3, 1},    // 96 bytes
    {16, 16, 2, 1},  // 512 bytes
    {8, 16, 4, 1},   // 512 bytes
    {2, 16, 3, 1},   // 96 bytes
    {8, 8, 6, 1},    // 384 bytes
    {4, 16, 6, 1},   // 384 bytes
    // pipelined, query values in registers (inner product, one-mean L2)
    {16, 8, 3, 3},   // 384 bytes
    {8, 8, 6, 3},    // 384 bytes
    {8, 16, 3, 3},   // 384 bytes
    {16, 16, 2, 3},  // 512 bytes
    {4, 8, 3, 3},    // 96 bytes
    {2, 16, 3, 3},   // 96 bytes
    {16, 8, 4, 3},   // 512 bytes
    // pipelined two blocks ahead, single round
    {16, 8, 3, 5},   // 384 bytes
    {8, 16, 3, 5},   // 384 bytes
    {4, 8, 3, 5},    // 96 bytes
    {2, 16, 3, 5},   // 96 bytes
    {8, 8, 6, 5},    // 384 bytes
    {16, 16, 2, 5},  // 512 bytes
    // pipelined, registers allocated for at least six waves per SIMD
    {4, 8, 3, 9},    // 96 bytes
    {2, 16, 3, 9},   // 96 bytes
};
constexpr int kNumCandShapes = sizeof(kCandShapes) / sizeof(kCandShapes[0]);

using CandKernel = void (*)(CandArgs);

// variant: 0 = IP, 1 = L2 one mean, 2 = L2 several means, 3 = L2 masked,
//          4 = L2 masked several means
// pipe bits: 1 = software-pipelined, 2 = query in registers, 4 = two blocks ahead,
//            8 = registers for at least six waves per SIMD
template <int B1, int B2, int S>
constexpr CandKernel cand_kernel_for(int variant)
{
    constexpr CandShape sh = kCandShapes[S];
    constexpr int depth = (sh.pipe & 1) ? ((sh.pipe & 4) ? 2 : 1) : 0;
    constexpr int W = (sh.pipe & 8) ? 6 : 1;
    switch (variant) {
    case 0: return k_cand<B1, B2, LVQ_IP, false, false, sh.g, sh.ch, sh.nch, depth, (sh.pipe & 2) != 0, W>;
    case 1: return k_cand<B1, B2, LVQ_L2, false, false, sh.g, sh.ch, sh.nch, depth, (sh.pipe & 2) != 0, W>;
    case 2:
        if constexpr ((sh.pipe & 2) == 0) return k_cand<B1, B2, LVQ_L2, true, false, sh.g, sh.ch, sh.nch, depth, false, W>;
        return nullptr;
    default: break;
    }
    if constexpr (S == 0) {
        if (variant == 3) return k_cand<B1, B2, LVQ_L2, false, true, sh.g, sh.ch, sh.nch, 0, false, 1>;
        if (variant == 4) return k_cand<B1, B2, LVQ_L2, true, true, sh.g, sh.ch, sh.nch, 0, false, 1>;
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
    case 7: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 7>(variant);
    case 8: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 8>(variant);
    case 9: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 9>(variant);
    case 10: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 10>(variant);
    case 11: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 11>(variant);
    case 12: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 12>(variant);
    case 13: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 13>(variant);
    case 14: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 14>(variant);
    case 15: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 15>(variant);
    case 16: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 16>(variant);
    case 17: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 17>(variant);
    case 18: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 18>(variant);
    case 19: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 19>(variant);
    case 20: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 20>(variant);
    case 21: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 21>(variant);
    case 22: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 22>(variant);
    case 23: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 23>(variant);
    case 24: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 24>(variant);
    case 25: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 25>(variant);
    case 26: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 26>(variant);
    case 27: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 27>(variant);
    case 28: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 28>(variant);
    case 29: return B2 == 4 ? nullptr : cand_kernel_for<B1, B2, 29>(variant);
    default: return nullptr;
    }
}

}  // namespace lvq
