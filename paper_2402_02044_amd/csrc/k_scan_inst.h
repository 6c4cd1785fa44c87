// k_scan_inst.h -- instantiation table of k_scan for one first-level width.
#pragma once

#include "k_cand_inst.h"
#include "k_scan_impl.h"

namespace lvq {

using ScanKernel = void (*)(ScanArgs);

// variant: 0 = IP, 1 = L2, 2 = L2 masked (generic shape only)
template <int B1, int B2, int S>
constexpr ScanKernel scan_kernel_for(int variant)
{
    constexpr CandShape sh = kCandShapes[S];
    if (variant == 0) return k_scan<B1, B2, LVQ_IP, false, sh.g, sh.ch, sh.nch>;
    if (variant == 1) return k_scan<B1, B2, LVQ_L2, false, sh.g, sh.ch, sh.nch>;
    if constexpr (S == 0)
        if (variant == 2) return k_scan<B1, B2, LVQ_L2, true, sh.g, sh.ch, sh.nch>;
    return nullptr;
}

template <int B1, int B2>
inline ScanKernel scan_lookup(int variant, int shape)
{
    switch (shape) {
    case 0: return scan_kernel_for<B1, B2, 0>(variant);
    case 1: return B2 == 4 ? nullptr : scan_kernel_for<B1, B2, 1>(variant);
    case 3: return B2 == 4 ? nullptr : scan_kernel_for<B1, B2, 3>(variant);
    case 4: return B2 == 4 ? nullptr : scan_kernel_for<B1, B2, 4>(variant);
    default: return nullptr;
    }
}

}  // namespace lvq
