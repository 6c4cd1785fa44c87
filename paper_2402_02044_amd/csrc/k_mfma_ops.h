// k_mfma_ops.h -- operand helpers of the matrix-core scans: 16-bit vector
// types, exact conversion of integer codes to bf16 / fp16 MFMA fragments or
// to one FP32 value per lane, and the 32x32x16 and 32x32x2 MFMAs (FP32
// accumulation).  A 16-bit fragment of one MFMA step holds, per lane, 8
// consecutive kernel-order positions of one row (lane & 31) and K half
// (lane >> 5); the same layout serves as the A or the B operand.
#pragma once

#include "k_common.h"

namespace lvq {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint32_t opaque_and_m(uint32_t w, uint32_t m)
{
    uint32_t r;
    asm("v_and_b32 %0, %1, %2" : "=v"(r) : "s"(m), "v"(w));
    return r;
}

// Two floats holding small integers -> packed 16-bit pair (exact).
template <bool FP16>
__device__ __forceinline__ uint32_t pack2(float lo, float hi)
{
    if constexpr (FP16) {
        auto h = __builtin_amdgcn_cvt_pkrtz(lo, hi);
        return __builtin_bit_cast(uint32_t, h);
    } else {
        // bfloat16 = high half of the float (exact: <= 8 significant bits)
        return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
    }
}

// B fragment (8 codes of one MFMA step) from the lane's 16 loaded bytes.
// 8-bit codes: step s covers bytes 8s..8s+7.  4-bit codes: step s covers
// word s, fields in kernel order (0,2,4,6,1,3,5,7).
template <int B1, bool FP16>
__device__ __forceinline__ uint4 b_fragment(const uint4 &v, int s)
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint4 r;
    if constexpr (B1 == 8) {
        const uint32_t a = w[2 * s], b = w[2 * s + 1];
        r.x = pack2<FP16>(ub<0>(a), ub<1>(a));
        r.y = pack2<FP16>(ub<2>(a), ub<3>(a));
        r.z = pack2<FP16>(ub<0>(b), ub<1>(b));
        r.w = pack2<FP16>(ub<2>(b), ub<3>(b));
    } else {
        const uint32_t lo = opaque_and_m(w[s], 0x0F0F0F0Fu);
        const uint32_t hi = opaque_and_m(w[s] >> 4, 0x0F0F0F0Fu);
        r.x = pack2<FP16>(ub<0>(lo), ub<1>(lo));
        r.y = pack2<FP16>(ub<2>(lo), ub<3>(lo));
        r.z = pack2<FP16>(ub<0>(hi), ub<1>(hi));
        r.w = pack2<FP16>(ub<2>(hi), ub<3>(hi));
    }
    return r;
}

// B fragment of the residual level (8-bit codes at the primary's code
// positions).  Primary 8-bit: the same bytes as b_fragment.  Primary 4-bit:
// the lane's 32 residual bytes hold positions 8w..8w+7 of its four words w;
// step s takes bytes 8s..8s+7 in the primary's kernel field order
// (0,2,4,6,1,3,5,7).
template <int B1, bool FP16>
__device__ __forceinline__ uint4 r_fragment(const uint4 (&v)[B1 == 4 ? 2 : 1], int s)
{
    if constexpr (B1 == 8) {
        return b_fragment<8, FP16>(v[0], s);
    } else {
        const uint32_t w[8] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w};
        const uint32_t lo = w[2 * s], hi = w[2 * s + 1];
        uint4 r;
        r.x = pack2<FP16>(ub<0>(lo), ub<2>(lo));
        r.y = pack2<FP16>(ub<0>(hi), ub<2>(hi));
        r.z = pack2<FP16>(ub<1>(lo), ub<3>(lo));
        r.w = pack2<FP16>(ub<1>(hi), ub<3>(hi));
        return r;
    }
}

// FP32 operands: one code (exact as a float) and one query value per lane.
// The lane's 16 loaded bytes as words whose bytes are its codes in kernel
// order, code t = byte t % 4 of word t / 4: 8-bit codes as loaded; 4-bit
// codes split into the low fields (0,2,4,6) and the high fields (1,3,5,7) of
// each word, the order of b_fragment.
template <int B1>
__device__ __forceinline__ void code_words(const uint4 &v, uint32_t (&w)[B1 == 8 ? 4 : 8])
{
    const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if constexpr (B1 == 8) {
            w[i] = x[i];
        } else {
            w[2 * i] = opaque_and_m(x[i], 0x0F0F0F0Fu);
            w[2 * i + 1] = opaque_and_m(x[i] >> 4, 0x0F0F0F0Fu);
        }
    }
}

// The lane's residual bytes of a chunk (8-bit codes, one per first-level
// position) as words in code_words' order: byte e of word s is the residual
// code of code 4 s + e.  8-bit first level: the 16 bytes as loaded.  4-bit
// first level: the 32 bytes hold, at bytes 8w .. 8w + 7, the codes of fields
// 0..7 of first-level word w, regrouped as fields (0,2,4,6) and (1,3,5,7).
template <int B1>
__device__ __forceinline__ void resid_words(const uint4 (&v)[B1 == 8 ? 1 : 2], uint32_t (&w)[B1 == 8 ? 4 : 8])
{
    if constexpr (B1 == 8) {
        w[0] = v[0].x;
        w[1] = v[0].y;
        w[2] = v[0].z;
        w[3] = v[0].w;
    } else {
        const uint32_t x[8] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            // bytes (0,2) of the low word then (0,2) of the high word; then (1,3), (1,3)
            w[2 * s] = __builtin_amdgcn_perm(x[2 * s + 1], x[2 * s], 0x06040200u);
            w[2 * s + 1] = __builtin_amdgcn_perm(x[2 * s + 1], x[2 * s], 0x07050301u);
        }
    }
}

// 32x32 FP32 scores += (32 rows x 2 codes) x (2 positions x 32 queries):
// lane l gives row (l & 31)'s code and query (l & 31)'s value at K index
// l >> 5.
__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <bool FP16>
__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c)
{
    if constexpr (FP16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}

}  // namespace
}  // namespace lvq
