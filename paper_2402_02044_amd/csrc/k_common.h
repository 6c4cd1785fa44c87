// k_common.h -- device helpers shared by the similarity kernels.
#pragma once

#include "lvq_internal.h"

namespace lvq {

// Byte k of a 32-bit word as float; the backend selects v_cvt_f32_ubyte{k}.
template <int K>
__device__ __forceinline__ float ub(uint32_t w)
{
    return (float)((w >> (8 * K)) & 0xFFu);
}

// Sum over aligned groups of G lanes (G <= 16) with DPP row operations; every
// lane of the group ends with the bitwise-identical total.
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group size");
    if (G >= 2)  // quad_perm [1,0,3,2]
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    if (G >= 4)  // quad_perm [2,3,0,1]
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    if (G >= 8)  // row_half_mirror
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    if (G >= 16)  // row_mirror
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
    return v;
}

// Ranking key: the k best entries are the k smallest keys.  High word: the
// score mapped to an order-preserving unsigned integer (ascending for L2,
// descending for IP, NaN last); low word: the slot (ties to the lower slot).
__device__ __forceinline__ uint32_t score_order(float s, int metric)
{
    if (s != s) return 0xFFFFFFFFu;
    uint32_t u = __float_as_uint(metric == LVQ_IP ? -s : s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint64_t make_key(float s, int32_t slot, int metric)
{
    return ((uint64_t)score_order(s, metric) << 32) | (uint32_t)slot;
}

constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ float key_score(uint64_t key, int metric)
{
    uint32_t u = (uint32_t)(key >> 32);
    uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float v = __uint_as_float(b);
    return metric == LVQ_IP ? -v : v;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o)
{
    uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
    return ((uint64_t)hi << 32) | lo;
}

// The wave-wide reductions below expect every lane of the wavefront active.
// DPP row operations leave each 16-lane row with its reduction in every lane
// (lane pairs xor 1, xor 2, then the half-row and row mirrors); the four row
// results are read out with readlane, so the total is wave-uniform.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint64_t min_u64(uint64_t a, uint64_t b)
{
    return b < a ? b : a;
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_min_u64(uint64_t v)
{
    const uint64_t o = ((uint64_t)dpp_u32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp_u32<CTRL>((uint32_t)v);
    return min_u64(v, o);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    v = dpp_min_u64<0xB1>(v);    // quad_perm [1,0,3,2]
    v = dpp_min_u64<0x4E>(v);    // quad_perm [2,3,0,1]
    v = dpp_min_u64<0x141>(v);   // row_half_mirror
    v = dpp_min_u64<0x140>(v);   // row_mirror
    return min_u64(min_u64(readlane_u64(v, 0), readlane_u64(v, 16)),
                   min_u64(readlane_u64(v, 32), readlane_u64(v, 48)));
}

__device__ __forceinline__ int wave_sum_i32(int v)
{
    uint32_t u = (uint32_t)v;
    u += dpp_u32<0xB1>(u);
    u += dpp_u32<0x4E>(u);
    u += dpp_u32<0x141>(u);
    u += dpp_u32<0x140>(u);
    return (int)((uint32_t)__builtin_amdgcn_readlane((int)u, 0) + (uint32_t)__builtin_amdgcn_readlane((int)u, 16) +
                 (uint32_t)__builtin_amdgcn_readlane((int)u, 32) + (uint32_t)__builtin_amdgcn_readlane((int)u, 48));
}

// One whole wavefront selects the k smallest keys of keys[0..n) (LDS) in ascending
// order into out[0..k); entries equal to a selected key are taken together
// (duplicates of an entry are kept as separate results, as many as fit).
// Returns the number of keys written (< k when fewer than k are valid).
// keys[] is consumed (selected entries are overwritten with kNoKey).
__device__ __forceinline__ int wave_select_smallest(uint64_t *keys, int n, int k, uint64_t *out)
{
    const int lane = threadIdx.x & 63;
    uint64_t mine = kNoKey;
    for (int i = lane; i < n; i += 64) mine = keys[i] < mine ? keys[i] : mine;
    int r = 0;
    while (r < k) {
        uint64_t best = wave_min_u64(mine);
        if (best == kNoKey) break;
        int cnt = 0;
        if (mine == best) {
            // one pass: take out the copies of best, keep the smallest of the rest
            uint64_t next = kNoKey;
            for (int i = lane; i < n; i += 64) {
                const uint64_t x = keys[i];
                if (x == best) {
                    keys[i] = kNoKey;
                    ++cnt;
                } else {
                    next = x < next ? x : next;
                }
            }
            mine = next;
        }
        cnt = wave_sum_i32(cnt);
        for (int c = 0; c < cnt && r < k; ++c, ++r)
            if (lane == 0) out[r] = best;
    }
    return r;
}

// Bitonic sort, ascending, of 64*E keys held E per lane (element i = e*64 +
// lane); fully unrolled so every register index is static.
template <int E>
__device__ __forceinline__ void wave_bitonic_sort(uint64_t (&v)[E])
{
    const int lane = threadIdx.x & 63;
    constexpr int N = 64 * E;
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int je = j >> 6;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int pe = e ^ je;
                    if (pe > e) {
                        const bool asc = ((e * 64) & size) == 0;
                        const uint64_t a = v[e], b = v[pe];
                        const bool swap = asc ? (a > b) : (a < b);
                        v[e] = swap ? b : a;
                        v[pe] = swap ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = e * 64 + lane;
                    const uint64_t o = shfl_xor_u64(v[e], j);
                    const bool asc = (i & size) == 0;
                    const bool lower = (lane & j) == 0;
                    const bool take_min = lower == asc;
                    const uint64_t mn = o < v[e] ? o : v[e], mx = o < v[e] ? v[e] : o;
                    v[e] = take_min ? mn : mx;
                }
            }
        }
    }
}

template <int E>
__device__ __forceinline__ int wave_sort_compact_e(uint64_t *buf, int n, int k)
{
    const int lane = threadIdx.x & 63;
    uint64_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * 64 + lane;
        v[e] = i < n ? buf[i] : kNoKey;
    }
    wave_bitonic_sort<E>(v);
    int valid = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * 64 + lane;
        if (i < k) buf[i] = v[e];
        valid += v[e] != kNoKey;
    }
    valid = wave_sum_i32(valid);
    return valid < k ? valid : k;
}

// Keep the k smallest of buf[0..n) (ascending) in buf[0..k) and return how
// many are valid keys (< k when fewer survive).  One whole wavefront.
__device__ __forceinline__ int wave_compact(uint64_t *buf, int n, int k, uint64_t *scratch)
{
    if (n <= 64 && k <= 64) return wave_sort_compact_e<1>(buf, n, k);
    if (n <= 128 && k <= 128) return wave_sort_compact_e<2>(buf, n, k);
    if (n <= 256 && k <= 256) return wave_sort_compact_e<4>(buf, n, k);
    if (n <= 512 && k <= 512) return wave_sort_compact_e<8>(buf, n, k);
    const int lane = threadIdx.x & 63;
    const int got = wave_select_smallest(buf, n, k, scratch);
    for (int i = lane; i < k; i += 64) buf[i] = i < got ? scratch[i] : kNoKey;
    return got;
}

// wave_compact with sorts of at most 128 keys and the selection loop beyond:
// little code and few registers, for kernels that compact short buffers.
__device__ __forceinline__ int wave_compact_lean(uint64_t *buf, int n, int k, uint64_t *scratch)
{
    if (n <= 64 && k <= 64) return wave_sort_compact_e<1>(buf, n, k);
    const int lane = threadIdx.x & 63;
    const int got = wave_select_smallest(buf, n, k, scratch);
    for (int i = lane; i < k; i += 64) buf[i] = i < got ? scratch[i] : kNoKey;
    return got;
}

}  // namespace lvq
