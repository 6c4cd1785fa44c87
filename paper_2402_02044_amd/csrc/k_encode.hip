// k_encode.hip -- LVQ encoding on gfx950 (Eq. 1-3, the residual level of
// Sec. 2.3, multi-means Def. 1), writing the packed row format of lvq.h.
//
// Encoding decides integer codes from binary32 arithmetic, so every operation
// is rounded on its own: no contraction into fused multiply-adds (the pragma
// below and -ffp-contract=off on this file), IEEE division, IEEE denormals.
// The result is bit-identical to a scalar binary32 evaluation of the same
// operation sequence:
//   nearest mean   s_m = sum_j (x_j - mu_mj)^2, sequential in j; ties to lower m;
//                  means marked retired are not candidates
//   Eq. 1          t = x - mu*, u = max t, l = min t
//   Eq. 2/3        Delta = (u - l) / (2^B1 - 1), inv = 1 / Delta,
//                  c1 = clamp(floor((t - l) * inv + 1/2), 0, 2^B1 - 1);
//                  Delta below the smallest normal -> Delta = 0, codes 0
//   residual       Delta2 = Delta / (2^B2 - 1), r = t - (Delta c1 + l),
//                  c2 = clamp(floor((r + Delta/2) * (1/Delta2) + 1/2), 0, 2^B2 - 1)
//
// Launch shape: four waves per workgroup; a vector is handled by a group of G
// lanes (G in {8, 16, 32, 64}: the fewest that leave each lane at most four
// packing units), staged through LDS so the packed words are written with
// coalesced 32-bit stores.  Code positions map to dimensions arithmetically
// (no table lookups on the packing path).
#pragma clang fp contract(off)

#include <float.h>

#include "lvq_internal.h"

namespace lvq {
namespace {

template <int G>
__device__ __forceinline__ float group_max(float v)
{
    for (int o = G / 2; o > 0; o >>= 1) {
        float w = __shfl_xor(v, o, G);
        v = w > v ? w : v;
    }
    return v;
}

template <int G>
__device__ __forceinline__ float group_min(float v)
{
    for (int o = G / 2; o > 0; o >>= 1) {
        float w = __shfl_xor(v, o, G);
        v = w < v ? w : v;
    }
    return v;
}

template <int G>
__device__ __forceinline__ int group_and(int v)
{
    for (int o = G / 2; o > 0; o >>= 1) v &= __shfl_xor(v, o, G);
    return v;
}

// Dimension held at code position p of the first-level layout (-1 for
// padding): sequential layouts hold dimension p; Turbo holds dimension
// 16k + w of its block in field k of word w (blocks of 128 positions at 4
// bits, 64 at 8 bits).  Residual codes use the same positions.
__device__ __forceinline__ int pos_dim_of(const Format &f, int p)
{
    if (p >= f.npos) return -1;
    int dim = p;
    if (f.layout == LVQ_TURBO) {
        const int bsh = f.bits1 == 4 ? 7 : 6;   // positions per block: 128 or 64
        const int fsh = f.bits1 == 4 ? 3 : 2;   // fields per word: 8 or 4
        const int r = p & ((1 << bsh) - 1);
        dim = ((p >> bsh) << bsh) + 16 * (r & ((1 << fsh) - 1)) + (r >> fsh);
    }
    return dim < f.dim ? dim : -1;
}

// Per-vector quantisation constants.
struct Steps {
    float l, delta, inv, half, inv2;
    unsigned top1, top2;
    bool step1, step2;
};

// One packing unit: U consecutive code positions, i.e. PW = U*B1/32 words of
// first-level codes and RW = U*B2/32 words of residual codes (U = 8 when a
// level is 4-bit, else 4).  Each field's codes are computed once: the
// first-level code, then the residual code from the same t.  Positions past
// the code area or holding no dimension get code 0.
template <int B1, int B2>
__device__ __forceinline__ void pack_unit(const float *ts, const Format &f, int unit, const Steps &st,
                                          uint32_t (&pw)[(B1 == 4 || B2 == 4 ? 8 : 4) * B1 / 32],
                                          uint32_t (&rw)[B2 ? (B1 == 4 || B2 == 4 ? 8 : 4) * B2 / 32 : 1])
{
#pragma clang fp contract(off)
    constexpr int U = (B1 == 4 || B2 == 4) ? 8 : 4;
    constexpr int PER1 = 32 / B1;
#pragma unroll
    for (int w = 0; w < U * B1 / 32; ++w) pw[w] = 0u;
#pragma unroll
    for (int w = 0; w < (B2 ? U * B2 / 32 : 1); ++w) rw[w] = 0u;
    const bool turbo = f.layout == LVQ_TURBO;
#pragma unroll
    for (int h = 0; h < U / PER1; ++h) {          // first-level words of the unit
        const int p0 = unit * U + h * PER1;       // first position of the word
        const int base = pos_dim_of(f, p0);       // its dimension (field 0)
        const int ds = turbo ? 16 : 1;            // dimension step between fields
#pragma unroll
        for (int k = 0; k < PER1; ++k) {
            // Branch-free: every field runs the same sequence, and fields
            // with no dimension, or a vector with no step, keep code 0.  With
            // no step inv (inv2) is 0, so the values stay in [0, top] (a NaN
            // fails the comparisons and becomes 0).
            const int dim = base + ds * k;
            const bool valid = base >= 0 && dim < f.dim && p0 + k < f.npos;
            const float t = ts[valid ? dim : 0];
            float a = t - st.l;
            float b = a * st.inv;
            float c = b + 0.5f;
            float v = floorf(c);
            v = v > 0.0f ? v : 0.0f;
            v = v > (float)st.top1 ? (float)st.top1 : v;
            const unsigned c1 = valid && st.step1 ? (unsigned)v : 0u;
            unsigned c2 = 0u;
            if constexpr (B2 != 0) {
                float y = st.delta * v;
                y = y + st.l;
                const float r = t - y;
                float a2 = r - (-st.half);
                float b2 = a2 * st.inv2;
                float c2f = b2 + 0.5f;
                float v2 = floorf(c2f);
                v2 = v2 > 0.0f ? v2 : 0.0f;
                v2 = v2 > (float)st.top2 ? (float)st.top2 : v2;
                c2 = valid && st.step1 && st.step2 ? (unsigned)v2 : 0u;
            }
            const int q = h * PER1 + k;            // field index within the unit
            pw[q / PER1] |= c1 << (B1 * (q % PER1));
            if constexpr (B2 != 0) rw[q / (32 / B2)] |= c2 << (B2 * (q % (32 / B2)));
        }
    }
}

// Floats between consecutive staged vectors in LDS: d rounded up to a
// multiple of four (float4 staging), and an odd multiple of four so that the
// vectors of one wave start in distinct bank groups (with d a multiple of 32,
// a stride of d would send every group's read of dimension j to one bank).
__host__ __device__ inline int stage_stride(int d)
{
    int s = (d + 3) & ~3;
    if (((s >> 2) & 1) == 0) s += 4;
    return s;
}

template <int B1, int B2, int G>
__global__ __launch_bounds__(256) void k_encode(EncodeArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ float lds[];
    constexpr int V = 256 / G;   // vectors per workgroup (four waves)
    const int grp = threadIdx.x / G;
    const int g = threadIdx.x % G;
    const int d = a.f.dim;
    const int64_t i = (int64_t)blockIdx.x * V + grp;
    const bool active = i < a.n;
    const int stride = stage_stride(d);
    float *ts = lds + (size_t)grp * stride;

    // stage x, check finiteness.  Rows of a multiple of four floats are read
    // as float4, four loads per lane issued before any is used.
    int finite = 1;
    const bool vec4 = (d & 3) == 0;
    if (active) {
        const float *x = a.x + i * d;
        if (vec4) {
            const int d4 = d >> 2;
            const float4 *x4 = reinterpret_cast<const float4 *>(x);
            float4 *t4 = reinterpret_cast<float4 *>(ts);
            for (int q0 = g; q0 < d4; q0 += 4 * G) {
                float4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = x4[min(q0 + u * G, d4 - 1)];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (q0 + u * G < d4) {
                        t4[q0 + u * G] = v[u];
                        if (!isfinite(v[u].x) || !isfinite(v[u].y) || !isfinite(v[u].z) || !isfinite(v[u].w))
                            finite = 0;
                    }
            }
        } else {
            for (int j = g; j < d; j += G) {
                float v = x[j];
                ts[j] = v;
                if (!isfinite(v)) finite = 0;
            }
        }
    }
    // means for the nearest-mean search, staged in LDS as [mean][dim] rows
    // of the staging stride when they fit: the lanes of a group read four
    // dimensions of their means with one 16-byte load, and the odd
    // multiple-of-four stride keeps those loads free of bank conflicts
    const int M = a.n_means;
    float *mt = lds + (size_t)V * stride;
    if (a.means_lds) {
        for (int e = threadIdx.x; e < M * d; e += 256) {
            const int m = e / d, j = e - m * d;
            mt[m * stride + j] = a.means[e];
        }
    }
    finite = group_and<G>(finite);
    __syncthreads();

    // Def. 1: nearest mean, sequential binary32 sum per mean, ties to lower m
    int mstar = 0;
    if (M > 1 && active && finite) {
        float best = 0.0f;
        int bm = -1;
        // two means per pass (m0 and m0 + G), each summed in dimension order
        for (int m0 = g; m0 < M; m0 += 2 * G) {
            const bool two = m0 + G < M;
            const int m1 = two ? m0 + G : m0;
            float s0 = 0.0f, s1 = 0.0f;
            if (a.means_lds && vec4) {
                const float4 *x4 = reinterpret_cast<const float4 *>(ts);
                const float4 *a4 = reinterpret_cast<const float4 *>(mt + m0 * stride);
                const float4 *b4 = reinterpret_cast<const float4 *>(mt + m1 * stride);
                auto step = [](float x, float mu, float &acc) {
                    float e = x - mu;
                    e = e * e;
                    acc = acc + e;
                };
#pragma unroll 4
                for (int q = 0; q < (d >> 2); ++q) {
                    const float4 xv = x4[q], av = a4[q], bv = b4[q];
                    step(xv.x, av.x, s0);
                    step(xv.x, bv.x, s1);
                    step(xv.y, av.y, s0);
                    step(xv.y, bv.y, s1);
                    step(xv.z, av.z, s0);
                    step(xv.z, bv.z, s1);
                    step(xv.w, av.w, s0);
                    step(xv.w, bv.w, s1);
                }
            } else if (a.means_lds) {
#pragma unroll 8
                for (int j = 0; j < d; ++j) {
                    const float x = ts[j];
                    float e0 = x - mt[m0 * stride + j];
                    float e1 = x - mt[m1 * stride + j];
                    e0 = e0 * e0;
                    e1 = e1 * e1;
                    s0 = s0 + e0;
                    s1 = s1 + e1;
                }
            } else {
#pragma unroll 8
                for (int j = 0; j < d; ++j) {
                    const float x = ts[j];
                    const float *mr = a.means_t + (int64_t)j * a.means_t_stride;
                    float e0 = x - mr[m0];
                    float e1 = x - mr[m1];
                    e0 = e0 * e0;
                    e1 = e1 * e1;
                    s0 = s0 + e0;
                    s1 = s1 + e1;
                }
            }
            // retired means are never chosen
            const bool ok0 = a.mean_active[m0] != 0;
            const bool ok1 = two && a.mean_active[m1] != 0;
            if (ok0 && (bm < 0 || s0 < best)) {
                best = s0;
                bm = m0;
            }
            if (ok1 && (bm < 0 || s1 < best)) {
                best = s1;
                bm = m1;
            }
        }
        // group argmin over (s, m): lexicographic
        for (int o = G / 2; o > 0; o >>= 1) {
            float ob = __shfl_xor(best, o, G);
            int om = __shfl_xor(bm, o, G);
            bool take = (bm < 0) || (om >= 0 && (ob < best || (ob == best && om < bm)));
            if (take) {
                best = ob;
                bm = om;
            }
        }
        mstar = bm < 0 ? 0 : bm;
    }
    __syncthreads();

    // Eq. 1: t = x - mu*, bounds
    float u = -FLT_MAX, l = FLT_MAX;
    if (active) {
        const float *mu = a.means + (int64_t)mstar * d;
        if (vec4) {
            const int d4 = d >> 2;
            const float4 *mu4 = reinterpret_cast<const float4 *>(mu);
            float4 *t4 = reinterpret_cast<float4 *>(ts);
            for (int q0 = g; q0 < d4; q0 += 4 * G) {
                float4 mv[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) mv[w] = mu4[min(q0 + w * G, d4 - 1)];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int q = q0 + w * G;
                    if (q >= d4) continue;
                    float4 t = t4[q];
                    t.x = t.x - mv[w].x;
                    t.y = t.y - mv[w].y;
                    t.z = t.z - mv[w].z;
                    t.w = t.w - mv[w].w;
                    t4[q] = t;
                    if (!isfinite(t.x) || !isfinite(t.y) || !isfinite(t.z) || !isfinite(t.w)) finite = 0;
                    u = fmaxf(fmaxf(u, fmaxf(t.x, t.y)), fmaxf(t.z, t.w));
                    l = fminf(fminf(l, fminf(t.x, t.y)), fminf(t.z, t.w));
                }
            }
        } else {
            for (int j = g; j < d; j += G) {
                float t = ts[j] - mu[j];
                ts[j] = t;
                if (!isfinite(t)) finite = 0;
                u = t > u ? t : u;
                l = t < l ? t : l;
            }
        }
    }
    u = group_max<G>(u);
    l = group_min<G>(l);
    finite = group_and<G>(finite);
    __syncthreads();
    if (!active) return;

    Steps st;
    st.top1 = (1u << B1) - 1u;
    st.top2 = B2 ? (1u << B2) - 1u : 0u;
    float delta = 0.0f, inv = 0.0f, delta2 = 0.0f, inv2 = 0.0f, half = 0.0f;
    bool have_step = false, have_step2 = false;
    if (finite) {
        float span = u - l;
        if (!isfinite(span)) finite = 0;
        else {
            delta = span / (float)st.top1;
            if (delta >= FLT_MIN) {
                have_step = true;
                inv = 1.0f / delta;
                if (B2) {
                    delta2 = delta / (float)st.top2;
                    if (delta2 >= FLT_MIN) {
                        have_step2 = true;
                        inv2 = 1.0f / delta2;
                        half = 0.5f * delta;
                    } else {
                        delta2 = 0.0f;
                    }
                }
            } else {
                delta = 0.0f;
            }
        }
    }
    st.l = l;
    st.delta = delta;
    st.inv = inv;
    st.half = half;
    st.inv2 = inv2;
    st.step1 = have_step;
    st.step2 = have_step2;

    // destination slot
    int64_t slot = i;
    const bool store = a.free_stack != nullptr;
    if (store) {
        slot = a.free_stack[a.free_top - 1 - i];
        if (g == 0) {
            a.slots_out[i] = (int32_t)slot;
            if (a.list_out) a.list_out[i] = (int32_t)slot;
        }
    }
    if (!finite && g == 0) atomicOr(a.err, kErrNonFinite);

    uint32_t *row = reinterpret_cast<uint32_t *>(a.rows + slot * a.f.row_bytes);
    // header: lanes 0..7 of the group
    if (g < 8) {
        const int w = g;
        if (store && w == 4) {
            // insert and delete epochs in one 64-bit store: a scan running
            // beside this insert reads the pair whole (old or new), and
            // either way finds the row invisible at its own, older epoch
            const uint64_t ep = ((uint64_t)(finite ? kLiveEpoch : a.epoch) << 32) | a.epoch;
            __hip_atomic_store(reinterpret_cast<uint64_t *>(row + 4), ep, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else if (!(store && w == 5)) {
            uint32_t v = 0;
            const uint64_t ext = store ? (a.ext_ids ? a.ext_ids[i] : (uint64_t)slot) : 0ull;
            switch (w) {
            case 0: v = finite ? __float_as_uint(l) : 0x7FC00000u; break;
            case 1: v = finite ? __float_as_uint(delta) : 0u; break;
            case 2: v = finite ? __float_as_uint(delta2) : 0u; break;
            case 3: v = (finite ? (uint32_t)mstar : 0u) | (store ? 0x100u : 0u); break;
            case 4: case 5: v = 0u; break;   // epochs of an encode-only row
            case 6: v = (uint32_t)ext; break;
            default: v = (uint32_t)(ext >> 32); break;
            }
            row[w] = v;
        }
    }
    // codes: unit u covers positions [U u, U u + U); a non-finite vector
    // stores zero codes
    constexpr int U = (B1 == 4 || B2 == 4) ? 8 : 4;
    constexpr int PW = U * B1 / 32, RW = B2 ? U * B2 / 32 : 0;
    const int row_words = a.f.row_bytes / 4;
    const int units = (a.f.npos + U - 1) / U;
    uint32_t *codes = row + 8;
    uint32_t *res = B2 && a.resid ? reinterpret_cast<uint32_t *>(a.resid + slot * a.f.resid_bytes) : nullptr;
    const int res_words = a.f.resid_bytes / 4;
    if (!finite) st.step1 = false;
    for (int unit = g; unit < units; unit += G) {
        uint32_t pw[PW], rw[B2 ? RW : 1];
        pack_unit<B1, B2>(ts, a.f, unit, st, pw, rw);
#pragma unroll
        for (int w = 0; w < PW; ++w)
            if (8 + unit * PW + w < row_words) codes[unit * PW + w] = pw[w];
        if constexpr (B2 != 0) {
            if (res) {
#pragma unroll
                for (int w = 0; w < RW; ++w)
                    if (unit * RW + w < res_words) res[unit * RW + w] = rw[w];
            }
        }
    }
    // zero padding after the last unit
    for (int w = 8 + units * PW + g; w < row_words; w += G) row[w] = 0u;
    if constexpr (B2 != 0) {
        if (res)
            for (int w = units * RW + g; w < res_words; w += G) res[w] = 0u;
    }
}

}  // namespace

template <int B1, int B2>
static hipError_t launch_encode_t(const EncodeArgs &a, int G, size_t lds, int64_t blocks, hipStream_t s)
{
    switch (G) {
    case 8: hipLaunchKernelGGL((k_encode<B1, B2, 8>), dim3((unsigned)blocks), dim3(256), lds, s, a); break;
    case 16: hipLaunchKernelGGL((k_encode<B1, B2, 16>), dim3((unsigned)blocks), dim3(256), lds, s, a); break;
    case 32: hipLaunchKernelGGL((k_encode<B1, B2, 32>), dim3((unsigned)blocks), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL((k_encode<B1, B2, 64>), dim3((unsigned)blocks), dim3(256), lds, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_encode(const EncodeArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    // lanes per vector: the fewest (8..64) giving each lane at most four
    // packing units
    const int U = (a.f.bits1 == 4 || a.f.bits2 == 4) ? 8 : 4;
    const int units = (a.f.npos + U - 1) / U;
    int G = 8;
    while (G < 64 && units > 4 * G) G *= 2;
    const int V = 256 / G;
    size_t lds = (size_t)V * stage_stride(a.f.dim) * sizeof(float);
    if (a.means_lds) lds += (size_t)a.n_means * stage_stride(a.f.dim) * sizeof(float);
    const int64_t blocks = (a.n + V - 1) / V;
    const int b1 = a.f.bits1, b2 = a.f.bits2;
    if (b1 == 4 && b2 == 0) return launch_encode_t<4, 0>(a, G, lds, blocks, s);
    if (b1 == 4 && b2 == 4) return launch_encode_t<4, 4>(a, G, lds, blocks, s);
    if (b1 == 4 && b2 == 8) return launch_encode_t<4, 8>(a, G, lds, blocks, s);
    if (b1 == 8 && b2 == 0) return launch_encode_t<8, 0>(a, G, lds, blocks, s);
    if (b1 == 8 && b2 == 4) return launch_encode_t<8, 4>(a, G, lds, blocks, s);
    if (b1 == 8 && b2 == 8) return launch_encode_t<8, 8>(a, G, lds, blocks, s);
    return hipErrorInvalidValue;
}

}  // namespace lvq
