// k_encode.hip -- LVQ encoding on gfx950 (Eq. 1-3, the residual level of
// Sec. 2.3, multi-means Def. 1), writing the packed row format of lvq.h.
//
// Encoding decides integer codes from binary32 arithmetic, so every operation
// is rounded on its own: no contraction into fused multiply-adds (the pragma
// below and -ffp-contract=off on this file), IEEE division, IEEE denormals.
// The result is bit-identical to a scalar binary32 evaluation of the same
// operation sequence:
//   nearest mean   s_m = sum_j (x_j - mu_mj)^2, sequential in j; ties to lower m
//   Eq. 1          t = x - mu*, u = max t, l = min t
//   Eq. 2/3        Delta = (u - l) / (2^B1 - 1), inv = 1 / Delta,
//                  c1 = clamp(floor((t - l) * inv + 1/2), 0, 2^B1 - 1);
//                  Delta below the smallest normal -> Delta = 0, codes 0
//   residual       Delta2 = Delta / (2^B2 - 1), r = t - (Delta c1 + l),
//                  c2 = clamp(floor((r + Delta/2) * (1/Delta2) + 1/2), 0, 2^B2 - 1)
//
// Launch shape: one 64-lane wavefront per workgroup; a vector is handled by a
// group of G lanes (G = 16 for d <= 256, else 64), staged through LDS so the
// packed words are written with coalesced 32-bit stores.
#pragma clang fp contract(off)

#include <float.h>

#include "lvq_internal.h"

namespace lvq {
namespace {

__device__ __forceinline__ unsigned quantize(float t, float lo, float inv, unsigned top)
{
#pragma clang fp contract(off)
    float a = t - lo;
    float b = a * inv;
    float c = b + 0.5f;
    float v = floorf(c);
    if (!(v > 0.0f)) return 0u;
    if (v > (float)top) return top;
    return (unsigned)v;
}

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

// Codes of one packed 32-bit word at word index `wi` of a code array of
// `bits`-bit fields.  `residual` selects the second level.
__device__ __forceinline__ uint32_t pack_word(const float *ts, const int32_t *pos_dim, int npos,
                                              int wi, int bits, bool residual, float l, float delta,
                                              float inv, unsigned top1, float half, float inv2,
                                              unsigned top2, bool have_step, bool have_step2)
{
#pragma clang fp contract(off)
    const int per = 32 / bits;
    uint32_t word = 0;
    for (int k = 0; k < per; ++k) {
        int p = wi * per + k;
        if (p >= npos) break;
        int j = pos_dim[p];
        if (j < 0) continue;
        float t = ts[j];
        unsigned c1 = have_step ? quantize(t, l, inv, top1) : 0u;
        unsigned v = c1;
        if (residual) {
            v = 0u;
            if (have_step2) {
                float y = delta * (float)c1;
                y = y + l;
                float r = t - y;
                v = quantize(r, -half, inv2, top2);
            }
        }
        word |= v << (bits * k);
    }
    return word;
}

template <int G>
__global__ __launch_bounds__(64) void k_encode(EncodeArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ float lds[];
    constexpr int V = 64 / G;
    const int lane = threadIdx.x;
    const int grp = lane / G;
    const int g = lane % G;
    const int d = a.f.dim;
    const int64_t i = (int64_t)blockIdx.x * V + grp;
    const bool active = i < a.n;
    float *ts = lds + (size_t)grp * d;

    // stage x, check finiteness
    int finite = 1;
    if (active) {
        const float *x = a.x + i * d;
        for (int j = g; j < d; j += G) {
            float v = x[j];
            ts[j] = v;
            if (!isfinite(v)) finite = 0;
        }
    }
    finite = group_and<G>(finite);
    __syncthreads();

    // Def. 1: nearest mean, sequential binary32 sum per mean, ties to lower m
    int mstar = 0;
    if (a.n_means > 1 && finite) {
        float best = 0.0f;
        int bm = -1;
        for (int m = g; m < a.n_means; m += G) {
            float s = 0.0f;
            for (int j = 0; j < d; ++j) {
                float e = ts[j] - a.means_t[(int64_t)j * a.means_t_stride + m];
                float e2 = e * e;
                s = s + e2;
            }
            if (bm < 0 || s < best) {
                best = s;
                bm = m;
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
        for (int j = g; j < d; j += G) {
            float t = ts[j] - mu[j];
            ts[j] = t;
            if (!isfinite(t)) finite = 0;
            u = t > u ? t : u;
            l = t < l ? t : l;
        }
    }
    u = group_max<G>(u);
    l = group_min<G>(l);
    finite = group_and<G>(finite);
    __syncthreads();
    if (!active) return;

    const unsigned top1 = (1u << a.f.bits1) - 1u;
    const unsigned top2 = a.f.bits2 ? (1u << a.f.bits2) - 1u : 0u;
    float delta = 0.0f, inv = 0.0f, delta2 = 0.0f, inv2 = 0.0f, half = 0.0f;
    bool have_step = false, have_step2 = false;
    if (finite) {
        float span = u - l;
        if (!isfinite(span)) finite = 0;
        else {
            delta = span / (float)top1;
            if (delta >= FLT_MIN) {
                have_step = true;
                inv = 1.0f / delta;
                if (a.f.bits2) {
                    delta2 = delta / (float)top2;
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
    const int row_words = a.f.row_bytes / 4;
    const int code_words = a.f.code_bytes / 4;
    for (int w = g; w < row_words; w += G) {
        if (store && w == 4) {
            // insert and delete epochs in one 64-bit store: a scan running
            // beside this insert reads the pair whole (old or new), and
            // either way finds the row invisible at its own, older epoch
            const uint64_t ep = ((uint64_t)(finite ? kLiveEpoch : a.epoch) << 32) | a.epoch;
            __hip_atomic_store(reinterpret_cast<uint64_t *>(row + 4), ep, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        if (store && w == 5) continue;
        uint32_t v = 0;
        if (w < 8) {
            uint64_t ext = store ? (a.ext_ids ? a.ext_ids[i] : (uint64_t)slot) : 0ull;
            switch (w) {
            case 0: v = finite ? __float_as_uint(l) : 0x7FC00000u; break;
            case 1: v = finite ? __float_as_uint(delta) : 0u; break;
            case 2: v = finite ? __float_as_uint(delta2) : 0u; break;
            case 3: v = (finite ? (uint32_t)mstar : 0u) | (store ? 0x100u : 0u); break;
            case 4: case 5: v = 0u; break;   // epochs of an encode-only row
            case 6: v = (uint32_t)ext; break;
            default: v = (uint32_t)(ext >> 32); break;
            }
        } else if (finite && w - 8 < code_words) {
            v = pack_word(ts, a.pos_dim, a.f.npos, w - 8, a.f.bits1, false, l, delta, inv, top1,
                          half, inv2, top2, have_step, have_step2);
        }
        row[w] = v;
    }
    if (a.f.bits2 && a.resid) {
        uint32_t *res = reinterpret_cast<uint32_t *>(a.resid + slot * a.f.resid_bytes);
        const int rwords = a.f.resid_bytes / 4;
        for (int w = g; w < rwords; w += G) {
            uint32_t v = 0;
            if (finite)
                v = pack_word(ts, a.pos_dim, a.f.npos, w, a.f.bits2, true, l, delta, inv, top1,
                              half, inv2, top2, have_step, have_step2);
            res[w] = v;
        }
    }
}

}  // namespace

hipError_t launch_encode(const EncodeArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int G = a.f.dim <= 256 ? 16 : 64;
    const int V = 64 / G;
    const size_t lds = (size_t)V * a.f.dim * sizeof(float);
    const int64_t blocks = (a.n + V - 1) / V;
    if (G == 16)
        hipLaunchKernelGGL(k_encode<16>, dim3((unsigned)blocks), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL(k_encode<64>, dim3((unsigned)blocks), dim3(64), lds, s, a);
    return hipGetLastError();
}

}  // namespace lvq
