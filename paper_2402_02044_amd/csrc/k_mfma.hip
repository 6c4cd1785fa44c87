// k_mfma.hip -- matrix-core scan: first-level instantiations, the 16-bit
// query fragment precompute, and the host-side launch helpers.
#include "k_mfma_impl.h"

namespace lvq {
namespace {

// Queries (nq x dim, bf16 or fp16 bits) -> A fragments in [tile][block][chunk]
// [step][lane][8] order over kernel-order code positions, zero at padding and
// past nq; plus sum(q) and <q, mu_m> from the same 16-bit values.
template <int B1>
__global__ __launch_bounds__(256) void k_prep16(const uint16_t *q, int64_t nq, int dim, int kpos, int qb, int fp16,
                                                const int32_t *kdim, const float *means, int n_means, uint16_t *frag,
                                                float *qsum, float *cm)
{
    constexpr int CHUNK_POS = B1 == 8 ? 32 : 64;
    constexpr int STEPS = B1 == 8 ? 2 : 4;
    const int nchunk = kpos / CHUNK_POS;
    const int tq = 32 * qb;
    const int64_t tile = blockIdx.x;
    const int64_t per_tile = (int64_t)qb * nchunk * STEPS * 64 * 8;
    for (int64_t e = threadIdx.x; e < per_tile; e += 256) {
        const int j = (int)(e % 8);
        const int l = (int)((e / 8) % 64);
        const int s = (int)((e / 512) % STEPS);
        const int c = (int)((e / (512 * STEPS)) % nchunk);
        const int b = (int)(e / (512 * STEPS * nchunk));
        const int half = l >> 5;
        const int p = B1 == 8 ? c * 32 + half * 16 + s * 8 + j : c * 64 + half * 32 + s * 8 + j;
        const int64_t gq = tile * tq + 32 * b + (l & 31);
        uint16_t v = 0;
        if (gq < nq) {
            const int d = kdim[p];
            if (d >= 0) v = q[gq * dim + d];
        }
        frag[tile * per_tile + e] = v;
    }
    // sums over the tile's queries: one wave per query
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i < tq; i += 4) {
        const int64_t gq = tile * tq + i;
        if (gq >= nq) continue;
        auto val = [&](int d) -> float {
            const uint16_t h = q[gq * dim + d];
            if (fp16) return (float)__builtin_bit_cast(_Float16, h);
            return __uint_as_float((uint32_t)h << 16);
        };
        float s = 0.0f;
        for (int d = lane; d < dim; d += 64) s += val(d);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) qsum[gq] = s;
        for (int m = 0; m < n_means; ++m) {
            float t = 0.0f;
            for (int d = lane; d < dim; d += 64) t = fmaf(val(d), means[(int64_t)m * dim + d], t);
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
            if (lane == 0) cm[gq * n_means + m] = t;
        }
    }
}

}  // namespace

MfmaKernelPtr mfma_kernel_first(int bits1, int kpos, int fp16, int *qb)
{
    if (bits1 == 8) return fp16 ? (MfmaKernelPtr)mfma_lookup<8, 0, true>(kpos, qb) : (MfmaKernelPtr)mfma_lookup<8, 0, false>(kpos, qb);
    if (bits1 == 4) return fp16 ? (MfmaKernelPtr)mfma_lookup<4, 0, true>(kpos, qb) : (MfmaKernelPtr)mfma_lookup<4, 0, false>(kpos, qb);
    return nullptr;
}
int mfma_query_block(int bits1, int bits2, int kpos)
{
    if (bits1 != 4 && bits1 != 8) return 0;
    if (kpos % (bits1 == 8 ? 32 : 64)) return 0;
    int qb = 0;
    const MfmaKernelPtr k = bits2 == 0 ? mfma_kernel_first(bits1, kpos, 0, &qb)
                                       : bits2 == 8 ? mfma_kernel_full(bits1, kpos, 0, &qb) : nullptr;
    return k ? qb : 0;
}

size_t mfma_lds_bytes(int qb, int n_means, int k, int capq)
{
    const int tq = 32 * qb;
    size_t b = (size_t)tq * 4 + (size_t)tq * n_means * 4;
    b = (b + 15) & ~(size_t)15;
    b += (size_t)tq * (8 + 4 + 4) + (tq & 1) * 4 + 8;
    b += (size_t)tq * capq * 8;
    b += (size_t)kWaves * k * 8;
    return b;
}

// Largest per-query key buffer (<= 512 keys, the register sort's reach, or
// k + one round when k is larger) that fits lds_max; 0 if even k + one round
// does not.
int mfma_capq(int qb, int n_means, int k, size_t lds_max)
{
    const int need = k + kRowsPerIter;
    int cap = need > 512 ? need : 512;
    while (cap > need && mfma_lds_bytes(qb, n_means, k, cap) > lds_max) cap -= 16;
    if (cap < need) cap = need;
    return mfma_lds_bytes(qb, n_means, k, cap) <= lds_max ? cap : 0;
}

hipError_t launch_prep16(const void *q, int64_t nq, int dim, int kpos, int bits1, int qb, int prec,
                         const int32_t *kdim, const float *means, int n_means, void *frag, float *qsum, float *cm,
                         hipStream_t s)
{
    if (!qb) return hipErrorInvalidValue;
    const int64_t tiles = (nq + 32 * qb - 1) / (32 * qb);
    auto kern = bits1 == 8 ? k_prep16<8> : k_prep16<4>;
    hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(256), 0, s, (const uint16_t *)q, nq, dim, kpos, qb,
                       prec == LVQ_FP16 ? 1 : 0, kdim, means, n_means, (uint16_t *)frag, qsum, cm);
    return hipGetLastError();
}

hipError_t launch_scan_mfma(const ScanArgs &a, int bits1, int bits2, int prec, hipStream_t s)
{
    int qb = 0;
    const int fp16 = prec == LVQ_FP16 ? 1 : 0;
    MfmaKernelPtr kern = bits2 == 0 ? mfma_kernel_first(bits1, a.kpos, fp16, &qb)
                                    : bits2 == 8 ? mfma_kernel_full(bits1, a.kpos, fp16, &qb) : nullptr;
    if (!kern) return hipErrorInvalidValue;
    const int64_t qtiles = (a.nq + 32 * qb - 1) / (32 * qb);
    const int64_t ntiles = qtiles * a.n_parts;
    const int64_t grid = (ntiles + 7) / 8 * 8;
    const size_t lds = mfma_lds_bytes(qb, a.n_means, a.k, a.capq);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace lvq
