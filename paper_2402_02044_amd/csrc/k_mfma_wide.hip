// k_mfma_wide.hip -- the queries-in-LDS matrix-core scan (k_mfma_wide_impl.h):
// bf16 / fp16 first-level instantiations, the FP32 query fragments, and the
// host-side helpers and launch of every form.
#include "k_mfma_wide_impl.h"

namespace lvq {
namespace {

// Instantiated position counts: 32-query blocks per workgroup (as many as
// the query fragments' LDS allows, at most four) and row blocks per wave
// (one with four query blocks: two spilled 32 registers and ran 4% slower at
// C4).
template <int B1, int PREC>
WideKernel wide_lookup_16(int kpos, int *qb, int *rb)
{
    switch (kpos) {
    case 96: *qb = 4; *rb = 1; return B1 == 8 ? k_scan_mfma_wide<8, 0, 96, 4, 1, PREC> : nullptr;
    case 128: *qb = 4; *rb = 1; return k_scan_mfma_wide<B1, 0, 128, 4, 1, PREC>;
    case 256: *qb = 4; *rb = 1; return k_scan_mfma_wide<B1, 0, 256, 4, 1, PREC>;
    case 384: *qb = 4; *rb = 1; return k_scan_mfma_wide<B1, 0, 384, 4, 1, PREC>;
    case 512: *qb = 4; *rb = 1; return k_scan_mfma_wide<B1, 0, 512, 4, 1, PREC>;
    case 768: *qb = 2; *rb = 2; return k_scan_mfma_wide<B1, 0, 768, 2, 2, PREC>;
    case 1024: *qb = 2; *rb = 2; return k_scan_mfma_wide<B1, 0, 1024, 2, 2, PREC>;
    default: return nullptr;
    }
}

// prec LVQ_BF16 / LVQ_FP16 or LVQ_FP32; bits2 0 (first level) or 8.
WideKernel wide_kernel(int bits1, int bits2, int kpos, int prec, int *qb, int *rb)
{
    if (bits1 != 4 && bits1 != 8) return nullptr;
    if (prec == LVQ_FP32) {
        if (bits2 == 0) return wide_kernel_f32(bits1, kpos, qb, rb);
        if (bits2 == 8) return wide_kernel_f32r(bits1, kpos, qb, rb);
        return nullptr;
    }
    if (bits2 == 8) return wide_kernel_16r(bits1, kpos, prec, qb, rb);
    if (bits2 != 0) return nullptr;
    if (prec == LVQ_BF16) return bits1 == 8 ? wide_lookup_16<8, LVQ_BF16>(kpos, qb, rb) : wide_lookup_16<4, LVQ_BF16>(kpos, qb, rb);
    if (prec == LVQ_FP16) return bits1 == 8 ? wide_lookup_16<8, LVQ_FP16>(kpos, qb, rb) : wide_lookup_16<4, LVQ_FP16>(kpos, qb, rb);
    return nullptr;
}

// LDS bytes of a launch: FP32 and both-level forms carry the c_m table of
// every mean (and each row's mean id); 16-bit both-level forms each row's
// Delta2.
size_t wide_lds(int qb, int kpos, int rb, int prec, int bits2, int n_means)
{
    const bool mm = prec == LVQ_FP32 || bits2 != 0, ch2 = prec != LVQ_FP32 && bits2 != 0;
    return wide_lds_bytes(qb, kpos, rb, prec == LVQ_FP32 ? 4 : 2, mm ? n_means : 0, 12 + (mm ? 4 : 0) + (ch2 ? 4 : 0));
}

// FP32 query fragments from kernel-order queries (nq x kpos, zero at padding
// positions): [tile][block][chunk][step][lane] float4s, element e of step s
// being the value for MFMA 4 s + e, whose lane l holds position
// CHUNK_POS c + (CHUNK_POS / 2)(l >> 5) + 4 s + e of query 32 block + (l & 31)
// (zero past nq) -- the positions of the codes that code_words hands that lane.
__global__ __launch_bounds__(256) void k_frag32(const float *qk, int64_t nq, int kpos, int chunk_pos, int qb,
                                                float4 *frag)
{
    const int nchunk = kpos / chunk_pos, steps = chunk_pos / 8;
    const int64_t per_tile = (int64_t)qb * nchunk * steps * 64;
    const int64_t tile = blockIdx.x;
    for (int64_t e = threadIdx.x; e < per_tile; e += 256) {
        const int l = (int)(e % 64);
        const int s = (int)((e / 64) % steps);
        const int c = (int)((e / (64 * steps)) % nchunk);
        const int b = (int)(e / (64 * steps * nchunk));
        const int64_t gq = tile * 32 * qb + 32 * b + (l & 31);
        const int p = c * chunk_pos + (l >> 5) * (chunk_pos / 2) + 4 * s;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (gq < nq) v = *reinterpret_cast<const float4 *>(qk + gq * kpos + p);
        frag[tile * per_tile + e] = v;
    }
}

}  // namespace

int mfma_wide_query_block(int bits1, int bits2, int kpos, int prec, int k, int n_means, size_t lds_max)
{
    if ((bits1 != 4 && bits1 != 8) || kpos % (bits1 == 8 ? 32 : 64)) return 0;
    if (k < 1 || k > kWideMaxK || n_means < 1 || (prec != LVQ_FP32 && bits2 == 0 && n_means != 1)) return 0;
    int qb = 0, rb = 0;
    if (!wide_kernel(bits1, bits2, kpos, prec, &qb, &rb)) return 0;
    return wide_lds(qb, kpos, rb, prec, bits2, n_means) <= lds_max ? qb : 0;
}

int mfma_wide_sorted(int k)
{
    int ks = 64;
    while (ks < k) ks *= 2;
    return ks;
}

int mfma_wide_cap(int k)
{
    return mfma_wide_sorted(k) + kWidePending;
}

hipError_t launch_scan_mfma_wide(const ScanArgs &a, int bits1, int bits2, int prec, int64_t grid, size_t lds_max,
                                 hipStream_t s)
{
    int qb = 0, rb = 0;
    WideKernel kern = wide_kernel(bits1, bits2, a.kpos, prec, &qb, &rb);
    if (!kern || grid < 8 || grid % 8 || a.k < 1 || a.k > kWideMaxK || a.mks != mfma_wide_sorted(a.k) ||
        a.mcap != mfma_wide_cap(a.k) || a.n_means < 1 || (prec != LVQ_FP32 && bits2 == 0 && a.n_means != 1))
        return hipErrorInvalidValue;
    const size_t lds = wide_lds(qb, a.kpos, rb, prec, bits2, a.n_means);
    if (lds > lds_max) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * wide_waves(rb)), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_frag32(const float *qk, int64_t nq, int kpos, int bits1, int qb, void *frag, hipStream_t s)
{
    const int chunk_pos = bits1 == 8 ? 32 : 64;
    if (qb < 1 || (bits1 != 4 && bits1 != 8) || kpos % chunk_pos) return hipErrorInvalidValue;
    if (nq <= 0) return hipSuccess;
    const int64_t tiles = (nq + 32 * qb - 1) / (32 * qb);
    hipLaunchKernelGGL(k_frag32, dim3((unsigned)tiles), dim3(256), 0, s, qk, nq, kpos, chunk_pos, qb,
                       reinterpret_cast<float4 *>(frag));
    return hipGetLastError();
}

}  // namespace lvq
