// k_mfma.hip -- exhaustive inner-product top-k on the matrix cores (MFMA):
// bfloat16 / float16 queries times first-level integer codes converted
// exactly to the same type (codes <= 255 are exact in both), FP32
// accumulation, then the per-row affine epilogue of Sec. 3.2
//   <q, x_hat> = c_m + l sum(q) + Delta <q, c1>
// and a fused threshold top-k per query (Sec. 2.1).
//
// Tiling.  A workgroup holds TQ = 32*QB queries; each of its four waves keeps
// all of them in registers as MFMA A fragments (v_mfma_f32_32x32x16, K order
// permuted consistently on both operands), and streams its own 32-row blocks
// of the store: a lane loads half of one row's codes per chunk (16 bytes),
// converts them to the MFMA type (byte -> f32 -> packed 16-bit) and feeds QB
// MFMAs per 16-deep step.  The next row block's codes are prefetched while
// the current one is multiplied.  Workgroups are mapped to (part, query tile)
// XCD-aware: each XCD walks a contiguous, part-major range of the tiles, so
// the workgroups running together on one XCD read the same rows through its
// L2.  Keys of candidates beating a query's running k-th best go to an LDS
// buffer that is compacted to k keys when it could overflow.
#include "k_common.h"

namespace lvq {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRowsPerWave = 32;
constexpr int kWaves = 4;
constexpr int kRowsPerIter = kRowsPerWave * kWaves;   // rows per workgroup round

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

// KPOS: code positions per row (kernel order); QB: 32-query blocks per
// workgroup.  Chunks: 16 bytes per lane half, i.e. 32 (8-bit) or 64 (4-bit)
// positions; steps per chunk: 2 (8-bit) or 4 (4-bit).
template <int B1, int KPOS, int QB, bool FP16>
__global__ __launch_bounds__(256, 1) void k_scan_mfma(ScanArgs a)
{
    constexpr int TQ = 32 * QB;
    constexpr int CHUNK_POS = B1 == 8 ? 32 : 64;
    constexpr int NCHUNK = KPOS / CHUNK_POS;
    constexpr int STEPS = B1 == 8 ? 2 : 4;
    static_assert(KPOS % CHUNK_POS == 0, "KPOS");

    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int half = lane >> 5, col = lane & 31;
    const int k = a.k;
    const int capq = a.capq;   // >= k + kRowsPerIter
    const int nm = a.n_means;

    // XCD-aware tile mapping: workgroup w runs on XCD w % 8; XCD x walks the
    // part-major tile sequence [x * per_xcd, (x+1) * per_xcd).
    const int64_t qtiles = (a.nq + TQ - 1) / TQ;
    const int64_t ntiles = qtiles * a.n_parts;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int part = (int)(tile / qtiles);
    const int64_t q0 = (tile % qtiles) * TQ;
    const int nqt = (int)min<int64_t>(TQ, a.nq - q0);
    const int64_t r0 = (int64_t)part * a.rows_per_part;
    const int64_t r1 = min<int64_t>(a.n_rows, r0 + a.rows_per_part);

    // LDS: per-query sum(q), c_m table, thresholds, counts, key buffers
    // (offsets are taken from the LDS base so every pointer stays in the LDS
    // address space: a round trip through an integer would turn the accesses
    // into flat ones, which wait for all outstanding global loads)
    float *qsum = reinterpret_cast<float *>(smem);              // TQ
    float *cmt = qsum + TQ;                                      // TQ x nm
    const size_t off = (((size_t)TQ * (1 + nm)) * sizeof(float) + 15) & ~(size_t)15;
    uint64_t *thr = reinterpret_cast<uint64_t *>(smem + off);    // TQ
    float *thr_f = reinterpret_cast<float *>(thr + TQ);          // TQ
    int *cnt = reinterpret_cast<int *>(thr_f + TQ);              // TQ
    uint64_t *buf = reinterpret_cast<uint64_t *>(cnt + TQ + (TQ & 1));
    uint64_t *tmp = buf + (size_t)TQ * capq;                     // 4 x k

    for (int t = tid; t < TQ; t += 256) {
        const bool in = t < nqt;
        qsum[t] = in ? a.qsum[q0 + t] : 0.0f;
        thr[t] = kNoKey;
        thr_f[t] = -__builtin_inff();
        cnt[t] = 0;
    }
    for (int t = tid; t < TQ * nm; t += 256) {
        const int qi = t / nm, m = t % nm;
        cmt[t] = qi < nqt ? a.cm[(q0 + qi) * nm + m] : 0.0f;
    }

    // A fragments: q16 holds, per query tile, [block][chunk][step][lane][8]
    uint4 afr[QB][NCHUNK][STEPS];
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.q16) + (tile % qtiles) * (int64_t)QB * NCHUNK * STEPS * 64;
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
            for (int c = 0; c < NCHUNK; ++c)
#pragma unroll
                for (int s = 0; s < STEPS; ++s) afr[b][c][s] = src[((b * NCHUNK + c) * STEPS + s) * 64 + lane];
    }
    __syncthreads();

    // Row blocks: lane (col, half) reads 16 bytes per chunk of row col.  The
    // next block's chunk c is loaded into the same registers as soon as the
    // current chunk c has been converted, so its latency overlaps the rest of
    // the current block.
    auto row_ptr = [&](int64_t rb, bool &in) {
        const int64_t slot = rb + col;
        in = slot < r1;
        return a.rows + (in ? slot : r0) * a.row_bytes;
    };

    uint4 vcur[NCHUNK];
    float4 hcur = make_float4(0.f, 0.f, 0.f, 0.f), hnext = hcur;
    uint2 ecur = make_uint2(1u, 0u), enext = ecur;
    bool icur = false, inext = false;
    int64_t rb = r0 + (int64_t)wave * kRowsPerWave;
    if (rb < r1) {
        const uint8_t *row = row_ptr(rb, icur);
        hcur = *reinterpret_cast<const float4 *>(row);
        ecur = *reinterpret_cast<const uint2 *>(row + 16);
#pragma unroll
        for (int c = 0; c < NCHUNK; ++c)
            vcur[c] = *reinterpret_cast<const uint4 *>(row + kHeaderBytes + c * 32 + half * 16);
    }

    for (int64_t base = r0; base < r1; base += kRowsPerIter) {
        const bool mine = rb < r1;
        const int64_t rb_next = rb + kRowsPerIter;
        // unconditional (clamped) prefetch: a load under a branch would make
        // every later wait count it as the most recent outstanding load
        const uint8_t *nrow = row_ptr(rb_next, inext);
        hnext = *reinterpret_cast<const float4 *>(nrow);
        enext = *reinterpret_cast<const uint2 *>(nrow + 16);
        if (mine) {
            f32x16 acc[QB];
#pragma unroll
            for (int b = 0; b < QB; ++b)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[b][i] = 0.0f;
#pragma unroll
            for (int c = 0; c < NCHUNK; ++c) {
#pragma unroll
                for (int s = 0; s < STEPS; ++s) {
                    const uint4 bfr = b_fragment<B1, FP16>(vcur[c], s);
#pragma unroll
                    for (int b = 0; b < QB; ++b) acc[b] = mfma<FP16>(afr[b][c][s], bfr, acc[b]);
                }
                vcur[c] = *reinterpret_cast<const uint4 *>(nrow + kHeaderBytes + c * 32 + half * 16);
            }
            // Epilogue: lane holds row `col` of the block and, per query block,
            // 16 queries: 8*g + 4*half + r (g, r < 4), i.e. four runs of four
            // consecutive queries, whose constants are read as float4.  All
            // scores are formed first; the append path runs only when some
            // lane has a score reaching its query's threshold.
            const int64_t slot = rb + col;
            const bool live = icur && ((__float_as_uint(hcur.w) >> 8) & 1u) && ecur.x <= a.epoch &&
                              a.epoch < ecur.y;
            const int mid = min((int)(__float_as_uint(hcur.w) & 0xFFu), nm - 1);
#pragma unroll
            for (int b = 0; b < QB; ++b) {
                float sc[16];
                bool pass[16];
                bool any = false;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int q4 = 32 * b + 8 * g + 4 * half;
                    const float4 qs = *reinterpret_cast<const float4 *>(qsum + q4);
                    const float4 tf = *reinterpret_cast<const float4 *>(thr_f + q4);
                    float4 cmv;
                    if (nm == 1) {
                        cmv = *reinterpret_cast<const float4 *>(cmt + q4);
                    } else {
                        cmv.x = cmt[(q4 + 0) * nm + mid];
                        cmv.y = cmt[(q4 + 1) * nm + mid];
                        cmv.z = cmt[(q4 + 2) * nm + mid];
                        cmv.w = cmt[(q4 + 3) * nm + mid];
                    }
                    const float qsv[4] = {qs.x, qs.y, qs.z, qs.w};
                    const float tfv[4] = {tf.x, tf.y, tf.z, tf.w};
                    const float cmq[4] = {cmv.x, cmv.y, cmv.z, cmv.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 4 * g + r;
                        sc[i] = fmaf(hcur.y, acc[b][i], fmaf(hcur.x, qsv[r], cmq[r]));
                        // tfv never rejects a score that can enter the top k
                        pass[i] = live && (q4 + r) < nqt && sc[i] >= tfv[r];
                        any |= pass[i];
                    }
                }
                if (__ballot(any)) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        if (!pass[i]) continue;
                        const int qi = 32 * b + 8 * (i >> 2) + 4 * half + (i & 3);
                        const uint64_t key = make_key(sc[i], (int32_t)slot, LVQ_IP);
                        if (key < thr[qi]) {
                            const int pos = atomicAdd(&cnt[qi], 1);
                            if (pos < capq) buf[(size_t)qi * capq + pos] = key;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // compaction: one LDS read per lane finds the queries whose buffer
        // could overflow next round; wave w compacts the ones with qi % 4 == w
        const bool last = base + kRowsPerIter >= r1;
        for (int q0w = 0; q0w < TQ; q0w += 64) {
            const int qi_l = q0w + lane;
            const bool need = qi_l < nqt && (last || min(cnt[qi_l], capq) > capq - kRowsPerIter) &&
                              (qi_l & (kWaves - 1)) == wave;
            uint64_t m = __ballot(need);
            while (m) {
                const int bit = __builtin_ctzll(m);
                m &= m - 1;
                const int qi = q0w + bit;
                const int n = min(cnt[qi], capq);
                uint64_t *qb = buf + (size_t)qi * capq;
                const int got = wave_compact(qb, n, k, tmp + (size_t)wave * k);
                if (lane == 0) {
                    cnt[qi] = got;
                    thr[qi] = got == k ? qb[k - 1] : kNoKey;
                    // Share the bound: this part holds k candidates whose score
                    // order is <= that of its k-th key, so no candidate with a
                    // larger score order (worse score) can reach the final top
                    // k in any part.  Ties stay admitted.
                    uint32_t gb = a.gthr[q0 + qi];
                    if (got == k) gb = min(gb, atomicMin(&a.gthr[q0 + qi], (uint32_t)(qb[k - 1] >> 32)));
                    thr_f[qi] = gb == 0xFFFFFFFFu ? -__builtin_inff() : key_score((uint64_t)gb << 32, LVQ_IP);
                }
            }
        }
        __syncthreads();
        rb = rb_next;
        hcur = hnext;
        ecur = enext;
        icur = inext;
    }
    for (int qi = wave; qi < nqt; qi += kWaves) {
        uint64_t *dst = a.part_keys + ((q0 + qi) * a.n_parts + part) * (int64_t)k;
        const int got = r1 > r0 ? cnt[qi] : 0;
        for (int i = lane; i < k; i += 64) dst[i] = i < got ? buf[(size_t)qi * capq + i] : kNoKey;
    }
}

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

using MfmaKernel = void (*)(ScanArgs);

template <int B1, bool FP16>
MfmaKernel mfma_lookup(int kpos, int *qb)
{
    switch (kpos) {
    case 96: *qb = 2; return B1 == 8 ? k_scan_mfma<8, 96, 2, FP16> : nullptr;
    case 128: *qb = 2; return k_scan_mfma<B1, 128, 2, FP16>;
    case 256: *qb = 2; return k_scan_mfma<B1, 256, 2, FP16>;
    case 384: *qb = 2; return k_scan_mfma<B1, 384, 2, FP16>;
    case 512: *qb = 2; return k_scan_mfma<B1, 512, 2, FP16>;
    case 768: *qb = 1; return k_scan_mfma<B1, 768, 1, FP16>;
    case 1024: *qb = 1; return k_scan_mfma<B1, 1024, 1, FP16>;
    default: return nullptr;
    }
}

}  // namespace

int mfma_query_block(int bits1, int kpos)
{
    if (bits1 != 4 && bits1 != 8) return 0;
    if (kpos % (bits1 == 8 ? 32 : 64)) return 0;
    int qb = 0;
    return (bits1 == 8 ? mfma_lookup<8, false>(kpos, &qb) : mfma_lookup<4, false>(kpos, &qb)) ? qb : 0;
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

hipError_t launch_prep16(const void *q, int64_t nq, int dim, int kpos, int bits1, int prec, const int32_t *kdim,
                         const float *means, int n_means, void *frag, float *qsum, float *cm, hipStream_t s)
{
    const int qb = mfma_query_block(bits1, kpos);
    if (!qb) return hipErrorInvalidValue;
    const int64_t tiles = (nq + 32 * qb - 1) / (32 * qb);
    auto kern = bits1 == 8 ? k_prep16<8> : k_prep16<4>;
    hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(256), 0, s, (const uint16_t *)q, nq, dim, kpos, qb,
                       prec == LVQ_FP16 ? 1 : 0, kdim, means, n_means, (uint16_t *)frag, qsum, cm);
    return hipGetLastError();
}

hipError_t launch_scan_mfma(const ScanArgs &a, int bits1, int prec, hipStream_t s)
{
    int qb = 0;
    MfmaKernel kern = nullptr;
    if (bits1 == 8)
        kern = prec == LVQ_FP16 ? mfma_lookup<8, true>(a.kpos, &qb) : mfma_lookup<8, false>(a.kpos, &qb);
    else
        kern = prec == LVQ_FP16 ? mfma_lookup<4, true>(a.kpos, &qb) : mfma_lookup<4, false>(a.kpos, &qb);
    if (!kern) return hipErrorInvalidValue;
    const int64_t qtiles = (a.nq + 32 * qb - 1) / (32 * qb);
    const int64_t ntiles = qtiles * a.n_parts;
    const int64_t grid = (ntiles + 7) / 8 * 8;
    const size_t lds = mfma_lds_bytes(qb, a.n_means, a.k, a.capq);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace lvq
