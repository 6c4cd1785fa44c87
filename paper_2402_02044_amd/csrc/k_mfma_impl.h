// k_mfma_impl.h -- exhaustive inner-product top-k on the matrix cores (MFMA):
// bfloat16 / float16 queries times integer codes converted exactly to the
// same type (codes <= 255 are exact in both), FP32 accumulation, then the
// per-row affine epilogue of Sec. 3.2
//   <q, x_hat> = c_m + l sum(q) + Delta <q, c1>                 (first level)
//   <q, x_hat> = c_m + (l - Delta/2) sum(q) + Delta <q, c1> + Delta2 <q, c2>
//                                                   (both levels, Sec. 2.3)
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
#pragma once

#include "k_mfma_ops.h"

namespace lvq {
namespace {

constexpr int kRowsPerWave = 32;
constexpr int kWaves = 4;
constexpr int kRowsPerIter = kRowsPerWave * kWaves;   // rows per workgroup round

// KPOS: code positions per row (kernel order); QB: 32-query blocks per
// workgroup; B2: 0 (first level) or 8 (both levels: the residual codes feed a
// second accumulator from the same query fragments).  Chunks: 16 bytes of
// first-level codes per lane half, i.e. 32 (8-bit) or 64 (4-bit) positions,
// and the residual bytes of the same positions (16 or 32 bytes); steps per
// chunk: 2 (8-bit) or 4 (4-bit).
template <int B1, int B2, int KPOS, int QB, bool FP16>
__global__ __launch_bounds__(256, 1) void k_scan_mfma(ScanArgs a)
{
    constexpr int TQ = 32 * QB;
    constexpr int CHUNK_POS = B1 == 8 ? 32 : 64;
    constexpr int NCHUNK = KPOS / CHUNK_POS;
    constexpr int STEPS = B1 == 8 ? 2 : 4;
    constexpr int RV = B1 == 4 ? 2 : 1;                   // residual uint4 loads per lane and chunk
    constexpr int RNCH = B2 ? NCHUNK : 1;                 // residual register chunks
    static_assert(KPOS % CHUNK_POS == 0, "KPOS");
    static_assert(B2 == 0 || B2 == 8, "residual width");

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
        // query slots past the batch admit nothing (+inf): the append test
        // needs no per-query range check
        thr_f[t] = in ? -__builtin_inff() : __builtin_inff();
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
    // Rows are the slots at list positions [r0, r1).  A lane's slot for a
    // block is read one block ahead of its row loads; positions past the part
    // read the list at r0 (a valid slot) and are masked out.
    auto slot_at = [&](int64_t pos) -> int64_t { return a.list[pos < r1 ? pos : r0]; };
    auto res_ptr = [&](int64_t slot) { return a.resid + slot * a.resid_bytes + half * (RV * 16); };

    uint4 vcur[NCHUNK];
    uint4 rcur[RNCH][RV];
    float4 hcur = make_float4(0.f, 0.f, 0.f, 0.f), hnext = hcur;
    uint2 ecur = make_uint2(1u, 0u), enext = ecur;
    bool icur = false, inext = false;
    int64_t rb = r0 + (int64_t)wave * kRowsPerWave;
    int64_t s_cur = 0, s_next = 0;
    if (rb < r1) {
        icur = rb + col < r1;
        s_cur = slot_at(rb + col);
        s_next = slot_at(rb + kRowsPerIter + col);
        const uint8_t *row = a.rows + s_cur * a.row_bytes;
        hcur = *reinterpret_cast<const float4 *>(row);
        ecur = *reinterpret_cast<const uint2 *>(row + 16);
#pragma unroll
        for (int c = 0; c < NCHUNK; ++c)
            vcur[c] = *reinterpret_cast<const uint4 *>(row + kHeaderBytes + c * 32 + half * 16);
        if constexpr (B2 != 0) {
            const uint8_t *res = res_ptr(s_cur);
#pragma unroll
            for (int c = 0; c < NCHUNK; ++c)
#pragma unroll
                for (int u = 0; u < RV; ++u)
                    rcur[c][u] = *reinterpret_cast<const uint4 *>(res + c * (2 * RV * 16) + u * 16);
        }
    }

    for (int64_t base = r0; base < r1; base += kRowsPerIter) {
        const bool mine = rb < r1;
        // shared per-query bounds for this round's compactions, loaded now so
        // their latency hides behind the round's products
        uint32_t gb_lane[(TQ + 63) / 64];
#pragma unroll
        for (int h = 0; h < (TQ + 63) / 64; ++h) {
            const int qi_l = 64 * h + lane;
            gb_lane[h] = a.gthr[q0 + (qi_l < nqt ? qi_l : 0)];
        }
        const int64_t rb_next = rb + kRowsPerIter;
        // unconditional (clamped) prefetch: a load under a branch would make
        // every later wait count it as the most recent outstanding load
        inext = rb_next + col < r1;
        const uint8_t *nrow = a.rows + s_next * a.row_bytes;
        const uint8_t *nres = B2 ? res_ptr(s_next) : nullptr;
        const int64_t s_after = slot_at(rb_next + kRowsPerIter + col);
        hnext = *reinterpret_cast<const float4 *>(nrow);
        enext = *reinterpret_cast<const uint2 *>(nrow + 16);
        if (mine) {
            f32x16 acc[QB], acc2[B2 ? QB : 1];
#pragma unroll
            for (int b = 0; b < QB; ++b)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[b][i] = 0.0f;
            if constexpr (B2 != 0) {
#pragma unroll
                for (int b = 0; b < QB; ++b)
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc2[b][i] = 0.0f;
            }
#pragma unroll
            for (int c = 0; c < NCHUNK; ++c) {
#pragma unroll
                for (int s = 0; s < STEPS; ++s) {
                    const uint4 bfr = b_fragment<B1, FP16>(vcur[c], s);
#pragma unroll
                    for (int b = 0; b < QB; ++b) acc[b] = mfma<FP16>(afr[b][c][s], bfr, acc[b]);
                    if constexpr (B2 != 0) {
                        const uint4 rfr = r_fragment<B1, FP16>(rcur[c], s);
#pragma unroll
                        for (int b = 0; b < QB; ++b) acc2[b] = mfma<FP16>(afr[b][c][s], rfr, acc2[b]);
                    }
                }
                vcur[c] = *reinterpret_cast<const uint4 *>(nrow + kHeaderBytes + c * 32 + half * 16);
                if constexpr (B2 != 0) {
#pragma unroll
                    for (int u = 0; u < RV; ++u)
                        rcur[c][u] = *reinterpret_cast<const uint4 *>(nres + c * (2 * RV * 16) + u * 16);
                }
            }
            // Epilogue: lane holds row `col` of the block and, per query block,
            // 16 queries: 8*g + 4*half + r (g, r < 4), i.e. four runs of four
            // consecutive queries, whose constants are read as float4.  All
            // scores are formed first; the append path runs only when some
            // lane has a score reaching its query's threshold.
            const int64_t slot = s_cur;
            const bool live = icur && ((__float_as_uint(hcur.w) >> 8) & 1u) && ecur.x <= a.epoch &&
                              a.epoch < ecur.y;
            const int mid = min((int)(__float_as_uint(hcur.w) & 0xFFu), nm - 1);
            // both levels: x_hat = mu + (l - Delta/2) + Delta c1 + Delta2 c2
            const float lp = B2 ? hcur.x - 0.5f * hcur.y : hcur.x;
#pragma unroll
            for (int b = 0; b < QB; ++b) {
                // the block's per-query constants, all read before any is used
                float4 qsA[4], tfA[4], cmA[4];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int q4 = 32 * b + 8 * g + 4 * half;
                    qsA[g] = *reinterpret_cast<const float4 *>(qsum + q4);
                    tfA[g] = *reinterpret_cast<const float4 *>(thr_f + q4);
                }
                if (nm == 1) {
#pragma unroll
                    for (int g = 0; g < 4; ++g)
                        cmA[g] = *reinterpret_cast<const float4 *>(cmt + 32 * b + 8 * g + 4 * half);
                } else {
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int q4 = 32 * b + 8 * g + 4 * half;
                        cmA[g] = make_float4(cmt[(q4 + 0) * nm + mid], cmt[(q4 + 1) * nm + mid],
                                             cmt[(q4 + 2) * nm + mid], cmt[(q4 + 3) * nm + mid]);
                    }
                }
                float sc[16];
                uint32_t passm = 0u;   // bit i: score i reaches its query's bound
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float qsv[4] = {qsA[g].x, qsA[g].y, qsA[g].z, qsA[g].w};
                    const float tfv[4] = {tfA[g].x, tfA[g].y, tfA[g].z, tfA[g].w};
                    const float cmv[4] = {cmA[g].x, cmA[g].y, cmA[g].z, cmA[g].w};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 4 * g + r;
                        const float cmq = cmv[r];
                        float v = fmaf(hcur.y, acc[b][i], fmaf(lp, qsv[r], cmq));
                        if constexpr (B2 != 0) v = fmaf(hcur.z, acc2[b][i], v);
                        sc[i] = v;
                        // tfv never rejects a score that can enter the top k
                        passm |= (live && v >= tfv[r]) ? 1u << i : 0u;
                    }
                }
                if (__ballot(passm != 0u)) {
                    // Append: the bound test above already admits only
                    // scores that can reach the top k; the buffer keeps room
                    // for one round of appends, so no key is lost.
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        if (!((passm >> i) & 1u)) continue;
                        const int qi = 32 * b + 8 * (i >> 2) + 4 * half + (i & 3);
                        const int pos = atomicAdd(&cnt[qi], 1);
                        if (pos < capq) buf[(size_t)qi * capq + pos] = make_key(sc[i], (int32_t)slot, LVQ_IP);
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
            const uint32_t gpre = gb_lane[q0w / 64];
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
                // the shared bound as read at the start of this round
                uint32_t gb = __shfl(gpre, bit, 64);
                if (lane == 0) {
                    cnt[qi] = got;
                    thr[qi] = got == k ? qb[k - 1] : kNoKey;
                    // Share the bound: this part holds k candidates whose score
                    // order is <= that of its k-th key, so no candidate with a
                    // larger score order (worse score) can reach the final top
                    // k in any part.  Ties stay admitted.  The update does not
                    // wait for the atomic (no return value): other parts see it
                    // at their next round.
                    if (got == k) {
                        const uint32_t mine = (uint32_t)(qb[k - 1] >> 32);
                        gb = min(gb, mine);
                        __hip_atomic_fetch_min(&a.gthr[q0 + qi], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    thr_f[qi] = gb == 0xFFFFFFFFu ? -__builtin_inff() : key_score((uint64_t)gb << 32, LVQ_IP);
                }
            }
        }
        __syncthreads();
        rb = rb_next;
        s_cur = s_next;
        s_next = s_after;
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

using MfmaKernel = void (*)(ScanArgs);

// Instantiated position counts and their query blocks per workgroup (one
// block where two would not fit the registers: long rows, and both levels
// from 384 positions on, which hold the residual codes as well).
template <int B1, int B2, bool FP16>
MfmaKernel mfma_lookup(int kpos, int *qb)
{
    constexpr int QB_MID = B2 ? 1 : 2;   // 384 and 512 positions
    switch (kpos) {
    case 96: *qb = 2; return B1 == 8 ? k_scan_mfma<8, B2, 96, 2, FP16> : nullptr;
    case 128: *qb = 2; return k_scan_mfma<B1, B2, 128, 2, FP16>;
    case 256: *qb = 2; return k_scan_mfma<B1, B2, 256, 2, FP16>;
    case 384: *qb = QB_MID; return k_scan_mfma<B1, B2, 384, QB_MID, FP16>;
    case 512: *qb = QB_MID; return k_scan_mfma<B1, B2, 512, QB_MID, FP16>;
    case 768: *qb = 1; return k_scan_mfma<B1, B2, 768, 1, FP16>;
    case 1024: *qb = 1; return k_scan_mfma<B1, B2, 1024, 1, FP16>;
    default: return nullptr;
    }
}

}  // namespace
}  // namespace lvq
