// k_mfma_wide_impl.h -- exhaustive inner-product top-k on the matrix cores
// with the queries staged in LDS (Sec. 3.2 similarity, Sec. 2.1 k-NN):
//   <q, x_hat> = c_m + l' sum(q) + <q, y>,
//   y = Delta c1 (first level, l' = l) or Delta c1 + Delta2 c2 (both levels,
//   l' = l - Delta / 2).
// 16-bit forms: bf16 / fp16 queries times codes converted exactly to the
// same type (v_mfma_f32_32x32x16), Delta applied to the FP32 accumulator; at
// both levels a second accumulator chain takes the residual codes, scaled by
// Delta2.  FP32 forms: FP32 queries times one FP32 value per lane
// (v_mfma_f32_32x32x2): the exactly converted first-level code (Delta applied
// to the accumulator) or, at both levels, y decoded per lane as the vector
// path decodes it (Delta c1 rounded, then fused with Delta2 c2).  c_m is one
// value per query with one mean; at both levels and in FP32 the row's mean
// picks it from an LDS table [mean][query], so any number of means whose
// table fits.
//
// Tiling.  A workgroup of eight waves (two per SIMD) copies the MFMA
// fragments of TQ = 32*QB queries into LDS once per tile, so every code
// fragment a wave converts (FP32: every code a lane converts) feeds QB MFMAs,
// one per 32-query block.  The codes are the A operand and the queries the B
// operand: lane l then owns query (l & 31) of every block -- its sum(q), c_m
// (one mean) and admission bound stay in registers -- and rows 8*(i/4) + 4*(l >> 5) +
// (i % 4), i < 16, of each 32-row block.  A wave scores RB = 1 or 2 blocks
// of 32 rows per round (two: each query fragment it reads from LDS feeds two
// MFMAs; one where the accumulators of four query blocks or of two chains
// take the registers); its 16-byte code pieces stream through a ring of
// loads a few chunks ahead, which runs on into the next round's rows.
//
// Top-k.  Each query keeps, in the workgroup's region of device memory, its
// KS best keys so far (sorted, KS = k rounded up to a power of two >= 64)
// followed by the keys pending a merge.  The epilogue tests a lane's 16
// scores against its query's bound; each passing score takes a pending slot
// with one LDS atomic and writes its key.  After the round's appends (a
// barrier), queries with 64 or more pending keys are merged by their owner
// wave: 64 keys at a time are sorted in registers and folded into the sorted
// list by one bitonic merge, and the bound becomes the k-th key, shared with
// the other row parts through gthr (an atomic minimum of score-order keys).
// The merges overlap the next round's products and end before its first
// barrier, which precedes its appends.  Workgroups are persistent, one per
// compute unit, and walk the part-major (part, query tile) sequence
// XCD-aware: the workgroups of one XCD take consecutive tiles, which read
// the same rows through its L2.  The both-level forms also read each row's
// residual codes through the ring (the decoded FP32 form its header a round
// ahead).
#pragma once

#include <type_traits>

#include "k_mfma_ops.h"

namespace lvq {
namespace {

// Waves per workgroup: two per SIMD, with 256 registers each, whether a
// wave scores two 32-row blocks per round (each query fragment read from LDS
// feeds two MFMAs) or one (where four query blocks, or a second accumulator
// chain, take the registers of the second block).  Three waves per SIMD with
// one block each spilled about 80 registers in the both-level forms and
// served 13% fewer queries.
__host__ __device__ constexpr int wide_waves(int)
{
    return 8;
}
// Chunks of codes in flight: a divisor of the chunk count, so that the ring
// slot of chunk c is c % RING in every round.  Up to four (eight in the
// 16-bit first-level forms with one row block per wave); two when each
// chunk also brings residual codes (the registers of a deeper ring would
// spill).
__host__ __device__ constexpr int wide_ring(int nchunk, bool resid)
{
    return resid ? (nchunk % 2 == 0 ? 2 : nchunk % 3 == 0 ? 3 : 1)
                 : (nchunk % 4 == 0 ? 4 : nchunk % 3 == 0 ? 3 : nchunk % 2 == 0 ? 2 : 1);
}
constexpr int kWideMerge = 64;                       // pending keys that trigger a merge
constexpr int kWidePending = 512 + kWideMerge;       // pending room: < 64 carried + a round of <= 512 rows
constexpr int kWideMaxK = 512;

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = __shfl((uint32_t)v, src, 64);
    const uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic merge of a bitonic sequence of 64*E keys held E per lane
// (element i = e*64 + lane).
template <int E>
__device__ __forceinline__ void wave_bitonic_merge(uint64_t (&v)[E])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 32 * E; j > 0; j >>= 1) {
        if (j >= 64) {
            const int je = j >> 6;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int pe = e ^ je;
                if (pe > e) {
                    const uint64_t a = v[e], b = v[pe];
                    v[e] = a < b ? a : b;
                    v[pe] = a < b ? b : a;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint64_t o = shfl_xor_u64(v[e], j);
                const bool lower = (lane & j) == 0;
                v[e] = lower ? (o < v[e] ? o : v[e]) : (o < v[e] ? v[e] : o);
            }
        }
    }
}

// One wave folds the pend keys appended at rq[KS + poff ..] into query
// region rq's sorted KS = 64*E best (rq[0 .. KS)), 64 at a time: the chunk is sorted,
// reversed and compared position-wise with the last 64 of the sorted list
// (the half-cleaner of the bitonic sequence list ++ reversed chunk, whose
// lower half is the KS smallest of both), then merged.  The list goes back to
// rq[0..KS); when out is set, its first k keys go there too.  Returns the
// number of valid keys among the first k; *kth receives the k-th.
template <int E>
__device__ __forceinline__ int merge_region(uint64_t *rq, int poff, int pend, int k, uint64_t *out, uint64_t *kth)
{
    constexpr int KS = 64 * E;
    const int lane = threadIdx.x & 63;
    uint64_t top[E];
#pragma unroll
    for (int e = 0; e < E; ++e) top[e] = rq[e * 64 + lane];
    for (int c = 0; c < pend; c += 64) {
        uint64_t x[1] = {c + lane < pend ? rq[KS + poff + c + lane] : kNoKey};
        wave_bitonic_sort<1>(x);
        const uint64_t xr = shfl_u64(x[0], 63 - lane);
        top[E - 1] = xr < top[E - 1] ? xr : top[E - 1];
        wave_bitonic_merge<E>(top);
    }
    int valid = 0;
    uint64_t kk = kNoKey;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * 64 + lane;
        rq[i] = top[e];
        if (i < k) {
            if (out) out[i] = top[e];
            valid += top[e] != kNoKey;
        }
        if (i == k - 1) kk = top[e];
    }
    *kth = readlane_u64(kk, (k - 1) & 63);
    return wave_sum_i32(valid);
}

__device__ __forceinline__ int merge_region_ks(int ks, uint64_t *rq, int poff, int pend, int k, uint64_t *out,
                                               uint64_t *kth)
{
    if (ks == 64) return merge_region<1>(rq, poff, pend, k, out, kth);
    if (ks == 128) return merge_region<2>(rq, poff, pend, k, out, kth);
    if (ks == 256) return merge_region<4>(rq, poff, pend, k, out, kth);
    return merge_region<8>(rq, poff, pend, k, out, kth);
}

// LDS bytes of a workgroup: query fragments (esize bytes per value),
// per-wave row constants (row_bytes per row: l, Delta, slot; with a c_m table
// also the mean id; with a residual chain also Delta2), per-query bounds and
// pending counts, and the c_m table ([mean][query], n_tab means; 0 for none).
__host__ __device__ constexpr size_t wide_lds_bytes(int qb, int kpos, int rb, int esize, int n_tab, int row_bytes)
{
    return (size_t)32 * qb * kpos * esize + (size_t)wide_waves(rb) * 32 * rb * row_bytes + (size_t)32 * qb * 8 +
           (size_t)32 * qb * n_tab * 4;
}

template <int B1, int B2, int KPOS, int QB, int RB, int PREC>
__global__ __launch_bounds__(64 * wide_waves(RB), 1) void k_scan_mfma_wide(ScanArgs a)
{
    constexpr bool F32 = PREC == LVQ_FP32, FP16 = PREC == LVQ_FP16;
    constexpr bool RES = B2 != 0;         // both levels: residual codes read with the codes
    constexpr bool DEC = RES && F32;      // FP32: A values Delta c1 + Delta2 c2 decoded per lane
    constexpr bool CH2 = RES && !F32;     // 16-bit: a second accumulator chain for the residual codes
    constexpr bool MM = F32 || RES;       // several means: c_m of (row mean, query) from the LDS table
    static_assert(!RES || B2 == 8, "both levels: 8-bit residual codes");
    constexpr int WAVES = wide_waves(RB);
    constexpr int RW = 32 * RB;               // rows per wave and round
    constexpr int RROUND = WAVES * RW;        // rows per round
    constexpr int TQ = 32 * QB;
    constexpr int CHUNK_POS = B1 == 8 ? 32 : 64;
    constexpr int NCHUNK = KPOS / CHUNK_POS;
    // 16-byte query fragments per chunk and block: 8 positions each in 16
    // bits, 4 in FP32 (one per lane and MFMA)
    constexpr int STEPS = F32 ? CHUNK_POS / 8 : CHUNK_POS / 16;
    // eight chunks in flight where the registers allow it (16-bit first
    // level, one row block per wave): a row missing in L2 then waits less
    constexpr int RING = (!RES && !F32 && RB == 1 && NCHUNK % 8 == 0) ? 8 : wide_ring(NCHUNK, RES);
    // residual 16-byte pieces per lane and chunk (one 8-bit code per
    // first-level position)
    constexpr int RP = RES ? CHUNK_POS / 32 : 1;
    constexpr int NFRAG = QB * NCHUNK * STEPS * 64;   // 16-byte fragments per query tile
    static_assert(KPOS % CHUNK_POS == 0, "KPOS");
    static_assert(NCHUNK % RING == 0, "every round starts at ring slot 0");
    static_assert(RROUND + kWideMerge <= kWidePending, "pending room");

    extern __shared__ __align__(16) unsigned char smem[];
    uint4 *qf = reinterpret_cast<uint4 *>(smem);
    float *rl = reinterpret_cast<float *>(qf + NFRAG);              // [wave][RW] l', NaN if not scored
    float *rd = rl + WAVES * RW;                                    // [wave][RW] Delta (1 when decoded)
    int32_t *rs = reinterpret_cast<int32_t *>(rd + WAVES * RW);     // [wave][RW] slot
    int32_t *rm = rs + WAVES * RW;                                  // [wave][RW] mean id (c_m table)
    float *rd2 = reinterpret_cast<float *>(rm + (MM ? WAVES * RW : 0));     // [wave][RW] Delta2 (two chains)
    float *thr_f = rd2 + (CH2 ? WAVES * RW : 0);                    // TQ admission bounds
    int *cnt = reinterpret_cast<int *>(thr_f + TQ);                 // TQ pending keys
    float *cmt = reinterpret_cast<float *>(cnt + TQ);               // [mean][TQ] c_m

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int half = lane >> 5, col = lane & 31;
    const int k = a.k, cap = a.mcap, ks = a.mks;
    const bool one_mean = a.n_means == 1;
    uint64_t *region = a.mkeys + (size_t)blockIdx.x * TQ * cap;
    float *wl = rl + wave * RW, *wd = rd + wave * RW, *wd2 = rd2 + wave * RW;
    int32_t *ws = rs + wave * RW, *wm = rm + wave * RW;

    const int64_t qtiles = (a.nq + TQ - 1) / TQ;
    const int64_t ntiles = qtiles * a.n_parts;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t gx = gridDim.x / 8;   // workgroups per XCD; the grid is a multiple of 8
    for (int64_t it = blockIdx.x / 8; it < per_xcd; it += gx) {
        const int64_t tile = (int64_t)(blockIdx.x % 8) * per_xcd + it;
        if (tile >= ntiles) break;
        const int part = (int)(tile / qtiles);
        const int64_t qt = tile % qtiles;
        const int64_t q0 = qt * TQ;
        const int nqt = (int)min<int64_t>(TQ, a.nq - q0);
        const int64_t r0 = (int64_t)part * a.rows_per_part;
        const int64_t r1 = min<int64_t>(a.n_rows, r0 + a.rows_per_part);
        auto out_keys = [&](int qi) { return a.part_keys + ((q0 + qi) * a.n_parts + part) * (int64_t)k; };

        __syncthreads();   // the previous tile is done with LDS
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.q16) + qt * NFRAG;
            for (int e = tid; e < NFRAG; e += 64 * WAVES) qf[e] = src[e];
        }
        for (int t = tid; t < TQ; t += 64 * WAVES) {
            // query slots past the batch admit nothing
            thr_f[t] = t < nqt ? -__builtin_inff() : __builtin_inff();
            cnt[t] = 0;
        }
        if (MM && !one_mean) {
            for (int t = tid; t < a.n_means * TQ; t += 64 * WAVES) {
                const int m = t / TQ, qi = t % TQ;
                cmt[t] = qi < nqt ? a.cm[(q0 + qi) * a.n_means + m] : 0.0f;
            }
        }
        for (int t = tid; t < TQ * ks; t += 64 * WAVES) region[(size_t)(t / ks) * cap + t % ks] = kNoKey;
        float qs[QB], cq[QB], tau[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const int qi = 32 * b + col;
            const bool in = qi < nqt;
            qs[b] = in ? a.qsum[q0 + qi] : 0.0f;
            cq[b] = in && one_mean ? a.cm[q0 + qi] : 0.0f;
            tau[b] = in ? -__builtin_inff() : __builtin_inff();
        }
        __syncthreads();

        if (r0 >= r1) {
            // an empty part contributes no keys
            for (int qi = wave; qi < nqt; qi += WAVES)
                for (int i = lane; i < k; i += 64) out_keys(qi)[i] = kNoKey;
            continue;
        }
        // Rows are the slots at list positions [r0, r1); positions past the
        // part read the slot at r0 (valid) and are not scored.  Row block j
        // of the wave in round r: positions r0 + RROUND * r + RW * wave +
        // 32 * j + (0..31).
        auto slot_at = [&](int64_t pos) -> int32_t { return a.list[pos < r1 ? pos : r0]; };
        auto codes = [&](int32_t slot) { return a.rows + (int64_t)slot * a.row_bytes + kHeaderBytes + half * 16; };
        auto resid = [&](int32_t slot) { return a.resid + (int64_t)slot * a.resid_bytes + half * 16 * RP; };
        auto header = [&](int32_t slot) { return a.rows + (int64_t)slot * a.row_bytes; };
        const int64_t wrow = (int64_t)wave * RW + col;
        int32_t sc[RB], sn[RB];
        uint4 ring[RING][RB], rring[RING][RB][RP];
        // decoded: the headers of the round's rows, read a round ahead
        float4 hd[RB];
        uint2 ep[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            sc[j] = slot_at(r0 + wrow + 32 * j);
            sn[j] = slot_at(r0 + RROUND + wrow + 32 * j);
            const uint8_t *p = codes(sc[j]);
#pragma unroll
            for (int c = 0; c < RING; ++c) ring[c][j] = *reinterpret_cast<const uint4 *>(p + c * 32);
            if constexpr (RES) {
                const uint8_t *r = resid(sc[j]);
#pragma unroll
                for (int c = 0; c < RING; ++c)
#pragma unroll
                    for (int w = 0; w < RP; ++w)
                        rring[c][j][w] = *reinterpret_cast<const uint4 *>(r + c * 32 * RP + 16 * w);
            }
            if constexpr (DEC) {
                hd[j] = *reinterpret_cast<const float4 *>(header(sc[j]));
                ep[j] = *reinterpret_cast<const uint2 *>(header(sc[j]) + 16);
            }
        }
        f32x16 acc[RB][QB], acc2[CH2 ? RB : 1][CH2 ? QB : 1];
        for (int64_t base = r0; base < r1; base += RROUND) {
            const bool last = base + RROUND >= r1;
            int32_t sa[RB];
#pragma unroll
            for (int j = 0; j < RB; ++j) sa[j] = slot_at(base + 2 * RROUND + wrow + 32 * j);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
                for (int b = 0; b < QB; ++b)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        acc[j][b][i] = 0.0f;
                        if constexpr (CH2) acc2[j][b][i] = 0.0f;
                    }
            // decoding scales of the lane's own rows
            float s1[RB], s2[RB];
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                s1[j] = DEC ? hd[j].y : 0.0f;
                s2[j] = DEC ? hd[j].z : 0.0f;
            }
            // The products.  Halfway through, the rows' headers (their lines
            // were read with the first codes; decoded: the next round's) and
            // the other parts' shared bounds for the lane's queries are
            // loaded.
            float4 hn[RB];
            uint2 en[RB];
            uint32_t gb[QB];
#pragma unroll
            for (int c = 0; c < NCHUNK; ++c) {
                // Chunks are scheduling regions: the compiler otherwise sinks
                // each ring load to its use and waits on it there.
                __builtin_amdgcn_sched_barrier(0);
                if (c == NCHUNK / 2) {
#pragma unroll
                    for (int j = 0; j < RB; ++j) {
                        const uint32_t *h = reinterpret_cast<const uint32_t *>(header(DEC ? sn[j] : sc[j]));
                        hn[j] = make_float4(__uint_as_float(h[0]), __uint_as_float(h[1]), __uint_as_float(h[2]),
                                            __uint_as_float(h[3]));
                        en[j] = make_uint2(h[4], h[5]);
                    }
#pragma unroll
                    for (int b = 0; b < QB; ++b) {
                        const int qi = 32 * b + col;
                        gb[b] = a.gthr[q0 + (qi < nqt ? qi : 0)];
                    }
                }
                uint4 v[RB], rv[RB][RP];
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    v[j] = ring[c % RING][j];
                    const bool cur = c + RING < NCHUNK;
                    const int cn = cur ? c + RING : c + RING - NCHUNK;
                    ring[c % RING][j] = *reinterpret_cast<const uint4 *>(codes(cur ? sc[j] : sn[j]) + cn * 32);
                    if constexpr (RES) {
                        const uint8_t *r = resid(cur ? sc[j] : sn[j]) + cn * 32 * RP;
#pragma unroll
                        for (int w = 0; w < RP; ++w) {
                            rv[j][w] = rring[c % RING][j][w];
                            rring[c % RING][j][w] = *reinterpret_cast<const uint4 *>(r + 16 * w);
                        }
                    }
                }
                if constexpr (F32) {
                    // code 4 s + e of the lane's piece is byte e of word s
                    // (and so is its residual code)
                    uint32_t cw[RB][STEPS], rw[RB][DEC ? STEPS : 1];
#pragma unroll
                    for (int j = 0; j < RB; ++j) {
                        code_words<B1>(v[j], cw[j]);
                        if constexpr (DEC) resid_words<B1>(rv[j], rw[j]);
                    }
#pragma unroll
                    for (int s = 0; s < STEPS; ++s) {
                        float4 bq[QB];
#pragma unroll
                        for (int b = 0; b < QB; ++b)
                            bq[b] = reinterpret_cast<const float4 *>(qf)[((b * NCHUNK + c) * STEPS + s) * 64 + lane];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            float af[RB];
#pragma unroll
                            for (int j = 0; j < RB; ++j) {
                                const float c1 = (float)((cw[j][s] >> (8 * e)) & 0xFFu);
                                if constexpr (DEC) {
                                    const float c2 = (float)((rw[j][DEC ? s : 0] >> (8 * e)) & 0xFFu);
                                    af[j] = fmaf(s2[j], c2, s1[j] * c1);
                                } else {
                                    af[j] = c1;
                                }
                            }
#pragma unroll
                            for (int b = 0; b < QB; ++b) {
                                const float bv = e == 0 ? bq[b].x : e == 1 ? bq[b].y : e == 2 ? bq[b].z : bq[b].w;
#pragma unroll
                                for (int j = 0; j < RB; ++j) acc[j][b] = mfma_f32(af[j], bv, acc[j][b]);
                            }
                        }
                    }
                } else {
                    // the chunk's query fragments are read first, so that
                    // their LDS latency overlaps the conversions and products
                    uint4 bqs[STEPS][QB];
#pragma unroll
                    for (int s = 0; s < STEPS; ++s)
#pragma unroll
                        for (int b = 0; b < QB; ++b) bqs[s][b] = qf[((b * NCHUNK + c) * STEPS + s) * 64 + lane];
#pragma unroll
                    for (int s = 0; s < STEPS; ++s) {
                        uint4 af[RB], af2[RB];
#pragma unroll
                        for (int j = 0; j < RB; ++j) {
                            af[j] = b_fragment<B1, FP16>(v[j], s);
                            if constexpr (CH2) af2[j] = r_fragment<B1, FP16>(rv[j], s);
                        }
#pragma unroll
                        for (int b = 0; b < QB; ++b) {
                            const uint4 bq = bqs[s][b];
#pragma unroll
                            for (int j = 0; j < RB; ++j) {
                                acc[j][b] = mfma<FP16>(af[j], bq, acc[j][b]);
                                if constexpr (CH2) acc2[j][b] = mfma<FP16>(af2[j], bq, acc2[j][b]);
                            }
                        }
                    }
                    // LDS reads of the chunk ahead of its products (up to
                    // 768 positions; longer rows spill with it)
                    if constexpr (KPOS <= 768) {
                        __builtin_amdgcn_sched_group_barrier(0x100, STEPS * QB, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, STEPS * QB * RB * (CH2 ? 2 : 1), 0);
                    }
                }
            }

            // the previous round's merges are done: their bounds are in thr_f
            __syncthreads();
            // (branch-free, so that the LDS reads of all blocks go out together)
            float tf[QB];
#pragma unroll
            for (int b = 0; b < QB; ++b) tf[b] = thr_f[32 * b + col];
#pragma unroll
            for (int b = 0; b < QB; ++b) {
                const float other = key_score((uint64_t)gb[b] << 32, LVQ_IP);
                tau[b] = fmaxf(tau[b], fmaxf(tf[b], gb[b] != 0xFFFFFFFFu ? other : -__builtin_inff()));
            }
            // Row constants of the round to the wave's LDS area: half 0
            // writes l' (NaN for rows not scored: dead, outside the snapshot,
            // past the part) and the slot, half 1 Delta (1 when decoded) and
            // the mean id.
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                const float4 H = DEC ? hd[j] : hn[j];
                const uint2 E = DEC ? ep[j] : en[j];
                const uint32_t f = __float_as_uint(H.w);
                const bool live = base + wrow + 32 * j < r1 && ((f >> 8) & 1u) && E.x <= a.epoch && a.epoch < E.y;
                if (half == 0) {
                    wl[32 * j + col] = live ? (RES ? H.x - 0.5f * H.y : H.x) : __builtin_nanf("");
                    ws[32 * j + col] = sc[j];
                    if constexpr (CH2) wd2[32 * j + col] = H.z;
                } else {
                    wd[32 * j + col] = DEC ? 1.0f : H.y;
                    if constexpr (MM) {
                        const int mid = (int)(f & 0xFFu);
                        wm[32 * j + col] = mid < a.n_means ? mid : 0;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // Lane rows 32*j + 8*g + 4*half + r4, r4 < 4: the score of (row,
            // query 32*b + col) is c_m + l' sum(q) + Delta <q, c1> (decoded:
            // + <q, y>; two chains: + Delta2 <q, c2>).  A score that reaches
            // its query's bound (a NaN score, from a row not scored, never
            // does) takes the next pending slot of that query by an LDS
            // atomic and writes its key there.  With several means c_m comes
            // from the LDS table by the row's mean id, else from the lane's
            // registers.
            auto epilogue = [&](auto tab) {
                constexpr bool TAB = decltype(tab)::value;
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    auto cmv = [&](int b, int m) {
                        if constexpr (TAB) return cmt[m * TQ + 32 * b + col];
                        else return cq[b];
                    };
                    auto score = [&](int b, int i, float l, float dlt, float d2, int m) {
                        const float t = fmaf(dlt, acc[j][b][i], fmaf(l, qs[b], cmv(b, m)));
                        if constexpr (CH2) return fmaf(d2, acc2[j][b][i], t);
                        else return t;
                    };
                    if constexpr (CH2) {
                        // One sweep: each score that reaches its bound is
                        // appended at once.  A score here costs three
                        // products and three LDS values (l', Delta, Delta2;
                        // c_m by mean), so a first sweep for the largest
                        // score per block, as below, costs more than it
                        // saves.
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const float4 L = *reinterpret_cast<const float4 *>(wl + 32 * j + 8 * g + 4 * half);
                            const float4 D = *reinterpret_cast<const float4 *>(wd + 32 * j + 8 * g + 4 * half);
                            int4 M4 = make_int4(0, 0, 0, 0);
                            if constexpr (TAB) M4 = *reinterpret_cast<const int4 *>(wm + 32 * j + 8 * g + 4 * half);
                            const float4 D2 = *reinterpret_cast<const float4 *>(wd2 + 32 * j + 8 * g + 4 * half);
                            const float lr[4] = {L.x, L.y, L.z, L.w}, dr[4] = {D.x, D.y, D.z, D.w};
                            const float d2r[4] = {D2.x, D2.y, D2.z, D2.w};
                            const int mr[4] = {M4.x, M4.y, M4.z, M4.w};
#pragma unroll
                            for (int b = 0; b < QB; ++b)
#pragma unroll
                                for (int r4 = 0; r4 < 4; ++r4) {
                                    const float sv = score(b, 4 * g + r4, lr[r4], dr[r4], d2r[r4], mr[r4]);
                                    if (sv >= tau[b]) {
                                        // the slot read and the atomic share one LDS wait;
                                        // the position is clamped (the pending room holds
                                        // a round's keys, so it never is)
                                        const int32_t slot = ws[32 * j + 8 * g + 4 * half + r4];
                                        const int qi = 32 * b + col;
                                        const int pos = min(atomicAdd(&cnt[qi], 1), kWidePending - 1);
                                        region[(size_t)qi * cap + ks + pos] = make_key(sv, slot, LVQ_IP);
                                    }
                                }
                        }
                        continue;
                    }
                    // One product chain: a first sweep takes each lane's
                    // largest score per query block; only blocks where some
                    // lane reaches its bound are scored again, appending
                    // each passing key.  A branch per score in the first
                    // sweep measured slower here.
                    float mx[QB];
#pragma unroll
                    for (int b = 0; b < QB; ++b) mx[b] = -__builtin_inff();
                    // the rows' l' and Delta stay in registers for the
                    // passing blocks' second scoring (not in the decoded
                    // forms with two query blocks, where they would spill)
                    constexpr bool KEEP = !(DEC && QB > 1);
                    float4 Lk[KEEP ? 4 : 1], Dk[KEEP ? 4 : 1];
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const float4 L = *reinterpret_cast<const float4 *>(wl + 32 * j + 8 * g + 4 * half);
                        const float4 D = *reinterpret_cast<const float4 *>(wd + 32 * j + 8 * g + 4 * half);
                        if constexpr (KEEP) {
                            Lk[g] = L;
                            Dk[g] = D;
                        }
                        int4 M4 = make_int4(0, 0, 0, 0);
                        if constexpr (TAB) M4 = *reinterpret_cast<const int4 *>(wm + 32 * j + 8 * g + 4 * half);
                        float4 D2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                        if constexpr (CH2) D2 = *reinterpret_cast<const float4 *>(wd2 + 32 * j + 8 * g + 4 * half);
                        const float lr[4] = {L.x, L.y, L.z, L.w}, dr[4] = {D.x, D.y, D.z, D.w};
                        const float d2r[4] = {D2.x, D2.y, D2.z, D2.w};
                        const int mr[4] = {M4.x, M4.y, M4.z, M4.w};
#pragma unroll
                        for (int b = 0; b < QB; ++b)
#pragma unroll
                            for (int r4 = 0; r4 < 4; ++r4) {
                                const float sv = score(b, 4 * g + r4, lr[r4], dr[r4], d2r[r4], mr[r4]);
                                mx[b] = fmaxf(mx[b], sv);   // a NaN score leaves mx[b]
                            }
                    }
#pragma unroll
                    for (int b = 0; b < QB; ++b) {
                        if (!__ballot(mx[b] >= tau[b])) continue;
                        const int qi = 32 * b + col;
                        uint64_t *dst = region + (size_t)qi * cap + ks;
                        if constexpr (!KEEP) {
#pragma unroll 4
                            for (int i = 0; i < 16; ++i) {
                                const int m = 32 * j + 8 * (i >> 2) + 4 * half + (i & 3);
                                const float sv = score(b, i, wl[m], wd[m], 0.0f, TAB ? wm[m] : 0);
                                if (sv >= tau[b]) {
                                    const int32_t slot = ws[m];
                                    const int pos = min(atomicAdd(&cnt[qi], 1), kWidePending - 1);
                                    dst[pos] = make_key(sv, slot, LVQ_IP);
                                }
                            }
                            continue;
                        }
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int m0 = 32 * j + 8 * g + 4 * half;
                            float4 L, D;
                            if constexpr (KEEP) {
                                L = Lk[g];
                                D = Dk[g];
                            } else {
                                L = *reinterpret_cast<const float4 *>(wl + m0);
                                D = *reinterpret_cast<const float4 *>(wd + m0);
                            }
                            int4 M4 = make_int4(0, 0, 0, 0);
                            if constexpr (TAB) M4 = *reinterpret_cast<const int4 *>(wm + m0);
                            const float lr[4] = {L.x, L.y, L.z, L.w}, dr[4] = {D.x, D.y, D.z, D.w};
                            const int mr[4] = {M4.x, M4.y, M4.z, M4.w};
#pragma unroll
                            for (int r4 = 0; r4 < 4; ++r4) {
                                const float sv = score(b, 4 * g + r4, lr[r4], dr[r4], 0.0f, mr[r4]);
                                if (sv >= tau[b]) {
                                    const int32_t slot = ws[m0 + r4];
                                    const int pos = min(atomicAdd(&cnt[qi], 1), kWidePending - 1);
                                    dst[pos] = make_key(sv, slot, LVQ_IP);
                                }
                            }
                        }
                    }
                }
            };
            if constexpr (MM) {
                if (!one_mean)
                    epilogue(std::true_type{});
                else
                    epilogue(std::false_type{});
            } else {
                epilogue(std::false_type{});
            }
            // the round's appends are done
            __syncthreads();
            // Merges: the queries with at least 64 pending keys (every query
            // after the last round), by wave (query % WAVES), the only wave
            // that reads or resets their counts here; they end before the
            // next round's first barrier.  After the last round the merged
            // list's first k keys are the tile's result.
            // (the counts are read before any merge: a wave's merges reset
            // only its own queries' counts)
            constexpr int NQW = (TQ + 63) / 64;
            int cv[NQW];
#pragma unroll
            for (int t = 0; t < NQW; ++t) cv[t] = 64 * t + lane < nqt ? cnt[64 * t + lane] : 0;
#pragma unroll
            for (int t = 0; t < NQW; ++t) {
                const int qw = 64 * t, qi_l = qw + lane;
                uint64_t m = __ballot(qi_l < nqt && qi_l % WAVES == wave && (last || cv[t] >= kWideMerge));
                while (m) {
                    const int qi = qw + __builtin_ctzll(m);
                    m &= m - 1;
                    uint64_t kth;
                    const int got = merge_region_ks(ks, region + (size_t)qi * cap, 0, min(cnt[qi], kWidePending), k,
                                                    last ? out_keys(qi) : nullptr, &kth);
                    uint32_t gbq = a.gthr[q0 + qi];
                    if (got == k) {
                        // this part holds k candidates at least as good as
                        // kth, so no worse score can enter the final top k
                        const uint32_t mine = (uint32_t)(kth >> 32);
                        gbq = min(gbq, mine);
                        if (lane == 0)
                            __hip_atomic_fetch_min(&a.gthr[q0 + qi], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (lane == 0) {
                        cnt[qi] = 0;
                        if (gbq != 0xFFFFFFFFu) thr_f[qi] = fmaxf(thr_f[qi], key_score((uint64_t)gbq << 32, LVQ_IP));
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                sc[j] = sn[j];
                sn[j] = sa[j];
                if constexpr (DEC) {
                    hd[j] = hn[j];
                    ep[j] = en[j];
                }
            }
        }
    }
}

}  // namespace

using WideKernel = void (*)(ScanArgs);

// Instantiations in their own units, by first-level bits and position count
// (nullptr when not instantiated; *qb = 32-query blocks per workgroup, *rb =
// row blocks per wave): FP32 first level (k_mfma_wide32.hip), FP32 both
// levels with 8-bit residual codes (k_mfma_wide32r.hip), bf16 / fp16 both
// levels (k_mfma_wide16r.hip, prec LVQ_BF16 or LVQ_FP16).
WideKernel wide_kernel_f32(int bits1, int kpos, int *qb, int *rb);
WideKernel wide_kernel_f32r(int bits1, int kpos, int *qb, int *rb);
WideKernel wide_kernel_16r(int bits1, int kpos, int prec, int *qb, int *rb);

}  // namespace lvq
