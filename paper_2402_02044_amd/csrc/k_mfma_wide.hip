// k_mfma_wide.hip -- exhaustive inner-product top-k on the matrix cores with
// the queries staged in LDS (first level; Sec. 3.2 similarity, Sec. 2.1 k-NN):
//   <q, x_hat> = c_m + l sum(q) + Delta <q, c1>
// (one mean: c_m = <q, mu> is one value per query) with bf16 / fp16 queries
// times codes converted exactly to the same type (v_mfma_f32_32x32x16), or
// FP32 queries times codes converted exactly to FP32 (v_mfma_f32_32x32x2),
// both with FP32 accumulation.
//
// Tiling.  A workgroup of eight waves (two per SIMD) copies the MFMA
// fragments of TQ = 32*QB queries into LDS once per tile, so every code
// fragment a wave converts (FP32: every code a lane converts) feeds QB MFMAs,
// one per 32-query block.  The codes are the A operand and the queries the B
// operand: lane l then owns query (l & 31) of every block -- its sum(q), c_m
// and admission bound stay in registers -- and rows 8*(i/4) + 4*(l >> 5) +
// (i % 4), i < 16, of each 32-row block.  A wave scores RB = 2 blocks of 32
// rows per round, so each query fragment it reads from LDS feeds two MFMAs;
// its 16-byte code pieces stream through a ring of loads a few chunks ahead,
// which runs on into the next round's rows.
//
// Top-k.  Each query keeps, in the workgroup's region of device memory, its
// KS best keys so far (sorted, KS = k rounded up to a power of two >= 64)
// followed by the keys pending a merge.  The epilogue tests a lane's 16
// scores against its query's bound; a lane with passing scores reserves room
// with one LDS atomic and writes its keys.  After the round's appends (a
// barrier), queries with 64 or more pending keys are merged by their owner
// wave: 64 keys at a time are sorted in registers and folded into the sorted
// list by one bitonic merge, and the bound becomes the k-th key, shared with
// the other row parts through gthr (an atomic minimum of score-order keys).
// The merges overlap the next round's products and end before its first
// barrier, which precedes its appends.  Workgroups are persistent, one per
// compute unit, and walk the part-major (part, query tile) sequence
// XCD-aware: the workgroups of one XCD take consecutive tiles, which read
// the same rows through its L2.
#include "k_mfma_ops.h"

namespace lvq {
namespace {

// Waves per workgroup by row blocks per wave: three per SIMD with one
// 32-row block (each query fragment read from LDS feeds one MFMA), two per
// SIMD with two (it feeds two, at twice the accumulator registers).
__host__ __device__ constexpr int wide_waves(int rb)
{
    return rb == 2 ? 8 : 12;
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
// per-wave row constants (l, Delta, slot of its rows), per-query bounds and
// pending counts.
__host__ __device__ constexpr size_t wide_lds_bytes(int qb, int kpos, int rb, int esize)
{
    return (size_t)32 * qb * kpos * esize + (size_t)wide_waves(rb) * 32 * rb * 12 + (size_t)32 * qb * 8;
}

template <int B1, int KPOS, int QB, int RB, int PREC>
__global__ __launch_bounds__(64 * wide_waves(RB), 1) void k_scan_mfma_wide(ScanArgs a)
{
    constexpr bool F32 = PREC == LVQ_FP32, FP16 = PREC == LVQ_FP16;
    constexpr int WAVES = wide_waves(RB);
    constexpr int RW = 32 * RB;               // rows per wave and round
    constexpr int RROUND = WAVES * RW;        // rows per round
    constexpr int TQ = 32 * QB;
    constexpr int CHUNK_POS = B1 == 8 ? 32 : 64;
    constexpr int NCHUNK = KPOS / CHUNK_POS;
    // 16-byte query fragments per chunk and block: 8 positions each in 16
    // bits, 4 in FP32 (one per lane and MFMA)
    constexpr int STEPS = F32 ? CHUNK_POS / 8 : CHUNK_POS / 16;
    constexpr int RING = NCHUNK < 4 ? NCHUNK : 4;
    constexpr int NFRAG = QB * NCHUNK * STEPS * 64;   // 16-byte fragments per query tile
    static_assert(KPOS % CHUNK_POS == 0, "KPOS");
    static_assert(RROUND + kWideMerge <= kWidePending, "pending room");

    extern __shared__ __align__(16) unsigned char smem[];
    uint4 *qf = reinterpret_cast<uint4 *>(smem);
    float *rl = reinterpret_cast<float *>(qf + NFRAG);              // [wave][RW] l, NaN if not scored
    float *rd = rl + WAVES * RW;                                    // [wave][RW] Delta
    int32_t *rs = reinterpret_cast<int32_t *>(rd + WAVES * RW);     // [wave][RW] slot
    float *thr_f = reinterpret_cast<float *>(rs + WAVES * RW);      // TQ admission bounds
    int *cnt = reinterpret_cast<int *>(thr_f + TQ);                 // TQ pending keys

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int half = lane >> 5, col = lane & 31;
    const int k = a.k, cap = a.mcap, ks = a.mks;
    uint64_t *region = a.mkeys + (size_t)blockIdx.x * TQ * cap;
    float *wl = rl + wave * RW, *wd = rd + wave * RW;
    int32_t *ws = rs + wave * RW;

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
        for (int t = tid; t < TQ * ks; t += 64 * WAVES) region[(size_t)(t / ks) * cap + t % ks] = kNoKey;
        float qs[QB], cq[QB], tau[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const int qi = 32 * b + col;
            const bool in = qi < nqt;
            qs[b] = in ? a.qsum[q0 + qi] : 0.0f;
            cq[b] = in ? a.cm[q0 + qi] : 0.0f;
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
        const int64_t wrow = (int64_t)wave * RW + col;
        int32_t sc[RB], sn[RB];
        uint4 ring[RING][RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            sc[j] = slot_at(r0 + wrow + 32 * j);
            sn[j] = slot_at(r0 + RROUND + wrow + 32 * j);
            const uint8_t *p = codes(sc[j]);
#pragma unroll
            for (int c = 0; c < RING; ++c) ring[c][j] = *reinterpret_cast<const uint4 *>(p + c * 32);
        }
        f32x16 acc[RB][QB];
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
                    for (int i = 0; i < 16; ++i) acc[j][b][i] = 0.0f;
            // The products.  Halfway through, the rows' headers (their lines
            // were read with the first codes) and the other parts' shared
            // bounds for the lane's queries are loaded.
            float4 hd[RB];
            uint2 ep[RB];
            uint32_t gb[QB];
#pragma unroll
            for (int c = 0; c < NCHUNK; ++c) {
                if (c == NCHUNK / 2) {
#pragma unroll
                    for (int j = 0; j < RB; ++j) {
                        const uint8_t *h = a.rows + (int64_t)sc[j] * a.row_bytes;
                        hd[j] = *reinterpret_cast<const float4 *>(h);
                        ep[j] = *reinterpret_cast<const uint2 *>(h + 16);
                    }
#pragma unroll
                    for (int b = 0; b < QB; ++b) {
                        const int qi = 32 * b + col;
                        gb[b] = a.gthr[q0 + (qi < nqt ? qi : 0)];
                    }
                }
                uint4 v[RB];
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    v[j] = ring[c % RING][j];
                    const uint8_t *p = codes(c + RING < NCHUNK ? sc[j] : sn[j]);
                    ring[c % RING][j] =
                        *reinterpret_cast<const uint4 *>(p + (c + RING < NCHUNK ? c + RING : c + RING - NCHUNK) * 32);
                }
                if constexpr (F32) {
                    // code 4 s + e of the lane's piece is byte e of word s
                    uint32_t cw[RB][STEPS];
#pragma unroll
                    for (int j = 0; j < RB; ++j) code_words<B1>(v[j], cw[j]);
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
                            for (int j = 0; j < RB; ++j) af[j] = (float)((cw[j][s] >> (8 * e)) & 0xFFu);
#pragma unroll
                            for (int b = 0; b < QB; ++b) {
                                const float bv = e == 0 ? bq[b].x : e == 1 ? bq[b].y : e == 2 ? bq[b].z : bq[b].w;
#pragma unroll
                                for (int j = 0; j < RB; ++j) acc[j][b] = mfma_f32(af[j], bv, acc[j][b]);
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < STEPS; ++s) {
                        uint4 af[RB];
#pragma unroll
                        for (int j = 0; j < RB; ++j) af[j] = b_fragment<B1, FP16>(v[j], s);
#pragma unroll
                        for (int b = 0; b < QB; ++b) {
                            const uint4 bq = qf[((b * NCHUNK + c) * STEPS + s) * 64 + lane];
#pragma unroll
                            for (int j = 0; j < RB; ++j) acc[j][b] = mfma<FP16>(af[j], bq, acc[j][b]);
                        }
                    }
                }
            }

            // the previous round's merges are done: their bounds are in thr_f
            __syncthreads();
#pragma unroll
            for (int b = 0; b < QB; ++b) {
                tau[b] = fmaxf(tau[b], thr_f[32 * b + col]);
                if (gb[b] != 0xFFFFFFFFu) tau[b] = fmaxf(tau[b], key_score((uint64_t)gb[b] << 32, LVQ_IP));
            }
            // Row constants of the round to the wave's LDS area: half 0
            // writes l (NaN for rows not scored: dead, outside the snapshot,
            // past the part) and the slot, half 1 Delta.
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                const uint32_t f = __float_as_uint(hd[j].w);
                const bool live = base + wrow + 32 * j < r1 && ((f >> 8) & 1u) && ep[j].x <= a.epoch &&
                                  a.epoch < ep[j].y;
                if (half == 0) {
                    wl[32 * j + col] = live ? hd[j].x : __builtin_nanf("");
                    ws[32 * j + col] = sc[j];
                } else {
                    wd[32 * j + col] = hd[j].y;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // Lane rows 32*j + 8*g + 4*half + r4, r4 < 4: the score of (row,
            // query 32*b + col) is c_m + l sum(q) + Delta <q, c1>.  A query
            // block whose lanes' largest scores all stay below their bounds
            // is done; else each lane counts its scores that reach the bound
            // (a NaN score, from a row not scored, never does), reserves
            // room with one LDS atomic and writes their keys.
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                auto score = [&](int b, int i, float l, float dlt) {
                    return fmaf(dlt, acc[j][b][i], fmaf(l, qs[b], cq[b]));
                };
                float mx[QB];
#pragma unroll
                for (int b = 0; b < QB; ++b) mx[b] = -__builtin_inff();
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float4 L = *reinterpret_cast<const float4 *>(wl + 32 * j + 8 * g + 4 * half);
                    const float4 D = *reinterpret_cast<const float4 *>(wd + 32 * j + 8 * g + 4 * half);
                    const float lr[4] = {L.x, L.y, L.z, L.w}, dr[4] = {D.x, D.y, D.z, D.w};
#pragma unroll
                    for (int b = 0; b < QB; ++b)
#pragma unroll
                        for (int r4 = 0; r4 < 4; ++r4) {
                            const float sv = score(b, 4 * g + r4, lr[r4], dr[r4]);
                            mx[b] = sv > mx[b] ? sv : mx[b];
                        }
                }
#pragma unroll
                for (int b = 0; b < QB; ++b) {
                    if (!__ballot(mx[b] >= tau[b])) continue;
                    // one score per iteration (a uniform index into the
                    // accumulators)
                    int np = 0;
#pragma unroll 4
                    for (int i = 0; i < 16; ++i) {
                        const int m = 32 * j + 8 * (i >> 2) + 4 * half + (i & 3);
                        np += score(b, i, wl[m], wd[m]) >= tau[b] ? 1 : 0;
                    }
                    const int qi = 32 * b + col;
                    int pos = np ? atomicAdd(&cnt[qi], np) : 0;
                    uint64_t *dst = region + (size_t)qi * cap + ks;
#pragma unroll 4
                    for (int i = 0; i < 16; ++i) {
                        const int m = 32 * j + 8 * (i >> 2) + 4 * half + (i & 3);
                        const float sv = score(b, i, wl[m], wd[m]);
                        if (sv >= tau[b]) {
                            if (pos < kWidePending) dst[pos] = make_key(sv, ws[m], LVQ_IP);
                            ++pos;
                        }
                    }
                }
            }
            // the round's appends are done
            __syncthreads();
            // Merges: the queries with at least 64 pending keys (every query
            // after the last round), by wave (query % WAVES), the only wave
            // that reads or resets their counts here; they end before the
            // next round's first barrier.  After the last round the merged
            // list's first k keys are the tile's result.
            for (int qw = 0; qw < TQ; qw += 64) {
                const int qi_l = qw + lane;
                uint64_t m = __ballot(qi_l < nqt && qi_l % WAVES == wave && (last || cnt[qi_l] >= kWideMerge));
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
            }
        }
    }
}

using WideKernel = void (*)(ScanArgs);

// Instantiated position counts: 32-query blocks per workgroup (as many as
// the query fragments' LDS allows, at most four) and row blocks per wave.
template <int B1, int PREC>
WideKernel wide_lookup_16(int kpos, int *qb, int *rb)
{
    switch (kpos) {
    case 96: *qb = 4; *rb = 2; return B1 == 8 ? k_scan_mfma_wide<8, 96, 4, 2, PREC> : nullptr;
    case 128: *qb = 4; *rb = 2; return k_scan_mfma_wide<B1, 128, 4, 2, PREC>;
    case 256: *qb = 4; *rb = 2; return k_scan_mfma_wide<B1, 256, 4, 2, PREC>;
    case 384: *qb = 4; *rb = 2; return k_scan_mfma_wide<B1, 384, 4, 2, PREC>;
    case 512: *qb = 4; *rb = 2; return k_scan_mfma_wide<B1, 512, 4, 2, PREC>;
    case 768: *qb = 2; *rb = 2; return k_scan_mfma_wide<B1, 768, 2, 2, PREC>;
    case 1024: *qb = 2; *rb = 2; return k_scan_mfma_wide<B1, 1024, 2, 2, PREC>;
    default: return nullptr;
    }
}

// FP32 query values take twice the LDS of 16-bit ones.
template <int B1>
WideKernel wide_lookup_32(int kpos, int *qb, int *rb)
{
    switch (kpos) {
    case 96: *qb = 4; *rb = 2; return B1 == 8 ? k_scan_mfma_wide<8, 96, 4, 2, LVQ_FP32> : nullptr;
    case 128: *qb = 4; *rb = 2; return k_scan_mfma_wide<B1, 128, 4, 2, LVQ_FP32>;
    case 256: *qb = 4; *rb = 2; return k_scan_mfma_wide<B1, 256, 4, 2, LVQ_FP32>;
    case 384: *qb = 2; *rb = 2; return k_scan_mfma_wide<B1, 384, 2, 2, LVQ_FP32>;
    case 512: *qb = 2; *rb = 2; return k_scan_mfma_wide<B1, 512, 2, 2, LVQ_FP32>;
    case 768: *qb = 1; *rb = 2; return k_scan_mfma_wide<B1, 768, 1, 2, LVQ_FP32>;
    case 1024: *qb = 1; *rb = 2; return k_scan_mfma_wide<B1, 1024, 1, 2, LVQ_FP32>;
    default: return nullptr;
    }
}

template <int B1>
WideKernel wide_lookup(int kpos, int prec, int *qb, int *rb)
{
    if (prec == LVQ_BF16) return wide_lookup_16<B1, LVQ_BF16>(kpos, qb, rb);
    if (prec == LVQ_FP16) return wide_lookup_16<B1, LVQ_FP16>(kpos, qb, rb);
    if (prec == LVQ_FP32) return wide_lookup_32<B1>(kpos, qb, rb);
    return nullptr;
}

WideKernel wide_kernel(int bits1, int kpos, int prec, int *qb, int *rb)
{
    if (bits1 == 8) return wide_lookup<8>(kpos, prec, qb, rb);
    if (bits1 == 4) return wide_lookup<4>(kpos, prec, qb, rb);
    return nullptr;
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

int mfma_wide_query_block(int bits1, int kpos, int prec, int k, int n_means, size_t lds_max)
{
    if ((bits1 != 4 && bits1 != 8) || kpos % (bits1 == 8 ? 32 : 64)) return 0;
    if (k < 1 || k > kWideMaxK || n_means != 1) return 0;
    int qb = 0, rb = 0;
    if (!wide_kernel(bits1, kpos, prec, &qb, &rb)) return 0;
    return wide_lds_bytes(qb, kpos, rb, prec == LVQ_FP32 ? 4 : 2) <= lds_max ? qb : 0;
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

hipError_t launch_scan_mfma_wide(const ScanArgs &a, int bits1, int prec, int64_t grid, hipStream_t s)
{
    int qb = 0, rb = 0;
    WideKernel kern = wide_kernel(bits1, a.kpos, prec, &qb, &rb);
    if (!kern || grid < 8 || grid % 8 || a.k < 1 || a.k > kWideMaxK || a.mks != mfma_wide_sorted(a.k) ||
        a.mcap != mfma_wide_cap(a.k) || a.n_means != 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * wide_waves(rb)),
                       wide_lds_bytes(qb, a.kpos, rb, prec == LVQ_FP32 ? 4 : 2), s, a);
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
