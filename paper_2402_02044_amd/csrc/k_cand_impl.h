// k_cand_impl.h -- similarities between float queries and the stored LVQ rows
// of per-query candidate lists (Sec. 3.2), with an optional fused per-list
// top-k (Sec. 2.1; lazy deletes are scored but filtered, App. A).
//
// Arithmetic (binary32, FMA accumulation):
//   IP  <q, x_hat> = c_m + l' sum(q) + Delta <q, c1> [+ Delta2 <q, c2>]
//       with c_m = <q, mu_m> per query and mean, l' = l [- Delta/2 at FULL]
//   L2  sum_p ((q - mu_m)_p - (l' + Delta c1_p [+ Delta2 c2_p]))^2   (direct
//       form: no cancellation for near neighbours)
//
// Launch shape.  A workgroup of 256 lanes owns one candidate list at a time
// (one list per workgroup, or a persistent loop popping lists from a work
// counter in descending-length order).  A list's query data lives in LDS in a
// bank-conflict-free layout; a group of G lanes scores one candidate: its
// lanes fetch disjoint CH-byte pieces of the row (NCH pieces each, all issued
// before any is consumed), decode nibbles/bytes with mask + byte conversion,
// accumulate with FMAs, and reduce with DPP row operations.
#pragma once

#include "k_common.h"

namespace lvq {

template <int B1, int CH>
struct CandGeom {
    static constexpr int kWords = CH / 4;             // 32-bit words per piece
    static constexpr int kSlots = CH * 8 / B1;        // code positions per piece
    static constexpr int kF4 = kSlots / 4;            // float4 reads of q per piece
};

// residual bytes per piece for a residual of B2 bits
template <int B1, int B2, int CH>
struct ResGeom {
    static constexpr int kBytes = B2 == 0 ? 0 : CH * 8 / B1 * B2 / 8;
    static constexpr int kWords = kBytes / 4 > 0 ? kBytes / 4 : 1;
};

template <int N>
struct Words {
    uint32_t w[N];
};

template <int N>
__device__ __forceinline__ Words<N> load_words(const uint8_t *p)
{
    Words<N> r;
    if constexpr (N == 4) {
        uint4 v = *reinterpret_cast<const uint4 *>(p);
        r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
    } else if constexpr (N == 8) {
        uint4 v = *reinterpret_cast<const uint4 *>(p);
        uint4 u = *reinterpret_cast<const uint4 *>(p + 16);
        r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
        r.w[4] = u.x; r.w[5] = u.y; r.w[6] = u.z; r.w[7] = u.w;
    } else if constexpr (N == 2) {
        uint2 v = *reinterpret_cast<const uint2 *>(p);
        r.w[0] = v.x; r.w[1] = v.y;
    } else {
        for (int i = 0; i < N; ++i) r.w[i] = reinterpret_cast<const uint32_t *>(p)[i];
    }
    return r;
}

// w & m, opaque to the optimiser: it keeps the mask-then-convert decoding (one
// AND per four fields, then v_cvt_f32_ubyte{0..3}) instead of rewriting it
// into one bit-field extract per field.
__device__ __forceinline__ uint32_t opaque_and(uint32_t w, uint32_t m)
{
    uint32_t r;
    asm("v_and_b32 %0, %1, %2" : "=v"(r) : "s"(m), "v"(w));
    return r;
}

template <int N>
__device__ __forceinline__ void zero_unless(Words<N> &x, bool ok)
{
#pragma unroll
    for (int i = 0; i < N; ++i) x.w[i] = ok ? x.w[i] : 0u;
}

// Accumulators of one candidate.
struct Acc {
    float a_lo, a_hi;   // first level: low fields, high fields (x16 for 4-bit)
    float r_lo, r_hi;   // residual level
};

// ---- IP: accumulate one first-level word and its residual ---------------
// q: the 8 (B1 = 4) or 4 (B1 = 8) query values of the word's kernel slots.
template <int B1, int B2>
__device__ __forceinline__ void ip_word(uint32_t w, const float *q, const uint32_t *res, int wi, Acc &A)
{
    if constexpr (B1 == 4) {
        const uint32_t lo = opaque_and(w, 0x0F0F0F0Fu), hi = opaque_and(w, 0xF0F0F0F0u);
        A.a_lo = fmaf(q[0], ub<0>(lo), A.a_lo);
        A.a_lo = fmaf(q[1], ub<1>(lo), A.a_lo);
        A.a_lo = fmaf(q[2], ub<2>(lo), A.a_lo);
        A.a_lo = fmaf(q[3], ub<3>(lo), A.a_lo);
        A.a_hi = fmaf(q[4], ub<0>(hi), A.a_hi);
        A.a_hi = fmaf(q[5], ub<1>(hi), A.a_hi);
        A.a_hi = fmaf(q[6], ub<2>(hi), A.a_hi);
        A.a_hi = fmaf(q[7], ub<3>(hi), A.a_hi);
        if constexpr (B2 == 8) {
            const uint32_t r0 = res[2 * wi], r1 = res[2 * wi + 1];
            A.r_lo = fmaf(q[0], ub<0>(r0), A.r_lo);
            A.r_lo = fmaf(q[1], ub<2>(r0), A.r_lo);
            A.r_lo = fmaf(q[2], ub<0>(r1), A.r_lo);
            A.r_lo = fmaf(q[3], ub<2>(r1), A.r_lo);
            A.r_lo = fmaf(q[4], ub<1>(r0), A.r_lo);
            A.r_lo = fmaf(q[5], ub<3>(r0), A.r_lo);
            A.r_lo = fmaf(q[6], ub<1>(r1), A.r_lo);
            A.r_lo = fmaf(q[7], ub<3>(r1), A.r_lo);
        } else if constexpr (B2 == 4) {
            const uint32_t r = res[wi];
            const uint32_t rl = opaque_and(r, 0x0F0F0F0Fu), rh = opaque_and(r, 0xF0F0F0F0u);
            A.r_lo = fmaf(q[0], ub<0>(rl), A.r_lo);
            A.r_lo = fmaf(q[1], ub<1>(rl), A.r_lo);
            A.r_lo = fmaf(q[2], ub<2>(rl), A.r_lo);
            A.r_lo = fmaf(q[3], ub<3>(rl), A.r_lo);
            A.r_hi = fmaf(q[4], ub<0>(rh), A.r_hi);
            A.r_hi = fmaf(q[5], ub<1>(rh), A.r_hi);
            A.r_hi = fmaf(q[6], ub<2>(rh), A.r_hi);
            A.r_hi = fmaf(q[7], ub<3>(rh), A.r_hi);
        }
    } else {
        A.a_lo = fmaf(q[0], ub<0>(w), A.a_lo);
        A.a_lo = fmaf(q[1], ub<1>(w), A.a_lo);
        A.a_lo = fmaf(q[2], ub<2>(w), A.a_lo);
        A.a_lo = fmaf(q[3], ub<3>(w), A.a_lo);
        if constexpr (B2 == 8) {
            const uint32_t r = res[wi];
            A.r_lo = fmaf(q[0], ub<0>(r), A.r_lo);
            A.r_lo = fmaf(q[1], ub<1>(r), A.r_lo);
            A.r_lo = fmaf(q[2], ub<2>(r), A.r_lo);
            A.r_lo = fmaf(q[3], ub<3>(r), A.r_lo);
        } else if constexpr (B2 == 4) {
            const uint32_t h = res[wi >> 1] >> (16 * (wi & 1));
            const uint32_t rl = opaque_and(h, 0x0F0Fu), rh = opaque_and(h, 0xF0F0u);
            A.r_lo = fmaf(q[0], ub<0>(rl), A.r_lo);
            A.r_lo = fmaf(q[2], ub<1>(rl), A.r_lo);
            A.r_hi = fmaf(q[1], ub<0>(rh), A.r_hi);
            A.r_hi = fmaf(q[3], ub<1>(rh), A.r_hi);
        }
    }
}

// ---- L2: accumulate one first-level word (direct form) --------------------
// q: (q - mu_m) at the word's kernel slots; m: padding mask or nullptr.
struct L2Row {
    float lp;      // l' = l [- Delta/2]
    float dl;      // Delta
    float dl16;    // Delta / 16 (high nibbles arrive multiplied by 16)
    float d2;      // Delta2 (FULL) or 0
    float d216;    // Delta2 / 16
};

template <bool MASK, bool RES>
__device__ __forceinline__ void l2_acc(float qv, float c1, float s1, float c2, float s2,
                                       const L2Row &R, float mk, float &acc)
{
    float x = fmaf(s1, c1, R.lp);
    if constexpr (RES) x = fmaf(s2, c2, x);
    float t = qv - x;
    if constexpr (MASK) t *= mk;
    acc = fmaf(t, t, acc);
}

template <int B1, int B2, bool MASK>
__device__ __forceinline__ void l2_word(uint32_t w, const float *q, const float *m, const uint32_t *res,
                                        int wi, const L2Row &R, float &acc)
{
    if constexpr (B1 == 4) {
        const uint32_t lo = opaque_and(w, 0x0F0F0F0Fu), hi = opaque_and(w, 0xF0F0F0F0u);
        float c2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        float s2lo = R.d2, s2hi = R.d2;
        if constexpr (B2 == 8) {
            const uint32_t r0 = res[2 * wi], r1 = res[2 * wi + 1];
            c2[0] = ub<0>(r0); c2[1] = ub<2>(r0); c2[2] = ub<0>(r1); c2[3] = ub<2>(r1);
            c2[4] = ub<1>(r0); c2[5] = ub<3>(r0); c2[6] = ub<1>(r1); c2[7] = ub<3>(r1);
        } else if constexpr (B2 == 4) {
            const uint32_t r = res[wi];
            const uint32_t rl = opaque_and(r, 0x0F0F0F0Fu), rh = opaque_and(r, 0xF0F0F0F0u);
            c2[0] = ub<0>(rl); c2[1] = ub<1>(rl); c2[2] = ub<2>(rl); c2[3] = ub<3>(rl);
            c2[4] = ub<0>(rh); c2[5] = ub<1>(rh); c2[6] = ub<2>(rh); c2[7] = ub<3>(rh);
            s2hi = R.d216;
        }
        l2_acc<MASK, (B2 != 0)>(q[0], ub<0>(lo), R.dl, c2[0], s2lo, R, MASK ? m[0] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[1], ub<1>(lo), R.dl, c2[1], s2lo, R, MASK ? m[1] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[2], ub<2>(lo), R.dl, c2[2], s2lo, R, MASK ? m[2] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[3], ub<3>(lo), R.dl, c2[3], s2lo, R, MASK ? m[3] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[4], ub<0>(hi), R.dl16, c2[4], s2hi, R, MASK ? m[4] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[5], ub<1>(hi), R.dl16, c2[5], s2hi, R, MASK ? m[5] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[6], ub<2>(hi), R.dl16, c2[6], s2hi, R, MASK ? m[6] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[7], ub<3>(hi), R.dl16, c2[7], s2hi, R, MASK ? m[7] : 1.f, acc);
    } else {
        float c2[4] = {0, 0, 0, 0};
        float s2[4] = {R.d2, R.d2, R.d2, R.d2};
        if constexpr (B2 == 8) {
            const uint32_t r = res[wi];
            c2[0] = ub<0>(r); c2[1] = ub<1>(r); c2[2] = ub<2>(r); c2[3] = ub<3>(r);
        } else if constexpr (B2 == 4) {
            const uint32_t h = res[wi >> 1] >> (16 * (wi & 1));
            const uint32_t rl = opaque_and(h, 0x0F0Fu), rh = opaque_and(h, 0xF0F0u);
            c2[0] = ub<0>(rl); c2[2] = ub<1>(rl); c2[1] = ub<0>(rh); c2[3] = ub<1>(rh);
            s2[1] = R.d216; s2[3] = R.d216;
        }
        l2_acc<MASK, (B2 != 0)>(q[0], ub<0>(w), R.dl, c2[0], s2[0], R, MASK ? m[0] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[1], ub<1>(w), R.dl, c2[1], s2[1], R, MASK ? m[1] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[2], ub<2>(w), R.dl, c2[2], s2[2], R, MASK ? m[2] : 1.f, acc);
        l2_acc<MASK, (B2 != 0)>(q[3], ub<3>(w), R.dl, c2[3], s2[3], R, MASK ? m[3] : 1.f, acc);
    }
}

// LDS query table layout: for a table of kpos floats split into pieces of
// kSlots slots, the r-th float4 of piece u is stored at float4 index
// r * npieces + u, so the lanes of a group (consecutive pieces) read
// consecutive float4s.
template <int B1, int CH>
__device__ __forceinline__ int qtab_index(int s, int npieces)
{
    using Geo = CandGeom<B1, CH>;
    const int u = s / Geo::kSlots, w = s % Geo::kSlots;
    return ((w >> 2) * npieces + u) * 4 + (w & 3);
}

// One candidate's row data as loaded by a lane of its group.
template <int B1, int B2, int CH, int NCH>
struct PairRegs {
    Words<CandGeom<B1, CH>::kWords> wv[NCH];
    Words<ResGeom<B1, B2, CH>::kWords> rv[NCH];
    float4 hdr;
    uint2 ep;      // insertion / deletion epochs (loaded when a top-k is fused)
    int32_t slot;
    bool valid, work;
};

// Issue the loads of one candidate (entry e of a list ending at e1): the
// header and the pieces p0 + c*G + g of the first-level and residual codes.
// Branch-free: out-of-range pieces and invalid candidates load from a valid
// address (slot 0, piece 0) and are zeroed by a select, so the values stay in
// registers.
template <int B1, int B2, int G, int CH, int NCH>
__device__ __forceinline__ void load_pair(PairRegs<B1, B2, CH, NCH> &P, const CandArgs &a, int64_t e,
                                          int64_t e1, int32_t slot, int p0, int g, int npieces)
{
    using Geo = CandGeom<B1, CH>;
    using RGeo = ResGeom<B1, B2, CH>;
    P.valid = e < e1;
    P.slot = slot;
    const bool in_range = slot >= 0 && (int64_t)slot < a.capacity;
    P.work = P.valid && in_range;
    const int64_t s = P.work ? slot : 0;
    const uint8_t *row = a.rows + s * a.row_bytes;
    const uint8_t *res = B2 ? a.resid + s * a.resid_bytes : nullptr;
    if (p0 == 0) {
        float4 h = *reinterpret_cast<const float4 *>(row);
        P.hdr = P.work ? h : make_float4(0.f, 0.f, 0.f, 0.f);
        // the epoch pair is one 64-bit load (it is written as one 64-bit
        // store), issued with the row so the fused top-k never waits on it
        if (a.k > 0) {
            const uint2 ep = *reinterpret_cast<const uint2 *>(row + 16);
            P.ep = P.work ? ep : make_uint2(1u, 0u);
        } else {
            P.ep = make_uint2(1u, 0u);
        }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int u = p0 + c * G + g;
        const bool ok = P.work && u < npieces;
        const int uu = u < npieces ? u : 0;
        P.wv[c] = load_words<Geo::kWords>(row + kHeaderBytes + uu * CH);
        zero_unless(P.wv[c], ok);
        if constexpr (B2 != 0) {
            P.rv[c] = load_words<RGeo::kWords>(res + uu * RGeo::kBytes);
            zero_unless(P.rv[c], ok);
        }
    }
}

// Query values of the pieces a lane owns, held in registers for a whole list
// (single-round shapes: a lane handles the same pieces for every candidate).
template <int B1, int CH, int NCH>
struct QRegs {
    float4 v[NCH][CandGeom<B1, CH>::kF4];
};

// Accumulate the loaded pieces of one candidate; query values come from the
// LDS table tq or, when QREG is set, from registers.  Pieces past the end
// (u >= npieces) hold zero codes; their L2 contribution is dropped by a
// select, their IP contribution is zero already.
template <int B1, int B2, int METRIC, bool MASK, int G, int CH, int NCH, bool QREG>
__device__ __forceinline__ void accumulate_pair(const PairRegs<B1, B2, CH, NCH> &P, const float *tq,
                                                const QRegs<B1, CH, NCH> &qr, const float *mtab, int p0,
                                                int g, int npieces, const L2Row &R, Acc &A, float &l2acc)
{
    using Geo = CandGeom<B1, CH>;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int u = p0 + c * G + g;
        const bool ok = u < npieces;
        const int uu = ok ? u : 0;
        float qv[Geo::kSlots];
        float mv[MASK ? Geo::kSlots : 1];
#pragma unroll
        for (int r = 0; r < Geo::kF4; ++r) {
            float4 f = QREG ? qr.v[c][r] : reinterpret_cast<const float4 *>(tq)[r * npieces + uu];
            qv[4 * r] = f.x; qv[4 * r + 1] = f.y; qv[4 * r + 2] = f.z; qv[4 * r + 3] = f.w;
            if constexpr (MASK) {
                float4 mm = reinterpret_cast<const float4 *>(mtab)[r * npieces + uu];
                mv[4 * r] = mm.x; mv[4 * r + 1] = mm.y; mv[4 * r + 2] = mm.z; mv[4 * r + 3] = mm.w;
            }
        }
        constexpr int kQW = B1 == 4 ? 8 : 4;   // query values per word
        float part = 0.0f;
#pragma unroll
        for (int wi = 0; wi < Geo::kWords; ++wi) {
            if constexpr (METRIC == LVQ_IP)
                ip_word<B1, B2>(P.wv[c].w[wi], qv + kQW * wi, P.rv[c].w, wi, A);
            else
                l2_word<B1, B2, MASK>(P.wv[c].w[wi], qv + kQW * wi, MASK ? mv + kQW * wi : nullptr,
                                      P.rv[c].w, wi, R, part);
        }
        if constexpr (METRIC == LVQ_L2) l2acc += ok ? part : 0.0f;
    }
}

template <int B2>
__device__ __forceinline__ L2Row l2_row(float4 hdr)
{
    L2Row R;
    R.lp = B2 ? hdr.x - 0.5f * hdr.y : hdr.x;
    R.dl = hdr.y;
    R.dl16 = hdr.y * 0.0625f;
    R.d2 = B2 ? hdr.z : 0.0f;
    R.d216 = hdr.z * 0.0625f;
    return R;
}

// Final value of one candidate from its group's accumulators (all lanes of
// the group return the same value).
template <int B2, int METRIC, int G>
__device__ __forceinline__ float finish_pair(const Acc &A, float l2acc, float4 hdr, const float *cmt, int n_means,
                                             float qsum)
{
    if constexpr (METRIC == LVQ_IP) {
        float a1 = fmaf(A.a_hi, 0.0625f, A.a_lo);
        a1 = group_sum<G>(a1);
        const float l = hdr.x, dl = hdr.y, dl2 = hdr.z;
        const int mid = (int)(__float_as_uint(hdr.w) & 0xFFu);
        const float lp = B2 ? l - 0.5f * dl : l;
        float score = fmaf(lp, qsum, cmt[mid < n_means ? mid : 0]);
        score = fmaf(dl, a1, score);
        if constexpr (B2 != 0) {
            float a2 = fmaf(A.r_hi, 0.0625f, A.r_lo);
            a2 = group_sum<G>(a2);
            score = fmaf(dl2, a2, score);
        }
        return score;
    } else {
        return group_sum<G>(l2acc);
    }
}

// Slot of list entry e (the list starts at e0): ids[e], or for segmented
// lists the entry of the segment holding e (the last one starting at or
// before it, found by bisection; empty segments are never chosen).
__device__ __forceinline__ int32_t entry_id(const CandArgs &a, int64_t e, int64_t e0, bool seg,
                                            const int64_t *sstart, const int64_t *sbase, int nseg)
{
    if (!seg) return a.ids[e];
    const int64_t loc = e - e0;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sstart[mid] <= loc) lo = mid;
        else hi = mid - 1;
    }
    return a.seg_members[sbase[lo] + (loc - sstart[lo])];
}

// Table of a row's mean: its id, or through the list's map (a stale entry of
// a mean the list does not hold is clamped into range; such a row is never
// visible to the list's query).
__device__ __forceinline__ int table_of(uint32_t mid, bool sub, const uint8_t *tmap, int ntab)
{
    const int t = sub ? (int)tmap[mid] : (int)mid;
    return t < ntab ? t : ntab - 1;
}

// PIPE: 0 = no software pipeline; 1 or 2 = the loads of the candidates one
// or two blocks ahead are in flight while the current block is consumed.
// WAVES: the fewest waves per SIMD the register allocation must allow (1: no
// constraint); small tiles trade a few registers for more rows in flight.
template <int B1, int B2, int METRIC, bool MULTI, bool MASK, int G, int CH, int NCH, int PIPE, bool QREG, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8))) void k_cand(CandArgs a)
{
    static_assert(!QREG || (PIPE && !MULTI && !MASK), "register-resident query needs one table, one round");
    static_assert(PIPE >= 0 && PIPE <= 2, "pipeline depth");
    using Regs = PairRegs<B1, B2, CH, NCH>;
    constexpr int kPairsPerWave = 64 / G;
    constexpr int kPairsPerBlock = 4 * kPairsPerWave;

    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int grp = lane / G;
    const int g = lane % G;

    const int npieces = a.kchunks * 16 / CH;
    // L2 with several means: one table q - mu_m per mean, or, for lists that
    // hold rows of a few known means only (a.list_means: list_nmeans per
    // list), one table per listed mean and a map from mean id to table
    const bool sub = METRIC == LVQ_L2 && MULTI && a.list_means != nullptr;
    const int ntab = (METRIC == LVQ_L2 && MULTI) ? (sub ? a.list_nmeans : a.n_means) : 1;
    // several means (L2): the means in kernel order stay in LDS for the whole
    // launch when a.mu_lds is set, so a list's tables q - mu_m need no reads
    // of the means from memory
    const bool mu_lds = METRIC == LVQ_L2 && MULTI && a.mu_lds;
    float *qtab = reinterpret_cast<float *>(smem);
    float *mutab = qtab + (size_t)ntab * a.kpos;
    float *mtab = mutab + (mu_lds ? (size_t)ntab * a.kpos : 0);   // mask (L2, MASK)
    float *cmt = mtab + (MASK ? a.kpos : 0);                   // c_m (IP)
    const int cm_n = METRIC == LVQ_IP ? a.n_means : 0;
    // fused top-k: one key buffer of a.cw entries per wave, then 4k entries
    // for the merge of the four waves (also each wave's selection scratch)
    uint8_t *tmap = reinterpret_cast<uint8_t *>(cmt + ((cm_n + 1) & ~1));   // kMaxMeans bytes when sub
    // segmented lists (a.seg_members): entry i of a list is entry i of the
    // concatenation of its means' member ranges; sstart holds the segments'
    // first entries (nseg + 1), sbase their starts in seg_members
    const bool seg = a.seg_members != nullptr;
    const int nseg = seg ? a.list_nmeans : 0;
    int64_t *sstart = reinterpret_cast<int64_t *>(tmap + (sub ? kMaxMeans : 0));
    int64_t *sbase = sstart + (seg ? nseg + 1 : 0);
    uint64_t *keys = reinterpret_cast<uint64_t *>(sbase + (seg ? nseg + 1 : 0));
    uint64_t *wbuf = keys + (size_t)wave * a.cw;
    uint64_t *merge = keys + (size_t)4 * a.cw;
    __shared__ int s_item;
    __shared__ int s_got[4];

    if (mu_lds)
        for (int i = tid; i < ntab * a.kpos; i += 256) {
            const int t = i / a.kpos, sp = i - t * a.kpos;
            mutab[(size_t)t * a.kpos + qtab_index<B1, CH>(sp, npieces)] = a.muk[i];
        }
    for (int iter = 0;; ++iter) {
        int item;
        if (a.queue) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(a.queue, 1);
            __syncthreads();
            item = s_item;
        } else {
            item = iter == 0 ? (int)blockIdx.x : (int)a.nq;
        }
        if (item >= a.nq) break;
        const int64_t list = a.order ? a.order[item] : item;
        int64_t e0 = a.offsets[list], e1 = a.offsets[list + 1];
        if (e0 < 0 || e1 < e0 || e1 > a.total) {
            if (tid == 0) atomicOr(a.err, kErrBadOffsets);
            e1 = e0 = 0;
        }

        // ---- per-list query tables in LDS
        __syncthreads();
        const float *qk = a.qk + list * a.kpos;
        for (int sp = tid; sp < a.kpos; sp += 256) {
            const float v = qk[sp];
            const int j = qtab_index<B1, CH>(sp, npieces);
            for (int t = 0; t < ntab; ++t) {
                float w = v;
                const int64_t mt = sub ? a.list_means[list * ntab + t] : t;
                if (METRIC == LVQ_L2)
                    w -= mu_lds ? mutab[(size_t)t * a.kpos + j] : a.muk[mt * a.kpos + sp];
                qtab[(size_t)t * a.kpos + j] = w;
            }
        }
        if (MASK)
            for (int sp = tid; sp < a.kpos; sp += 256) mtab[qtab_index<B1, CH>(sp, npieces)] = a.kmask[sp];
        for (int m = tid; m < cm_n; m += 256) cmt[m] = a.cm[list * a.n_means + m];
        if (sub)
            for (int t = tid; t < ntab; t += 256) tmap[a.list_means[list * ntab + t]] = (uint8_t)t;
        if (seg)
            for (int p = tid; p < nseg; p += 256) {
                const int m = a.list_means[list * nseg + p];
                sbase[p] = a.seg_offs[m];
                sstart[p + 1] = a.seg_offs[m + 1] - a.seg_offs[m];   // sizes, summed below
            }
        __syncthreads();
        if (seg) {
            if (tid == 0) {
                sstart[0] = 0;
                for (int p = 0; p < nseg; ++p) sstart[p + 1] += sstart[p];
            }
            __syncthreads();
        }
        const float qsum = METRIC == LVQ_IP ? a.qsum[list] : 0.0f;
        QRegs<B1, CH, NCH> qr;
        if constexpr (QREG) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int u = c * G + g;
#pragma unroll
                for (int r = 0; r < CandGeom<B1, CH>::kF4; ++r) {
                    const float4 f = reinterpret_cast<const float4 *>(qtab)[r * npieces + (u < npieces ? u : 0)];
                    qr.v[c][r] = u < npieces ? f : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
        }

        // Per-wave pruned top-k: a wave appends the keys of its candidates
        // that beat its bound thr (its k-th best so far) to its own buffer and
        // compacts the buffer to its k best when the next block might not fit.
        int nw = 0;                 // keys in this wave's buffer (wave-uniform)
        uint64_t thr = kNoKey;      // this wave's bound (wave-uniform)
        const int k = a.k;
        const int64_t my = (int64_t)wave * kPairsPerWave + grp;   // entry offset inside a block of pairs

        Regs cur, nx1;
        int32_t slot_next = 0;
        if constexpr (PIPE) {
            // software pipeline: the rows of the candidates PIPE blocks ahead
            // and the id after them are in flight while the current one is
            // consumed
            const int64_t e = e0 + my;
            const int32_t s0 = e < e1 ? entry_id(a, e, e0, seg, sstart, sbase, nseg) : 0;
            load_pair<B1, B2, G, CH, NCH>(cur, a, e, e1, s0, 0, g, npieces);
            if constexpr (PIPE == 2) {
                const int64_t e_1 = e + kPairsPerBlock;
                const int32_t s1 = e_1 < e1 ? entry_id(a, e_1, e0, seg, sstart, sbase, nseg) : 0;
                load_pair<B1, B2, G, CH, NCH>(nx1, a, e_1, e1, s1, 0, g, npieces);
            }
            slot_next = e + PIPE * kPairsPerBlock < e1
                            ? entry_id(a, e + PIPE * kPairsPerBlock, e0, seg, sstart, sbase, nseg) : 0;
        }
        for (int64_t base = e0; base < e1; base += kPairsPerBlock) {
            const int64_t e = base + my;
            Acc A{0.f, 0.f, 0.f, 0.f};
            float l2acc = 0.0f;
            float4 hdr;
            uint2 ep;
            bool valid, work;
            int32_t slot;
            if constexpr (PIPE) {
                Regs nxt;
                const int64_t en = e + PIPE * kPairsPerBlock;
                load_pair<B1, B2, G, CH, NCH>(nxt, a, en, e1, slot_next, 0, g, npieces);
                slot_next = en + kPairsPerBlock < e1 ? entry_id(a, en + kPairsPerBlock, e0, seg, sstart, sbase, nseg) : 0;
                hdr = cur.hdr;
                ep = cur.ep;
                const float *tq = qtab + ((METRIC == LVQ_L2 && MULTI)
                                              ? (size_t)table_of(__float_as_uint(hdr.w) & 0xFFu, sub, tmap, ntab) * a.kpos
                                              : 0);
                const L2Row R = l2_row<B2>(hdr);
                accumulate_pair<B1, B2, METRIC, MASK, G, CH, NCH, QREG>(cur, tq, qr, mtab, 0, g, npieces, R, A,
                                                                        l2acc);
                valid = cur.valid;
                work = cur.work;
                slot = cur.slot;
                if constexpr (PIPE == 2) {
                    cur = nx1;
                    nx1 = nxt;
                } else {
                    cur = nxt;
                }
            } else {
                valid = e < e1;
                slot = valid ? entry_id(a, e, e0, seg, sstart, sbase, nseg) : 0;
                Regs P;
                load_pair<B1, B2, G, CH, NCH>(P, a, e, e1, slot, 0, g, npieces);
                hdr = P.hdr;
                ep = P.ep;
                work = P.work;
                const float *tq = qtab + ((METRIC == LVQ_L2 && MULTI)
                                              ? (size_t)table_of(__float_as_uint(hdr.w) & 0xFFu, sub, tmap, ntab) * a.kpos
                                              : 0);
                const L2Row R = l2_row<B2>(hdr);
                accumulate_pair<B1, B2, METRIC, MASK, G, CH, NCH, false>(P, tq, qr, mtab, 0, g, npieces, R, A,
                                                                         l2acc);
                for (int p0 = G * NCH; p0 < npieces; p0 += G * NCH) {
                    load_pair<B1, B2, G, CH, NCH>(P, a, e, e1, slot, p0, g, npieces);
                    accumulate_pair<B1, B2, METRIC, MASK, G, CH, NCH, false>(P, tq, qr, mtab, p0, g, npieces, R,
                                                                             A, l2acc);
                }
            }

            float score = finish_pair<B2, METRIC, G>(A, l2acc, hdr, cmt, a.n_means, qsum);
            if (valid && !work) {
                score = __uint_as_float(0x7FC00000u);
                if (g == 0 && !(a.neg_empty && slot < 0)) atomicOr(a.err, kErrBadSlot);
            }
            if (valid && g == 0 && a.dist) a.dist[e] = score;
            if (k > 0) {
                uint64_t key = kNoKey;
                if (work) {
                    const bool live = ((__float_as_uint(hdr.w) >> 8) & 1u) && ep.x <= a.epoch && a.epoch < ep.y;
                    if (live) key = make_key(score, slot, METRIC);
                }
                const bool pass = valid && g == 0 && key < thr;
                const uint64_t bal = __ballot(pass);
                const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                if (pass) wbuf[nw + below] = key;
                nw += __popcll(bal);
                // compact when the next block might not fit, and after the
                // last block (the merge takes at most k keys per wave)
                if (nw > a.cw - kPairsPerWave || (base + kPairsPerBlock >= e1 && nw > k)) {
                    const int got = wave_compact_lean(wbuf, nw, k, merge + (size_t)wave * k);
                    nw = got;
                    const uint64_t t = got == k ? wbuf[k - 1] : kNoKey;
                    thr = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t >> 32)) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t);
                }
            }
        }

        if (k > 0) {
            // each wave holds at most k keys; wave 0 merges the four
            if (lane == 0) s_got[wave] = nw;
            __syncthreads();
            if (wave == 0) {
                int n = 0;
                for (int w = 0; w < 4; ++w) {
                    const int gw = s_got[w];
                    for (int i = lane; i < gw; i += 64) merge[n + i] = keys[(size_t)w * a.cw + i];
                    n += gw;
                }
                const int got = wave_compact_lean(merge, n, k, keys);
                for (int i = lane; i < k; i += 64) {
                    int32_t sid = -1;
                    float sv = METRIC == LVQ_L2 ? __uint_as_float(0x7F800000u) : __uint_as_float(0xFF800000u);
                    if (i < got) {
                        sid = (int32_t)(uint32_t)merge[i];
                        sv = key_score(merge[i], METRIC);
                    }
                    a.topk_ids[list * k + i] = sid;
                    a.topk_dist[list * k + i] = sv;
                }
            }
        }
    }
}

// LDS bytes of one k_cand launch with per-wave key buffers of cw entries
inline size_t cand_lds_bytes_impl(int kpos, int ntab, bool mask, int n_means_ip, int k, int cw, bool map, int nseg)
{
    size_t b = (size_t)ntab * kpos * 4 + (mask ? (size_t)kpos * 4 : 0) + (size_t)((n_means_ip + 1) & ~1) * 4;
    if (map) b += kMaxMeans;
    if (nseg > 0) b += (size_t)2 * (nseg + 1) * 8;
    b = (b + 15) & ~(size_t)15;
    if (k > 0) b += ((size_t)4 * cw + (size_t)4 * k) * 8;
    return b;
}

}  // namespace lvq
