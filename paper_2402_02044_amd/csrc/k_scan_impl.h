// k_scan_impl.h -- exhaustive top-k over every live slot (the k-NN problem of
// Sec. 2.1), FP32 vector-ALU form.
//
// Grid: (query tile of TQ queries) x (part of the slot range).  Each
// workgroup keeps its TQ queries in LDS (bank-conflict-free layout shared
// with the candidate kernel) and streams its part of the store: a group of G
// lanes loads R rows at a time, decodes them once into registers
//   IP: y_p = Delta c1_p [+ Delta2 c2_p]          (score = c_m + l' sum q + <q, y>)
//   L2: x'_p = l' + Delta c1_p [+ Delta2 c2_p]    (score = sum (q' - x')^2,
//       padding positions forced to 0 so they contribute nothing)
// and reuses them for all TQ queries.  Scores that beat a query's running
// k-th best key are appended to a per-query LDS buffer that a wavefront
// compacts back to k keys when it fills; each (query, part) writes its k best
// keys, and k_topk_merge reduces the parts.
#pragma once

#include "k_cand_impl.h"

namespace lvq {

constexpr int kScanTQ = 16;  // queries per workgroup
constexpr int kScanR = 2;    // rows per lane group and round

inline size_t scan_lds_bytes_impl(int kpos, int n_means_ip, int k, int capq)
{
    size_t b = (size_t)kScanTQ * kpos * 4;                  // query tables
    b += (size_t)kScanTQ * (((n_means_ip + 1) & ~1) + 2) * 4; // c_m, sum q
    b = (b + 15) & ~(size_t)15;
    b += (size_t)kScanTQ * 16;                              // thresholds + counts
    b += (size_t)kScanTQ * capq * 8;                        // candidate buffers
    b += (size_t)4 * k * 8;                                  // per-wave select scratch
    return b;
}

// Per-query key buffer: up to 512 keys (the register sort's reach) while the
// workgroup keeps room for two resident workgroups per CU, at least k + one
// round of rows; 0 when that does not fit.
inline int scan_capq_impl(int kpos, int n_means_ip, int k, int rows_per_round, size_t lds_max)
{
    const int need = k + rows_per_round;
    int cap = need > 512 ? need : 512;
    while (cap > need && scan_lds_bytes_impl(kpos, n_means_ip, k, cap) > lds_max / 2) cap -= 16;
    if (cap < need) cap = need;
    return scan_lds_bytes_impl(kpos, n_means_ip, k, cap) <= lds_max ? cap : 0;
}

template <int B1, int B2, int METRIC, bool MASK, int G, int CH, int NCH>
__global__ __launch_bounds__(256) void k_scan(ScanArgs a)
{
    using Geo = CandGeom<B1, CH>;
    using RGeo = ResGeom<B1, B2, CH>;
    constexpr int R = kScanR;
    constexpr int TQ = kScanTQ;
    constexpr int NG = 256 / G;               // lane groups per workgroup
    constexpr int kRows = NG * R;             // rows per round
    constexpr int kVals = NCH * Geo::kSlots;  // decoded values per lane and row

    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int grp = tid / G, g = tid % G;
    const int npieces = a.kchunks * 16 / CH;
    const int cm_n = METRIC == LVQ_IP ? a.n_means : 0;
    const int cm_stride = ((cm_n + 1) & ~1) + 2;
    const int k = a.k;
    const int capq = a.capq;   // >= k + kRows

    // offsets from the LDS base keep every pointer in the LDS address space
    float *qtab = reinterpret_cast<float *>(smem);
    float *qc = qtab + (size_t)TQ * a.kpos;                 // [TQ][cm_stride]: c_m..., sum q
    const size_t off = (((size_t)TQ * a.kpos + (size_t)TQ * cm_stride) * sizeof(float) + 15) & ~(size_t)15;
    uint64_t *thr = reinterpret_cast<uint64_t *>(smem + off);
    int *cnt = reinterpret_cast<int *>(thr + TQ);
    uint64_t *buf = reinterpret_cast<uint64_t *>(cnt + 2 * TQ);
    uint64_t *tmp = buf + (size_t)TQ * capq;

    const int64_t q0 = (int64_t)blockIdx.x * TQ;
    const int nqt = (int)min<int64_t>(TQ, a.nq - q0);
    const int64_t r0 = (int64_t)blockIdx.y * a.rows_per_part;
    const int64_t r1 = min<int64_t>(a.n_rows, r0 + a.rows_per_part);

    for (int t = 0; t < TQ; ++t)
        for (int s = tid; s < a.kpos; s += 256) {
            float v = 0.0f;
            if (t < nqt) {
                v = a.qk[(q0 + t) * a.kpos + s];
                if (METRIC == LVQ_L2) v -= a.muk[s];
            }
            qtab[(size_t)t * a.kpos + qtab_index<B1, CH>(s, npieces)] = v;
        }
    for (int t = tid; t < TQ * cm_stride; t += 256) {
        const int qi = t / cm_stride, m = t % cm_stride;
        float v = 0.0f;
        if (qi < nqt) {
            if (m < cm_n) v = a.cm[(q0 + qi) * a.n_means + m];
            else if (m == cm_stride - 1 && METRIC == LVQ_IP) v = a.qsum[q0 + qi];
        }
        qc[t] = v;
    }
    if (tid < TQ) {
        thr[tid] = kNoKey;
        cnt[tid] = 0;
    }
    __syncthreads();

    for (int64_t base = r0; base < r1; base += kRows) {
        // ---- load R rows per group (all pieces issued first)
        Words<Geo::kWords> wv[R][NCH];
        Words<RGeo::kWords> rv[R][NCH];
        float4 hdr[R];
        bool live[R];
        int64_t slot[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int64_t pos = base + (int64_t)grp * R + rr;
            const bool in = pos < r1;
            slot[rr] = a.list[in ? pos : r0];   // list position -> slot
            const uint8_t *row = a.rows + slot[rr] * a.row_bytes;
            hdr[rr] = in ? *reinterpret_cast<const float4 *>(row) : make_float4(0.f, 0.f, 0.f, 0.f);
            uint2 ep = in ? *reinterpret_cast<const uint2 *>(row + 16) : make_uint2(1u, 0u);
            live[rr] = in && ((__float_as_uint(hdr[rr].w) >> 8) & 1u) && ep.x <= a.epoch && a.epoch < ep.y;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int u = c * G + g;
                if (in && u < npieces) {
                    wv[rr][c] = load_words<Geo::kWords>(row + kHeaderBytes + u * CH);
                    if constexpr (B2 != 0)
                        rv[rr][c] = load_words<RGeo::kWords>(a.resid + slot[rr] * a.resid_bytes +
                                                             u * RGeo::kBytes);
                } else {
#pragma unroll
                    for (int i = 0; i < Geo::kWords; ++i) wv[rr][c].w[i] = 0;
#pragma unroll
                    for (int i = 0; i < RGeo::kWords; ++i) rv[rr][c].w[i] = 0;
                }
            }
        }
        // ---- decode once per row
        float xv[R][kVals];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const float l = hdr[rr].x, dl = hdr[rr].y, dl2 = hdr[rr].z;
            const float lp = B2 ? l - 0.5f * dl : l;
            const float base_v = METRIC == LVQ_L2 ? lp : 0.0f;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int u = c * G + g;
                float mk[Geo::kSlots];
                if constexpr (MASK) {
#pragma unroll
                    for (int s = 0; s < Geo::kSlots; ++s) {
                        const int pos = u * Geo::kSlots + s;
                        mk[s] = (u < npieces && pos < a.kpos) ? a.kmask[pos] : 0.0f;
                    }
                }
#pragma unroll
                for (int wi = 0; wi < Geo::kWords; ++wi) {
                    const uint32_t w = wv[rr][c].w[wi];
                    float c1[B1 == 4 ? 8 : 4], c2[B1 == 4 ? 8 : 4], s1[B1 == 4 ? 8 : 4], s2[B1 == 4 ? 8 : 4];
                    if constexpr (B1 == 4) {
                        const uint32_t lo = w & 0x0F0F0F0Fu, hi = w & 0xF0F0F0F0u;
                        c1[0] = ub<0>(lo); c1[1] = ub<1>(lo); c1[2] = ub<2>(lo); c1[3] = ub<3>(lo);
                        c1[4] = ub<0>(hi); c1[5] = ub<1>(hi); c1[6] = ub<2>(hi); c1[7] = ub<3>(hi);
                        for (int s = 0; s < 4; ++s) { s1[s] = dl; s1[s + 4] = dl * 0.0625f; }
                        for (int s = 0; s < 8; ++s) { c2[s] = 0.f; s2[s] = dl2; }
                        if constexpr (B2 == 8) {
                            const uint32_t q0w = rv[rr][c].w[2 * wi], q1w = rv[rr][c].w[2 * wi + 1];
                            c2[0] = ub<0>(q0w); c2[1] = ub<2>(q0w); c2[2] = ub<0>(q1w); c2[3] = ub<2>(q1w);
                            c2[4] = ub<1>(q0w); c2[5] = ub<3>(q0w); c2[6] = ub<1>(q1w); c2[7] = ub<3>(q1w);
                        } else if constexpr (B2 == 4) {
                            const uint32_t r = rv[rr][c].w[wi];
                            const uint32_t rl = r & 0x0F0F0F0Fu, rh = r & 0xF0F0F0F0u;
                            c2[0] = ub<0>(rl); c2[1] = ub<1>(rl); c2[2] = ub<2>(rl); c2[3] = ub<3>(rl);
                            c2[4] = ub<0>(rh); c2[5] = ub<1>(rh); c2[6] = ub<2>(rh); c2[7] = ub<3>(rh);
                            for (int s = 4; s < 8; ++s) s2[s] = dl2 * 0.0625f;
                        }
                    } else {
                        c1[0] = ub<0>(w); c1[1] = ub<1>(w); c1[2] = ub<2>(w); c1[3] = ub<3>(w);
                        for (int s = 0; s < 4; ++s) { s1[s] = dl; c2[s] = 0.f; s2[s] = dl2; }
                        if constexpr (B2 == 8) {
                            const uint32_t r = rv[rr][c].w[wi];
                            c2[0] = ub<0>(r); c2[1] = ub<1>(r); c2[2] = ub<2>(r); c2[3] = ub<3>(r);
                        } else if constexpr (B2 == 4) {
                            const uint32_t h = (rv[rr][c].w[wi >> 1] >> (16 * (wi & 1))) & 0xFFFFu;
                            const uint32_t rl = h & 0x0F0Fu, rh = h & 0xF0F0u;
                            c2[0] = ub<0>(rl); c2[2] = ub<1>(rl); c2[1] = ub<0>(rh); c2[3] = ub<1>(rh);
                            s2[1] = dl2 * 0.0625f; s2[3] = dl2 * 0.0625f;
                        }
                    }
                    constexpr int QW = B1 == 4 ? 8 : 4;
#pragma unroll
                    for (int s = 0; s < QW; ++s) {
                        float v = fmaf(s1[s], c1[s], base_v);
                        if constexpr (B2 != 0) v = fmaf(s2[s], c2[s], v);
                        if constexpr (MASK) v *= mk[wi * QW + s];
                        xv[rr][c * Geo::kSlots + wi * QW + s] = v;
                    }
                }
            }
        }
        // ---- all queries of the tile
        for (int qi = 0; qi < nqt; ++qi) {
            const float *tq = qtab + (size_t)qi * a.kpos;
            float acc[R];
#pragma unroll
            for (int rr = 0; rr < R; ++rr) acc[rr] = 0.0f;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int u = c * G + g;
                if (u >= npieces) continue;
#pragma unroll
                for (int r4 = 0; r4 < Geo::kF4; ++r4) {
                    float4 f = reinterpret_cast<const float4 *>(tq)[r4 * npieces + u];
                    float qv[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int rr = 0; rr < R; ++rr) {
                            const float x = xv[rr][c * Geo::kSlots + 4 * r4 + e];
                            if constexpr (METRIC == LVQ_IP) {
                                acc[rr] = fmaf(qv[e], x, acc[rr]);
                            } else {
                                const float t = qv[e] - x;
                                acc[rr] = fmaf(t, t, acc[rr]);
                            }
                        }
                }
            }
            const float *qcq = qc + (size_t)qi * cm_stride;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                float sc = group_sum<G>(acc[rr]);
                if constexpr (METRIC == LVQ_IP) {
                    const int mid = (int)(__float_as_uint(hdr[rr].w) & 0xFFu);
                    const float l = hdr[rr].x, dl = hdr[rr].y;
                    const float lp = B2 ? l - 0.5f * dl : l;
                    sc = fmaf(lp, qcq[cm_stride - 1], qcq[mid < a.n_means ? mid : 0]) + sc;
                }
                if (live[rr] && g == 0) {
                    const uint64_t key = make_key(sc, (int32_t)slot[rr], METRIC);
                    if (key < thr[qi]) {
                        int pos = atomicAdd(&cnt[qi], 1);
                        if (pos < capq) buf[(size_t)qi * capq + pos] = key;
                    }
                }
            }
        }
        __syncthreads();
        // ---- compact buffers that could overflow next round
        const bool last = base + kRows >= r1;
        for (int qi = wave; qi < nqt; qi += 4) {
            const int n = min(cnt[qi], capq);
            if (last || n > capq - kRows) {
                uint64_t *qb = buf + (size_t)qi * capq;
                const int got = wave_compact(qb, n, k, tmp + (size_t)wave * k);
                if (lane == 0) {
                    cnt[qi] = got;
                    thr[qi] = got == k ? qb[k - 1] : kNoKey;
                }
            }
        }
        __syncthreads();
    }
    // ---- (query, part) results; an empty part writes no keys
    for (int qi = wave; qi < TQ; qi += 4) {
        if (qi >= nqt) continue;
        uint64_t *dst = a.part_keys + ((q0 + qi) * a.n_parts + blockIdx.y) * (int64_t)k;
        const int got = r1 > r0 ? cnt[qi] : 0;
        for (int i = lane; i < k; i += 64) dst[i] = i < got ? buf[(size_t)qi * capq + i] : kNoKey;
    }
}

}  // namespace lvq
