// k_graph.hip -- greedy graph search (Alg. 1) and the pieces of graph
// construction (App. A): neighbourhood pruning (Alg. 2) and reverse edges.
//
// Search: one workgroup per query.  LDS holds the query (kernel order for
// LVQ rows, natural order for float vectors) and the L2 padding mask, the
// candidate set -- at most W keys, best first -- and a hash set of every node
// proposed so far.  A key is (score order << 32) | (slot << 1) | explored: the
// explored flag travels with the key through the sorts without changing the
// (score, slot) order of distinct nodes.  Each step explores the best
// unexplored key: its out-neighbours not seen before are scored (4 or 16 lanes per
// neighbour) and merged, and the set is cut to the W best.  Deleted rows are
// traversed; the result is the k best live ones.  Over LVQ rows the
// similarity is the first level (Sec. 2.3: the first level traverses, both
// levels re-rank); over float vectors (construction) it is the binary32
// squared distance or inner product.
//
// Pruning: one workgroup per node.  Its candidates and current out-neighbours
// are scored against it into LDS keys, sorted by one wave and deduplicated;
// the best remaining candidate x* is kept and every candidate that x* is at
// least alpha times as similar to as the node is dropped, until R are kept.
#include <algorithm>
#include <type_traits>

#include "k_common.h"

namespace lvq {
namespace {

constexpr int kMaxHash = 16384;   // seen-set hash slots per query (int32 slot or -1)
constexpr int kMaxDegree = kGraphMaxDegree;
constexpr int kMaxWindow = 256;
constexpr int kPruneCap = kPruneChunk + kMaxDegree;   // candidates of one merge
constexpr int kFloat = 0;                             // MODE of float vectors

struct GraphArgs {
    const uint8_t *rows;
    int row_bytes, kchunks, kpos;
    int64_t capacity;
    const float *qk, *qsum, *cm, *muk, *kmask;
    int n_means, metric;
    int64_t nq;
    const int32_t *graph;
    int degree;
    const int32_t *entries;
    int n_entries;
    int window, k;
    uint32_t epoch;
    int32_t *ids;
    float *dist;
    int32_t *explored;
    uint32_t *err;
    const float *xf;
    int dim;
    const int32_t *qnodes;
    int hash_slots;
};

// Open-addressing hash set h of n slots (-1 marks an empty slot), linear
// probing from a multiplicative hash scaled to [0, n).  Insert: 1 if s was
// not there, 0 if it was, -1 if the set is full.
__device__ __forceinline__ uint32_t hash_home(int32_t s, uint32_t n)
{
    return (uint32_t)(((uint64_t)((uint32_t)s * 2654435761u) * n) >> 32);
}

__device__ __forceinline__ int hash_insert(int32_t *h, int32_t s, uint32_t n)
{
    uint32_t i = hash_home(s, n);
    for (uint32_t probe = 0; probe < n; ++probe) {
        const int32_t old = atomicCAS(&h[i], -1, s);
        if (old == -1) return 1;
        if (old == s) return 0;
        i = i + 1 == n ? 0 : i + 1;
    }
    return -1;
}

__device__ __forceinline__ bool hash_contains(const int32_t *h, int32_t s, uint32_t n)
{
    uint32_t i = hash_home(s, n);
    for (uint32_t probe = 0; probe < n; ++probe) {
        const int32_t v = h[i];
        if (v == s) return true;
        if (v == -1) return false;
        i = i + 1 == n ? 0 : i + 1;
    }
    return false;
}

// Similarity of two float vectors (one in LDS, one in global memory) by the
// G lanes of a group (G = 4 or 16); every lane of the group returns the value.
template <int METRIC, int G>
__device__ __forceinline__ float sim_f32(const float *u, const float *x, int dim, int g)
{
    float s = 0.0f;
    for (int j = g; j < dim; j += G) {
        const float v = x[j];
        if constexpr (METRIC == LVQ_IP) {
            s = fmaf(u[j], v, s);
        } else {
            const float t = u[j] - v;
            s = fmaf(t, t, s);
        }
    }
    return group_sum<G>(s);
}

// Similarity of one stored node to the query, by one lane.  LVQ rows: the
// first level in kernel order (qt less the mean when there is one mean, L2;
// IP adds l * sum(q) + <q, mu_m> from qsum / cm); the L2 padding mask is
// applied from chunk cpad on (the first 16-byte chunk of codes holding a
// padding position).  Float rows: binary32 squared distance or inner product.
template <int B1, int METRIC, bool ONE_MEAN>
__device__ __forceinline__ float score_rows(const GraphArgs &a, const float *qt, const float *mk, int32_t slot,
                                            float qsum, const float *cm, int cpad)
{
    const uint8_t *row = a.rows + (int64_t)slot * a.row_bytes;
    const float4 hdr = *reinterpret_cast<const float4 *>(row);
    const uint4 *code = reinterpret_cast<const uint4 *>(row + kHeaderBytes);
    const int mid = min((int)(__float_as_uint(hdr.w) & 0xFFu), a.n_means - 1);
    const float l = hdr.x, dl = hdr.y;
    const float *mu = a.muk + (int64_t)mid * a.kpos;
    constexpr int PER = B1 == 8 ? 4 : 8;   // positions per 32-bit word
    const float4 *q4 = reinterpret_cast<const float4 *>(qt);
    const float4 *m4 = reinterpret_cast<const float4 *>(mk);
    float s = 0.0f;
    // one 16-byte chunk; the mask is applied only in the chunks from cpad on,
    // which run in a loop of their own (same order of accumulation)
    auto chunk = [&](int c, auto masked_tag) {
        constexpr bool masked = decltype(masked_tag)::value;
        const uint4 v = code[c];
        const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w = wv[i];
            const int p0 = (4 * c + i) * PER;
            float cv[PER], qv[PER], mv[PER];
            if constexpr (B1 == 8) {
                cv[0] = ub<0>(w); cv[1] = ub<1>(w); cv[2] = ub<2>(w); cv[3] = ub<3>(w);
            } else {
                // kernel order of a 4-bit word: fields 0,2,4,6 (low nibbles), then 1,3,5,7
                const uint32_t lo = w & 0x0F0F0F0Fu, hi = (w >> 4) & 0x0F0F0F0Fu;
                cv[0] = ub<0>(lo); cv[1] = ub<1>(lo); cv[2] = ub<2>(lo); cv[3] = ub<3>(lo);
                cv[4] = ub<0>(hi); cv[5] = ub<1>(hi); cv[6] = ub<2>(hi); cv[7] = ub<3>(hi);
            }
#pragma unroll
            for (int h = 0; h < PER / 4; ++h) {
                const float4 q = q4[p0 / 4 + h];
                qv[4 * h] = q.x; qv[4 * h + 1] = q.y; qv[4 * h + 2] = q.z; qv[4 * h + 3] = q.w;
                if constexpr (masked) {
                    const float4 m = m4[p0 / 4 + h];
                    mv[4 * h] = m.x; mv[4 * h + 1] = m.y; mv[4 * h + 2] = m.z; mv[4 * h + 3] = m.w;
                }
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                if constexpr (METRIC == LVQ_IP) {
                    s = fmaf(qv[j], cv[j], s);
                } else {
                    const float qj = ONE_MEAN ? qv[j] : qv[j] - mu[p0 + j];
                    float t = qj - fmaf(dl, cv[j], l);
                    if constexpr (masked) t *= mv[j];
                    s = fmaf(t, t, s);
                }
            }
        }
    };
    const int split = METRIC == LVQ_L2 ? min(cpad, a.kchunks) : a.kchunks;
    for (int c = 0; c < split; ++c) chunk(c, std::false_type{});
    for (int c = split; c < a.kchunks; ++c) chunk(c, std::true_type{});
    if constexpr (METRIC == LVQ_IP) return fmaf(dl, s, fmaf(l, qsum, cm[mid]));
    return s;
}

template <int B1, int METRIC>
__device__ __forceinline__ float score_lane(const GraphArgs &a, const float *qt, const float *mk, int32_t slot,
                                            float qsum, const float *cm, int cpad)
{
    if constexpr (B1 == kFloat) {
        const float *x = a.xf + (int64_t)slot * a.dim;
        float s = 0.0f;
        if ((a.dim & 3) == 0) {
            const float4 *x4 = reinterpret_cast<const float4 *>(x);
            const float4 *q4 = reinterpret_cast<const float4 *>(qt);
            for (int c = 0; c < (a.dim >> 2); ++c) {
                const float4 v = x4[c], q = q4[c];
                if constexpr (METRIC == LVQ_IP) {
                    s = fmaf(q.x, v.x, s);
                    s = fmaf(q.y, v.y, s);
                    s = fmaf(q.z, v.z, s);
                    s = fmaf(q.w, v.w, s);
                } else {
                    const float t0 = q.x - v.x, t1 = q.y - v.y, t2 = q.z - v.z, t3 = q.w - v.w;
                    s = fmaf(t0, t0, s);
                    s = fmaf(t1, t1, s);
                    s = fmaf(t2, t2, s);
                    s = fmaf(t3, t3, s);
                }
            }
        } else {
            for (int j = 0; j < a.dim; ++j) {
                if constexpr (METRIC == LVQ_IP) {
                    s = fmaf(qt[j], x[j], s);
                } else {
                    const float t = qt[j] - x[j];
                    s = fmaf(t, t, s);
                }
            }
        }
        return s;
    } else if (METRIC == LVQ_IP || a.n_means != 1) {
        return score_rows<B1, METRIC, false>(a, qt, mk, slot, qsum, cm, cpad);
    } else {
        return score_rows<B1, METRIC, true>(a, qt, mk, slot, qsum, cm, cpad);
    }
}

__device__ __forceinline__ int32_t key_node(uint64_t k)
{
    return (int32_t)((uint32_t)k >> 1);
}

// Ascending sort of the wave's 64 keys (one per lane, all lanes active),
// the bitonic network of wave_bitonic_sort with each exchange distance's own
// data movement: DPP quad permutations for lanes 1 and 2 apart (11 of the 21
// stages), ds_swizzle's bit mode for 4 to 16 (within 32-lane halves) and
// ds_bpermute only for 32.
template <int J>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v)
{
    if constexpr (J == 1) return dpp_u32<0xB1>(v);   // quad_perm [1,0,3,2]
    else if constexpr (J == 2) return dpp_u32<0x4E>(v);   // quad_perm [2,3,0,1]
    else if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);
    else return __shfl_xor(v, J, 64);
}

template <int SIZE, int J>
__device__ __forceinline__ void sort64_stages(uint64_t &v, int lane)
{
    const uint64_t o = ((uint64_t)xor_lane_u32<J>((uint32_t)(v >> 32)) << 32) | xor_lane_u32<J>((uint32_t)v);
    const bool asc = (lane & SIZE) == 0;
    const bool lower = (lane & J) == 0;
    const uint64_t mn = o < v ? o : v, mx = o < v ? v : o;
    v = lower == asc ? mn : mx;
    if constexpr (J > 1) sort64_stages<SIZE, J / 2>(v, lane);
}

template <int SIZE = 2>
__device__ __forceinline__ void wave_sort64(uint64_t &v, int lane)
{
    sort64_stages<SIZE, SIZE / 2>(v, lane);
    if constexpr (SIZE < 64) wave_sort64<SIZE * 2>(v, lane);
}

// One wavefront (one 64-lane workgroup) per query.  Each step explores the
// best unexplored node x: lane t takes x's out-neighbour t, drops nodes that
// entered the set before, and scores the rest, one neighbour per lane.  The
// new keys are sorted across the wave (register bitonic sort), repeats of a
// node (equal keys, now adjacent) are dropped, and the keys are merged into
// the sorted set by binary searches: a new key lands at its index
// among the new keys plus the number of set keys below it, a set key moves
// down by the number of new keys below it.  Keys landing below W form the new
// set; the smallest position of an unexplored key is the next node.
template <int B1, int METRIC>
__global__ __launch_bounds__(64) void k_graph_search(GraphArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int64_t qi = blockIdx.x;
    if (qi >= a.nq) return;
    const int W = a.window;
    const int kq = (a.kpos + 3) & ~3;
    float *qt = reinterpret_cast<float *>(smem);                     // kq
    float *mk = qt + kq;                                             // kq
    uint64_t *cur = reinterpret_cast<uint64_t *>(mk + kq);           // W: the candidate set, ascending
    uint64_t *nxt = cur + W;                                         // W: the merged set
    uint64_t *skey = nxt + W;                                        // 64: a step's keys, ascending
    int32_t *hset = reinterpret_cast<int32_t *>(skey + 64);          // hash_slots: nodes that entered

    const float *qsrc = a.qk + qi * a.kpos;
    bool qok = true;
    if constexpr (B1 == kFloat) {
        if (a.qnodes) {
            const int32_t node = a.qnodes[qi];
            qok = node >= 0 && node < a.capacity;
            qsrc = a.xf + (int64_t)(qok ? node : 0) * a.dim;
        }
    }
    for (int p = lane; p < kq; p += 64) {
        float v = p < a.kpos ? qsrc[p] : 0.0f;
        if (B1 != kFloat && METRIC == LVQ_L2 && a.n_means == 1 && p < a.kpos) v -= a.muk[p];   // q - mu once
        qt[p] = v;
        mk[p] = METRIC == LVQ_L2 && B1 != kFloat && p < a.kpos ? a.kmask[p] : 1.0f;
    }
    const uint32_t hn = (uint32_t)a.hash_slots;
    for (int i = lane; i < a.hash_slots; i += 64) hset[i] = -1;
    if (lane == 0 && !qok) atomicOr(a.err, kErrBadSlot);
    // first 16-byte code chunk holding a padding position (L2 mask)
    int cpad = 1 << 30;
    if constexpr (B1 != kFloat && METRIC == LVQ_L2) {
        int first = 1 << 30;
        for (int p = lane; p < a.kpos; p += 64)
            if (a.kmask[p] == 0.0f) first = min(first, p);
        first = (int)wave_min_u64((uint64_t)(uint32_t)first);
        cpad = first == (1 << 30) ? first : first / (B1 == 8 ? 16 : 32);
    }
    const float qsum = B1 != kFloat && METRIC == LVQ_IP ? a.qsum[qi] : 0.0f;
    const float *cm = B1 != kFloat && METRIC == LVQ_IP ? a.cm + qi * a.n_means : nullptr;
    __syncthreads();

    int qn = 0, pick = 1 << 30, explored = 0, scored = 0;
    bool stop = false;
    // Merge the lanes' keys (kNoKey where none) into the set; returns the
    // number of distinct new nodes.
    auto merge = [&](uint64_t key) -> int {
        wave_sort64(key, lane);
        const uint32_t plo = __shfl_up((uint32_t)key, 1, 64), phi = __shfl_up((uint32_t)(key >> 32), 1, 64);
        const bool valid = key != kNoKey && !(lane > 0 && key == (((uint64_t)phi << 32) | plo));
        const uint64_t vm = __ballot(valid);
        const int nn = __popcll(vm);
        const int j = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(vm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)vm, 0u));
        if (valid) skey[j] = key;
        __syncthreads();
        int best = 1 << 30;
        bool full = false;
        if (valid) {
            int lo = 0, hi = qn;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cur[mid] < key) lo = mid + 1;
                else hi = mid;
            }
            const int p = j + lo;
            if (p < W) {
                nxt[p] = key;
                best = p;
                // remembered: not proposed again while in the set, and once
                // cut it could not re-enter (the W-th best only improves)
                full = hash_insert(hset, key_node(key), hn) < 0;
            }
        }
        for (int i = lane; i < qn; i += 64) {
            const uint64_t k = cur[i];
            int lo = 0, hi = nn;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (skey[mid] < k) lo = mid + 1;
                else hi = mid;
            }
            const int p = i + lo;
            if (p < W) {
                nxt[p] = k;
                if (!(k & 1ull) && p < best) best = p;
            }
        }
        if (__ballot(full)) {
            if (lane == 0) atomicOr(a.err, kErrOverflow);
            stop = true;
        }
        __syncthreads();
        pick = (int)wave_min_u64((uint64_t)(uint32_t)best);
        qn = min(W, qn + nn);
        uint64_t *t = cur;
        cur = nxt;
        nxt = t;
        return nn;
    };

    // entry nodes (at most 64), repeats dropped
    {
        int32_t s = lane < a.n_entries && qok ? a.entries[lane] : -1;
        if (s >= a.capacity) s = -1;
        uint64_t key = kNoKey;
        if (s >= 0) {
            const float v = score_lane<B1, METRIC>(a, qt, mk, s, qsum, cm, cpad);
            key = (make_key(v, 0, METRIC) & 0xFFFFFFFF00000000ull) | ((uint64_t)(uint32_t)s << 1);
        }
        scored = merge(key);
    }

    while (pick < qn && !stop) {
        const uint64_t kx = cur[pick];
        const int32_t x = key_node(kx);
        // the set's W-th key (its explored bit, which the mark below may
        // change, plays no part in comparisons with new keys)
        const uint64_t worst = qn == W ? cur[W - 1] : kNoKey;
        if (lane == 0) cur[pick] = kx | 1ull;   // explored; read by the merge after its barrier
        ++explored;
        // out-neighbours that never entered the set; one rejected before is
        // scored again and rejected again, since the set's W-th best only
        // improves
        int32_t y = lane < a.degree ? a.graph[(int64_t)x * a.degree + lane] : -1;
        if (y >= a.capacity) y = -1;
        if (y >= 0 && hash_contains(hset, y, hn)) y = -1;
        uint64_t key = kNoKey;
        if (y >= 0) {
            const float v = score_lane<B1, METRIC>(a, qt, mk, y, qsum, cm, cpad);
            key = (make_key(v, 0, METRIC) & 0xFFFFFFFF00000000ull) | ((uint64_t)(uint32_t)y << 1);
        }
        scored += __popcll(__ballot(y >= 0));
        // A full set keeps only keys below its W-th: when no lane has one, the
        // merge would change nothing but the explored mark, and the next node
        // is the first unexplored key of the set as it stands.
        if (!__ballot(key < worst)) {
            __syncthreads();   // the explored mark
            pick = 1 << 30;
            for (int base = 0; base < qn; base += 64) {
                const int i = base + lane;
                const uint64_t m = __ballot(i < qn && !(cur[i] & 1ull));
                if (m) {
                    pick = base + __builtin_ctzll(m);
                    break;
                }
            }
            continue;
        }
        merge(key);
    }

    // the k best live keys, in order
    int out = 0;
    for (int base = 0; base < qn && out < a.k; base += 64) {
        const int i = base + lane;
        bool live = false;
        uint64_t key = kNoKey;
        if (i < qn) {
            key = cur[i];
            if constexpr (B1 == kFloat) {
                live = true;
            } else {
                const uint8_t *row = a.rows + (int64_t)key_node(key) * a.row_bytes;
                const uint2 ep = *reinterpret_cast<const uint2 *>(row + 16);
                live = (row[13] & 1u) && ep.x <= a.epoch && a.epoch < ep.y;
            }
        }
        const uint64_t m = __ballot(live);
        const int pos = out + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (live && pos < a.k) {
            a.ids[qi * a.k + pos] = key_node(key);
            if (a.dist) a.dist[qi * a.k + pos] = key_score(key, METRIC);
        }
        out += __popcll(m);
    }
    for (int i = max(out, 0) + lane; i < a.k; i += 64) {
        a.ids[qi * a.k + i] = -1;
        if (a.dist)
            a.dist[qi * a.k + i] = METRIC == LVQ_L2 ? __uint_as_float(0x7F800000u) : __uint_as_float(0xFF800000u);
    }
    if (lane == 0 && a.explored) {
        a.explored[2 * qi] = explored;
        a.explored[2 * qi + 1] = scored;
    }
}

// ---- neighbourhood pruning (Alg. 2) ----------------------------------------

template <int METRIC, int G>
__global__ __launch_bounds__(256) void k_graph_prune(PruneLaunch a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int grp = tid / G, g = tid % G;
    const int64_t i = blockIdx.x;
    if (i >= a.m) return;
    float *xv = reinterpret_cast<float *>(smem);   // the node (dim)
    float *xs = xv + a.dim;                        // x* (dim)
    __shared__ uint64_t keys[512];
    __shared__ int32_t cid[kPruneCap];
    __shared__ int32_t kept[kMaxDegree];
    __shared__ uint8_t rm[kPruneCap];
    __shared__ int s_n, s_kept, s_pick, s_unique;

    const int32_t p = a.nodes[i];
    if (p < 0 || p >= a.n) {
        if (tid == 0) atomicOr(a.err, kErrBadSlot);
        return;
    }
    const uint8_t *del = a.deleted;
    int64_t c0, c1;
    if (del) {
        // delete consolidation: position j names out-neighbour j / R of p
        // and, when that one is deleted, its out-neighbour j % R
        c0 = 0;
        c1 = (int64_t)a.R * a.R;
    } else if (a.coffs) {
        const int64_t j = a.by_node ? (int64_t)p : i;
        c0 = a.coffs[j];
        c1 = a.coffs[j + 1];
    } else {
        c0 = i * a.cstride;
        c1 = c0 + a.cstride;
    }
    if (c0 < 0 || c1 < c0) {
        if (tid == 0) atomicOr(a.err, kErrBadOffsets);
        return;
    }
    for (int j = tid; j < a.dim; j += 256) xv[j] = a.xf[(int64_t)p * a.dim + j];
    if (tid == 0) s_kept = 0;
    __syncthreads();
    // the current out-neighbours (kept in LDS across chunks)
    if (tid == 0)
        for (int r = 0; r < a.R; ++r) {
            const int32_t y = a.graph[(int64_t)p * a.R + r];
            if (y >= 0 && y < a.n && y != p && !(del && del[y])) kept[s_kept++] = y;
        }
    __syncthreads();

    int64_t cs = c0;   // next position block (kPruneChunk positions) to read
    for (;;) {
        if (tid == 0) s_n = s_kept;
        for (int r = tid; r < s_kept; r += 256) cid[r] = kept[r];
        __syncthreads();
        // append whole position blocks, in order, while their candidates fit
        // beside the out-neighbours kept so far (the first block always fits:
        // R + kPruneChunk <= kPruneCap)
        for (;;) {
            const int have = s_n;   // last written before the preceding barrier
            const int64_t j = cs + tid;
            int32_t y = -1;
            if (j < c1) {
                if (del) {
                    const int32_t v = a.graph[(int64_t)p * a.R + j / a.R];
                    y = v >= 0 && v < a.n && del[v] ? a.graph[(int64_t)v * a.R + j % a.R] : -1;
                    if (y >= 0 && y < a.n && del[y]) y = -1;
                } else {
                    y = a.cids[j];
                }
                if (!(y >= 0 && y < a.n && y != p)) y = -1;
            }
            const int cnt = __syncthreads_count(y >= 0);
            if (cs >= c1 || have + cnt > kPruneCap) break;
            if (y >= 0) cid[atomicAdd(&s_n, 1)] = y;
            cs += kPruneChunk;
            __syncthreads();
        }
        const int nn = s_n;
        // similarities to the node
        for (int c = grp; c < nn; c += NG) {
            const int32_t y = cid[c];
            const float v = sim_f32<METRIC, G>(xv, a.xf + (int64_t)y * a.dim, a.dim, g);
            if (g == 0) keys[c] = make_key(v, y, METRIC);
        }
        __syncthreads();
        if (wave == 0 && nn > 0) wave_compact(keys, nn, nn, nullptr);   // nn <= 320: register sort
        __syncthreads();
        // equal keys (the same node) are adjacent
        for (int c = tid; c < nn; c += 256) rm[c] = c > 0 && keys[c] == keys[c - 1];
        __syncthreads();
        if (tid == 0) {
            int u = 0;
            for (int c = 0; c < nn; ++c) u += !rm[c];
            s_unique = u;
            s_kept = 0;
            s_pick = -1;
        }
        __syncthreads();
        if (!a.always && s_unique <= a.R) {
            if (tid == 0)
                for (int c = 0; c < nn; ++c)
                    if (!rm[c]) kept[s_kept++] = (int32_t)(uint32_t)keys[c];
            __syncthreads();
        } else {
            int pos = 0;
            for (;;) {
                if (tid == 0) {
                    int c = pos;
                    while (c < nn && rm[c]) ++c;
                    if (c < nn) {
                        kept[s_kept++] = (int32_t)(uint32_t)keys[c];
                        rm[c] = 1;
                        s_pick = s_kept < a.R ? c : -1;
                    } else {
                        s_pick = -1;
                    }
                }
                __syncthreads();
                const int c = s_pick;
                if (c < 0) break;
                pos = c + 1;
                const int32_t xstar = (int32_t)(uint32_t)keys[c];
                for (int j = tid; j < a.dim; j += 256) xs[j] = a.xf[(int64_t)xstar * a.dim + j];
                __syncthreads();
                for (int e = pos + grp; e < nn; e += NG) {
                    if (rm[e]) continue;   // uniform within the group
                    const int32_t y = (int32_t)(uint32_t)keys[e];
                    const float t = sim_f32<METRIC, G>(xs, a.xf + (int64_t)y * a.dim, a.dim, g);
                    const float sp = key_score(keys[e], METRIC);
                    const float at = a.alpha * t;
                    const bool drop = METRIC == LVQ_L2 ? at <= sp : at >= sp;
                    if (g == 0 && drop) rm[e] = 1;
                }
                __syncthreads();
            }
        }
        __syncthreads();
        if (cs >= c1) break;
    }
    for (int r = tid; r < a.R; r += 256) a.graph[(int64_t)p * a.R + r] = r < s_kept ? kept[r] : -1;
}

// ---- reverse edges ----------------------------------------------------------

constexpr int kScanItems = 2048;   // per block: 256 threads x 8

__global__ __launch_bounds__(256) void k_rev_count(const int32_t *graph, int R, const int32_t *nodes, int64_t m,
                                                    int64_t n, int32_t *cnt)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m * R; e += (int64_t)gridDim.x * 256) {
        const int32_t x = nodes[e / R];
        if (x < 0 || x >= n) continue;
        const int32_t y = graph[(int64_t)x * R + e % R];
        if (y >= 0 && y < n && y != x) atomicAdd(&cnt[y], 1);
    }
}

__global__ __launch_bounds__(256) void k_scan_local(const int32_t *cnt, int64_t n, int64_t *offs, int64_t *bsum)
{
    __shared__ int64_t part[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanItems + tid * 8;
    int64_t v[8], s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = base + k < n ? cnt[base + k] : 0;
        s += v[k];
    }
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {   // inclusive scan of the thread sums
        const int64_t y = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < n) offs[base + k] = run;
        run += v[k];
    }
    if (tid == 255) bsum[blockIdx.x] = part[255];
}

// exclusive scan of bsum[0..nb) in place; bsum[nb] = total
__global__ __launch_bounds__(1024) void k_scan_top(int64_t *bsum, int64_t nb)
{
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + tid;
        const int64_t x = i < nb ? bsum[i] : 0;
        sh[tid] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t y = tid >= o ? sh[tid - o] : 0;
            __syncthreads();
            sh[tid] += y;
            __syncthreads();
        }
        const int64_t c = carry;
        if (i < nb) bsum[i] = c + sh[tid] - x;
        __syncthreads();
        if (tid == 1023) carry = c + sh[1023];
        __syncthreads();
    }
    if (tid == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t *cnt, int64_t n, int64_t *offs, const int64_t *bsum,
                                                     int64_t nb, int32_t *touched, int32_t *ntouched)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        offs[i] += bsum[i / kScanItems];
        if (cnt[i] > 0) touched[atomicAdd(ntouched, 1)] = (int32_t)i;
    }
    if (i == 0) offs[n] = bsum[nb];
}

__global__ __launch_bounds__(256) void k_rev_fill(const int32_t *graph, int R, const int32_t *nodes, int64_t m,
                                                   int64_t n, const int64_t *offs, int32_t *cnt, int32_t *rev)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m * R; e += (int64_t)gridDim.x * 256) {
        const int32_t x = nodes[e / R];
        if (x < 0 || x >= n) continue;
        const int32_t y = graph[(int64_t)x * R + e % R];
        if (y >= 0 && y < n && y != x) {
            const int32_t k = atomicSub(&cnt[y], 1) - 1;   // counts return to zero
            rev[offs[y] + k] = x;
        }
    }
}

// Kept nodes with a deleted out-neighbour: out[0 .. *count).
__global__ __launch_bounds__(256) void k_graph_affected(const int32_t *graph, int R, int64_t n, const uint8_t *deleted,
                                                         int32_t *out, int32_t *count)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        if (deleted[p]) continue;
        bool hit = false;
        for (int r = 0; r < R && !hit; ++r) {
            const int32_t y = graph[p * R + r];
            hit = y >= 0 && y < n && deleted[y];
        }
        if (hit) out[atomicAdd(count, 1)] = (int32_t)p;
    }
}

// Rows of the flagged nodes (deleted != NULL) or of the listed nodes to -1.
__global__ __launch_bounds__(256) void k_graph_clear_rows(int32_t *graph, int R, int64_t n, const uint8_t *deleted,
                                                           const int32_t *nodes, int64_t m)
{
    const int64_t total = (deleted ? n : m) * R;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / R;
        if (deleted) {
            if (deleted[i]) graph[e] = -1;
        } else {
            const int32_t p = nodes[i];
            if (p >= 0 && p < n) graph[(int64_t)p * R + e % R] = -1;
        }
    }
}

unsigned grid_for(int64_t work)
{
    const int64_t b = (work + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

int graph_hash_slots(int window, int degree)
{
    // the nodes that enter a walk's candidate set: about 5.5 W on average and
    // under 8.5 W at most on 10^6-node graphs of out-degree 64; 8 (W + 64)
    // slots keep the table at most two-thirds full
    (void)degree;
    return std::min(kMaxHash, 8 * (window + 64));
}

size_t graph_lds_bytes(int kpos, int window, int degree)
{
    const size_t kq = (size_t)((kpos + 3) & ~3);
    return 2 * kq * 4 + (size_t)(2 * window + 64) * 8 + (size_t)graph_hash_slots(window, degree) * 4;
}

hipError_t launch_graph_search(const GraphLaunch &l, hipStream_t s)
{
    GraphArgs a;
    a.rows = l.rows;
    a.row_bytes = l.row_bytes;
    a.kchunks = l.kchunks;
    a.kpos = l.kpos;
    a.capacity = l.capacity;
    a.qk = l.qk;
    a.qsum = l.qsum;
    a.cm = l.cm;
    a.muk = l.muk;
    a.kmask = l.kmask;
    a.n_means = l.n_means;
    a.metric = l.metric;
    a.nq = l.nq;
    a.graph = l.graph;
    a.degree = l.degree;
    a.entries = l.entries;
    a.n_entries = l.n_entries;
    a.window = l.window;
    a.k = l.k;
    a.epoch = l.epoch;
    a.ids = l.ids;
    a.dist = l.dist;
    a.explored = l.explored;
    a.err = l.err;
    a.xf = l.xf;
    a.dim = l.dim;
    a.qnodes = l.qnodes;
    a.hash_slots = graph_hash_slots(l.window, l.degree);
    if (l.nq <= 0) return hipSuccess;
    if (l.window > kMaxWindow || l.degree > kMaxDegree || l.k > l.window || l.n_entries > kMaxDegree)
        return hipErrorInvalidValue;
    const size_t lds = graph_lds_bytes(l.kpos, l.window, l.degree);
    void (*kern)(GraphArgs) = nullptr;
    const bool ip = l.metric == LVQ_IP;
    if (!l.rows) {
        if (!l.xf || l.kpos != l.dim) return hipErrorInvalidValue;
        kern = ip ? k_graph_search<kFloat, LVQ_IP> : k_graph_search<kFloat, LVQ_L2>;
    } else if (l.bits1 == 8) {
        kern = ip ? k_graph_search<8, LVQ_IP> : k_graph_search<8, LVQ_L2>;
    } else if (l.bits1 == 4) {
        kern = ip ? k_graph_search<4, LVQ_IP> : k_graph_search<4, LVQ_L2>;
    }
    if (!kern) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)l.nq), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_graph_prune(const PruneLaunch &l, hipStream_t s)
{
    if (l.m <= 0) return hipSuccess;
    if (l.R < 1 || l.R > kMaxDegree || l.dim < 1 || l.dim > kGraphMaxDim || l.m > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    const size_t lds = (size_t)2 * l.dim * 4;
    void (*kern)(PruneLaunch) = l.dim <= 128
        ? (l.metric == LVQ_IP ? k_graph_prune<LVQ_IP, 4> : k_graph_prune<LVQ_L2, 4>)
        : (l.metric == LVQ_IP ? k_graph_prune<LVQ_IP, 16> : k_graph_prune<LVQ_L2, 16>);
    hipLaunchKernelGGL(kern, dim3((unsigned)l.m), dim3(256), lds, s, l);
    return hipGetLastError();
}

hipError_t launch_graph_affected(const int32_t *graph, int R, int64_t n, const uint8_t *deleted, int32_t *out,
                                 int32_t *count, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(count, 0, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_graph_affected, dim3(grid_for(n)), dim3(256), 0, s, graph, R, n, deleted, out, count);
    return hipGetLastError();
}

hipError_t launch_graph_clear_rows(int32_t *graph, int R, int64_t n, const uint8_t *deleted, const int32_t *nodes,
                                   int64_t m, hipStream_t s)
{
    const int64_t rows = deleted ? n : m;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_graph_clear_rows, dim3(grid_for(rows * R)), dim3(256), 0, s, graph, R, n, deleted, nodes, m);
    return hipGetLastError();
}

hipError_t launch_reverse_edges(const int32_t *graph, int R, const int32_t *nodes, int64_t m, int64_t n,
                                int32_t *cnt, int64_t *offs, int64_t *scratch, int32_t *rev, int32_t *touched,
                                int32_t *ntouched, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanItems - 1) / kScanItems;
    hipError_t e = launch_fill_i32(ntouched, 0, 1, s);
    if (e != hipSuccess) return e;
    if (m > 0) hipLaunchKernelGGL(k_rev_count, dim3(grid_for(m * R)), dim3(256), 0, s, graph, R, nodes, m, n, cnt);
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, offs, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, scratch, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cnt, n, offs, scratch, nb,
                       touched, ntouched);
    if (m > 0)
        hipLaunchKernelGGL(k_rev_fill, dim3(grid_for(m * R)), dim3(256), 0, s, graph, R, nodes, m, n, offs, cnt, rev);
    return hipGetLastError();
}

}  // namespace lvq
