// k_graph.hip -- greedy graph search (Alg. 1) over the stored LVQ rows with
// first-level similarities (Sec. 2.3: the first level traverses, both
// levels re-rank).
//
// One workgroup per query.  LDS holds the query in kernel order (and the L2
// padding mask), the candidate set -- at most W keys, best first -- and a
// hash set of every node proposed so far.  A key is (score order << 32) |
// (slot << 1) | explored: the explored flag travels with the key through the
// sorts without changing the (score, slot) order of distinct nodes.  Each
// step explores the best unexplored key: its out-neighbours not seen before
// are scored (16 lanes per neighbour) and merged, and the set is cut to the
// W best.  Deleted rows are traversed; the result is the k best live ones.
#include "k_common.h"

namespace lvq {
namespace {

constexpr int kHash = 16384;      // hash slots per query (int32 slot or -1)
constexpr int kMaxDegree = 64;
constexpr int kMaxWindow = 256;

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
};

__device__ __forceinline__ uint32_t hash_slot(int32_t s)
{
    return ((uint32_t)s * 2654435761u) >> (32 - 14);   // 14 bits: kHash slots
}

// Insert s into the hash set: 1 if it was not there, 0 if it was, -1 if the
// set is full.
__device__ __forceinline__ int hash_insert(int32_t *h, int32_t s)
{
    uint32_t i = hash_slot(s);
    for (int probe = 0; probe < kHash; ++probe) {
        const int32_t old = atomicCAS(&h[i], -1, s);
        if (old == -1) return 1;
        if (old == s) return 0;
        i = (i + 1) & (kHash - 1);
    }
    return -1;
}

// First-level similarity of row `slot` to the query, by the 16 lanes of a
// group (g = 0..15); every lane of the group returns the value.
template <int B1, int METRIC>
__device__ __forceinline__ float score16(const GraphArgs &a, const float *qt, const float *mk, int32_t slot, int g)
{
    const uint8_t *row = a.rows + (int64_t)slot * a.row_bytes;
    const float4 hdr = *reinterpret_cast<const float4 *>(row);
    const uint32_t *codes = reinterpret_cast<const uint32_t *>(row + kHeaderBytes);
    const int nwords = a.kchunks * 4;
    const int mid = min((int)(__float_as_uint(hdr.w) & 0xFFu), a.n_means - 1);
    const float l = hdr.x, dl = hdr.y;
    constexpr int PER = B1 == 8 ? 4 : 8;   // positions per 32-bit word
    float s_lo = 0.0f, s_hi = 0.0f;
    for (int w = g; w < nwords; w += 16) {
        const uint32_t c = codes[w];
        const int p0 = w * PER;
        float cv[PER];
        if constexpr (B1 == 8) {
            cv[0] = ub<0>(c); cv[1] = ub<1>(c); cv[2] = ub<2>(c); cv[3] = ub<3>(c);
        } else {
            // kernel order of a 4-bit word: fields 0,2,4,6 (low nibbles), then 1,3,5,7
            const uint32_t lo = c & 0x0F0F0F0Fu, hi = (c >> 4) & 0x0F0F0F0Fu;
            cv[0] = ub<0>(lo); cv[1] = ub<1>(lo); cv[2] = ub<2>(lo); cv[3] = ub<3>(lo);
            cv[4] = ub<0>(hi); cv[5] = ub<1>(hi); cv[6] = ub<2>(hi); cv[7] = ub<3>(hi);
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int p = p0 + j;
            if constexpr (METRIC == LVQ_IP) {
                s_lo = fmaf(qt[p], cv[j], s_lo);
            } else {
                const float qv = qt[p] - a.muk[(int64_t)mid * a.kpos + p];   // q - mu, kernel order
                float t = qv - fmaf(dl, cv[j], l);
                t *= mk[p];
                s_hi = fmaf(t, t, s_hi);
            }
        }
    }
    if constexpr (METRIC == LVQ_IP) {
        const float dot = group_sum<16>(s_lo);
        return fmaf(dl, dot, fmaf(l, a.qsum[0], a.cm[mid]));   // qsum / cm already offset to the query
    } else {
        return group_sum<16>(s_hi);
    }
}

template <int B1, int METRIC>
__global__ __launch_bounds__(256) void k_graph_search(GraphArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int grp = tid >> 4, g = tid & 15;   // 16 groups of 16 lanes
    const int64_t qi = blockIdx.x;
    if (qi >= a.nq) return;
    const int W = a.window;
    float *qt = reinterpret_cast<float *>(smem);                       // kpos
    float *mk = qt + a.kpos;                                           // kpos
    uint64_t *qkey = reinterpret_cast<uint64_t *>(mk + a.kpos);        // W + kMaxDegree (+ scratch)
    uint64_t *scratch = qkey + W + kMaxDegree;                         // kMaxWindow (selection scratch)
    int32_t *hset = reinterpret_cast<int32_t *>(scratch + kMaxWindow); // kHash
    __shared__ int32_t s_new[kMaxDegree];
    __shared__ int s_nnew, s_qn, s_pick, s_stop, s_explored, s_scored;

    for (int p = tid; p < a.kpos; p += 256) {
        qt[p] = a.qk[qi * a.kpos + p];
        mk[p] = METRIC == LVQ_L2 ? a.kmask[p] : 1.0f;
    }
    for (int i = tid; i < kHash; i += 256) hset[i] = -1;
    if (tid == 0) {
        s_nnew = 0;
        s_stop = 0;
        s_explored = 0;
        s_scored = 0;
    }
    __syncthreads();
    GraphArgs b = a;
    b.qsum = a.qsum + qi;
    b.cm = a.cm + qi * a.n_means;

    // entry nodes: deduplicated through the hash set, scored, sorted
    for (int i = tid; i < a.n_entries; i += 256) {
        const int32_t s = a.entries[i];
        if (s >= 0 && s < a.capacity && hash_insert(hset, s) == 1) s_new[atomicAdd(&s_nnew, 1)] = s;
    }
    __syncthreads();
    int qn = 0;
    auto score_new = [&](int base_n) {
        const int nn = s_nnew;
        for (int c = grp; c < nn; c += 16) {
            const int32_t s = s_new[c];
            const float v = score16<B1, METRIC>(b, qt, mk, s, g);
            if (g == 0) qkey[base_n + c] = (make_key(v, 0, METRIC) & 0xFFFFFFFF00000000ull) | ((uint64_t)(uint32_t)s << 1);
        }
    };
    score_new(0);
    __syncthreads();
    if (wave == 0) {
        const int n0 = s_nnew;
        if (lane == 0) s_scored = n0;
        const int got = wave_compact(qkey, n0, min(W, max(n0, 1)), scratch);
        if (lane == 0) s_qn = min(got, W);
    }
    __syncthreads();
    qn = s_qn;

    for (;;) {
        // the best unexplored key (the set is sorted)
        if (tid == 0) s_pick = 1 << 30;
        __syncthreads();
        for (int i = tid; i < qn; i += 256)
            if (!(qkey[i] & 1ull)) atomicMin(&s_pick, i);
        __syncthreads();
        const int pick = s_pick;
        if (pick >= qn || s_stop) break;
        const int32_t x = (int32_t)((uint32_t)qkey[pick] >> 1);
        __syncthreads();
        if (tid == 0) {
            qkey[pick] |= 1ull;
            s_nnew = 0;
            ++s_explored;
        }
        __syncthreads();
        // out-neighbours not seen before
        if (tid < a.degree) {
            const int32_t y = a.graph[(int64_t)x * a.degree + tid];
            if (y >= 0 && y < a.capacity) {
                const int r = hash_insert(hset, y);
                if (r == 1) s_new[atomicAdd(&s_nnew, 1)] = y;
                if (r < 0) {
                    s_stop = 1;
                    atomicOr(a.err, kErrOverflow);
                }
            }
        }
        __syncthreads();
        if (s_nnew == 0) continue;
        score_new(qn);
        __syncthreads();
        if (wave == 0) {
            const int n = qn + s_nnew;
            if (lane == 0) s_scored += s_nnew;
            const int got = wave_compact(qkey, n, W, scratch);
            if (lane == 0) s_qn = got;
        }
        __syncthreads();
        qn = s_qn;
    }

    // the k best live keys, in order
    if (wave == 0) {
        int out = 0;
        for (int base = 0; base < qn && out < a.k; base += 64) {
            const int i = base + lane;
            bool live = false;
            uint64_t key = kNoKey;
            if (i < qn) {
                key = qkey[i];
                const int32_t s = (int32_t)((uint32_t)key >> 1);
                const uint8_t *row = a.rows + (int64_t)s * a.row_bytes;
                const uint2 ep = *reinterpret_cast<const uint2 *>(row + 16);
                live = (row[13] & 1u) && ep.x <= a.epoch && a.epoch < ep.y;
            }
            const uint64_t m = __ballot(live);
            const int pos = out + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (live && pos < a.k) {
                a.ids[qi * a.k + pos] = (int32_t)((uint32_t)key >> 1);
                a.dist[qi * a.k + pos] = key_score(key, METRIC);
            }
            out += __popcll(m);
        }
        for (int i = max(out, 0) + lane; i < a.k; i += 64) {
            a.ids[qi * a.k + i] = -1;
            a.dist[qi * a.k + i] = METRIC == LVQ_L2 ? __uint_as_float(0x7F800000u) : __uint_as_float(0xFF800000u);
        }
        if (lane == 0 && a.explored) {
            a.explored[2 * qi] = s_explored;
            a.explored[2 * qi + 1] = s_scored;
        }
    }
}

}  // namespace

size_t graph_lds_bytes(int kpos, int window)
{
    return (size_t)2 * kpos * 4 + (size_t)(window + kMaxDegree + kMaxWindow) * 8 + (size_t)kHash * 4;
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
    if (l.nq <= 0) return hipSuccess;
    const size_t lds = graph_lds_bytes(l.kpos, l.window);
    void (*kern)(GraphArgs) = nullptr;
    if (l.bits1 == 8) kern = l.metric == LVQ_IP ? k_graph_search<8, LVQ_IP> : k_graph_search<8, LVQ_L2>;
    else if (l.bits1 == 4) kern = l.metric == LVQ_IP ? k_graph_search<4, LVQ_IP> : k_graph_search<4, LVQ_L2>;
    if (!kern) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)l.nq), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace lvq
