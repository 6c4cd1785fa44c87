// k_misc.hip -- per-query precompute (Sec. 3.2), store maintenance (lazy
// deletes and batched consolidation, App. A), top-k merge, the global mean
// (Sec. 2.3) and k-means for the M-LVQ centres (Sec. 3.2).
#include <float.h>

#include <algorithm>

#include "k_common.h"

namespace lvq {
namespace {

__device__ __forceinline__ float wave_sum_f32(float v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---- query precompute: the query in kernel order, sum(q), <q, mu_m> -------
// One 256-lane workgroup per query; wave w reduces the means w, w+4, ...
__global__ __launch_bounds__(256) void k_prep(PrepArgs a)
{
    const int64_t i = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const float *q = reinterpret_cast<const float *>(a.q) + i * a.dim;
    for (int s = tid; s < a.kpos; s += 256) {
        int j = a.kdim[s];
        a.qk[i * a.kpos + s] = j >= 0 ? q[j] : 0.0f;
    }
    if (wave == 0) {
        float s = 0.0f;
        for (int j = lane; j < a.dim; j += 64) s += q[j];
        s = wave_sum_f32(s);
        if (lane == 0) a.qsum[i] = s;
    }
    if (a.metric == LVQ_IP) {
        for (int m = wave; m < a.n_means; m += 4) {
            const float *mu = a.means + (int64_t)m * a.dim;
            float s = 0.0f;
            for (int j = lane; j < a.dim; j += 64) s = fmaf(q[j], mu[j], s);
            s = wave_sum_f32(s);
            if (lane == 0) a.cm[i * a.n_means + m] = s;
        }
    }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// fp32 -> bf16 (upper half, round to nearest even; NaN stays a quiet NaN) or
// fp16 (the hardware conversion, round to nearest even).
__global__ void k_cast16(const float *x, int64_t n, int prec, uint16_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[i];
        uint16_t h;
        if (prec == LVQ_BF16) {
            const uint32_t u = __float_as_uint(v);
            h = (u & 0x7FFFFFFFu) > 0x7F800000u ? (uint16_t)((u >> 16) | 0x40u)
                                                 : (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
        } else {
            const _Float16 f = (_Float16)v;
            h = __builtin_bit_cast(uint16_t, f);
        }
        out[i] = h;
    }
}

// ---- list order for the persistent launch ---------------------------------
// Lists are bucketed by floor(log2(length)), longest bucket first, so the
// work counter hands out long lists before short ones (longest-first
// scheduling).  The order inside a bucket does not affect any result.
__global__ __launch_bounds__(1024) void k_list_order(const int64_t *offsets, int64_t nq, int32_t *order)
{
    __shared__ int hist[64];
    __shared__ int base[64];
    const int tid = threadIdx.x;
    if (tid < 64) hist[tid] = 0;
    __syncthreads();
    for (int64_t i = tid; i < nq; i += 1024) {
        int64_t len = offsets[i + 1] - offsets[i];
        int b = len > 0 ? 63 - __clzll((unsigned long long)len) : 0;
        atomicAdd(&hist[63 - b], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int b = 0; b < 64; ++b) {
            base[b] = acc;
            acc += hist[b];
        }
    }
    __syncthreads();
    for (int64_t i = tid; i < nq; i += 1024) {
        int64_t len = offsets[i + 1] - offsets[i];
        int b = len > 0 ? 63 - __clzll((unsigned long long)len) : 0;
        int pos = atomicAdd(&base[63 - b], 1);
        order[pos] = (int32_t)i;
    }
}

// ---- merge of per-part top-k keys -----------------------------------------
// One wavefront per query selects the k smallest of n_parts * k keys.
__global__ __launch_bounds__(64) void k_topk_merge(const uint64_t *keys, int64_t nq, int n_parts, int k,
                                                   int metric, int32_t *ids, float *dist)
{
    extern __shared__ uint64_t mk[];
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    const int n = n_parts * k;
    for (int t = lane; t < n; t += 64) mk[t] = keys[i * n + t];
    uint64_t *out = mk + n;
    int got = wave_select_smallest(mk, n, k, out);
    for (int r = lane; r < k; r += 64) {
        int32_t sid = -1;
        float sv = metric == LVQ_L2 ? __uint_as_float(0x7F800000u) : __uint_as_float(0xFF800000u);
        if (r < got) {
            sid = (int32_t)(uint32_t)out[r];
            sv = key_score(out[r], metric);
        }
        ids[i * k + r] = sid;
        dist[i * k + r] = sv;
    }
}

// ---- store maintenance ----------------------------------------------------
__global__ void k_delete(StoreArgs a, const int32_t *slots, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = slots[i];
        if (s < 0 || (int64_t)s >= a.capacity) {
            atomicOr(a.err, kErrBadSlot);
            continue;
        }
        uint8_t *row = a.rows + (int64_t)s * a.row_bytes;
        uint32_t flags = row[13];
        uint32_t *del = reinterpret_cast<uint32_t *>(row + 20);
        if (!(flags & 1u) || *del != kLiveEpoch) {
            atomicOr(a.err, kErrBadSlot);
            continue;
        }
        *del = a.epoch;
    }
}

// Consolidation, pass 1: count reclaimable slots per 1024-slot block.
__device__ __forceinline__ bool reclaimable(const uint8_t *row, uint32_t safe_epoch)
{
    uint32_t flags = row[13];
    uint32_t del = *reinterpret_cast<const uint32_t *>(row + 20);
    return (flags & 1u) && del != kLiveEpoch && del <= safe_epoch;
}

__global__ __launch_bounds__(1024) void k_consolidate_count(StoreArgs a, uint32_t safe_epoch, int32_t *counts)
{
    __shared__ int wsum[16];
    const int64_t s = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int r = s < a.capacity && reclaimable(a.rows + s * a.row_bytes, safe_epoch);
    r = __popcll(__ballot(r));
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        counts[blockIdx.x] = t;
    }
}

// Exclusive prefix sums of counts[0..nb) in place, in ascending block order
// or (descending) from the last block down; returns the total.  One
// workgroup of 1024 threads: each thread sums a run of blocks, the run
// totals are scanned across the workgroup, then each thread writes its run.
__device__ int64_t block_exclusive_scan(int32_t *counts, int nb, bool descending)
{
    __shared__ int64_t wtot[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per, b1 = min(nb, b0 + per);
    auto at = [&](int i) -> int32_t & { return counts[descending ? nb - 1 - i : i]; };
    int64_t run = 0;
    for (int i = b0; i < b1; ++i) run += at(i);
    // inclusive scan of run totals within the wave, then across waves
    int64_t inc = run;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) before += wtot[w];
        total += wtot[w];
    }
    int64_t acc = before + inc - run;
    for (int i = b0; i < b1; ++i) {
        const int32_t c = at(i);
        at(i) = (int32_t)acc;
        acc += c;
    }
    return total;
}

// pass 2: exclusive offsets in descending block order (one workgroup)
__global__ __launch_bounds__(1024) void k_consolidate_scan(int32_t *counts, int nblocks, int64_t free_top,
                                                           int64_t *new_top)
{
    const int64_t total = block_exclusive_scan(counts, nblocks, true);
    if (threadIdx.x == 0) *new_top = free_top + total;
}

// pass 3: push reclaimable slots (descending slot order) and clear their rows
__global__ __launch_bounds__(1024) void k_consolidate_push(StoreArgs a, uint32_t safe_epoch,
                                                           const int32_t *offs, int32_t *stack,
                                                           int64_t free_top)
{
    __shared__ int wsum[16];
    const int64_t s = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool r = s < a.capacity && reclaimable(a.rows + s * a.row_bytes, safe_epoch);
    unsigned long long m = __ballot(r);
    // slots above s inside this wave
    int above = __popcll(lane == 63 ? 0ull : (m >> (lane + 1)));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int waves_above = 0;
    for (int w = wave + 1; w < 16; ++w) waves_above += wsum[w];
    if (r) {
        int64_t pos = free_top + offs[blockIdx.x] + waves_above + above;
        stack[pos] = (int32_t)s;
        uint32_t *h = reinterpret_cast<uint32_t *>(a.rows + s * a.row_bytes);
        for (int w = 0; w < 8; ++w) h[w] = 0u;
    }
}

// Occupied-slot list, pass 1: occupied slots per 1024-slot block.
__global__ __launch_bounds__(1024) void k_list_count(StoreArgs a, int32_t *counts)
{
    __shared__ int wsum[16];
    const int64_t s = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int r = s < a.capacity && (a.rows[s * a.row_bytes + 13] & 1u);
    r = __popcll(__ballot(r));
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        counts[blockIdx.x] = t;
    }
}

// pass 2: exclusive offsets in ascending block order (one workgroup)
__global__ __launch_bounds__(1024) void k_list_scan(int32_t *counts, int nblocks, int64_t *len)
{
    const int64_t total = block_exclusive_scan(counts, nblocks, false);
    if (threadIdx.x == 0) *len = total;
}

// pass 3: write the occupied slots in ascending order
__global__ __launch_bounds__(1024) void k_list_write(StoreArgs a, const int32_t *offs, int32_t *list)
{
    __shared__ int wsum[16];
    const int64_t s = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool r = s < a.capacity && (a.rows[s * a.row_bytes + 13] & 1u);
    const unsigned long long m = __ballot(r);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int waves_below = 0;
    for (int w = 0; w < wave; ++w) waves_below += wsum[w];
    if (r) list[offs[blockIdx.x] + waves_below + below] = (int32_t)s;
}

__global__ void k_gather_rows(StoreArgs a, const int32_t *slots, int64_t n, uint8_t *rows_out,
                              uint8_t *resid_out)
{
    const int64_t i = blockIdx.x;
    int32_t s = slots[i];
    if (s < 0 || (int64_t)s >= a.capacity) {
        if (threadIdx.x == 0) atomicOr(a.err, kErrBadSlot);
        return;
    }
    const uint32_t *src = reinterpret_cast<const uint32_t *>(a.rows + (int64_t)s * a.row_bytes);
    uint32_t *dst = reinterpret_cast<uint32_t *>(rows_out + i * a.row_bytes);
    for (int w = threadIdx.x; w < a.row_bytes / 4; w += blockDim.x) dst[w] = src[w];
    if (resid_out && a.resid) {
        src = reinterpret_cast<const uint32_t *>(a.resid + (int64_t)s * a.resid_bytes);
        dst = reinterpret_cast<uint32_t *>(resid_out + i * a.resid_bytes);
        for (int w = threadIdx.x; w < a.resid_bytes / 4; w += blockDim.x) dst[w] = src[w];
    }
}

// ---- global mean: binary64 column sums over row chunks, then a fixed-order
// sum of the chunk partials --------------------------------------------------
constexpr int kMeanRows = 4096;

__global__ __launch_bounds__(256) void k_mean_partial(const float *x, int64_t n, int dim, double *part)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dim) return;
    const int64_t r0 = (int64_t)blockIdx.y * kMeanRows;
    const int64_t r1 = r0 + kMeanRows < n ? r0 + kMeanRows : n;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)x[r * dim + j];
    part[(int64_t)blockIdx.y * dim + j] = s;
}

__global__ __launch_bounds__(256) void k_mean_final(const double *part, int nchunks, int64_t n, int dim, float *out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dim) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * dim + j];
    out[j] = (float)(s / (double)n);
}

// ---- k-means ----------------------------------------------------------------
__global__ __launch_bounds__(256) void k_km_assign(const float *x, int64_t n, int dim, const float *c, int k,
                                                   int32_t *assign)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float *xi = x + i * dim;
    float best = FLT_MAX;
    int bm = 0;
    for (int m = 0; m < k; ++m) {
        const float *cm = c + (int64_t)m * dim;
        float s = 0.0f;
        for (int j = 0; j < dim; ++j) {
            float e = xi[j] - cm[j];
            s = fmaf(e, e, s);
        }
        if (s < best) {
            best = s;
            bm = m;
        }
    }
    assign[i] = bm;
}

// one workgroup per (centre, 256-dim block): binary64 sums in row order
__global__ __launch_bounds__(256) void k_km_update(const float *x, int64_t n, int dim, const int32_t *assign,
                                                   int k, float *c)
{
    const int m = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dim) return;
    double s = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        if (assign[i] == m) {
            s += (double)x[i * dim + j];
            ++cnt;
        }
    if (cnt > 0) c[(int64_t)m * dim + j] = (float)(s / (double)cnt);
}

// ---- bandwidth probes (measurement): the loads of an access pattern with
// no arithmetic; each lane folds the words it read into one, and each block
// XORs its lanes' words into *sink, so no load can be dropped and the result
// is the XOR of every 32-bit word read.
__device__ __forceinline__ void block_xor_into(uint32_t acc, uint32_t *sink)
{
    __shared__ uint32_t part[4];
    for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicXor(sink, part[0] ^ part[1] ^ part[2] ^ part[3]);
}

__global__ __launch_bounds__(256) void k_bw_stream(const uint4 *src, int64_t n, uint32_t *sink)
{
    // workgroup b streams the contiguous range [b * chunk, (b + 1) * chunk),
    // eight coalesced 16-byte loads in flight per lane
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = min(n, lo + chunk);
    uint32_t acc = 0;
    int64_t i = lo + threadIdx.x;
    for (; i + 7 * 256 < hi; i += 8 * 256) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[i + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < hi; i += 256) {
        const uint4 v = src[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    block_xor_into(acc, sink);
}

// GL lanes per listed slot (GL in {4, 8, 16}, the smallest covering the
// pieces): the header and first-level code bytes the similarity kernels read
// (code16 pieces of 16 bytes) and, when resid is set, the residual row
// (res16 pieces).
template <int GL>
__global__ __launch_bounds__(256) void k_bw_gather(const uint8_t *rows, int row_bytes, int code16, const uint8_t *resid,
                                                    int resid_bytes, int res16, const int32_t *ids, int64_t n,
                                                    int64_t capacity, uint32_t *sink)
{
    const int g = threadIdx.x % GL;
    const int64_t stride = (int64_t)gridDim.x * (256 / GL);
    uint32_t acc = 0;
    for (int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / GL; i < n; i += stride) {
        const int32_t s = ids[i];
        if (s < 0 || s >= capacity) continue;
        const uint4 *r = reinterpret_cast<const uint4 *>(rows + (int64_t)s * row_bytes);
        for (int p = g; p < code16; p += GL) {
            const uint4 v = r[p];
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
        if (resid) {
            const uint4 *q = reinterpret_cast<const uint4 *>(resid + (int64_t)s * resid_bytes);
            for (int p = g; p < res16; p += GL) {
                const uint4 v = q[p];
                acc ^= v.x ^ v.y ^ v.z ^ v.w;
            }
        }
    }
    block_xor_into(acc, sink);
}

}  // namespace

hipError_t launch_prep(const PrepArgs &a, hipStream_t s)
{
    if (a.nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)a.nq), dim3(256), 0, s, a);
    return hipGetLastError();
}

static unsigned fill_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_bw_stream(const void *src, int64_t n16, uint32_t *sink, hipStream_t s)
{
    hipError_t e = launch_fill_u32(sink, 0u, 1, s);
    if (e != hipSuccess || n16 <= 0) return e;
    hipLaunchKernelGGL(k_bw_stream, dim3(8192), dim3(256), 0, s, reinterpret_cast<const uint4 *>(src), n16, sink);
    return hipGetLastError();
}

hipError_t launch_bw_gather(const uint8_t *rows, int row_bytes, int code16, const uint8_t *resid, int resid_bytes,
                            int res16, const int32_t *ids, int64_t n, int64_t capacity, uint32_t *sink, hipStream_t s)
{
    hipError_t e = launch_fill_u32(sink, 0u, 1, s);
    if (e != hipSuccess || n <= 0) return e;
    const int pieces = std::max(code16, resid ? res16 : 0);
    const int gl = pieces > 8 ? 16 : (pieces > 4 ? 8 : 4);
    const int64_t blocks = std::min<int64_t>((n * gl + 255) / 256, 16384);
    auto kern = gl == 16 ? k_bw_gather<16> : (gl == 8 ? k_bw_gather<8> : k_bw_gather<4>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, rows, row_bytes, code16, resid, resid_bytes,
                       res16, ids, n, capacity, sink);
    return hipGetLastError();
}

hipError_t launch_cast16(const float *x, int64_t n, int prec, void *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast16, dim3(fill_blocks(n)), dim3(256), 0, s, x, n, prec, reinterpret_cast<uint16_t *>(out));
    return hipGetLastError();
}

hipError_t launch_list_order(const int64_t *offsets, int64_t nq, int32_t *order, int32_t *, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_list_order, dim3(1), dim3(1024), 0, s, offsets, nq, order);
    return hipGetLastError();
}

hipError_t launch_topk_merge(const uint64_t *keys, int64_t nq, int n_parts, int k, int metric, int32_t *ids,
                             float *dist, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    size_t lds = ((size_t)n_parts * k + k) * sizeof(uint64_t);
    hipLaunchKernelGGL(k_topk_merge, dim3((unsigned)nq), dim3(64), lds, s, keys, nq, n_parts, k, metric, ids,
                       dist);
    return hipGetLastError();
}

hipError_t launch_delete(const StoreArgs &a, const int32_t *slots, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_delete, dim3(fill_blocks(n)), dim3(256), 0, s, a, slots, n);
    return hipGetLastError();
}

hipError_t launch_consolidate(const StoreArgs &a, uint32_t safe_epoch, int32_t *free_stack, int64_t free_top,
                              int32_t *block_counts, int64_t *new_top, hipStream_t s)
{
    const int nb = (int)((a.capacity + 1023) / 1024);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_consolidate_count, dim3(nb), dim3(1024), 0, s, a, safe_epoch, block_counts);
    hipLaunchKernelGGL(k_consolidate_scan, dim3(1), dim3(1024), 0, s, block_counts, nb, free_top, new_top);
    hipLaunchKernelGGL(k_consolidate_push, dim3(nb), dim3(1024), 0, s, a, safe_epoch, block_counts, free_stack,
                       free_top);
    return hipGetLastError();
}

hipError_t launch_build_list(const StoreArgs &a, int32_t *list, int32_t *block_counts, int64_t *len, hipStream_t s)
{
    const int nb = (int)((a.capacity + 1023) / 1024);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_list_count, dim3(nb), dim3(1024), 0, s, a, block_counts);
    hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, s, block_counts, nb, len);
    hipLaunchKernelGGL(k_list_write, dim3(nb), dim3(1024), 0, s, a, block_counts, list);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const StoreArgs &a, const int32_t *slots, int64_t n, uint8_t *rows_out,
                              uint8_t *resid_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)n), dim3(64), 0, s, a, slots, n, rows_out, resid_out);
    return hipGetLastError();
}

hipError_t launch_mean(const float *x, int64_t n, int dim, float *out, double *scratch, hipStream_t s)
{
    const int nchunks = (int)((n + kMeanRows - 1) / kMeanRows);
    dim3 g1((dim + 255) / 256, nchunks);
    hipLaunchKernelGGL(k_mean_partial, g1, dim3(256), 0, s, x, n, dim, scratch);
    hipLaunchKernelGGL(k_mean_final, dim3((dim + 255) / 256), dim3(256), 0, s, scratch, nchunks, n, dim, out);
    return hipGetLastError();
}

hipError_t launch_kmeans_assign(const float *x, int64_t n, int dim, const float *c, int k, int32_t *assign,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_km_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, dim, c, k, assign);
    return hipGetLastError();
}

hipError_t launch_kmeans_update(const float *x, int64_t n, int dim, const int32_t *assign, int k, float *c,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_km_update, dim3((dim + 255) / 256, k), dim3(256), 0, s, x, n, dim, assign, k, c);
    return hipGetLastError();
}

}  // namespace lvq

#include "k_cand_inst.h"
#include "k_scan_impl.h"

namespace lvq {

int num_tile_shapes() { return kNumCandShapes; }
TileShape tile_shape(int i) { return kCandShapes[i]; }
size_t cand_lds_bytes(int kpos, int ntab, bool mask, int n_means_ip, int k, int cw, bool map, int nseg)
{
    return cand_lds_bytes_impl(kpos, ntab, mask, n_means_ip, k, cw, map, nseg);
}
size_t scan_lds_bytes(int kpos, int n_means_ip, int k, int capq)
{
    return scan_lds_bytes_impl(kpos, n_means_ip, k, capq);
}
int scan_capq(int kpos, int n_means_ip, int k, int rows_per_round, size_t lds_max)
{
    return scan_capq_impl(kpos, n_means_ip, k, rows_per_round, lds_max);
}
int scan_rows_per_round(int g) { return 256 / g * kScanR; }

}  // namespace lvq
