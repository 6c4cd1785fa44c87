// k_probe.hip -- M-LVQ as a soft inverted index (the Sec. 3.2 remark that a
// query touches only a few centres): per-mean member lists of the occupied
// slots, the routing of each query to its nprobe nearest means, and the
// per-query list offsets over the members of the probed means, which the
// candidate kernel walks range by range.
//
// Routing ranks means by the Def. 1 distance s_m = sum_j (q_j - mu_mj)^2 in
// binary32, summed in dimension order with every operation rounded on its own
// (no contraction: the pragma below and -ffp-contract=off on this file), ties
// to the lower mean id, NaN last: the rule that assigns rows to means.
#pragma clang fp contract(off)

#include <algorithm>

#include "k_common.h"

namespace lvq {
namespace {

// ---- member lists ----------------------------------------------------------
// The mean id of a slot's row is header byte 12.  Each workgroup histograms a
// contiguous chunk of the occupied-slot list in LDS; the fill pass reserves
// one range per (workgroup, mean) with a single global atomic and places its
// slots with LDS atomics (the order inside a mean is unspecified).

__device__ __forceinline__ int slot_mean(const uint8_t *rows, int row_bytes, int32_t slot)
{
    return rows[(int64_t)slot * row_bytes + 12];
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *p, int n)
{
    for (int i = threadIdx.x; i < n; i += 256) p[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_member_count(const int32_t *list, int64_t n, int64_t chunk,
                                                      const uint8_t *rows, int row_bytes, int n_means,
                                                      unsigned long long *counts)
{
    __shared__ unsigned hist[kMaxMeans];
    for (int m = threadIdx.x; m < kMaxMeans; m += 256) hist[m] = 0u;
    __syncthreads();
    const int64_t a = (int64_t)blockIdx.x * chunk, b = min(n, a + chunk);
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
        const int m = slot_mean(rows, row_bytes, list[i]);
        atomicAdd(&hist[m < n_means ? m : 0], 1u);
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n_means; m += 256)
        if (hist[m]) atomicAdd(&counts[m], (unsigned long long)hist[m]);
}

// offsets[m] = sum of counts below m (offsets[n_means] = total); cursor = offsets
__global__ __launch_bounds__(256) void k_member_scan(const unsigned long long *counts, int n_means,
                                                     int64_t *offsets, unsigned long long *cursor)
{
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int m = 0; m < n_means; ++m) {
            offsets[m] = acc;
            cursor[m] = (unsigned long long)acc;
            acc += (int64_t)counts[m];
        }
        offsets[n_means] = acc;
    }
}

__global__ __launch_bounds__(256) void k_member_fill(const int32_t *list, int64_t n, int64_t chunk,
                                                     const uint8_t *rows, int row_bytes, int n_means,
                                                     const int64_t *offsets, unsigned long long *cursor,
                                                     int32_t *members)
{
    __shared__ unsigned hist[kMaxMeans];
    __shared__ unsigned reserved[kMaxMeans];
    __shared__ unsigned long long base[kMaxMeans];
    for (int m = threadIdx.x; m < kMaxMeans; m += 256) hist[m] = 0u;
    __syncthreads();
    const int64_t a = (int64_t)blockIdx.x * chunk, b = min(n, a + chunk);
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
        const int m = slot_mean(rows, row_bytes, list[i]);
        atomicAdd(&hist[m < n_means ? m : 0], 1u);
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n_means; m += 256) {
        base[m] = hist[m] ? atomicAdd(&cursor[m], (unsigned long long)hist[m]) : 0ull;
        reserved[m] = hist[m];
        hist[m] = 0u;
    }
    __syncthreads();
    // A row's mean id can change between the two passes only when a
    // consolidation running beside this build frees its slot (a row deleted
    // before every epoch still being read): such a slot is dropped rather
    // than written past its mean's range, and the entry it leaves keeps the
    // empty marker (-1) the lists were filled with.
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
        const int32_t slot = list[i];
        int m = slot_mean(rows, row_bytes, slot);
        m = m < n_means ? m : 0;
        const unsigned r = atomicAdd(&hist[m], 1u);
        const unsigned long long at = base[m] + r;
        if (at < (unsigned long long)offsets[m + 1] && r < reserved[m]) members[at] = slot;
    }
}

// live members of requested means: one workgroup per requested mean
__global__ __launch_bounds__(256) void k_members_live(const int32_t *req, int nreq, const int64_t *moffs,
                                                      const int32_t *members, const uint8_t *rows, int row_bytes,
                                                      uint32_t epoch, const int64_t *out_offs, int32_t *out,
                                                      unsigned long long *counts)
{
    for (int i = blockIdx.x; i < nreq; i += gridDim.x) {
        const int m = req[i];
        for (int64_t e = moffs[m] + threadIdx.x; e < moffs[m + 1]; e += 256) {
            const int32_t slot = members[e];
            if (slot < 0) continue;
            const uint8_t *row = rows + (int64_t)slot * row_bytes;
            const uint2 ep = *reinterpret_cast<const uint2 *>(row + 16);
            const bool live = (row[13] & 1u) && ep.x <= epoch && epoch < ep.y;
            if (!live) continue;
            const unsigned long long pos = atomicAdd(&counts[i], 1ull);
            if (out_offs) out[out_offs[i] + (int64_t)pos] = slot;
        }
    }
}

// ---- routing ----------------------------------------------------------------
// One wave per query; lane l scores means l, l + 64, ... (E per lane, M <=
// 64 E), each as a sequential sum over the dimensions; the (distance, mean)
// keys are sorted in registers and the first nprobe written out.
template <int E>
__global__ __launch_bounds__(256) void k_route(const float *q, int64_t nq, int dim, const float *means_t,
                                               int means_stride, int n_means, int nprobe, int32_t *probe)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t qi = (int64_t)blockIdx.x * 4 + wave;
    if (qi >= nq) return;
    const float *x = q + (int64_t)__builtin_amdgcn_readfirstlane((int)qi) * dim;
    float s[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s[e] = 0.0f;
    for (int j = 0; j < dim; ++j) {
        const float xj = x[j];
        const float *mr = means_t + (int64_t)j * means_stride;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int m = e * 64 + lane;
            const float mu = m < n_means ? mr[m] : 0.0f;
            float diff = xj - mu;
            float sq = diff * diff;
            s[e] = s[e] + sq;
        }
    }
    uint64_t key[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = e * 64 + lane;
        key[e] = m < n_means ? make_key(s[e], m, LVQ_L2) : kNoKey;
    }
    wave_bitonic_sort<E>(key);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int r = e * 64 + lane;
        if (r < nprobe) probe[qi * nprobe + r] = (int32_t)(uint32_t)key[e];
    }
}

// ---- candidate lists ----------------------------------------------------------
// qtot[q] = members of q's probed means; offsets by one workgroup's scan.
__global__ __launch_bounds__(256) void k_probe_count(const int32_t *probe, int64_t nq, int nprobe,
                                                     const int64_t *moffs, int64_t *qtot)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nq; i += (int64_t)gridDim.x * 256) {
        int64_t t = 0;
        for (int p = 0; p < nprobe; ++p) {
            const int m = probe[i * nprobe + p];
            t += moffs[m + 1] - moffs[m];
        }
        qtot[i] = t;
    }
}

// in-place exclusive scan of v[0..n) into v[0..n], v[n] = total: one
// workgroup of 1024 threads, 1024 entries per round with a running carry
__global__ __launch_bounds__(1024) void k_scan_i64(int64_t *v, int64_t n)
{
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t x = i < n ? v[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {   // Hillis-Steele inclusive scan
            const int64_t y = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        const int64_t c = carry;
        if (i < n) v[i] = c + sh[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry = c + sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) v[n] = carry;
}

}  // namespace

hipError_t launch_members(const int32_t *list, int64_t n, const uint8_t *rows, int row_bytes, int n_means,
                          unsigned long long *counts, unsigned long long *cursor, int64_t *offsets,
                          int32_t *members, hipStream_t s)
{
    if (n_means < 1 || n_means > kMaxMeans) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, counts, n_means);
    const int64_t chunk = 8192;
    const int64_t blocks = (n + chunk - 1) / chunk;
    if (blocks > 0)
        hipLaunchKernelGGL(k_member_count, dim3((unsigned)blocks), dim3(256), 0, s, list, n, chunk, rows, row_bytes,
                           n_means, counts);
    hipLaunchKernelGGL(k_member_scan, dim3(1), dim3(256), 0, s, counts, n_means, offsets, cursor);
    if (blocks > 0)
        hipLaunchKernelGGL(k_member_fill, dim3((unsigned)blocks), dim3(256), 0, s, list, n, chunk, rows, row_bytes,
                           n_means, offsets, cursor, members);
    return hipGetLastError();
}

hipError_t launch_mean_counts(const int32_t *list, int64_t n, const uint8_t *rows, int row_bytes, int n_means,
                              unsigned long long *counts, hipStream_t s)
{
    if (n_means < 1 || n_means > kMaxMeans) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, counts, n_means);
    const int64_t chunk = 8192;
    const int64_t blocks = (n + chunk - 1) / chunk;
    if (blocks > 0)
        hipLaunchKernelGGL(k_member_count, dim3((unsigned)blocks), dim3(256), 0, s, list, n, chunk, rows, row_bytes,
                           n_means, counts);
    return hipGetLastError();
}

hipError_t launch_members_live(const int32_t *req, int nreq, const int64_t *moffs, const int32_t *members,
                               const uint8_t *rows, int row_bytes, uint32_t epoch, const int64_t *out_offs,
                               int32_t *out, unsigned long long *counts, hipStream_t s)
{
    if (nreq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, counts, nreq);
    hipLaunchKernelGGL(k_members_live, dim3((unsigned)std::min(nreq, 4096)), dim3(256), 0, s, req, nreq, moffs,
                       members, rows, row_bytes, epoch, out_offs, out, counts);
    return hipGetLastError();
}

hipError_t launch_route(const float *q, int64_t nq, int dim, const float *means_t, int means_stride, int n_means,
                        int nprobe, int32_t *probe, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nq + 3) / 4)), block(256);
    if (n_means <= 64)
        hipLaunchKernelGGL(k_route<1>, grid, block, 0, s, q, nq, dim, means_t, means_stride, n_means, nprobe, probe);
    else if (n_means <= 128)
        hipLaunchKernelGGL(k_route<2>, grid, block, 0, s, q, nq, dim, means_t, means_stride, n_means, nprobe, probe);
    else if (n_means <= 256)
        hipLaunchKernelGGL(k_route<4>, grid, block, 0, s, q, nq, dim, means_t, means_stride, n_means, nprobe, probe);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_probe_offsets(const int32_t *probe, int64_t nq, int nprobe, const int64_t *moffs, int64_t *qoffs,
                                hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((nq + 255) / 256, 4096);
    if (nq > 0)
        hipLaunchKernelGGL(k_probe_count, dim3((unsigned)blocks), dim3(256), 0, s, probe, nq, nprobe, moffs, qoffs);
    hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, qoffs, nq);
    return hipGetLastError();
}


}  // namespace lvq
