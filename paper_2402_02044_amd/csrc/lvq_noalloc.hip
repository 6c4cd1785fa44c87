// lvq_noalloc.hip -- lvq_distances_noalloc: the candidate-list similarities
// of lvq_distances with their scratch (query tables in kernel order, sums of
// q, per-mean terms, list order, the persistent launch's work counter) in a
// fixed device array instead of the per-stream workspace, so that a call
// allocates no device memory (for callers that cannot: code under HIP graph
// capture, serving loops, harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "lvq_index.h"

namespace {

constexpr size_t kScratchBytes = LVQ_NOALLOC_SCRATCH_BYTES;

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it reaches the array only through the pointer
// hipGetSymbolAddress returns for each device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device, once set up

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace lvq {

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return LVQ_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return LVQ_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LVQ_ERR_DEVICE;
    g_scratch[device] = p;
    return LVQ_OK;
}

}  // namespace lvq

using namespace lvq;

extern "C" int lvq_distances_noalloc(lvq_index *ix, const float *q_dev, int64_t nq, const int64_t *offsets_dev,
                                     const int32_t *ids_dev, int64_t total, int32_t level, float *dist_dev,
                                     int32_t k, int32_t *topk_ids_dev, float *topk_dist_dev, void *stream)
{
    if (!ix || nq < 0 || nq > INT32_MAX) return LVQ_ERR_INVALID_ARG;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return LVQ_ERR_DEVICE;
    if (cur != ix->device) return LVQ_ERR_INVALID_ARG;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (cur >= 0 && cur < kMaxDevices) base = g_scratch[cur];
    }
    if (!base) return LVQ_ERR_DEVICE;   // lvq_create sets it up
    std::lock_guard<std::mutex> lk(ix->mu);
    // carve the scratch: every piece 256-byte aligned
    const size_t n = (size_t)std::max<int64_t>(nq, 1);
    const size_t b_qk = up256(sizeof(float) * n * ix->f.kpos), b_qsum = up256(sizeof(float) * n),
                 b_cm = up256(sizeof(float) * n * ix->n_means), b_order = up256(sizeof(int32_t) * n);
    if (b_qk + b_qsum + b_cm + b_order + 256 > kScratchBytes) return LVQ_ERR_SCRATCH;
    char *p = static_cast<char *>(base);
    DistScratch sc;
    sc.qk = reinterpret_cast<float *>(p);
    sc.qsum = reinterpret_cast<float *>(p + b_qk);
    sc.cm = reinterpret_cast<float *>(p + b_qk + b_qsum);
    sc.order = reinterpret_cast<int32_t *>(p + b_qk + b_qsum + b_cm);
    sc.queue = reinterpret_cast<int32_t *>(p + b_qk + b_qsum + b_cm + b_order);
    hipStream_t s = (hipStream_t)stream;
    int rc = host_begin_call(ix, s);
    if (rc) return rc;
    rc = host_distances(ix, q_dev, nq, offsets_dev, ids_dev, total, level, dist_dev, k, topk_ids_dev, topk_dist_dev,
                        s, -1, ix->epoch, false, nullptr, 0, nullptr, nullptr, &sc);
    if (rc == LVQ_OK && nq > 0) rc = host_note_query(ix, s, ix->epoch, false);
    ix->capturing = false;
    return rc;
}
