// lvq_serve.hip -- request server of the C ABI (lvq_server_* in lvq.h):
// continuous batching of k-NN query batches (the problem of Sec. 2.1) over
// an index that keeps changing through inserts and deletes (Sec. 2.2).
//
// Host threads:
//   submit (caller)  copies a batch's queries and queues the batch;
//   dispatcher       admits queued batches in arrival order once a stream
//                    slot is free and the device pool can hold the batch's
//                    buffers, then enqueues upload (through the slot's
//                    pinned staging buffer), first-level exhaustive
//                    top-k', two-level re-rank of those candidates and the
//                    download of the results on the slot's stream;
//   completer        polls the slots' completion events, stamps completion
//                    times, hands results to waiters and frees slot and pool
//                    space.
// Every computation runs in the library's kernels; this file schedules.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lvq_index.h"

using namespace lvq;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over one device region, with coalescing frees.
class Pool {
public:
    void reset(size_t bytes)
    {
        free_.clear();
        if (bytes) free_[0] = bytes;
        size_ = bytes;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;   // offset -> length
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Request {
    int64_t ticket = 0;
    int32_t nq = 0;
    std::vector<float> q;        // host copy of the queries until admission
    size_t off = 0, bytes = 0;   // pool region while admitted
    int slot = -1;
    uint32_t epoch = 0;
    int status = LVQ_OK;
    bool done = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<int32_t> ids;
    std::vector<float> dist;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float *q_host = nullptr;       // pinned query staging (max_batch x dim)
    int32_t *ids_host = nullptr;   // pinned result staging
    float *dist_host = nullptr;
    std::shared_ptr<Request> req;  // batch in flight (null: free)
    bool launched = false;         // `done` recorded; the completer may poll it
};

}  // namespace

struct lvq_server {
    lvq_index *ix = nullptr;
    lvq_server_config cfg{};
    int dim = 0;
    bool rerank = false;
    DevBuf pool_mem, offsets;
    Pool pool;
    std::vector<Slot> slots;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<int64_t, std::shared_ptr<Request>> requests;
    int64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0;
    int32_t in_flight = 0, peak_in_flight = 0, peak_queue = 0;
    std::mutex mu;
    std::condition_variable admit_cv, done_cv, work_cv;
    bool stop = false;
    std::thread dispatcher, completer;
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // device bytes of one admitted batch: fp32 queries, their 16-bit copy for
    // the matrix-core scan, first-level candidates, re-ranked results
    size_t batch_bytes(int64_t nq) const
    {
        size_t b = align_up(sizeof(float) * (size_t)nq * dim);
        if (cfg.precision != LVQ_FP32) b += align_up(2 * (size_t)nq * dim);
        b += 2 * align_up(4 * (size_t)nq * cfg.k_first);
        if (rerank) b += 2 * align_up(4 * (size_t)nq * cfg.k);
        return b;
    }

    int free_slot() const
    {
        for (size_t i = 0; i < slots.size(); ++i)
            if (!slots[i].req) return (int)i;
        return -1;
    }

    void finish(Slot &sl, int status);
    void run_dispatcher();
    void run_completer();
    int launch(Slot &sl, Request &r);
};

// Enqueue one admitted batch on its slot's stream.
int lvq_server::launch(Slot &sl, Request &r)
{
    hipStream_t s = sl.stream;
    const int64_t nq = r.nq;
    char *base = static_cast<char *>(pool_mem.p) + r.off;
    float *q32 = reinterpret_cast<float *>(base);
    base += align_up(sizeof(float) * (size_t)nq * dim);
    void *q16 = nullptr;
    if (cfg.precision != LVQ_FP32) {
        q16 = base;
        base += align_up(2 * (size_t)nq * dim);
    }
    int32_t *cand_ids = reinterpret_cast<int32_t *>(base);
    base += align_up(4 * (size_t)nq * cfg.k_first);
    float *cand_dist = reinterpret_cast<float *>(base);
    base += align_up(4 * (size_t)nq * cfg.k_first);
    int32_t *out_ids = cand_ids;
    float *out_dist = cand_dist;
    if (rerank) {
        out_ids = reinterpret_cast<int32_t *>(base);
        base += align_up(4 * (size_t)nq * cfg.k);
        out_dist = reinterpret_cast<float *>(base);
    }
    // the slot's staging buffer is free: its previous batch has completed
    std::memcpy(sl.q_host, r.q.data(), sizeof(float) * (size_t)nq * dim);
    std::vector<float>().swap(r.q);
    if (hipMemcpyAsync(q32, sl.q_host, sizeof(float) * (size_t)nq * dim, hipMemcpyHostToDevice, s) != hipSuccess)
        return LVQ_ERR_DEVICE;
    if (q16 && launch_cast16(q32, nq * dim, cfg.precision, q16, s) != hipSuccess) return LVQ_ERR_DEVICE;
    int rc;
    {
        std::lock_guard<std::mutex> lk(ix->mu);
        if ((rc = host_begin_call(ix, s))) return rc;
        r.epoch = ix->epoch;   // the batch reads the store as of its admission
        rc = host_topk(ix, q16 ? q16 : (const void *)q32, cfg.precision, nq, cfg.k_first, cfg.scan_level,
                       cand_ids, cand_dist, s, r.epoch);
        if (rc == LVQ_OK && rerank)
            rc = host_distances(ix, q32, nq, static_cast<const int64_t *>(offsets.p), cand_ids,
                                nq * (int64_t)cfg.k_first, cfg.rerank_level, nullptr, cfg.k, out_ids, out_dist, s,
                                -1, r.epoch, true);
        if (rc == LVQ_OK) rc = host_note_query(ix, s, r.epoch);
        ix->capturing = false;
    }
    if (rc) return rc;
    if (hipMemcpyAsync(sl.ids_host, out_ids, 4 * (size_t)nq * cfg.k, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(sl.dist_host, out_dist, 4 * (size_t)nq * cfg.k, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(sl.done, s) != hipSuccess)
        return LVQ_ERR_DEVICE;
    return LVQ_OK;
}

// Under `mu`: hand the slot's batch its results and free slot and pool space.
void lvq_server::finish(Slot &sl, int status)
{
    Request &r = *sl.req;
    r.t_done = now();
    r.status = status;
    if (status == LVQ_OK) {
        r.ids.assign(sl.ids_host, sl.ids_host + (size_t)r.nq * cfg.k);
        r.dist.assign(sl.dist_host, sl.dist_host + (size_t)r.nq * cfg.k);
    }
    r.done = true;
    pool.release(r.off, r.bytes);
    sl.req.reset();
    sl.launched = false;
    --in_flight;
    ++completed;
    done_cv.notify_all();
    admit_cv.notify_all();
}

void lvq_server::run_dispatcher()
{
    (void)hipSetDevice(ix->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        int si = -1;
        size_t off = 0;
        admit_cv.wait(lk, [&] {
            if (queue.empty()) return stop;
            si = free_slot();
            return si >= 0 && pool.alloc(queue.front()->bytes, &off);
        });
        if (queue.empty()) break;   // stopping and nothing queued
        std::shared_ptr<Request> r = queue.front();
        queue.pop_front();
        Slot &sl = slots[si];
        r->off = off;
        r->slot = si;
        r->t_admit = now();
        sl.req = r;
        sl.launched = false;
        ++in_flight;
        peak_in_flight = std::max(peak_in_flight, in_flight);
        lk.unlock();
        const int rc = launch(sl, *r);
        lk.lock();
        if (rc != LVQ_OK) {
            // nothing may still write the batch's buffers: wait for the stream
            lk.unlock();
            (void)hipStreamSynchronize(sl.stream);
            lk.lock();
            finish(sl, rc);
        } else {
            sl.launched = true;
            work_cv.notify_all();
        }
    }
}

void lvq_server::run_completer()
{
    (void)hipSetDevice(ix->device);
    std::vector<int> polled;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        polled.clear();
        for (size_t i = 0; i < slots.size(); ++i)
            if (slots[i].req && slots[i].launched) polled.push_back((int)i);
        if (polled.empty()) {
            if (stop && queue.empty() && in_flight == 0) break;
            work_cv.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        lk.unlock();
        std::vector<std::pair<int, int>> ended;
        for (int i : polled) {
            const hipError_t e = hipEventQuery(slots[i].done);
            if (e == hipSuccess) ended.push_back({i, LVQ_OK});
            else if (e != hipErrorNotReady) ended.push_back({i, LVQ_ERR_DEVICE});
        }
        lk.lock();
        for (auto &p : ended) finish(slots[p.first], p.second);
        if (ended.empty()) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

extern "C" {

int lvq_server_create(lvq_index *ix, const lvq_server_config *cfg, lvq_server **out)
{
    if (!ix || !cfg || !out) return LVQ_ERR_INVALID_ARG;
    *out = nullptr;
    lvq_server_config c = *cfg;
    if (c.slots < 1 || c.slots > 64 || c.max_batch < 1 || c.max_batch > 65536 || c.k < 1 || c.k > kMaxTopK)
        return LVQ_ERR_INVALID_ARG;
    if (c.precision != LVQ_FP32 && c.precision != LVQ_BF16 && c.precision != LVQ_FP16) return LVQ_ERR_INVALID_ARG;
    if (c.scan_level != LVQ_PRIMARY && c.scan_level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    if (c.rerank_level != LVQ_PRIMARY && c.rerank_level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    if (c.scan_level == LVQ_FULL || c.rerank_level == LVQ_PRIMARY) {
        c.rerank_level = LVQ_PRIMARY;   // one stage: the scan's top-k is the result
        c.k_first = c.k;
    } else if (c.k_first < c.k || c.k_first > kMaxTopK) {
        return LVQ_ERR_INVALID_ARG;
    }
    if ((c.scan_level == LVQ_FULL || c.rerank_level == LVQ_FULL) && ix->f.bits2 == 0) return LVQ_ERR_INVALID_ARG;
    if (c.pool_bytes < 0) return LVQ_ERR_INVALID_ARG;
    if (ix->cfg.capacity == 0) return LVQ_ERR_INVALID_ARG;
    if (c.precision != LVQ_FP32 &&
        (ix->cfg.metric != LVQ_IP ||
         !mfma_query_block(ix->f.bits1, c.scan_level == LVQ_FULL ? ix->f.bits2 : 0, ix->f.kpos)))
        return LVQ_ERR_UNSUPPORTED;

    lvq_server *sv = new (std::nothrow) lvq_server();
    if (!sv) return LVQ_ERR_OOM;
    sv->ix = ix;
    sv->cfg = c;
    sv->dim = ix->f.dim;
    sv->rerank = c.rerank_level == LVQ_FULL;
    sv->t0 = std::chrono::steady_clock::now();
    const size_t one = sv->batch_bytes(c.max_batch);
    if (c.pool_bytes == 0) sv->cfg.pool_bytes = (int64_t)(one * (size_t)c.slots);
    if ((size_t)sv->cfg.pool_bytes < one) {
        delete sv;
        return LVQ_ERR_INVALID_ARG;   // the largest batch could never be admitted
    }
    int rc = LVQ_OK;
    sv->slots.resize(c.slots);
    {
        std::lock_guard<std::mutex> lk(ix->mu);
        rc = host_alloc(ix, sv->pool_mem, (size_t)sv->cfg.pool_bytes);
        if (rc == LVQ_OK) rc = host_alloc(ix, sv->offsets, sizeof(int64_t) * ((size_t)c.max_batch + 1));
        for (int i = 0; i < c.slots && rc == LVQ_OK; ++i) {
            Slot &sl = sv->slots[i];
            if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void **)&sl.q_host, sizeof(float) * (size_t)c.max_batch * sv->dim, 0) != hipSuccess ||
                hipHostMalloc((void **)&sl.ids_host, 4 * (size_t)c.max_batch * c.k, 0) != hipSuccess ||
                hipHostMalloc((void **)&sl.dist_host, 4 * (size_t)c.max_batch * c.k, 0) != hipSuccess) {
                rc = LVQ_ERR_DEVICE;
                break;
            }
            // size the stream's scan workspace for every batch size up front
            rc = host_reserve(ix, sl.stream, c.max_batch, c.k_first, c.precision, c.scan_level,
                              sv->rerank ? c.k : 0, c.rerank_level);
        }
    }
    if (rc == LVQ_OK) {
        std::vector<int64_t> offs((size_t)c.max_batch + 1);
        for (size_t i = 0; i < offs.size(); ++i) offs[i] = (int64_t)i * c.k_first;
        if (hipMemcpy(sv->offsets.p, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
            rc = LVQ_ERR_DEVICE;
    }
    if (rc != LVQ_OK) {
        lvq_server_destroy(sv);
        return rc;
    }
    sv->pool.reset((size_t)sv->cfg.pool_bytes);
    sv->dispatcher = std::thread([sv] { sv->run_dispatcher(); });
    sv->completer = std::thread([sv] { sv->run_completer(); });
    *out = sv;
    return LVQ_OK;
}

int lvq_server_submit(lvq_server *sv, const float *q_host, int32_t nq, int64_t *ticket_out)
{
    if (!sv || !q_host || !ticket_out || nq < 1 || nq > sv->cfg.max_batch) return LVQ_ERR_INVALID_ARG;
    auto r = std::make_shared<Request>();
    r->t_submit = sv->now();
    r->nq = nq;
    r->bytes = sv->batch_bytes(nq);
    try {
        r->q.assign(q_host, q_host + (size_t)nq * sv->dim);
    } catch (...) {
        return LVQ_ERR_OOM;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return LVQ_ERR_INVALID_ARG;
    r->ticket = sv->next_ticket++;
    sv->requests[r->ticket] = r;
    sv->queue.push_back(r);
    ++sv->submitted;
    sv->peak_queue = std::max(sv->peak_queue, (int32_t)sv->queue.size());
    *ticket_out = r->ticket;
    sv->admit_cv.notify_all();
    return LVQ_OK;
}

int lvq_server_wait(lvq_server *sv, int64_t ticket, int32_t *ids_host, float *dist_host, lvq_request_info *info)
{
    if (!sv) return LVQ_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) {
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->status = LVQ_ERR_INVALID_ARG;
        }
        return LVQ_ERR_INVALID_ARG;
    }
    std::shared_ptr<Request> r = it->second;
    sv->done_cv.wait(lk, [&] { return r->done; });
    sv->requests.erase(ticket);
    lk.unlock();
    if (r->status == LVQ_OK) {
        if (ids_host) std::memcpy(ids_host, r->ids.data(), sizeof(int32_t) * r->ids.size());
        if (dist_host) std::memcpy(dist_host, r->dist.data(), sizeof(float) * r->dist.size());
    }
    if (info) {
        info->status = r->status;
        info->nq = r->nq;
        info->epoch = r->epoch;
        info->slot = r->slot;
        info->t_submit = r->t_submit;
        info->t_admit = r->t_admit;
        info->t_done = r->t_done;
    }
    return r->status;
}

int lvq_server_drain(lvq_server *sv)
{
    if (!sv) return LVQ_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->done_cv.wait(lk, [&] { return sv->queue.empty() && sv->in_flight == 0; });
    return LVQ_OK;
}

int lvq_server_get_stats(lvq_server *sv, lvq_server_stats *out)
{
    if (!sv || !out) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->pool_bytes = (int64_t)sv->pool.size();
    out->pool_peak = (int64_t)sv->pool.peak();
    out->batch_bytes_max = (int64_t)sv->batch_bytes(sv->cfg.max_batch);
    out->slots = (int32_t)sv->slots.size();
    out->peak_in_flight = sv->peak_in_flight;
    out->peak_queue = sv->peak_queue;
    out->queued = (int32_t)sv->queue.size();
    out->in_flight = sv->in_flight;
    return LVQ_OK;
}

int lvq_server_destroy(lvq_server *sv)
{
    if (!sv) return LVQ_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->admit_cv.notify_all();
        sv->work_cv.notify_all();
    }
    if (sv->dispatcher.joinable()) sv->dispatcher.join();   // admits what is queued, then ends
    if (sv->completer.joinable()) sv->completer.join();     // ends once nothing is in flight
    for (Slot &sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.q_host) (void)hipHostFree(sl.q_host);
        if (sl.ids_host) (void)hipHostFree(sl.ids_host);
        if (sl.dist_host) (void)hipHostFree(sl.dist_host);
    }
    {
        std::lock_guard<std::mutex> lk(sv->ix->mu);
        for (Slot &sl : sv->slots) {
            auto it = sv->ix->ws.find(sl.stream);
            if (it == sv->ix->ws.end()) continue;
            Workspace &w = it->second;
            for (DevBuf *b : {&w.qk, &w.qsum, &w.cm, &w.order, &w.queue, &w.part, &w.q16, &w.gthr})
                host_free(sv->ix, *b);
            sv->ix->ws.erase(it);
        }
        host_free(sv->ix, sv->pool_mem);
        host_free(sv->ix, sv->offsets);
    }
    delete sv;
    return LVQ_OK;
}

}  // extern "C"
