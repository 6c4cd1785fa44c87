// lvq_host.hip -- host side of the C ABI declared in include/lvq.h: argument
// checks, the device store, per-stream workspaces, epochs, and kernel
// dispatch.  Every computation of the path runs in the kernels; this file
// only validates, allocates and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "lvq_index.h"

namespace lvq {

bool make_format(const lvq_config &c, Format *f)
{
    if (c.dim < 1 || c.dim > 8192) return false;
    if (c.bits1 != 4 && c.bits1 != 8) return false;
    if (c.bits2 != 0 && c.bits2 != 4 && c.bits2 != 8) return false;
    if (c.layout != LVQ_SEQUENTIAL && c.layout != LVQ_TURBO) return false;
    if (c.align != 32 && c.align != 64 && c.align != 128) return false;
    if (c.metric != LVQ_L2 && c.metric != LVQ_IP) return false;
    auto up = [](int v, int m) { return (v + m - 1) / m * m; };
    int blk = c.layout == LVQ_TURBO ? (c.bits1 == 4 ? 128 : 64) : (c.bits1 == 4 ? 8 : 4);
    f->dim = c.dim;
    f->bits1 = c.bits1;
    f->bits2 = c.bits2;
    f->layout = c.layout;
    f->align = c.align;
    f->npos = up(c.dim, blk);
    f->code_bytes = f->npos * c.bits1 / 8;
    f->row_bytes = up(kHeaderBytes + f->code_bytes, c.align);
    f->resid_bytes = c.bits2 ? up(f->npos * c.bits2 / 8, c.align) : 0;
    f->kchunks = up(f->code_bytes, 16) / 16;
    f->kpos = f->kchunks * 16 * 8 / c.bits1;
    return true;
}

// dimension held at code position p (the row format of lvq.h)
static int pos_dim(const Format &f, int p)
{
    if (p >= f.npos) return -1;
    int dim = p;
    if (f.layout == LVQ_TURBO) {
        const int per = 32 / f.bits1, blk = f.bits1 == 4 ? 128 : 64;
        const int b = p / blk, r = p % blk, w = r / per, k = r % per;
        dim = b * blk + 16 * k + w;
    }
    return dim < f.dim ? dim : -1;
}

void kernel_order_dims(const Format &f, int32_t *kdim)
{
    for (int s = 0; s < f.kpos; ++s) {
        int p = s;
        if (f.bits1 == 4) {
            const int w = s / 8, r = s % 8;
            p = 8 * w + (r < 4 ? 2 * r : 2 * (r - 4) + 1);
        }
        kdim[s] = pos_dim(f, p);
    }
}

}  // namespace lvq

using namespace lvq;

namespace {

int map_hip(hipError_t e)
{
    if (e == hipSuccess) return LVQ_OK;
    if (e == hipErrorOutOfMemory) return LVQ_ERR_OOM;
    return LVQ_ERR_DEVICE;
}

#define LVQ_HIP(x)                         \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return map_hip(e_); \
    } while (0)

int dev_alloc(lvq_index *ix, DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p) return LVQ_OK;
    if (ix->capturing) return LVQ_ERR_INVALID_ARG;   // no allocation inside graph capture
    if (b.pinned) return LVQ_ERR_INVALID_ARG;        // a captured graph still reads it
    if (bytes == 0) bytes = 16;
    const int64_t grow = (int64_t)bytes - (int64_t)b.bytes;
    if (ix->cfg.mem_budget_bytes > 0 && ix->device_bytes + grow > ix->cfg.mem_budget_bytes)
        return LVQ_ERR_OOM;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return LVQ_ERR_OOM;
    if (b.p) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b.p);
    }
    ix->device_bytes += grow;
    b.p = p;
    b.bytes = bytes;
    return LVQ_OK;
}

void dev_free(lvq_index *ix, DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    ix->device_bytes -= (int64_t)b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

template <class T>
T *P(DevBuf &b)
{
    return reinterpret_cast<T *>(b.p);
}

bool finite_host(const float *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// Rebuild the device means tables for ids [0, n_means).
int upload_means(lvq_index *ix, const std::vector<float> &all)
{
    const Format &f = ix->f;
    const int M = ix->n_means, d = f.dim;
    std::vector<float> mt((size_t)d * kMaxMeans, 0.0f), mk((size_t)M * f.kpos, 0.0f);
    std::vector<int32_t> kd(f.kpos);
    kernel_order_dims(f, kd.data());
    for (int m = 0; m < M; ++m)
        for (int j = 0; j < d; ++j) mt[(size_t)j * kMaxMeans + m] = all[(size_t)m * d + j];
    for (int m = 0; m < M; ++m)
        for (int s = 0; s < f.kpos; ++s)
            if (kd[s] >= 0) mk[(size_t)m * f.kpos + s] = all[(size_t)m * d + kd[s]];
    int rc;
    if ((rc = dev_alloc(ix, ix->means, sizeof(float) * (size_t)kMaxMeans * d))) return rc;
    if ((rc = dev_alloc(ix, ix->means_t, sizeof(float) * (size_t)kMaxMeans * d))) return rc;
    if ((rc = dev_alloc(ix, ix->muk, sizeof(float) * (size_t)kMaxMeans * f.kpos))) return rc;
    LVQ_HIP(hipMemcpy(ix->means.p, all.data(), sizeof(float) * (size_t)M * d, hipMemcpyHostToDevice));
    LVQ_HIP(hipMemcpy(ix->means_t.p, mt.data(), sizeof(float) * mt.size(), hipMemcpyHostToDevice));
    LVQ_HIP(hipMemcpy(ix->muk.p, mk.data(), sizeof(float) * mk.size(), hipMemcpyHostToDevice));
    return LVQ_OK;
}

Workspace &workspace(lvq_index *ix, hipStream_t s) { return ix->ws[s]; }

// After a captured call on `s`: its workspace buffers (which the graph's
// kernels read and write) are never freed or grown again, and the occupied-
// slot list a captured scan walks is never recycled by consolidation.
void pin_after_capture(lvq_index *ix, hipStream_t s, bool reads_list)
{
    if (!ix->capturing) return;
    Workspace &w = ix->ws[s];
    for (DevBuf *b : {&w.qk, &w.qsum, &w.cm, &w.order, &w.queue, &w.part, &w.q16, &w.gthr, &w.mkeys, &w.members, &w.moffs,
                      &w.mcount, &w.mcursor, &w.probe, &w.qoffs, &w.qids})
        if (b->p) b->pinned = true;
    if (reads_list && ix->list_active >= 0) ix->lists[ix->list_active].captured = true;
}

// Record whether `s` is capturing a HIP graph: captured calls allocate
// nothing, skip cross-stream ordering and in-flight bookkeeping, and replay
// at the epoch of capture.
int begin_call(lvq_index *ix, hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    LVQ_HIP(hipStreamIsCapturing(s, &st));
    ix->capturing = st != hipStreamCaptureStatusNone;
    return LVQ_OK;
}

// Make work on `s` wait for the latest store update issued on another stream.
int order_after_updates(lvq_index *ix, hipStream_t s)
{
    if (ix->capturing) return LVQ_OK;
    if (ix->have_update && ix->update_stream != s) LVQ_HIP(hipStreamWaitEvent(s, ix->update_ev, 0));
    return LVQ_OK;
}

int note_update(lvq_index *ix, hipStream_t s)
{
    ix->version += 1;
    LVQ_HIP(hipEventRecord(ix->update_ev, s));
    ix->update_stream = s;
    ix->have_update = true;
    return LVQ_OK;
}

// may_create = false (the allocation-free entry point): with no spare event,
// wait for the oldest in-flight launch and take its event (lvq_create makes
// a few spare events, so one of the two lists is never empty).
int note_query(lvq_index *ix, hipStream_t s, uint32_t epoch, bool may_create = true)
{
    if (ix->capturing) return LVQ_OK;
    hipEvent_t ev;
    if (ix->spare_events.empty() && !may_create) {
        if (ix->inflight.empty()) return LVQ_ERR_DEVICE;
        LVQ_HIP(hipEventSynchronize(ix->inflight.front().ev));
        ix->spare_events.push_back(ix->inflight.front().ev);
        ix->inflight.pop_front();
    }
    if (!ix->spare_events.empty()) {
        ev = ix->spare_events.back();
        ix->spare_events.pop_back();
    } else {
        LVQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    LVQ_HIP(hipEventRecord(ev, s));
    ix->inflight.push_back({epoch, ++ix->query_seq, ev});
    // retire completed entries from the front
    while (!ix->inflight.empty() && hipEventQuery(ix->inflight.front().ev) == hipSuccess) {
        ix->spare_events.push_back(ix->inflight.front().ev);
        ix->inflight.pop_front();
    }
    return LVQ_OK;
}

// Bracket the main kernel with events when timing is enabled.
int timing_begin(lvq_index *ix, hipStream_t s)
{
    if (!ix->timing || ix->capturing) return LVQ_OK;
    hipEvent_t a, b;
    LVQ_HIP(hipEventCreate(&a));
    LVQ_HIP(hipEventCreate(&b));
    LVQ_HIP(hipEventRecord(a, s));
    ix->tev.push_back({a, b});
    return LVQ_OK;
}

int timing_end(lvq_index *ix, hipStream_t s)
{
    if (!ix->timing || ix->capturing || ix->tev.empty()) return LVQ_OK;
    LVQ_HIP(hipEventRecord(ix->tev.back().second, s));
    return LVQ_OK;
}

// Query prep into the given buffers (nq x kpos, nq, nq x n_means floats).
int prep_into(lvq_index *ix, const float *q, int64_t nq, float *qk, float *qsum, float *cm, hipStream_t s)
{
    const Format &f = ix->f;
    PrepArgs pa;
    pa.q = q;
    pa.nq = nq;
    pa.dim = f.dim;
    pa.kpos = f.kpos;
    pa.n_means = ix->n_means;
    pa.metric = ix->cfg.metric;
    pa.kdim = P<int32_t>(ix->kdim);
    pa.means = P<float>(ix->means);
    pa.qk = qk;
    pa.qsum = qsum;
    pa.cm = cm;
    LVQ_HIP(launch_prep(pa, s));
    return LVQ_OK;
}

int prep_queries(lvq_index *ix, Workspace &w, const float *q, int64_t nq, hipStream_t s)
{
    const Format &f = ix->f;
    int rc;
    if ((rc = dev_alloc(ix, w.qk, sizeof(float) * (size_t)std::max<int64_t>(nq, 1) * f.kpos))) return rc;
    if ((rc = dev_alloc(ix, w.qsum, sizeof(float) * (size_t)std::max<int64_t>(nq, 1)))) return rc;
    if ((rc = dev_alloc(ix, w.cm, sizeof(float) * (size_t)std::max<int64_t>(nq, 1) * ix->n_means))) return rc;
    return prep_into(ix, q, nq, P<float>(w.qk), P<float>(w.qsum), P<float>(w.cm), s);
}

// Default tile shape: the instantiated shape whose round covers the code
// bytes with the least waste, preferring more lanes per candidate.
int default_shape(const Format &f, void *(*lookup)(int, int, int), int bits2, int variant)
{
    const int bytes = f.kchunks * 16;
    int best = -1;
    double best_cost = 1e30;
    for (int i = 0; i < num_tile_shapes(); ++i) {
        if (!lookup(bits2, variant, i)) continue;
        TileShape t = tile_shape(i);
        const int round = t.g * t.ch * t.nch;
        const int rounds = (bytes + round - 1) / round;
        if (t.pipe && rounds > 1) continue;
        const double waste = (double)rounds * round / bytes;
        const double cost = waste * 16.0 / t.g + (rounds > 1 ? 0.5 * rounds : 0.0);
        if (cost < best_cost) {
            best_cost = cost;
            best = i;
        }
    }
    return best;
}

bool shape_fits(const Format &f, void *(*lookup)(int, int, int), int bits2, int variant, int shape)
{
    if (shape < 0 || shape >= num_tile_shapes() || !lookup(bits2, variant, shape)) return false;
    TileShape t = tile_shape(shape);
    return !t.pipe || t.g * t.ch * t.nch >= f.kchunks * 16;
}

}  // namespace

namespace lvq {

int host_begin_call(lvq_index *ix, hipStream_t s) { return begin_call(ix, s); }
int host_note_query(lvq_index *ix, hipStream_t s, uint32_t epoch, bool may_create)
{
    return note_query(ix, s, epoch, may_create);
}
int host_alloc(lvq_index *ix, DevBuf &b, size_t bytes) { return dev_alloc(ix, b, bytes); }
void host_free(lvq_index *ix, DevBuf &b) { dev_free(ix, b); }

}  // namespace lvq

extern "C" {

const char *lvq_strerror(int code)
{
    switch (code) {
    case LVQ_OK: return "ok";
    case LVQ_ERR_INVALID_ARG: return "invalid argument";
    case LVQ_ERR_UNSUPPORTED: return "unsupported configuration";
    case LVQ_ERR_OOM: return "out of device memory or over the memory budget";
    case LVQ_ERR_CAPACITY: return "not enough free slots";
    case LVQ_ERR_DEVICE: return "HIP runtime error";
    case LVQ_ERR_NONFINITE: return "non-finite input vector";
    case LVQ_ERR_BAD_SLOT: return "slot out of range or not live";
    case LVQ_ERR_SCRATCH: return "request exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown error";
    }
}

int lvq_row_format(const lvq_config *cfg, int32_t *row_bytes, int32_t *resid_bytes, int32_t *code_positions)
{
    Format f;
    if (!cfg || !make_format(*cfg, &f)) return LVQ_ERR_INVALID_ARG;
    if (row_bytes) *row_bytes = f.row_bytes;
    if (resid_bytes) *resid_bytes = f.resid_bytes;
    if (code_positions) *code_positions = f.npos;
    return LVQ_OK;
}

int lvq_create(const lvq_config *cfg, const float *means_host, int32_t n_means, lvq_index **out)
{
    if (!cfg || !out || !means_host) return LVQ_ERR_INVALID_ARG;
    *out = nullptr;
    Format f;
    if (!make_format(*cfg, &f)) return LVQ_ERR_INVALID_ARG;
    if (n_means < 1 || n_means > kMaxMeans || cfg->capacity < 0 || cfg->capacity > INT32_MAX)
        return LVQ_ERR_INVALID_ARG;
    if (!finite_host(means_host, (size_t)n_means * cfg->dim)) return LVQ_ERR_NONFINITE;
    lvq_index *ix = new (std::nothrow) lvq_index();
    if (!ix) return LVQ_ERR_OOM;
    ix->cfg = *cfg;
    ix->f = f;
    ix->n_means = n_means;
    int rc = LVQ_OK;
    do {
        if (hipGetDevice(&ix->device) != hipSuccess) { rc = LVQ_ERR_DEVICE; break; }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ix->device) == hipSuccess) {
            ix->n_cu = prop.multiProcessorCount;
            ix->lds_max = prop.sharedMemPerBlock;
        }
        std::vector<float> all(means_host, means_host + (size_t)n_means * cfg->dim);
        if ((rc = upload_means(ix, all))) break;
        std::vector<int32_t> kd(f.kpos);
        kernel_order_dims(f, kd.data());
        std::vector<float> km(f.kpos);
        for (int s = 0; s < f.kpos; ++s) km[s] = kd[s] >= 0 ? 1.0f : 0.0f;
        if ((rc = dev_alloc(ix, ix->kdim, sizeof(int32_t) * f.kpos))) break;
        if ((rc = dev_alloc(ix, ix->kmask, sizeof(float) * f.kpos))) break;
        if ((rc = dev_alloc(ix, ix->err, 16))) break;
        if ((rc = dev_alloc(ix, ix->scratch, 4096))) break;
        if ((rc = dev_alloc(ix, ix->mean_active, kMaxMeans))) break;
        if ((rc = dev_alloc(ix, ix->mean_counts, sizeof(uint64_t) * kMaxMeans))) break;
        ix->retired.assign(kMaxMeans, 0);
        if (hipMemset(ix->mean_active.p, 1, kMaxMeans)) {
            rc = LVQ_ERR_DEVICE;
            break;
        }
        if (hipMemcpy(ix->kdim.p, kd.data(), sizeof(int32_t) * f.kpos, hipMemcpyHostToDevice) ||
            hipMemcpy(ix->kmask.p, km.data(), sizeof(float) * f.kpos, hipMemcpyHostToDevice) ||
            hipMemset(ix->err.p, 0, 16)) {
            rc = LVQ_ERR_DEVICE;
            break;
        }
        const int64_t cap = cfg->capacity;
        if (cap > 0) {
            if ((rc = dev_alloc(ix, ix->rows, (size_t)cap * f.row_bytes))) break;
            if (f.resid_bytes && (rc = dev_alloc(ix, ix->resid, (size_t)cap * f.resid_bytes))) break;
            if ((rc = dev_alloc(ix, ix->stack, sizeof(int32_t) * (size_t)cap))) break;
            if (hipMemset(ix->rows.p, 0, (size_t)cap * f.row_bytes) ||
                (f.resid_bytes && hipMemset(ix->resid.p, 0, (size_t)cap * f.resid_bytes))) {
                rc = LVQ_ERR_DEVICE;
                break;
            }
            std::vector<int32_t> st(cap);
            for (int64_t i = 0; i < cap; ++i) st[i] = (int32_t)(cap - 1 - i);
            if (hipMemcpy(ix->stack.p, st.data(), sizeof(int32_t) * cap, hipMemcpyHostToDevice)) {
                rc = LVQ_ERR_DEVICE;
                break;
            }
        }
        ix->free_top = cap;
        if (cap > 0) {
            ix->lists.resize(1);
            if ((rc = dev_alloc(ix, ix->lists[0].buf, sizeof(int32_t) * (size_t)cap))) break;
            ix->list_active = 0;
            ix->list_len = 0;
        }
        if (hipEventCreateWithFlags(&ix->update_ev, hipEventDisableTiming)) { rc = LVQ_ERR_DEVICE; break; }
        for (int i = 0; i < 8 && rc == LVQ_OK; ++i) {
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming)) rc = LVQ_ERR_DEVICE;
            else ix->spare_events.push_back(ev);
        }
        if (rc) break;
        if ((rc = noalloc_setup(ix->device))) break;
    } while (0);
    if (rc) {
        lvq_destroy(ix);
        return rc;
    }
    *out = ix;
    return LVQ_OK;
}

int lvq_destroy(lvq_index *ix)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    for (auto &kv : ix->ws) {
        Workspace &w = kv.second;
        for (DevBuf *b : {&w.qk, &w.qsum, &w.cm, &w.order, &w.queue, &w.part, &w.q16, &w.gthr, &w.mkeys, &w.members, &w.moffs,
                          &w.mcount, &w.mcursor, &w.probe, &w.qoffs, &w.qids})
            dev_free(ix, *b);
    }
    for (DevBuf *b : {&ix->means, &ix->means_t, &ix->muk, &ix->kmask, &ix->kdim, &ix->rows,
                      &ix->resid, &ix->stack, &ix->err, &ix->scratch, &ix->mean_active, &ix->mean_counts})
        dev_free(ix, *b);
    for (SlotList &l : ix->lists) dev_free(ix, l.buf);
    for (auto &f : ix->inflight) (void)hipEventDestroy(f.ev);
    for (auto e : ix->spare_events) (void)hipEventDestroy(e);
    if (ix->update_ev) (void)hipEventDestroy(ix->update_ev);
    delete ix;
    return LVQ_OK;
}

int lvq_set_means(lvq_index *ix, const float *means_host, int32_t n_means, int32_t *first_id_out, void *stream)
{
    if (!ix || !means_host || n_means < 1 || n_means > kMaxMeans) return LVQ_ERR_INVALID_ARG;
    const Format &f = ix->f;
    const int d = f.dim;
    if (!finite_host(means_host, (size_t)n_means * d)) return LVQ_ERR_NONFINITE;
    hipStream_t s = (hipStream_t)stream;
    // tables for the new ids only: work already queued reads ids below the old count
    std::vector<float> mt((size_t)d * n_means), mk((size_t)n_means * f.kpos, 0.0f);
    std::vector<int32_t> kd(f.kpos);
    kernel_order_dims(f, kd.data());
    for (int m = 0; m < n_means; ++m)
        for (int j = 0; j < d; ++j) mt[(size_t)j * n_means + m] = means_host[(size_t)m * d + j];
    for (int m = 0; m < n_means; ++m)
        for (int t = 0; t < f.kpos; ++t)
            if (kd[t] >= 0) mk[(size_t)m * f.kpos + t] = means_host[(size_t)m * d + kd[t]];
    int first = 0;
    {
        std::lock_guard<std::mutex> lk(ix->mu);
        if (ix->n_means + n_means > kMaxMeans) return LVQ_ERR_CAPACITY;
        int rc = begin_call(ix, s);
        if (rc) return rc;
        if (ix->capturing) {
            ix->capturing = false;
            return LVQ_ERR_INVALID_ARG;
        }
        if ((rc = order_after_updates(ix, s))) return rc;
        first = ix->n_means;
        LVQ_HIP(hipMemcpyAsync(P<float>(ix->means) + (size_t)first * d, means_host, sizeof(float) * mt.size(),
                               hipMemcpyHostToDevice, s));
        LVQ_HIP(hipMemcpy2DAsync(P<float>(ix->means_t) + first, sizeof(float) * kMaxMeans, mt.data(),
                                 sizeof(float) * n_means, sizeof(float) * n_means, d, hipMemcpyHostToDevice, s));
        LVQ_HIP(hipMemcpyAsync(P<float>(ix->muk) + (size_t)first * f.kpos, mk.data(), sizeof(float) * mk.size(),
                               hipMemcpyHostToDevice, s));
        ix->n_means += n_means;
        if ((rc = note_update(ix, s))) return rc;
    }
    // the host sources must outlive the copies
    LVQ_HIP(hipStreamSynchronize(s));
    if (first_id_out) *first_id_out = first;
    return LVQ_OK;
}

static int encode_common(lvq_index *ix, const float *x, int64_t n, uint8_t *rows, uint8_t *resid,
                         const uint64_t *ext, int32_t *slots_out, bool store, hipStream_t s)
{
    EncodeArgs a;
    a.x = x;
    a.n = n;
    a.means = P<float>(ix->means);
    a.means_t = P<float>(ix->means_t);
    a.means_t_stride = kMaxMeans;
    a.n_means = ix->n_means;
    a.means_lds = ix->n_means > 1 && (size_t)ix->n_means * ix->f.dim * sizeof(float) <= 32768 ? 1 : 0;
    a.mean_active = P<uint8_t>(ix->mean_active);
    a.f = ix->f;
    a.rows = rows;
    a.resid = resid;
    a.free_stack = store ? P<int32_t>(ix->stack) : nullptr;
    a.free_top = ix->free_top;
    a.list_out = store ? P<int32_t>(ix->lists[ix->list_active].buf) + ix->list_len : nullptr;
    a.slots_out = slots_out;
    a.ext_ids = ext;
    a.epoch = ix->epoch;
    a.err = P<uint32_t>(ix->err);
    LVQ_HIP(launch_encode(a, s));
    return LVQ_OK;
}

int lvq_encode(lvq_index *ix, const float *x_dev, int64_t n, uint8_t *rows_dev, uint8_t *resid_dev, void *stream)
{
    if (!ix || n < 0 || (n > 0 && (!x_dev || !rows_dev))) return LVQ_ERR_INVALID_ARG;
    if (ix->f.bits2 && n > 0 && !resid_dev) return LVQ_ERR_INVALID_ARG;
    if (n == 0) return LVQ_OK;
    std::lock_guard<std::mutex> lk(ix->mu);
    return encode_common(ix, x_dev, n, rows_dev, resid_dev, nullptr, nullptr, false, (hipStream_t)stream);
}

int lvq_insert(lvq_index *ix, const float *x_dev, int64_t n, const uint64_t *ext_ids_dev, int32_t *slots_out_dev,
               void *stream)
{
    if (!ix || n < 0 || (n > 0 && (!x_dev || !slots_out_dev))) return LVQ_ERR_INVALID_ARG;
    if (n == 0) return LVQ_OK;
    std::lock_guard<std::mutex> lk(ix->mu);
    if (n > ix->free_top) return LVQ_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    ix->epoch += 1;
    rc = encode_common(ix, x_dev, n, P<uint8_t>(ix->rows), P<uint8_t>(ix->resid), ext_ids_dev, slots_out_dev,
                       true, s);
    if (rc) return rc;
    ix->free_top -= n;
    ix->list_len += n;
    return note_update(ix, s);
}

static StoreArgs store_args(lvq_index *ix)
{
    StoreArgs a;
    a.rows = P<uint8_t>(ix->rows);
    a.resid = P<uint8_t>(ix->resid);
    a.row_bytes = ix->f.row_bytes;
    a.resid_bytes = ix->f.resid_bytes;
    a.capacity = ix->cfg.capacity;
    a.epoch = ix->epoch;
    a.err = P<uint32_t>(ix->err);
    return a;
}

int lvq_delete(lvq_index *ix, const int32_t *slots_dev, int64_t n, void *stream)
{
    if (!ix || n < 0 || (n > 0 && !slots_dev)) return LVQ_ERR_INVALID_ARG;
    if (n == 0) return LVQ_OK;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    ix->epoch += 1;
    LVQ_HIP(launch_delete(store_args(ix), slots_dev, n, s));
    return note_update(ix, s);
}

int lvq_consolidate(lvq_index *ix, void *stream, int64_t *n_freed_out)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    if (n_freed_out) *n_freed_out = 0;
    const int64_t cap = ix->cfg.capacity;
    if (cap == 0) return LVQ_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    // the oldest epoch an unfinished query may still observe, and the oldest
    // launch still running
    uint32_t safe = ix->epoch;
    uint64_t oldest = UINT64_MAX;
    for (auto it = ix->inflight.begin(); it != ix->inflight.end();) {
        if (hipEventQuery(it->ev) == hipSuccess) {
            ix->spare_events.push_back(it->ev);
            it = ix->inflight.erase(it);
        } else {
            safe = std::min(safe, it->epoch);
            oldest = std::min(oldest, it->seq);
            ++it;
        }
    }
    // a list buffer for the compacted list: a retired one no running query
    // reads, else a new one
    int next = -1;
    for (int i = 0; i < (int)ix->lists.size(); ++i)
        if (i != ix->list_active && ix->lists[i].retire_seq < oldest && !ix->lists[i].captured) {
            next = i;
            break;
        }
    if (next < 0) {
        SlotList fresh_list;
        if ((rc = dev_alloc(ix, fresh_list.buf, sizeof(int32_t) * (size_t)cap))) return rc;
        ix->lists.push_back(fresh_list);
        next = (int)ix->lists.size() - 1;
    }
    const int nb = (int)((cap + 1023) / 1024);
    if ((rc = dev_alloc(ix, ix->scratch, sizeof(int32_t) * (size_t)nb + 64))) return rc;
    int32_t *counts = P<int32_t>(ix->scratch);
    int64_t *tail = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(ix->scratch.p) +
                                                ((sizeof(int32_t) * (size_t)nb + 15) & ~(size_t)15));
    LVQ_HIP(launch_consolidate(store_args(ix), safe, P<int32_t>(ix->stack), ix->free_top, counts, tail, s));
    LVQ_HIP(launch_build_list(store_args(ix), P<int32_t>(ix->lists[next].buf), counts, tail + 1, s));
    int64_t got[2] = {0, 0};   // new stack top, list length
    LVQ_HIP(hipMemcpyAsync(got, tail, sizeof(got), hipMemcpyDeviceToHost, s));
    LVQ_HIP(hipStreamSynchronize(s));
    if (n_freed_out) *n_freed_out = got[0] - ix->free_top;
    ix->free_top = got[0];
    ix->lists[ix->list_active].retire_seq = ix->query_seq;   // every launch so far may read it
    ix->list_active = next;
    ix->list_len = got[1];
    return note_update(ix, s);
}

}  // extern "C"

int lvq::host_distances(lvq_index *ix, const float *q_dev, int64_t nq, const int64_t *offsets_dev,
                        const int32_t *ids_dev, int64_t total, int32_t level, float *dist_dev, int32_t k,
                        int32_t *topk_ids_dev, float *topk_dist_dev, hipStream_t s, int force_shape,
                        uint32_t epoch, bool neg_empty, const int32_t *list_means, int list_nmeans,
                        const int64_t *seg_offs, const int32_t *seg_members, const DistScratch *fixed)
{
    if (!ix || nq < 0 || total < 0 || nq > INT32_MAX) return LVQ_ERR_INVALID_ARG;
    const bool segmented = seg_members != nullptr;
    if (segmented && (!seg_offs || !list_means)) return LVQ_ERR_INVALID_ARG;
    if (level != LVQ_PRIMARY && level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    if (k < 0 || k > kMaxTopK) return LVQ_ERR_INVALID_ARG;
    if (nq == 0) return LVQ_OK;
    if (!q_dev || !offsets_dev || (total > 0 && !ids_dev && !segmented)) return LVQ_ERR_INVALID_ARG;
    if (k == 0 && !dist_dev) return LVQ_ERR_INVALID_ARG;
    if (k > 0 && (!topk_ids_dev || !topk_dist_dev)) return LVQ_ERR_INVALID_ARG;
    if (ix->cfg.capacity == 0) return LVQ_ERR_INVALID_ARG;
    if (level == LVQ_FULL && ix->f.bits2 == 0) return LVQ_ERR_INVALID_ARG;
    const Format &f = ix->f;
    const int bits2 = level == LVQ_FULL ? f.bits2 : 0;
    const bool l2 = ix->cfg.metric == LVQ_L2;
    const bool multi = l2 && ix->n_means > 1;
    const bool masked = l2 && f.kpos != f.dim;
    const int variant = !l2 ? 0 : (masked ? (multi ? 4 : 3) : (multi ? 2 : 1));
    auto lookup = f.bits1 == 4 ? cand_kernel_b4 : cand_kernel_b8;
    int shape = force_shape >= 0 ? force_shape : ix->cand_shape[level == LVQ_FULL][k > 0];
    if (!shape_fits(f, lookup, bits2, variant, shape)) {
        if (force_shape >= 0) return LVQ_ERR_UNSUPPORTED;
        shape = default_shape(f, lookup, bits2, variant);
    }
    void *kern = shape >= 0 ? lookup(bits2, variant, shape) : nullptr;
    if (!kern) return LVQ_ERR_UNSUPPORTED;
    const bool sub = multi && list_means != nullptr;
    if (list_means && (list_nmeans < 1 || list_nmeans > ix->n_means)) return LVQ_ERR_INVALID_ARG;
    const int nseg = segmented ? list_nmeans : 0;
    const int ntab = multi ? (sub ? list_nmeans : ix->n_means) : 1;
    // top-k key buffer per wave: about 2k + one block of candidates (a block
    // holds at most 32 per wave), at least 64 and at most 2048 entries,
    // halved while the launch does not fit the workgroup's LDS
    int cw = 64;
    while (cw < 2 * k + 32 && cw < 2048) cw *= 2;
    size_t lds = cand_lds_bytes(f.kpos, ntab, masked, l2 ? 0 : ix->n_means, k, cw, sub, nseg);
    while (lds > ix->lds_max && cw / 2 >= k + 32) {
        cw /= 2;
        lds = cand_lds_bytes(f.kpos, ntab, masked, l2 ? 0 : ix->n_means, k, cw, sub, nseg);
    }
    if (lds > ix->lds_max) return LVQ_ERR_UNSUPPORTED;
    // several means: a second set of tables keeps the means in LDS if it fits
    int mu_lds = 0;
    if (multi && !sub) {
        const size_t with = cand_lds_bytes(f.kpos, 2 * ntab, masked, 0, k, cw, false, nseg);
        if (with <= ix->lds_max) {
            mu_lds = 1;
            lds = with;
        }
    }

    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    DistScratch sc;
    if (fixed) {
        sc = *fixed;
        if ((rc = prep_into(ix, q_dev, nq, sc.qk, sc.qsum, sc.cm, s))) return rc;
    } else {
        Workspace &w = workspace(ix, s);
        if ((rc = prep_queries(ix, w, q_dev, nq, s))) return rc;
        if ((rc = dev_alloc(ix, w.order, sizeof(int32_t) * (size_t)nq))) return rc;
        if ((rc = dev_alloc(ix, w.queue, 64))) return rc;
        sc = {P<float>(w.qk), P<float>(w.qsum), P<float>(w.cm), P<int32_t>(w.order), P<int32_t>(w.queue)};
    }

    CandArgs a;
    a.rows = P<uint8_t>(ix->rows);
    a.resid = P<uint8_t>(ix->resid);
    a.row_bytes = f.row_bytes;
    a.resid_bytes = f.resid_bytes;
    a.kchunks = f.kchunks;
    a.kpos = f.kpos;
    a.capacity = ix->cfg.capacity;
    a.qk = sc.qk;
    a.qsum = sc.qsum;
    a.cm = sc.cm;
    a.muk = P<float>(ix->muk);
    a.kmask = P<float>(ix->kmask);
    a.n_means = ix->n_means;
    a.offsets = offsets_dev;
    a.ids = ids_dev;
    a.nq = nq;
    a.total = total;
    a.dist = dist_dev;
    a.k = k;
    a.topk_ids = topk_ids_dev;
    a.topk_dist = topk_dist_dev;
    a.epoch = epoch;
    a.err = P<uint32_t>(ix->err);
    a.neg_empty = neg_empty ? 1 : 0;
    a.cw = cw;
    a.mu_lds = mu_lds;
    a.list_means = (sub || segmented) ? list_means : nullptr;
    a.list_nmeans = (sub || segmented) ? list_nmeans : 0;
    a.seg_offs = segmented ? seg_offs : nullptr;
    a.seg_members = segmented ? seg_members : nullptr;
    // persistent launch: lists longest-first from a device work counter
    a.order = sc.order;
    a.queue = sc.queue;
    LVQ_HIP(launch_fill_i32(a.queue, 0, 1, s));
    LVQ_HIP(launch_list_order(offsets_dev, nq, sc.order, nullptr, s));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t grid = std::min<int64_t>(nq, (int64_t)ix->n_cu * per_cu);
    ix->last_wg = grid;
    ix->last_lists = nq;
    ix->last_parts = 0;
    if (!fixed && (rc = timing_begin(ix, s))) return rc;
    hipLaunchKernelGGL(reinterpret_cast<void (*)(CandArgs)>(kern), dim3((unsigned)grid), dim3(256), lds, s, a);
    LVQ_HIP(hipGetLastError());
    return fixed ? LVQ_OK : timing_end(ix, s);
}

extern "C" {

int lvq_distances(lvq_index *ix, const float *q_dev, int64_t nq, const int64_t *offsets_dev, const int32_t *ids_dev,
                  int64_t total, int32_t level, float *dist_dev, int32_t k, int32_t *topk_ids_dev,
                  float *topk_dist_dev, void *stream)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    int rc = begin_call(ix, (hipStream_t)stream);
    if (rc) return rc;
    rc = host_distances(ix, q_dev, nq, offsets_dev, ids_dev, total, level, dist_dev, k, topk_ids_dev,
                        topk_dist_dev, (hipStream_t)stream, -1, ix->epoch, false);
    if (rc == LVQ_OK) rc = note_query(ix, (hipStream_t)stream, ix->epoch);
    if (rc == LVQ_OK) pin_after_capture(ix, (hipStream_t)stream, false);
    ix->capturing = false;
    return rc;
}

int lvq_set_tile(lvq_index *ix, int32_t level, int32_t topk, int32_t shape)
{
    if (!ix || (level != LVQ_PRIMARY && level != LVQ_FULL) || shape < -1 || shape >= num_tile_shapes())
        return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    ix->cand_shape[level == LVQ_FULL][topk != 0] = shape;
    return LVQ_OK;
}

int lvq_num_tile_shapes(void) { return num_tile_shapes(); }

int lvq_tile_shape(int32_t shape, int32_t *lanes, int32_t *piece_bytes, int32_t *pieces, int32_t *pipe)
{
    if (shape < 0 || shape >= num_tile_shapes()) return LVQ_ERR_INVALID_ARG;
    const TileShape t = tile_shape(shape);
    if (lanes) *lanes = t.g;
    if (piece_bytes) *piece_bytes = t.ch;
    if (pieces) *pieces = t.nch;
    if (pipe) *pipe = t.pipe;
    return LVQ_OK;
}

int lvq_autotune(lvq_index *ix, const float *q_dev, int64_t nq, const int64_t *offsets_dev, const int32_t *ids_dev,
                 int64_t total, int32_t level, int32_t k, int32_t *shape_out, float *ms_out, void *stream)
{
    if (!ix || nq < 1 || total < 0 || k < 0 || k > kMaxTopK) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    ix->capturing = false;
    float *dist = nullptr;
    int32_t *ti = nullptr;
    float *td = nullptr;
    LVQ_HIP(hipMalloc((void **)&dist, sizeof(float) * (size_t)std::max<int64_t>(total, 1)));
    if (k > 0) {
        LVQ_HIP(hipMalloc((void **)&ti, sizeof(int32_t) * (size_t)nq * k));
        LVQ_HIP(hipMalloc((void **)&td, sizeof(float) * (size_t)nq * k));
    }
    hipEvent_t a, b;
    LVQ_HIP(hipEventCreate(&a));
    LVQ_HIP(hipEventCreate(&b));
    int best = -1;
    float best_ms = 0.0f;
    int rc = LVQ_OK;
    for (int i = 0; i < num_tile_shapes() && rc == LVQ_OK; ++i) {
        if (host_distances(ix, q_dev, nq, offsets_dev, ids_dev, total, level, dist, k, ti, td, s, i, ix->epoch,
                           false) != LVQ_OK)
            continue;   // shape not available for this format
        float ms = 0.0f;
        if (hipEventRecord(a, s) != hipSuccess) { rc = LVQ_ERR_DEVICE; break; }
        for (int r = 0; r < 3 && rc == LVQ_OK; ++r)
            rc = host_distances(ix, q_dev, nq, offsets_dev, ids_dev, total, level, dist, k, ti, td, s, i, ix->epoch,
                                false);
        if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
            rc = LVQ_ERR_DEVICE;
            break;
        }
        if (best < 0 || ms < best_ms) {
            best = i;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(s);
    (void)hipFree(dist);
    if (ti) (void)hipFree(ti);
    if (td) (void)hipFree(td);
    if (rc) return rc;
    if (best < 0) return LVQ_ERR_UNSUPPORTED;
    ix->cand_shape[level == LVQ_FULL][k > 0] = best;
    if (shape_out) *shape_out = best;
    if (ms_out) *ms_out = best_ms / 3.0f;
    return LVQ_OK;
}

}  // extern "C"

static int topk_mfma(lvq_index *ix, const void *q_dev, int32_t prec, int64_t nq, int32_t k, int32_t level,
                     int32_t *ids_dev, float *dist_dev, hipStream_t s, uint32_t epoch);

// Row parts of the FP32 scan: enough workgroups (query tiles x parts) for
// about four per compute unit, parts of at least 1024 rows, and a merge that
// holds parts * k keys (+ k) of 8 bytes in one workgroup's LDS.
static int64_t scan_parts_fp32(const lvq_index *ix, int64_t nq, int32_t k, int64_t n_rows)
{
    const int64_t qtiles = (nq + 15) / 16;
    int64_t parts = std::max<int64_t>(1, (4 * (int64_t)ix->n_cu + qtiles - 1) / qtiles);
    parts = std::min<int64_t>(parts, std::max<int64_t>(1, n_rows / 1024));
    return std::min<int64_t>(parts, std::max<int64_t>(1, (int64_t)(ix->lds_max / 8 - k) / k));
}

// Row parts of the MFMA scan (one resident workgroup per compute unit).
// Time model: whole rounds of workgroups over the compute units, each
// workgroup streaming n_rows / parts rows, plus a per-part overhead (a part
// starts with a loose top-k bound and adds k keys to the merge) of 2% of a
// part's scan per extra part.  Parts keep at least 64 row rounds, and the
// merge (parts * k keys, + k) fits one workgroup's LDS.
static int64_t scan_parts_mfma(const lvq_index *ix, int64_t qtiles, int32_t k, int64_t n_rows)
{
    const int64_t max_parts = std::max<int64_t>(
        1, std::min<int64_t>(n_rows / (64 * 128), (int64_t)(ix->lds_max / 8 - k) / k));
    int64_t parts = 1;
    double best = 0.0;
    for (int64_t p = 1; p <= max_parts; ++p) {
        const int64_t rounds = (qtiles * p + ix->n_cu - 1) / ix->n_cu;
        const double cost = (double)rounds / (double)p * (1.0 + 0.02 * (double)p);
        if (p == 1 || cost < best) {
            best = cost;
            parts = p;
        }
    }
    return parts;
}

// Row parts and persistent grid of the wide MFMA scan (one workgroup per
// compute unit, a multiple of 8 for the XCD-aware tile walk).  Time model:
// each workgroup runs ceil(tiles per XCD / workgroups per XCD) tiles of
// N = n_rows / parts rows, plus a per-tile cost in 16-bit row equivalents:
// 10,240 for staging the queries and the final merge, and the appends of a
// part's loose bound.  A 32 x 32 block of scores holds a key beating the
// running k-th best of t rows with probability about min(1, 1024 k / t), so
// the blocks that append add about 512 k (1 + ln(N / 1024 k)) rows' worth.
// An FP32 row costs about 8 16-bit ones (a sixteenth of the matrix-core
// rate, half the queries per tile).  Parts keep at least 8 rounds of rows,
// and the merge (parts * k keys, + k) fits one workgroup's LDS.
static int64_t scan_parts_wide(const lvq_index *ix, int64_t qtiles, int32_t k, int64_t n_rows, int32_t prec,
                               int64_t *grid)
{
    const int64_t slots = std::max<int64_t>(8, ix->n_cu / 8 * 8);
    const int64_t max_parts = std::max<int64_t>(
        1, std::min<int64_t>(n_rows / 4096, (int64_t)(ix->lds_max / 8 - k) / k));
    int64_t parts = 1;
    double best = 0.0;
    for (int64_t p = 1; p <= max_parts; ++p) {
        const int64_t tiles = qtiles * p;
        const int64_t g = std::min<int64_t>(slots, (tiles + 7) / 8 * 8);
        const int64_t per_xcd = (tiles + 7) / 8;
        const int64_t iters = (per_xcd + g / 8 - 1) / (g / 8);
        const double rows = (double)((n_rows + p - 1) / p), warm = 1024.0 * k;
        const double row_cost = prec == LVQ_FP32 ? 8.0 : 1.0;
        const double cost = (double)iters * (rows + (10240.0 + 0.5 * warm * (1.0 + std::log(std::max(1.0, rows / warm)))) / row_cost);
        if (p == 1 || cost < best) {
            best = cost;
            parts = p;
        }
    }
    *grid = std::min<int64_t>(slots, (qtiles * parts + 7) / 8 * 8);
    return parts;
}

int lvq::host_topk(lvq_index *ix, const void *q_dev, int32_t prec, int64_t nq, int32_t k, int32_t level,
                   int32_t *ids_dev, float *dist_dev, hipStream_t s, uint32_t epoch)
{
    if (nq < 0 || nq > INT32_MAX || k < 1 || k > kMaxTopK) return LVQ_ERR_INVALID_ARG;
    if (level != LVQ_PRIMARY && level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    if (prec != LVQ_FP32 && prec != LVQ_BF16 && prec != LVQ_FP16 && prec != LVQ_FP32_VALU)
        return LVQ_ERR_INVALID_ARG;
    if (nq == 0) return LVQ_OK;
    if (!q_dev || !ids_dev || !dist_dev) return LVQ_ERR_INVALID_ARG;
    if (level == LVQ_FULL && ix->f.bits2 == 0) return LVQ_ERR_INVALID_ARG;
    const Format &f = ix->f;
    if (prec == LVQ_BF16 || prec == LVQ_FP16)
        return topk_mfma(ix, q_dev, prec, nq, k, level, ids_dev, dist_dev, s, epoch);
    const bool l2 = ix->cfg.metric == LVQ_L2;
    // the inner product runs on the FP32 matrix cores when the format, k and
    // the means' c_m table allow
    // (LVQ_FP32_VALU: the vector path whatever the format)
    if (prec == LVQ_FP32 && !l2 &&
        mfma_wide_query_block(f.bits1, level == LVQ_FULL ? f.bits2 : 0, f.kpos, LVQ_FP32, k, ix->n_means,
                              ix->lds_max))
        return topk_mfma(ix, q_dev, LVQ_FP32, nq, k, level, ids_dev, dist_dev, s, epoch);
    if (l2 && ix->n_means > 1) return LVQ_ERR_UNSUPPORTED;
    const bool masked = l2 && f.kpos != f.dim;
    const int variant = !l2 ? 0 : (masked ? 2 : 1);
    const int bits2 = level == LVQ_FULL ? f.bits2 : 0;
    auto lookup = f.bits1 == 4 ? scan_kernel_b4 : scan_kernel_b8;
    // a scan processes the whole row in one round
    int shape = -1;
    for (int i = 0; i < num_tile_shapes(); ++i) {
        if (!lookup(bits2, variant, i)) continue;
        TileShape t = tile_shape(i);
        if (t.g * t.ch * t.nch < f.kchunks * 16) continue;
        if (shape < 0) { shape = i; continue; }
        TileShape b = tile_shape(shape);
        if (t.g * t.ch * t.nch < b.g * b.ch * b.nch) shape = i;
    }
    if (shape < 0) return LVQ_ERR_UNSUPPORTED;
    void *kern = lookup(bits2, variant, shape);
    const TileShape sh = tile_shape(shape);
    const int rpr = scan_rows_per_round(sh.g);
    const int capq = scan_capq(f.kpos, l2 ? 0 : ix->n_means, k, rpr, ix->lds_max);
    if (!capq) return LVQ_ERR_UNSUPPORTED;
    const size_t lds = scan_lds_bytes(f.kpos, l2 ? 0 : ix->n_means, k, capq);

    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    Workspace &w = workspace(ix, s);
    if ((rc = prep_queries(ix, w, (const float *)q_dev, nq, s))) return rc;
    const int64_t n_rows = ix->list_len;
    const int64_t qtiles = (nq + 15) / 16;
    const int64_t parts = scan_parts_fp32(ix, nq, k, n_rows);
    const int64_t rows_per_part = std::max<int64_t>(1, (n_rows + parts - 1) / parts);
    if ((rc = dev_alloc(ix, w.part, sizeof(uint64_t) * (size_t)nq * parts * k))) return rc;

    ScanArgs a;
    a.rows = P<uint8_t>(ix->rows);
    a.resid = P<uint8_t>(ix->resid);
    a.row_bytes = f.row_bytes;
    a.resid_bytes = f.resid_bytes;
    a.kchunks = f.kchunks;
    a.kpos = f.kpos;
    a.list = P<int32_t>(ix->lists[ix->list_active].buf);
    a.n_rows = n_rows;
    a.qk = P<float>(w.qk);
    a.qsum = P<float>(w.qsum);
    a.cm = P<float>(w.cm);
    a.muk = P<float>(ix->muk);
    a.kmask = P<float>(ix->kmask);
    a.q16 = nullptr;
    a.n_means = ix->n_means;
    a.nq = nq;
    a.k = k;
    a.epoch = epoch;
    a.rows_per_part = rows_per_part;
    a.n_parts = (int)parts;
    a.capq = capq;
    a.gthr = nullptr;
    a.part_keys = P<uint64_t>(w.part);
    a.err = P<uint32_t>(ix->err);
    ix->last_wg = qtiles * parts;
    ix->last_lists = 0;
    ix->last_parts = (int32_t)parts;
    if ((rc = timing_begin(ix, s))) return rc;
    hipLaunchKernelGGL(reinterpret_cast<void (*)(ScanArgs)>(kern), dim3((unsigned)qtiles, (unsigned)parts), dim3(256),
                       lds, s, a);
    LVQ_HIP(hipGetLastError());
    if ((rc = timing_end(ix, s))) return rc;
    LVQ_HIP(launch_topk_merge(a.part_keys, nq, (int)parts, k, ix->cfg.metric, ids_dev, dist_dev, s));
    return LVQ_OK;
}

extern "C" {

int lvq_topk(lvq_index *ix, const void *q_dev, int32_t prec, int64_t nq, int32_t k, int32_t level, int32_t *ids_dev,
             float *dist_dev, void *stream)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ix, s);
    if (rc) return rc;
    rc = host_topk(ix, q_dev, prec, nq, k, level, ids_dev, dist_dev, s, ix->epoch);
    if (rc == LVQ_OK && nq > 0) rc = note_query(ix, s, ix->epoch);
    if (rc == LVQ_OK) pin_after_capture(ix, s, true);
    ix->capturing = false;
    return rc;
}

}  // extern "C"

// Exhaustive top-k on the matrix cores: inner product; bf16 / fp16 queries
// at either level, FP32 queries on the wide kernel only.
static int topk_mfma(lvq_index *ix, const void *q_dev, int32_t prec, int64_t nq, int32_t k, int32_t level,
                     int32_t *ids_dev, float *dist_dev, hipStream_t s, uint32_t epoch)
{
    const Format &f = ix->f;
    if (ix->cfg.metric != LVQ_IP) return LVQ_ERR_UNSUPPORTED;
    const int bits2 = level == LVQ_FULL ? f.bits2 : 0;
    if (bits2 != 0 && bits2 != 8) return LVQ_ERR_UNSUPPORTED;   // both levels need 8-bit residual codes
    // the wide kernel (queries in LDS) when it takes the case; else the
    // register-resident kernel (16-bit queries only)
    const int qbw = mfma_wide_query_block(f.bits1, bits2, f.kpos, prec, k, ix->n_means, ix->lds_max);
    if (prec == LVQ_FP32 && !qbw) return LVQ_ERR_UNSUPPORTED;
    const int qb = qbw ? qbw : mfma_query_block(f.bits1, bits2, f.kpos);
    if (!qb) return LVQ_ERR_UNSUPPORTED;
    const int capq = qbw ? 0 : mfma_capq(qb, ix->n_means, k, ix->lds_max);
    if (!qbw && !capq) return LVQ_ERR_UNSUPPORTED;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    Workspace &w = workspace(ix, s);
    const int tq = 32 * qb;
    const int64_t qtiles = (nq + tq - 1) / tq;
    if (prec == LVQ_FP32) {
        // kernel-order FP32 queries, sum(q) and c_m, then their MFMA fragments
        if ((rc = prep_queries(ix, w, (const float *)q_dev, nq, s))) return rc;
        if ((rc = dev_alloc(ix, w.q16, (size_t)qtiles * tq * f.kpos * 4))) return rc;
        LVQ_HIP(launch_frag32(P<float>(w.qk), nq, f.kpos, f.bits1, qb, w.q16.p, s));
    } else {
        if ((rc = dev_alloc(ix, w.q16, (size_t)qtiles * tq * f.kpos * 2))) return rc;
        if ((rc = dev_alloc(ix, w.qsum, sizeof(float) * (size_t)nq))) return rc;
        if ((rc = dev_alloc(ix, w.cm, sizeof(float) * (size_t)nq * ix->n_means))) return rc;
        LVQ_HIP(launch_prep16(q_dev, nq, f.dim, f.kpos, f.bits1, qb, prec, P<int32_t>(ix->kdim), P<float>(ix->means),
                              ix->n_means, w.q16.p, P<float>(w.qsum), P<float>(w.cm), s));
    }
    const int64_t n_rows = ix->list_len;
    int64_t grid = 0;
    const int64_t parts =
        qbw ? scan_parts_wide(ix, qtiles, k, n_rows, prec, &grid) : scan_parts_mfma(ix, qtiles, k, n_rows);
    const int64_t rows_per_part = std::max<int64_t>(1, (n_rows + parts - 1) / parts);
    if ((rc = dev_alloc(ix, w.part, sizeof(uint64_t) * (size_t)nq * parts * k))) return rc;
    if ((rc = dev_alloc(ix, w.gthr, sizeof(uint32_t) * (size_t)nq))) return rc;
    if (qbw && (rc = dev_alloc(ix, w.mkeys, sizeof(uint64_t) * (size_t)grid * tq * mfma_wide_cap(k)))) return rc;
    LVQ_HIP(launch_fill_u32(P<uint32_t>(w.gthr), 0xFFFFFFFFu, nq, s));
    ScanArgs a;
    a.rows = P<uint8_t>(ix->rows);
    a.resid = P<uint8_t>(ix->resid);
    a.row_bytes = f.row_bytes;
    a.resid_bytes = f.resid_bytes;
    a.kchunks = f.kchunks;
    a.kpos = f.kpos;
    a.list = P<int32_t>(ix->lists[ix->list_active].buf);
    a.n_rows = n_rows;
    a.qk = nullptr;
    a.qsum = P<float>(w.qsum);
    a.cm = P<float>(w.cm);
    a.muk = nullptr;
    a.kmask = nullptr;
    a.q16 = w.q16.p;
    a.n_means = ix->n_means;
    a.nq = nq;
    a.k = k;
    a.epoch = epoch;
    a.rows_per_part = rows_per_part;
    a.n_parts = (int)parts;
    a.capq = capq;
    a.gthr = P<uint32_t>(w.gthr);
    a.part_keys = P<uint64_t>(w.part);
    a.err = P<uint32_t>(ix->err);
    a.mkeys = qbw ? P<uint64_t>(w.mkeys) : nullptr;
    a.mcap = qbw ? mfma_wide_cap(k) : 0;
    a.mks = qbw ? mfma_wide_sorted(k) : 0;
    ix->last_wg = qbw ? grid : (qtiles * parts + 7) / 8 * 8;
    ix->last_lists = 0;
    ix->last_parts = (int32_t)parts;
    if ((rc = timing_begin(ix, s))) return rc;
    if (qbw)
        LVQ_HIP(launch_scan_mfma_wide(a, f.bits1, bits2, prec, grid, ix->lds_max, s));
    else
        LVQ_HIP(launch_scan_mfma(a, f.bits1, bits2, prec, s));
    if ((rc = timing_end(ix, s))) return rc;
    LVQ_HIP(launch_topk_merge(a.part_keys, nq, (int)parts, k, LVQ_IP, ids_dev, dist_dev, s));
    return LVQ_OK;
}

// Per-mean member lists of stream s's workspace, rebuilt after any update.
static int ensure_members(lvq_index *ix, Workspace &w, hipStream_t s)
{
    if (w.members_version == ix->version) return LVQ_OK;
    const int M = ix->n_means;
    const int64_t n = ix->list_len;
    int rc;
    if ((rc = dev_alloc(ix, w.members, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)))) return rc;
    if ((rc = dev_alloc(ix, w.moffs, sizeof(int64_t) * (size_t)(kMaxMeans + 1)))) return rc;
    if ((rc = dev_alloc(ix, w.mcount, sizeof(uint64_t) * (size_t)kMaxMeans))) return rc;
    if ((rc = dev_alloc(ix, w.mcursor, sizeof(uint64_t) * (size_t)kMaxMeans))) return rc;
    if (n > 0) LVQ_HIP(launch_fill_i32(P<int32_t>(w.members), -1, n, s));
    LVQ_HIP(launch_members(n > 0 ? P<int32_t>(ix->lists[ix->list_active].buf) : nullptr, n, P<uint8_t>(ix->rows),
                           ix->f.row_bytes, M, P<unsigned long long>(w.mcount), P<unsigned long long>(w.mcursor),
                           P<int64_t>(w.moffs), P<int32_t>(w.members), s));
    w.members_version = ix->version;
    return LVQ_OK;
}

// Soft inverted index: route, build the probed means' candidate lists, and
// run the candidate kernel's fused top-k over them.
static int probe_topk(lvq_index *ix, const float *q_dev, int64_t nq, int32_t nprobe, int32_t k, int32_t level,
                      int32_t *probe_out_dev, int32_t *ids_dev, float *dist_dev, hipStream_t s)
{
    if (nq < 0 || nq > INT32_MAX || k < 1 || k > kMaxTopK) return LVQ_ERR_INVALID_ARG;
    if (level != LVQ_PRIMARY && level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    if (level == LVQ_FULL && ix->f.bits2 == 0) return LVQ_ERR_INVALID_ARG;
    const int M = ix->n_means;
    if (nprobe < 1 || nprobe > M) return LVQ_ERR_INVALID_ARG;
    if (nq == 0) return LVQ_OK;
    if (!q_dev || !ids_dev || !dist_dev || ix->cfg.capacity == 0) return LVQ_ERR_INVALID_ARG;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    Workspace &w = workspace(ix, s);
    if ((rc = ensure_members(ix, w, s))) return rc;
    int32_t *probe = probe_out_dev;
    if (!probe) {
        if ((rc = dev_alloc(ix, w.probe, sizeof(int32_t) * (size_t)nq * nprobe))) return rc;
        probe = P<int32_t>(w.probe);
    }
    if ((rc = dev_alloc(ix, w.qoffs, sizeof(int64_t) * (size_t)(nq + 1)))) return rc;
    LVQ_HIP(launch_route(q_dev, nq, ix->f.dim, P<float>(ix->means_t), kMaxMeans, M, nprobe, probe, s));
    LVQ_HIP(launch_probe_offsets(probe, nq, nprobe, P<int64_t>(w.moffs), P<int64_t>(w.qoffs), s));
    // the lists are the probed means' member ranges, walked in place
    return host_distances(ix, q_dev, nq, P<int64_t>(w.qoffs), nullptr, INT64_MAX, level, nullptr, k, ids_dev,
                          dist_dev, s, -1, ix->epoch, true, probe, nprobe, P<int64_t>(w.moffs),
                          P<int32_t>(w.members));
}

extern "C" {

int lvq_probe_topk(lvq_index *ix, const float *q_dev, int64_t nq, int32_t nprobe, int32_t k, int32_t level,
                   int32_t *probe_out_dev, int32_t *ids_dev, float *dist_dev, void *stream)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ix, s);
    if (rc) return rc;
    rc = probe_topk(ix, q_dev, nq, nprobe, k, level, probe_out_dev, ids_dev, dist_dev, s);
    if (rc == LVQ_OK && nq > 0) rc = note_query(ix, s, ix->epoch);
    if (rc == LVQ_OK) pin_after_capture(ix, s, true);
    ix->capturing = false;
    return rc;
}

int lvq_graph_search(lvq_index *ix, const float *q_dev, int64_t nq, const int32_t *graph_dev, int32_t degree,
                     const int32_t *entries_dev, int32_t n_entries, int32_t window, int32_t k, int32_t *ids_dev,
                     float *dist_dev, int32_t *explored_dev, void *stream)
{
    if (!ix || nq < 0 || nq > INT32_MAX || degree < 1 || degree > 64 || n_entries < 1 || n_entries > 64 ||
        k < 1 || window < k || window > 256)
        return LVQ_ERR_INVALID_ARG;
    if (nq > 0 && (!q_dev || !graph_dev || !entries_dev || !ids_dev || !dist_dev)) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    if (ix->cfg.capacity == 0) return LVQ_ERR_INVALID_ARG;
    const Format &f = ix->f;
    if (graph_lds_bytes(f.kpos, window, degree) > ix->lds_max) return LVQ_ERR_UNSUPPORTED;
    if (nq == 0) return LVQ_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ix, s);
    if (rc) return rc;
    if ((rc = order_after_updates(ix, s)) == LVQ_OK) {
        Workspace &w = workspace(ix, s);
        if ((rc = prep_queries(ix, w, q_dev, nq, s)) == LVQ_OK) {
            GraphLaunch l;
            l.rows = P<uint8_t>(ix->rows);
            l.row_bytes = f.row_bytes;
            l.kchunks = f.kchunks;
            l.kpos = f.kpos;
            l.bits1 = f.bits1;
            l.metric = ix->cfg.metric;
            l.capacity = ix->cfg.capacity;
            l.qk = P<float>(w.qk);
            l.qsum = P<float>(w.qsum);
            l.cm = P<float>(w.cm);
            l.muk = P<float>(ix->muk);
            l.kmask = P<float>(ix->kmask);
            l.n_means = ix->n_means;
            l.nq = nq;
            l.graph = graph_dev;
            l.degree = degree;
            l.entries = entries_dev;
            l.n_entries = n_entries;
            l.window = window;
            l.k = k;
            l.epoch = ix->epoch;
            l.ids = ids_dev;
            l.dist = dist_dev;
            l.explored = explored_dev;
            l.err = P<uint32_t>(ix->err);
            if ((rc = timing_begin(ix, s)) == LVQ_OK) {
                hipError_t e = launch_graph_search(l, s);
                rc = e == hipSuccess ? timing_end(ix, s) : map_hip(e);
            }
        }
    }
    if (rc == LVQ_OK) rc = note_query(ix, s, ix->epoch);
    if (rc == LVQ_OK) pin_after_capture(ix, s, false);
    ix->capturing = false;
    return rc;
}

int lvq_retire_means(lvq_index *ix, const int32_t *ids_host, int32_t n, void *stream)
{
    if (!ix || n < 0 || (n > 0 && !ids_host)) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> next = ix->retired;
    for (int32_t i = 0; i < n; ++i) {
        if (ids_host[i] < 0 || ids_host[i] >= ix->n_means) return LVQ_ERR_INVALID_ARG;
        next[ids_host[i]] = 1;
    }
    int active = 0;
    for (int m = 0; m < ix->n_means; ++m) active += !next[m];
    if (active == 0) return LVQ_ERR_INVALID_ARG;
    int rc = begin_call(ix, s);
    if (rc) return rc;
    if (ix->capturing) {
        ix->capturing = false;
        return LVQ_ERR_UNSUPPORTED;
    }
    if ((rc = order_after_updates(ix, s))) return rc;
    ix->retired = next;
    std::vector<uint8_t> act(kMaxMeans);
    for (int m = 0; m < kMaxMeans; ++m) act[m] = !ix->retired[m];
    LVQ_HIP(hipMemcpyAsync(ix->mean_active.p, act.data(), kMaxMeans, hipMemcpyHostToDevice, s));
    LVQ_HIP(hipStreamSynchronize(s));   // the host flags must outlive the copy
    return note_update(ix, s);
}

int lvq_add_means(lvq_index *ix, const float *means_host, int32_t n, int32_t *ids_out_host, void *stream)
{
    if (!ix || !means_host || !ids_out_host || n < 1 || n > kMaxMeans) return LVQ_ERR_INVALID_ARG;
    const Format &f = ix->f;
    const int d = f.dim;
    if (!finite_host(means_host, (size_t)n * d)) return LVQ_ERR_NONFINITE;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ix, s);
    if (rc) return rc;
    if (ix->capturing) {
        ix->capturing = false;
        return LVQ_ERR_UNSUPPORTED;
    }
    if ((rc = order_after_updates(ix, s))) return rc;
    // rows per id over the occupied slots: a retired id none refers to is free
    std::vector<uint64_t> cnt(kMaxMeans, 0);
    if (ix->list_len > 0) {
        LVQ_HIP(launch_mean_counts(P<int32_t>(ix->lists[ix->list_active].buf), ix->list_len, P<uint8_t>(ix->rows),
                                   f.row_bytes, ix->n_means, P<unsigned long long>(ix->mean_counts), s));
        LVQ_HIP(hipMemcpyAsync(cnt.data(), ix->mean_counts.p, sizeof(uint64_t) * ix->n_means,
                               hipMemcpyDeviceToHost, s));
        LVQ_HIP(hipStreamSynchronize(s));
    }
    std::vector<int32_t> ids;
    for (int m = 0; m < ix->n_means && (int)ids.size() < n; ++m)
        if (ix->retired[m] && cnt[m] == 0) ids.push_back(m);
    int next_new = ix->n_means;
    while ((int)ids.size() < n && next_new < kMaxMeans) ids.push_back(next_new++);
    if ((int)ids.size() < n) return LVQ_ERR_CAPACITY;
    std::vector<int32_t> kd(f.kpos);
    kernel_order_dims(f, kd.data());
    std::vector<float> col((size_t)d * n), mk((size_t)n * f.kpos, 0.0f);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < d; ++j) col[(size_t)i * d + j] = means_host[(size_t)i * d + j];
        for (int t = 0; t < f.kpos; ++t)
            if (kd[t] >= 0) mk[(size_t)i * f.kpos + t] = means_host[(size_t)i * d + kd[t]];
    }
    for (int i = 0; i < n; ++i) {
        const int m = ids[i];
        LVQ_HIP(hipMemcpyAsync(P<float>(ix->means) + (size_t)m * d, means_host + (size_t)i * d, sizeof(float) * d,
                               hipMemcpyHostToDevice, s));
        // column m of the transposed table: d values with a stride of kMaxMeans
        LVQ_HIP(hipMemcpy2DAsync(P<float>(ix->means_t) + m, sizeof(float) * kMaxMeans, col.data() + (size_t)i * d,
                                 sizeof(float), sizeof(float), d, hipMemcpyHostToDevice, s));
        LVQ_HIP(hipMemcpyAsync(P<float>(ix->muk) + (size_t)m * f.kpos, mk.data() + (size_t)i * f.kpos,
                               sizeof(float) * f.kpos, hipMemcpyHostToDevice, s));
        ix->retired[m] = 0;
    }
    ix->n_means = std::max(ix->n_means, next_new);
    std::vector<uint8_t> act(kMaxMeans);
    for (int m = 0; m < kMaxMeans; ++m) act[m] = !ix->retired[m];
    LVQ_HIP(hipMemcpyAsync(ix->mean_active.p, act.data(), kMaxMeans, hipMemcpyHostToDevice, s));
    if ((rc = note_update(ix, s))) return rc;
    LVQ_HIP(hipStreamSynchronize(s));   // the host sources must outlive the copies
    for (int i = 0; i < n; ++i) ids_out_host[i] = ids[i];
    return LVQ_OK;
}

int lvq_mean_members(lvq_index *ix, const int32_t *mean_ids_host, int32_t n, int64_t *offsets_host,
                     int32_t *slots_dev, int64_t cap, void *stream)
{
    if (!ix || n < 0 || (n > 0 && (!mean_ids_host || !offsets_host)) || cap < 0 || (cap > 0 && !slots_dev))
        return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    for (int32_t i = 0; i < n; ++i)
        if (mean_ids_host[i] < 0 || mean_ids_host[i] >= ix->n_means) return LVQ_ERR_INVALID_ARG;
    if (offsets_host) offsets_host[0] = 0;
    if (n == 0) return LVQ_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ix, s);
    if (rc) return rc;
    if (ix->capturing) {
        ix->capturing = false;
        return LVQ_ERR_UNSUPPORTED;
    }
    if ((rc = order_after_updates(ix, s))) return rc;
    Workspace &w = workspace(ix, s);
    if ((rc = ensure_members(ix, w, s))) return rc;
    // requested ids and, later, the output offsets share the probe buffer
    if ((rc = dev_alloc(ix, w.probe, sizeof(int32_t) * (size_t)n))) return rc;
    if ((rc = dev_alloc(ix, w.qoffs, sizeof(int64_t) * (size_t)(n + 1)))) return rc;
    if ((rc = dev_alloc(ix, w.qids, sizeof(uint64_t) * (size_t)n))) return rc;
    LVQ_HIP(hipMemcpyAsync(w.probe.p, mean_ids_host, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    const uint32_t epoch = ix->epoch;
    unsigned long long *counts = P<unsigned long long>(w.qids);
    LVQ_HIP(launch_members_live(P<int32_t>(w.probe), n, P<int64_t>(w.moffs), P<int32_t>(w.members), P<uint8_t>(ix->rows),
                                ix->f.row_bytes, epoch, nullptr, nullptr, counts, s));
    std::vector<uint64_t> c(n);
    LVQ_HIP(hipMemcpyAsync(c.data(), counts, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s));
    LVQ_HIP(hipStreamSynchronize(s));
    for (int32_t i = 0; i < n; ++i) offsets_host[i + 1] = offsets_host[i] + (int64_t)c[i];
    if (offsets_host[n] > cap) return LVQ_ERR_CAPACITY;
    LVQ_HIP(hipMemcpyAsync(w.qoffs.p, offsets_host, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    LVQ_HIP(launch_members_live(P<int32_t>(w.probe), n, P<int64_t>(w.moffs), P<int32_t>(w.members), P<uint8_t>(ix->rows),
                                ix->f.row_bytes, epoch, P<int64_t>(w.qoffs), slots_dev, counts, s));
    LVQ_HIP(hipStreamSynchronize(s));   // offsets_host is read by the copy above
    ix->capturing = false;
    return LVQ_OK;
}

}  // extern "C"

int lvq::host_reserve(lvq_index *ix, hipStream_t s, int64_t max_nq, int32_t k_first, int32_t prec,
                      int32_t scan_level, int32_t k_rerank, int32_t rerank_level)
{
    if (max_nq < 1 || max_nq > INT32_MAX || k_first < 1 || k_first > kMaxTopK || k_rerank < 0 ||
        k_rerank > kMaxTopK)
        return LVQ_ERR_INVALID_ARG;
    if (scan_level != LVQ_PRIMARY && scan_level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    if (k_rerank > 0 && rerank_level != LVQ_PRIMARY && rerank_level != LVQ_FULL) return LVQ_ERR_INVALID_ARG;
    const Format &f = ix->f;
    const int64_t n_rows = ix->cfg.capacity;   // the part counts grow with the rows scanned
    size_t qk = 0, part = 0, q16 = 0, gthr = 0, order = 0, mkeys = 0;
    const size_t qsum = sizeof(float) * (size_t)max_nq;
    const size_t cm = sizeof(float) * (size_t)max_nq * kMaxMeans;   // any mean count the index may reach
    if (prec == LVQ_FP32 || k_rerank > 0) qk = sizeof(float) * (size_t)max_nq * f.kpos;
    if (prec == LVQ_FP32) {
        for (int64_t nq = 1; nq <= max_nq; ++nq)
            part = std::max(part, sizeof(uint64_t) * (size_t)(nq * scan_parts_fp32(ix, nq, k_first, n_rows) * k_first));
        // the FP32 matrix-core scan (inner product; its query block does not
        // depend on the mean count, which only decides whether the c_m table
        // fits)
        const int qbf = ix->cfg.metric == LVQ_IP
                            ? mfma_wide_query_block(f.bits1, scan_level == LVQ_FULL ? f.bits2 : 0, f.kpos, LVQ_FP32,
                                                    k_first, 1, ix->lds_max)
                            : 0;
        if (qbf) {
            const int64_t tq = 32 * qbf;
            q16 = (size_t)((max_nq + tq - 1) / tq) * tq * f.kpos * 4;
            for (int64_t nq = 1; nq <= max_nq; ++nq) {
                int64_t grid = 0;
                const int64_t parts = scan_parts_wide(ix, (nq + tq - 1) / tq, k_first, n_rows, LVQ_FP32, &grid);
                part = std::max(part, sizeof(uint64_t) * (size_t)(nq * parts * k_first));
                mkeys = std::max(mkeys, sizeof(uint64_t) * (size_t)grid * tq * mfma_wide_cap(k_first));
            }
            gthr = sizeof(uint32_t) * (size_t)max_nq;
        }
    } else {
        const int bits2 = scan_level == LVQ_FULL ? f.bits2 : 0;
        const int qbw = mfma_wide_query_block(f.bits1, bits2, f.kpos, prec, k_first, kMaxMeans, ix->lds_max);
        const int qb = qbw ? qbw : mfma_query_block(f.bits1, bits2, f.kpos);
        if (!qb) return LVQ_ERR_UNSUPPORTED;
        // the wide kernel when it takes any mean count the index may reach;
        // else reserve for both kernels (the register-resident one serves
        // what the wide one cannot)
        const int qbw_any = mfma_wide_query_block(f.bits1, bits2, f.kpos, prec, k_first, 1, ix->lds_max);
        const int qbo = mfma_query_block(f.bits1, bits2, f.kpos);
        for (int kind = 0; kind < 2; ++kind) {
            const bool wide = kind == 0;
            const int q = wide ? qbw_any : (qbw ? 0 : qbo);
            if (!q) continue;
            const int64_t tq = 32 * q;
            q16 = std::max(q16, (size_t)((max_nq + tq - 1) / tq) * tq * f.kpos * 2);
            for (int64_t nq = 1; nq <= max_nq; ++nq) {
                const int64_t qtiles = (nq + tq - 1) / tq;
                int64_t grid = 0;
                const int64_t parts = wide ? scan_parts_wide(ix, qtiles, k_first, n_rows, prec, &grid)
                                           : scan_parts_mfma(ix, qtiles, k_first, n_rows);
                part = std::max(part, sizeof(uint64_t) * (size_t)(nq * parts * k_first));
                if (wide) mkeys = std::max(mkeys, sizeof(uint64_t) * (size_t)grid * tq * mfma_wide_cap(k_first));
            }
        }
        gthr = sizeof(uint32_t) * (size_t)max_nq;
    }
    if (k_rerank > 0) order = sizeof(int32_t) * (size_t)max_nq;
    Workspace &w = workspace(ix, s);
    int rc;
    if (qk && (rc = dev_alloc(ix, w.qk, qk))) return rc;
    if ((rc = dev_alloc(ix, w.qsum, qsum))) return rc;
    if ((rc = dev_alloc(ix, w.cm, cm))) return rc;
    if (part && (rc = dev_alloc(ix, w.part, part))) return rc;
    if (q16 && (rc = dev_alloc(ix, w.q16, q16))) return rc;
    if (gthr && (rc = dev_alloc(ix, w.gthr, gthr))) return rc;
    if (mkeys && (rc = dev_alloc(ix, w.mkeys, mkeys))) return rc;
    if (order && (rc = dev_alloc(ix, w.order, order))) return rc;
    if (k_rerank > 0 && (rc = dev_alloc(ix, w.queue, 64))) return rc;
    return LVQ_OK;
}

extern "C" {

int lvq_read_rows(lvq_index *ix, const int32_t *slots_dev, int64_t n, uint8_t *rows_dev, uint8_t *resid_dev,
                  void *stream)
{
    if (!ix || n < 0 || (n > 0 && (!slots_dev || !rows_dev))) return LVQ_ERR_INVALID_ARG;
    if (n == 0) return LVQ_OK;
    std::lock_guard<std::mutex> lk(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    LVQ_HIP(launch_gather_rows(store_args(ix), slots_dev, n, rows_dev, resid_dev, s));
    return LVQ_OK;
}

int lvq_bw_stream(const void *src_dev, int64_t bytes, uint32_t *sink_dev, void *stream)
{
    if (!sink_dev || bytes < 0 || (bytes & 15) || (bytes > 0 && (!src_dev || ((uintptr_t)src_dev & 15))))
        return LVQ_ERR_INVALID_ARG;
    LVQ_HIP(launch_bw_stream(src_dev, bytes / 16, sink_dev, (hipStream_t)stream));
    return LVQ_OK;
}

int lvq_bw_gather(lvq_index *ix, const int32_t *ids_dev, int64_t n, int32_t level, uint32_t *sink_dev, void *stream)
{
    if (!ix || !sink_dev || n < 0 || (n > 0 && !ids_dev) || (level != LVQ_PRIMARY && level != LVQ_FULL))
        return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    const Format &f = ix->f;
    if (level == LVQ_FULL && !f.bits2) return LVQ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int rc = order_after_updates(ix, s);
    if (rc) return rc;
    const bool full = level == LVQ_FULL;
    LVQ_HIP(launch_bw_gather(P<uint8_t>(ix->rows), f.row_bytes, (kHeaderBytes + 16 * f.kchunks) / 16,
                             full ? P<uint8_t>(ix->resid) : nullptr, f.resid_bytes, f.resid_bytes / 16, ids_dev, n,
                             ix->cfg.capacity, sink_dev, s));
    return LVQ_OK;
}

int lvq_get_stats(lvq_index *ix, lvq_stats *out)
{
    if (!ix || !out) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    out->capacity = ix->cfg.capacity;
    out->free_slots = ix->free_top;
    out->live_estimate = ix->cfg.capacity - ix->free_top;
    out->device_bytes = ix->device_bytes;
    out->n_means = ix->n_means;
    out->row_bytes = ix->f.row_bytes;
    out->resid_bytes = ix->f.resid_bytes;
    out->code_positions = ix->f.npos;
    out->epoch = ix->epoch;
    out->last_workgroups = ix->last_wg;
    out->last_lists = ix->last_lists;
    out->last_parts = ix->last_parts;
    return LVQ_OK;
}

int lvq_set_timing(lvq_index *ix, int enable)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    ix->timing = enable != 0;
    return LVQ_OK;
}

int lvq_kernel_time(lvq_index *ix, double *ms_out, int64_t *launches_out)
{
    if (!ix || !ms_out) return LVQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ix->mu);
    double total = 0.0;
    for (auto &p : ix->tev) {
        LVQ_HIP(hipEventSynchronize(p.second));
        float ms = 0.0f;
        LVQ_HIP(hipEventElapsedTime(&ms, p.first, p.second));
        total += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (launches_out) *launches_out = (int64_t)ix->tev.size();
    ix->tev.clear();
    *ms_out = total;
    return LVQ_OK;
}

int lvq_sync(lvq_index *ix, void *stream)
{
    if (!ix) return LVQ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    LVQ_HIP(hipStreamSynchronize(s));
    uint32_t e = 0;
    {
        std::lock_guard<std::mutex> lk(ix->mu);
        LVQ_HIP(hipMemcpy(&e, ix->err.p, sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (e) LVQ_HIP(hipMemset(ix->err.p, 0, sizeof(uint32_t)));
    }
    if (e & kErrNonFinite) return LVQ_ERR_NONFINITE;
    if (e & kErrBadSlot) return LVQ_ERR_BAD_SLOT;
    if (e & (kErrBadOffsets | kErrOverflow)) return LVQ_ERR_INVALID_ARG;
    return LVQ_OK;
}

int lvq_mean(const float *x_dev, int64_t n, int32_t dim, float *mean_out_dev, void *stream)
{
    if (!x_dev || !mean_out_dev || n < 1 || dim < 1) return LVQ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nchunks = (n + 4095) / 4096;
    double *scratch = nullptr;
    LVQ_HIP(hipMallocAsync((void **)&scratch, sizeof(double) * (size_t)nchunks * dim, s));
    hipError_t e = launch_mean(x_dev, n, dim, mean_out_dev, scratch, s);
    hipError_t e2 = hipFreeAsync(scratch, s);
    LVQ_HIP(e);
    LVQ_HIP(e2);
    return LVQ_OK;
}

int lvq_kmeans(const float *x_dev, int64_t n, int32_t dim, int32_t k, const int64_t *init_idx_host, int32_t iters,
               float *means_out_dev, void *stream)
{
    if (!x_dev || !means_out_dev || !init_idx_host || n < 1 || dim < 1 || k < 1 || k > n || iters < 0)
        return LVQ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    for (int m = 0; m < k; ++m) {
        if (init_idx_host[m] < 0 || init_idx_host[m] >= n) return LVQ_ERR_INVALID_ARG;
        LVQ_HIP(hipMemcpyAsync(means_out_dev + (size_t)m * dim, x_dev + (size_t)init_idx_host[m] * dim,
                               sizeof(float) * dim, hipMemcpyDeviceToDevice, s));
    }
    int32_t *assign = nullptr;
    LVQ_HIP(hipMallocAsync((void **)&assign, sizeof(int32_t) * (size_t)n, s));
    hipError_t e = hipSuccess;
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
        e = launch_kmeans_assign(x_dev, n, dim, means_out_dev, k, assign, s);
        if (e == hipSuccess) e = launch_kmeans_update(x_dev, n, dim, assign, k, means_out_dev, s);
    }
    hipError_t e2 = hipFreeAsync(assign, s);
    LVQ_HIP(e);
    LVQ_HIP(e2);
    return LVQ_OK;
}

}  // extern "C"

// ---- graph construction (App. A) ---------------------------------------------

namespace {

int graph_device_lds(size_t *out)
{
    int dev = 0;
    hipDeviceProp_t prop;
    LVQ_HIP(hipGetDevice(&dev));
    LVQ_HIP(hipGetDeviceProperties(&prop, dev));
    *out = prop.sharedMemPerBlock;
    return LVQ_OK;
}

int graph_kernel_error(uint32_t e)
{
    if (e & kErrBadSlot) return LVQ_ERR_BAD_SLOT;
    if (e & kErrBadOffsets) return LVQ_ERR_INVALID_ARG;
    return LVQ_OK;   // a search that stopped at the seen-set capacity still yields candidates
}

// Device buffers of one construction call, released on every exit path.
struct GraphScratch {
    std::vector<void *> bufs;
    hipStream_t s;
    explicit GraphScratch(hipStream_t st) : s(st) {}
    template <typename T>
    int alloc(T **p, size_t count)
    {
        *p = nullptr;
        void *q = nullptr;
        LVQ_HIP(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
        bufs.push_back(q);
        *p = static_cast<T *>(q);
        return LVQ_OK;
    }
    ~GraphScratch()
    {
        (void)hipStreamSynchronize(s);
        for (void *q : bufs) (void)hipFree(q);
    }
};

// The update routine of graph construction (App. A) for the nodes of
// `order`, `passes` times (alpha = 1 first when there are two passes):
// their rows are cleared, then batch by batch each node's window nearest
// nodes found from `entry` are pruned into its out-neighbours and it joins
// their out-neighbours (pruned on overflow).  A batch is at most max_batch
// nodes and, in the first pass, at most the number already in the graph
// (in_graph before the first node, plus the nodes inserted so far).
int graph_update(const float *x_dev, int64_t n, int dim, int metric, const std::vector<int32_t> &order,
                 int64_t in_graph, int R, int window, float alpha, int passes, int32_t entry, int32_t max_batch,
                 int32_t *graph_dev, hipStream_t s)
{
    if (dim < 1 || dim > kGraphMaxDim || (metric != LVQ_L2 && metric != LVQ_IP) || R < 1 || R > kGraphMaxDegree ||
        window < R || window > 256 || !(alpha > 0.0f) || !std::isfinite(alpha) || max_batch < 1)
        return LVQ_ERR_INVALID_ARG;
    size_t lds_max = 0;
    int rc = graph_device_lds(&lds_max);
    if (rc) return rc;
    if (graph_lds_bytes(dim, window, R) > lds_max) return LVQ_ERR_UNSUPPORTED;
    const int64_t count = (int64_t)order.size();
    if (count == 0) return LVQ_OK;
    const int64_t B = std::min<int64_t>(max_batch, count);
    GraphScratch sc(s);
    int32_t *order_d, *res, *cnt, *rev, *touched, *ntouched, *entry_d;
    int64_t *offs, *scan;
    uint32_t *err;
    const int64_t nb = (n + 2047) / 2048;
    if ((rc = sc.alloc(&order_d, (size_t)count)) || (rc = sc.alloc(&res, (size_t)(B * window))) ||
        (rc = sc.alloc(&cnt, (size_t)n)) || (rc = sc.alloc(&offs, (size_t)n + 1)) ||
        (rc = sc.alloc(&scan, (size_t)nb + 1)) || (rc = sc.alloc(&rev, (size_t)(B * R))) ||
        (rc = sc.alloc(&touched, (size_t)(B * R))) || (rc = sc.alloc(&ntouched, 1)) ||
        (rc = sc.alloc(&entry_d, 1)) || (rc = sc.alloc(&err, 1)))
        return rc;
    LVQ_HIP(hipMemcpyAsync(order_d, order.data(), sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice, s));
    LVQ_HIP(hipMemcpyAsync(entry_d, &entry, sizeof(int32_t), hipMemcpyHostToDevice, s));
    LVQ_HIP(launch_graph_clear_rows(graph_dev, R, n, nullptr, order_d, count, s));
    LVQ_HIP(launch_fill_i32(cnt, 0, n, s));
    LVQ_HIP(launch_fill_u32(err, 0, 1, s));
    for (int pass = 0; pass < passes; ++pass) {
        const float a = (passes == 2 && pass == 0) ? 1.0f : alpha;
        for (int64_t b = 0; b < count;) {
            const int64_t now = pass == 0 ? in_graph + b : n;
            const int64_t bs = std::min<int64_t>({B, std::max<int64_t>(1, now), count - b});
            const int32_t *nodes = order_d + b;
            GraphLaunch g{};
            g.capacity = n;
            g.kpos = dim;
            g.metric = metric;
            g.n_means = 1;
            g.nq = bs;
            g.graph = graph_dev;
            g.degree = R;
            g.entries = entry_d;
            g.n_entries = 1;
            g.window = window;
            g.k = window;
            g.ids = res;
            g.err = err;
            g.xf = x_dev;
            g.dim = dim;
            g.qnodes = nodes;
            LVQ_HIP(launch_graph_search(g, s));
            PruneLaunch p{};
            p.xf = x_dev;
            p.dim = dim;
            p.metric = metric;
            p.n = n;
            p.nodes = nodes;
            p.m = bs;
            p.cids = res;
            p.cstride = window;
            p.always = 1;
            p.graph = graph_dev;
            p.R = R;
            p.alpha = a;
            p.err = err;
            LVQ_HIP(launch_graph_prune(p, s));
            LVQ_HIP(launch_reverse_edges(graph_dev, R, nodes, bs, n, cnt, offs, scan, rev, touched, ntouched, s));
            int32_t nt = 0;
            LVQ_HIP(hipMemcpyAsync(&nt, ntouched, sizeof(nt), hipMemcpyDeviceToHost, s));
            LVQ_HIP(hipStreamSynchronize(s));
            PruneLaunch r = p;
            r.nodes = touched;
            r.m = nt;
            r.coffs = offs;
            r.by_node = 1;
            r.cids = rev;
            r.cstride = 0;
            r.always = 0;
            LVQ_HIP(launch_graph_prune(r, s));
            b += bs;
        }
    }
    uint32_t herr = 0;
    LVQ_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    LVQ_HIP(hipStreamSynchronize(s));
    return graph_kernel_error(herr);
}

}  // namespace

extern "C" {

int lvq_graph_prune(const float *x_dev, int64_t n, int32_t dim, int32_t metric, const int32_t *nodes_dev, int64_t m,
                    const int64_t *cand_offsets_dev, const int32_t *cand_ids_dev, int32_t degree, float alpha,
                    int32_t *graph_dev, void *stream)
{
    if (n < 1 || n > INT32_MAX || dim < 1 || dim > kGraphMaxDim || (metric != LVQ_L2 && metric != LVQ_IP) || m < 0 ||
        m > INT32_MAX || degree < 1 || degree > kGraphMaxDegree || !(alpha > 0.0f) || !std::isfinite(alpha))
        return LVQ_ERR_INVALID_ARG;
    if (m == 0) return LVQ_OK;
    if (!x_dev || !nodes_dev || !cand_offsets_dev || !cand_ids_dev || !graph_dev) return LVQ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    GraphScratch sc(s);
    uint32_t *err = nullptr;
    int rc = sc.alloc(&err, 1);
    if (rc) return rc;
    LVQ_HIP(launch_fill_u32(err, 0, 1, s));
    PruneLaunch l{};
    l.xf = x_dev;
    l.dim = dim;
    l.metric = metric;
    l.n = n;
    l.nodes = nodes_dev;
    l.m = m;
    l.coffs = cand_offsets_dev;
    l.by_node = 0;
    l.cids = cand_ids_dev;
    l.always = 1;
    l.graph = graph_dev;
    l.R = degree;
    l.alpha = alpha;
    l.err = err;
    LVQ_HIP(launch_graph_prune(l, s));
    uint32_t herr = 0;
    LVQ_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    LVQ_HIP(hipStreamSynchronize(s));
    return graph_kernel_error(herr);
}

int lvq_graph_build(const float *x_dev, int64_t n, int32_t dim, int32_t metric, int64_t first, int32_t degree,
                    int32_t window, float alpha, int32_t passes, int32_t entry, int32_t max_batch, int32_t *graph_dev,
                    void *stream)
{
    if (!x_dev || !graph_dev || n < 1 || n > INT32_MAX || first < 0 || first > n || passes < 1 || passes > 2 ||
        entry < 0 || entry >= n || (first > 0 && entry >= first))
        return LVQ_ERR_INVALID_ARG;
    std::vector<int32_t> order;
    order.reserve((size_t)(n - first));
    if (first == 0) {
        order.push_back(entry);
        for (int64_t v = 0; v < n; ++v)
            if (v != entry) order.push_back((int32_t)v);
    } else {
        for (int64_t v = first; v < n; ++v) order.push_back((int32_t)v);
    }
    return graph_update(x_dev, n, dim, metric, order, first, degree, window, alpha, passes, entry, max_batch,
                        graph_dev, (hipStream_t)stream);
}

int lvq_graph_insert(const float *x_dev, int64_t n, int32_t dim, int32_t metric, const int32_t *nodes_host,
                     int64_t m, int32_t degree, int32_t window, float alpha, int32_t entry, int32_t max_batch,
                     int32_t *graph_dev, void *stream)
{
    if (!x_dev || !graph_dev || n < 1 || n > INT32_MAX || m < 0 || m > n || (m > 0 && !nodes_host) || entry < 0 ||
        entry >= n)
        return LVQ_ERR_INVALID_ARG;
    std::vector<int32_t> order(nodes_host, nodes_host + m);
    std::vector<int32_t> sorted = order;
    std::sort(sorted.begin(), sorted.end());
    for (size_t i = 0; i < sorted.size(); ++i)
        if (sorted[i] < 0 || sorted[i] >= n || sorted[i] == entry || (i > 0 && sorted[i] == sorted[i - 1]))
            return LVQ_ERR_INVALID_ARG;
    return graph_update(x_dev, n, dim, metric, order, n - m, degree, window, alpha, 1, entry, max_batch, graph_dev,
                        (hipStream_t)stream);
}

int lvq_graph_delete(const float *x_dev, int64_t n, int32_t dim, int32_t metric, const uint8_t *deleted_dev,
                     int32_t degree, float alpha, int32_t *graph_dev, void *stream)
{
    if (!x_dev || !deleted_dev || !graph_dev || n < 1 || n > INT32_MAX || dim < 1 || dim > kGraphMaxDim ||
        (metric != LVQ_L2 && metric != LVQ_IP) || degree < 1 || degree > kGraphMaxDegree || !(alpha > 0.0f) ||
        !std::isfinite(alpha))
        return LVQ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    GraphScratch sc(s);
    int32_t *affected, *count;
    uint32_t *err;
    int rc;
    if ((rc = sc.alloc(&affected, (size_t)n)) || (rc = sc.alloc(&count, 1)) || (rc = sc.alloc(&err, 1))) return rc;
    LVQ_HIP(launch_fill_u32(err, 0, 1, s));
    LVQ_HIP(launch_graph_affected(graph_dev, degree, n, deleted_dev, affected, count, s));
    int32_t na = 0;
    LVQ_HIP(hipMemcpyAsync(&na, count, sizeof(na), hipMemcpyDeviceToHost, s));
    LVQ_HIP(hipStreamSynchronize(s));
    PruneLaunch p{};
    p.xf = x_dev;
    p.dim = dim;
    p.metric = metric;
    p.n = n;
    p.nodes = affected;
    p.m = na;
    p.always = 0;
    p.graph = graph_dev;
    p.R = degree;
    p.alpha = alpha;
    p.err = err;
    p.deleted = deleted_dev;
    LVQ_HIP(launch_graph_prune(p, s));
    LVQ_HIP(launch_graph_clear_rows(graph_dev, degree, n, deleted_dev, nullptr, 0, s));
    uint32_t herr = 0;
    LVQ_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    LVQ_HIP(hipStreamSynchronize(s));
    return graph_kernel_error(herr);
}

}  // extern "C"
