// lvq_index.h -- the library-owned index object and the host-side entry
// points shared by lvq_host.hip (the C ABI) and lvq_serve.hip (the request
// server).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "lvq_internal.h"

namespace lvq {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool pinned = false;   // read by a captured HIP graph: never freed or grown while the index lives
};

// Scratch of one host_distances call given by the caller (the allocation-free
// entry point): query tables (nq x kpos), sums of q (nq), mean terms
// (nq x n_means), list order (nq) and the persistent launch's work counter.
struct DistScratch {
    float *qk, *qsum, *cm;
    int32_t *order, *queue;
};

// Per-stream scratch of the query entry points.
struct Workspace {
    DevBuf qk, qsum, cm, order, queue, part, q16, gthr, mkeys;
    // soft inverted index: this stream's per-mean member lists (built at
    // store version members_version) and per-call routing / candidate lists
    DevBuf members, moffs, mcount, mcursor, probe, qoffs, qids;
    uint64_t members_version = ~0ull;
};

// A query launch that may still be reading the store, the epoch it reads,
// and its launch sequence number.
struct InFlight {
    uint32_t epoch;
    uint64_t seq;
    hipEvent_t ev;
};

// A list of occupied slots the exhaustive scans walk.  The active list grows
// by appends (inserts); consolidation writes a compacted list into another
// buffer and retires the active one, which is reused once every query
// launched before the switch (seq <= retire_seq) has completed.
struct SlotList {
    DevBuf buf;
    uint64_t retire_seq = 0;
    bool captured = false;   // a captured scan reads it: never reused for another list
};

}  // namespace lvq

struct lvq_index {
    lvq_config cfg;
    lvq::Format f;
    int device = 0;
    int n_cu = 256;
    size_t lds_max = 65536;    // LDS bytes one workgroup may allocate
    int n_means = 0;
    // device store
    lvq::DevBuf means, means_t, muk, kmask, kdim, rows, resid, stack, err, scratch;
    lvq::DevBuf mean_active, mean_counts;   // kMaxMeans flags (0 = retired); counts per mean id
    std::vector<uint8_t> retired;           // host copy of the retired flags
    int64_t free_top = 0;   // host view of the free-slot stack top
    uint32_t epoch = 1;
    std::vector<lvq::SlotList> lists;
    int list_active = -1;
    int64_t list_len = 0;   // entries of the active list
    uint64_t query_seq = 0; // launches recorded as in flight so far
    uint64_t version = 0;   // store updates so far (any insert, delete, consolidation, means change)
    int64_t device_bytes = 0;
    std::map<hipStream_t, lvq::Workspace> ws;
    std::deque<lvq::InFlight> inflight;
    std::vector<hipEvent_t> spare_events;
    hipEvent_t update_ev = nullptr;   // recorded after the latest store update
    hipStream_t update_stream = nullptr;
    bool have_update = false;
    std::mutex mu;                    // guards every field above
    int cand_shape[2][2] = {{-1, -1}, {-1, -1}};   // tuned [level][topk]
    bool capturing = false;   // the current call's stream is capturing a HIP graph
    bool timing = false;
    int64_t last_wg = 0, last_lists = 0;   // shape of the latest similarity launch (lvq_stats)
    int32_t last_parts = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
};

namespace lvq {

// The functions below expect the caller to hold ix->mu.

// Record whether `s` is capturing a HIP graph (captured calls allocate
// nothing and keep no in-flight record).
int host_begin_call(lvq_index *ix, hipStream_t s);

// Exhaustive top-k over the slots live at `epoch` (lvq_topk's semantics);
// records no in-flight entry (host_note_query does).
int host_topk(lvq_index *ix, const void *q_dev, int32_t prec, int64_t nq, int32_t k, int32_t level,
              int32_t *ids_dev, float *dist_dev, hipStream_t s, uint32_t epoch);

// Candidate-list similarities (lvq_distances' semantics) with the fused top-k
// filtered at `epoch`.  neg_empty: a negative slot marks an empty list entry
// (no error, left out of the top-k) instead of an invalid one.  list_means
// (nq x list_nmeans, optional): the only means the rows of each list can
// belong to (L2 with several means then builds a list's tables for those).
// seg_offs / seg_members (optional, with list_means): segmented lists, entry
// i of list q being entry i of the concatenated member ranges of q's means
// (ids_dev unused).
int host_distances(lvq_index *ix, const float *q_dev, int64_t nq, const int64_t *offsets_dev,
                   const int32_t *ids_dev, int64_t total, int32_t level, float *dist_dev, int32_t k,
                   int32_t *topk_ids_dev, float *topk_dist_dev, hipStream_t s, int force_shape, uint32_t epoch,
                   bool neg_empty, const int32_t *list_means = nullptr, int list_nmeans = 0,
                   const int64_t *seg_offs = nullptr, const int32_t *seg_members = nullptr,
                   const DistScratch *fixed = nullptr);

// Mark the work queued so far on `s` as a query reading the store at `epoch`
// (consolidation keeps the slots that query may still see).  may_create =
// false never creates an event: without a spare one it waits for the oldest
// in-flight launch and reuses its event.
int host_note_query(lvq_index *ix, hipStream_t s, uint32_t epoch, bool may_create = true);

// Per-device set-up of the allocation-free entry point's fixed scratch
// (called by lvq_create with the index's device current).
int noalloc_setup(int device);

// Size the workspace of stream `s` for every query batch of up to max_nq
// queries through host_topk (k_first, prec, scan_level) followed by
// host_distances (k_rerank at `rerank_level`, 0 for none), so that such calls
// on `s` allocate nothing.
int host_reserve(lvq_index *ix, hipStream_t s, int64_t max_nq, int32_t k_first, int32_t prec, int32_t scan_level,
                 int32_t k_rerank, int32_t rerank_level);

// Device buffers not tied to a stream, drawn from the index's memory budget.
int host_alloc(lvq_index *ix, DevBuf &b, size_t bytes);
void host_free(lvq_index *ix, DevBuf &b);

}  // namespace lvq
