// lvq_internal.h -- declarations shared by the host side of the library and
// the kernel translation units.  Not part of the public ABI (see lvq.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lvq.h"

namespace lvq {

constexpr int kHeaderBytes = 32;
constexpr uint32_t kLiveEpoch = 0xFFFFFFFFu;   // delete epoch of a live row
constexpr int kMaxMeans = 256;
constexpr int kMaxTopK = 1024;

// sticky error bits raised by kernels
enum : uint32_t { kErrNonFinite = 1u, kErrBadSlot = 2u, kErrBadOffsets = 4u, kErrOverflow = 8u };

// Storage format (mirrors the row description in lvq.h).
struct Format {
    int dim, bits1, bits2, layout, align;
    int npos;        // code positions (dims padded to the layout block)
    int code_bytes;  // first-level code bytes
    int row_bytes;   // header + codes, padded to align
    int resid_bytes; // residual row stride (0 without a residual level)
    int kchunks;     // 16-byte chunks of first-level codes read by the kernels
    int kpos;        // code positions covered by those chunks
};

bool make_format(const lvq_config &cfg, Format *f);

// Kernel order of code positions.  For 4-bit codes the fields of a 32-bit
// word are visited as (0,2,4,6,1,3,5,7): the low nibble of each byte first,
// then the high nibble, so one mask exposes four fields to byte-wise
// conversion; 8-bit codes keep their natural order.  kdim[s] is the
// dimension held at kernel slot s, or -1.
void kernel_order_dims(const Format &f, int32_t *kdim /* kpos entries */);

// ---- argument blocks -------------------------------------------------------

struct EncodeArgs {
    const float *x;          // n x dim
    int64_t n;
    const float *means;      // M x dim
    const float *means_t;    // dim rows of means_t_stride (transposed copy, coalesced assignment)
    int means_t_stride;
    int n_means;
    int means_lds;           // stage the means in LDS (small M x dim)
    const uint8_t *mean_active;  // n_means flags: 0 = retired (not chosen by the nearest-mean search)
    Format f;
    uint8_t *rows;           // output rows (row i at rows + slot(i) * row_bytes)
    uint8_t *resid;
    // store mode (insert): slots popped from the free stack
    const int32_t *free_stack;  // NULL for pure encode
    int64_t free_top;           // stack top before the pop
    int32_t *slots_out;
    const uint64_t *ext_ids;
    int32_t *list_out;          // store mode: vector i's slot is appended at list_out[i]
    uint32_t epoch;
    uint32_t *err;
};

struct PrepArgs {
    const void *q;           // nq x dim (fp32)
    int64_t nq;
    int dim, kpos, n_means, metric;
    const int32_t *kdim;     // kpos entries
    const float *means;      // M x dim
    float *qk;               // nq x kpos (kernel order, zero at padding)
    float *qsum;             // nq
    float *cm;               // nq x M (IP: <q, mu_m>)
};

struct CandArgs {
    const uint8_t *rows;
    const uint8_t *resid;
    int row_bytes, resid_bytes;
    int kchunks, kpos;
    int64_t capacity;
    const float *qk, *qsum, *cm;
    const float *muk;        // M x kpos means in kernel order (L2)
    const float *kmask;      // kpos: 1 at real positions, 0 at padding (L2)
    int n_means;
    const int64_t *offsets;
    const int32_t *ids;
    int64_t nq, total;
    float *dist;             // may be NULL
    int k;
    int32_t *topk_ids;
    float *topk_dist;
    uint32_t epoch;
    uint32_t *err;
    const int32_t *order;    // list processing order (NULL: identity)
    int32_t *queue;          // persistent work counter (NULL: one list per block)
    int neg_empty;           // a negative id is an empty entry, not an error
    int cw;                  // top-k key buffer entries per wave (>= k + 32)
    int mu_lds;              // L2 with several means: keep muk in LDS for the launch
    const int32_t *list_means;   // the means each list's rows belong to (nq x list_nmeans),
    int list_nmeans;             // or NULL for any mean
    const int64_t *seg_offs;     // segmented lists: member ranges per mean (n_means + 1) and the
    const int32_t *seg_members;  // members; a list is its means' ranges in list_means order
};

struct ScanArgs {
    const uint8_t *rows;
    const uint8_t *resid;
    int row_bytes, resid_bytes, kchunks, kpos;
    const int32_t *list;     // occupied slots; entries [0, n_rows) are scanned
    int64_t n_rows;
    const float *qk, *qsum, *cm, *muk, *kmask;
    const void *q16;         // MFMA forms: nq x kpos bf16/fp16 in kernel order
    int n_means;
    int64_t nq;
    int k;
    uint32_t epoch;
    int64_t rows_per_part;
    int n_parts;
    int capq;                // per-query key buffer capacity in LDS
    uint32_t *gthr;          // nq: order key bound of the k-th best score seen by any part
    uint64_t *part_keys;     // nq x n_parts x k sortable keys
    uint32_t *err;
    uint64_t *mkeys;         // wide matrix-core scan: per-workgroup key regions (mcap keys per query:
    int mcap, mks;           //   mks sorted best keys, then the keys appended since they were merged)
};

struct StoreArgs {
    uint8_t *rows;
    uint8_t *resid;
    int row_bytes, resid_bytes;
    int64_t capacity;
    uint32_t epoch;
    uint32_t *err;
};

// ---- launchers (each returns hipSuccess or the launch error) --------------

hipError_t launch_encode(const EncodeArgs &a, hipStream_t s);
hipError_t launch_prep(const PrepArgs &a, hipStream_t s);
// Kernel tables: k_cand / k_scan instantiations by first-level width, level
// residual width (0 at the first level), variant and tile shape; nullptr when
// not instantiated.  cand variants: 0 IP, 1 L2, 2 L2 several means, 3 L2
// masked, 4 L2 masked several means.  scan variants: 0 IP, 1 L2, 2 L2 masked.
struct TileShape {
    int g, ch, nch;   // lanes per candidate, bytes per piece, pieces per lane and round
    int pipe;         // bit 0: software-pipelined single-round candidate loop;
                      // bit 1: query values held in registers for a whole list;
                      // bit 2: the pipeline runs two blocks of candidates ahead
};
int num_tile_shapes();
TileShape tile_shape(int i);
void *cand_kernel_b4(int bits2, int variant, int shape);
void *cand_kernel_b8(int bits2, int variant, int shape);
void *scan_kernel_b4(int bits2, int variant, int shape);
void *scan_kernel_b8(int bits2, int variant, int shape);
size_t cand_lds_bytes(int kpos, int ntab, bool mask, int n_means_ip, int k, int cw, bool map = false,
                      int nseg = 0);
size_t scan_lds_bytes(int kpos, int n_means_ip, int k, int capq);
int scan_capq(int kpos, int n_means_ip, int k, int rows_per_round, size_t lds_max);
int scan_rows_per_round(int g);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
// Soft inverted index (k_probe.hip): per-mean member lists of `list`
// (counts, cursor: n_means entries; offsets: n_means + 1; members: n entries,
// filled beforehand with -1), routing of queries to their nprobe nearest
// means, and the list offsets of the probed means' members (qoffs: nq + 1).
hipError_t launch_members(const int32_t *list, int64_t n, const uint8_t *rows, int row_bytes, int n_means,
                          unsigned long long *counts, unsigned long long *cursor, int64_t *offsets,
                          int32_t *members, hipStream_t s);
hipError_t launch_route(const float *q, int64_t nq, int dim, const float *means_t, int means_stride, int n_means,
                        int nprobe, int32_t *probe, hipStream_t s);
hipError_t launch_probe_offsets(const int32_t *probe, int64_t nq, int nprobe, const int64_t *moffs, int64_t *qoffs,
                                hipStream_t s);
// Greedy graph search (k_graph.hip): one workgroup per query.
struct GraphLaunch {
    const uint8_t *rows;
    int row_bytes, kchunks, kpos, bits1, metric;
    int64_t capacity;
    const float *qk, *qsum, *cm, *muk, *kmask;
    int n_means;
    int64_t nq;
    const int32_t *graph;    // capacity x degree slots, -1: no edge
    int degree;
    const int32_t *entries;
    int n_entries;
    int window, k;
    uint32_t epoch;
    int32_t *ids;
    float *dist;
    int32_t *explored;       // nq x 2 (explored, scored), may be NULL
    uint32_t *err;
    // float mode (graph construction): rows == NULL, the nodes are the float
    // vectors xf (capacity x dim); query i is xf[qnodes[i]] (kpos = dim)
    const float *xf;
    int dim;
    const int32_t *qnodes;
};
// Seen-set hash slots of a walk (a power of two, at most 16384) and the
// search kernel's LDS bytes.
int graph_hash_slots(int window, int degree);
size_t graph_lds_bytes(int kpos, int window, int degree);
hipError_t launch_graph_search(const GraphLaunch &l, hipStream_t s);

// Neighbourhood pruning (Alg. 2) over float vectors, one workgroup per node.
// Node i = nodes[i]; its candidates are cids[coffs[j] .. coffs[j + 1]) with
// j = i (by_node 0) or j = the node (by_node 1), or cids[i * cstride ..
// (i + 1) * cstride) when coffs is NULL; -1 entries are skipped.  They are
// taken in groups of whole blocks of kPruneChunk positions, as many blocks
// as fit (at most kPruneChunk + R candidates) beside the out-neighbours kept
// so far, each group merged with those; `always` 0 prunes only a merge
// holding more than R distinct nodes.  With `deleted` (n flags) the
// candidate positions are instead the R x R table of p's out-neighbours'
// out-neighbours, of which only the kept out-neighbours of deleted ones
// count, and p's own deleted out-neighbours are dropped (delete
// consolidation).
constexpr int kPruneChunk = 256;
constexpr int kGraphMaxDegree = 64;
constexpr int kGraphMaxDim = 4096;
struct PruneLaunch {
    const float *xf;
    int dim, metric;
    int64_t n;
    const int32_t *nodes;
    int64_t m;
    const int64_t *coffs;
    int by_node;
    const int32_t *cids;
    int cstride;
    int always;
    int32_t *graph;
    int R;
    float alpha;
    uint32_t *err;
    const uint8_t *deleted;
};
hipError_t launch_graph_prune(const PruneLaunch &l, hipStream_t s);
// Kept nodes with a deleted out-neighbour into out[0 .. *count); rows of the
// flagged (deleted) or listed (nodes, m) nodes set to -1.
hipError_t launch_graph_affected(const int32_t *graph, int R, int64_t n, const uint8_t *deleted, int32_t *out,
                                 int32_t *count, hipStream_t s);
hipError_t launch_graph_clear_rows(int32_t *graph, int R, int64_t n, const uint8_t *deleted, const int32_t *nodes,
                                   int64_t m, hipStream_t s);

// Reverse edges of the out-neighbours of nodes[0..m): cnt (n, all zero on
// entry and on return) counts them; offs (n + 1) receives the CSR offsets by
// target node, rev the sources, touched[0 .. *ntouched) the targets.
// scratch: at least (n + 2047) / 2048 + 1 int64.
hipError_t launch_reverse_edges(const int32_t *graph, int R, const int32_t *nodes, int64_t m, int64_t n,
                                int32_t *cnt, int64_t *offs, int64_t *scratch, int32_t *rev, int32_t *touched,
                                int32_t *ntouched, hipStream_t s);

hipError_t launch_mean_counts(const int32_t *list, int64_t n, const uint8_t *rows, int row_bytes, int n_means,
                              unsigned long long *counts, hipStream_t s);
// Live members (flag set, insert epoch <= epoch < delete epoch) of the means
// req[0..nreq): counts[i] (zeroed here) receives their number; with out_offs,
// the slots of mean i are also written at out[out_offs[i] ..] in no order.
hipError_t launch_members_live(const int32_t *req, int nreq, const int64_t *moffs, const int32_t *members,
                               const uint8_t *rows, int row_bytes, uint32_t epoch, const int64_t *out_offs,
                               int32_t *out, unsigned long long *counts, hipStream_t s);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Bandwidth probes (measurement): *sink = XOR of every 32-bit word read.
hipError_t launch_bw_stream(const void *src, int64_t n16, uint32_t *sink, hipStream_t s);
hipError_t launch_bw_gather(const uint8_t *rows, int row_bytes, int code16, const uint8_t *resid, int resid_bytes,
                            int res16, const int32_t *ids, int64_t n, int64_t capacity, uint32_t *sink, hipStream_t s);
hipError_t launch_list_order(const int64_t *offsets, int64_t nq, int32_t *order, int32_t *scratch,
                             hipStream_t s);
// bits2: 0 scans the first level, 8 both levels (8-bit residual codes).
hipError_t launch_scan_mfma(const ScanArgs &a, int bits1, int bits2, int prec, hipStream_t s);
typedef void (*MfmaKernelPtr)(ScanArgs);
MfmaKernelPtr mfma_kernel_first(int bits1, int kpos, int fp16, int *qb);
MfmaKernelPtr mfma_kernel_full(int bits1, int kpos, int fp16, int *qb);
// MFMA exhaustive scan: 32-query blocks per workgroup for a format (0 when
// the code width / position count has no instantiation), its LDS bytes, and
// the query-fragment precompute for bf16 / fp16 queries.
int mfma_query_block(int bits1, int bits2, int kpos);
size_t mfma_lds_bytes(int qb, int n_means, int k, int capq);
int mfma_capq(int qb, int n_means, int k, size_t lds_max);
// The wide matrix-core scan (queries staged in LDS, inner product, k <=
// 512): prec LVQ_BF16 / LVQ_FP16 at the first level with one mean, or
// LVQ_FP32 on the FP32 MFMA at the first level (bits2 0) or both levels
// (bits2 8) with any mean count whose c_m table fits the LDS.  The 32-query
// blocks per workgroup (0 when the format, precision, k, means or the LDS
// bytes rule it out), the sorted keys kept per query (k rounded up to a
// power of two, at least 64) and the key-region capacity per query, and the
// launch of a persistent grid (a multiple of 8 workgroups, each owning
// 32*qb*cap keys of a.mkeys; a.mks and a.mcap as these functions give them).
// The FP32 forms read a.q16 as the fragments launch_frag32 writes from
// kernel-order queries (nq x kpos FP32, as prep_queries leaves them):
// 32*qb*kpos*4 bytes per tile of 32*qb queries; and a.cm as nq x n_means.
int mfma_wide_query_block(int bits1, int bits2, int kpos, int prec, int k, int n_means, size_t lds_max);
int mfma_wide_sorted(int k);
int mfma_wide_cap(int k);
hipError_t launch_scan_mfma_wide(const ScanArgs &a, int bits1, int bits2, int prec, int64_t grid, size_t lds_max,
                                 hipStream_t s);
hipError_t launch_frag32(const float *qk, int64_t nq, int kpos, int bits1, int qb, void *frag, hipStream_t s);
hipError_t launch_prep16(const void *q, int64_t nq, int dim, int kpos, int bits1, int qb, int prec,
                         const int32_t *kdim, const float *means, int n_means, void *frag, float *qsum, float *cm,
                         hipStream_t s);
// fp32 -> bf16 / fp16 (LVQ_BF16 / LVQ_FP16), round to nearest even, n values.
hipError_t launch_cast16(const float *x, int64_t n, int prec, void *out, hipStream_t s);
hipError_t launch_topk_merge(const uint64_t *part_keys, int64_t nq, int n_parts, int k, int metric,
                             int32_t *ids, float *dist, hipStream_t s);
hipError_t launch_delete(const StoreArgs &a, const int32_t *slots, int64_t n, hipStream_t s);
hipError_t launch_consolidate(const StoreArgs &a, uint32_t safe_epoch, int32_t *free_stack,
                              int64_t free_top, int32_t *block_counts, int64_t *new_top,
                              hipStream_t s);
// The occupied slots (flags bit 0), ascending, into list; count to *len.
hipError_t launch_build_list(const StoreArgs &a, int32_t *list, int32_t *block_counts, int64_t *len,
                             hipStream_t s);
hipError_t launch_gather_rows(const StoreArgs &a, const int32_t *slots, int64_t n, uint8_t *rows_out,
                              uint8_t *resid_out, hipStream_t s);
hipError_t launch_mean(const float *x, int64_t n, int dim, float *out, double *scratch, hipStream_t s);
hipError_t launch_kmeans_assign(const float *x, int64_t n, int dim, const float *c, int k,
                                int32_t *assign, hipStream_t s);
hipError_t launch_kmeans_update(const float *x, int64_t n, int dim, const int32_t *assign, int k,
                                float *c, hipStream_t s);

}  // namespace lvq
