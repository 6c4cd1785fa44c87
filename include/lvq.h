/*
 * lvq.h -- C ABI of the MI355X (gfx950) LVQ library.
 *
 * Locally-adaptive Vector Quantization after "Locally-Adaptive Quantization
 * for Streaming Vector Search" (arXiv 2402.02044): per-vector LVQ encoding
 * (Sec. 2.3, Eq. 1-3), the two-level residual variant LVQ-B1xB2 (Sec. 2.3),
 * multi-means LVQ (Sec. 3.2, Def. 1), the Turbo code layout (Sec. 3.1,
 * App. B), and similarities between float queries and stored codes
 * (Sec. 3.2) over candidate lists and as an exhaustive top-k (Sec. 2.1).
 *
 * Conventions for every entry point
 *  - Pointers named *_dev are device pointers (HBM of the current device); the
 *    caller owns them and keeps them alive until the stream has passed the
 *    call.  Pointers named *_host are host pointers read before return.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously on it; argument checks are synchronous.
 *  - Return value: LVQ_OK (0) or a negative LVQ_ERR_* code; no C++ exception
 *    crosses the ABI.  Errors found inside kernels (an out-of-range slot, a
 *    non-finite input vector) set a sticky per-index error word, write NaN to
 *    the affected outputs, and are reported (and cleared) by lvq_sync.
 *  - The library owns the store (rows, residual rows, means, free-slot list)
 *    and its workspace, all in device memory it allocates itself, counted
 *    against lvq_config.mem_budget_bytes.
 *  - HIP graphs: lvq_distances, lvq_topk, lvq_probe_topk and
 *    lvq_graph_search may be captured into a graph on `stream` once an
 *    uncaptured call of the same size has sized the stream's workspace (a
 *    captured call allocates nothing and otherwise fails with
 *    LVQ_ERR_INVALID_ARG); lvq_distances_noalloc needs no such call.  A
 *    captured call replays at the store epoch of capture and does not order
 *    itself after store updates on other streams; no other entry point may
 *    be captured.  After a capture the stream's workspace is fixed for the
 *    index's life, so that no replay reads or writes freed memory: a later
 *    call on that stream that would need a larger workspace fails with
 *    LVQ_ERR_INVALID_ARG (use another stream).  The occupied-slot list a
 *    captured lvq_topk or lvq_probe_topk scans is never recycled by
 *    lvq_consolidate (each later consolidation writes a new list buffer), so
 *    replays keep scanning the slots listed at capture; a row deleted after
 *    the capture and then freed by a consolidation is no longer seen by
 *    them (its slot is cleared or holds a row inserted after the capture).
 *    Re-capture after consolidations to replay the current store.
 *  - Matrices are row-major and dense: x_dev is n x dim float32, q_dev is
 *    nq x dim (float32, or bfloat16 / float16 for lvq_topk's MFMA forms).
 *  - Similarity: LVQ_L2 returns the squared Euclidean distance to the
 *    reconstruction (smaller is better); LVQ_IP returns the inner product with
 *    it (larger is better).  Ties rank the lower slot first; NaN ranks last.
 */
#ifndef LVQ_H
#define LVQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lvq_index lvq_index;            /* opaque, owned by the library */

typedef enum { LVQ_L2 = 0, LVQ_IP = 1 } lvq_metric;
typedef enum { LVQ_SEQUENTIAL = 0, LVQ_TURBO = 1 } lvq_layout;
typedef enum { LVQ_PRIMARY = 1, LVQ_FULL = 2 } lvq_level;
/* LVQ_FP32_VALU: FP32 on the vector ALUs only (the plain kernel), for
 * lvq_topk; it computes what LVQ_FP32 computes, in another order. */
typedef enum { LVQ_FP32 = 0, LVQ_BF16 = 1, LVQ_FP16 = 2, LVQ_FP32_VALU = 3 } lvq_precision;

enum {
    LVQ_OK = 0,
    LVQ_ERR_INVALID_ARG = -1,
    LVQ_ERR_UNSUPPORTED = -2,
    LVQ_ERR_OOM = -3,          /* device allocation failed or memory budget exceeded */
    LVQ_ERR_CAPACITY = -4,     /* not enough free slots */
    LVQ_ERR_DEVICE = -5,       /* HIP runtime error */
    LVQ_ERR_NONFINITE = -6,    /* an input vector had a non-finite component */
    LVQ_ERR_BAD_SLOT = -7,     /* a slot id out of range (or not live for lvq_delete) */
    LVQ_ERR_SCRATCH = -8       /* lvq_distances_noalloc: the call needs more than its fixed scratch */
};

/* Index configuration.
 *  dim       vector dimensionality d (1..8192)
 *  bits1     first-level bits B1: 4 or 8 (Eq. 3)
 *  bits2     residual bits B2: 0 (one level), 4 or 8 (Sec. 2.3, LVQ-B1xB2)
 *  metric    LVQ_L2 or LVQ_IP
 *  layout    LVQ_SEQUENTIAL (dimension j at code position j) or LVQ_TURBO
 *            (Sec. 3.1: per 64-byte block of sixteen 32-bit words, dimension
 *            16k + w of the block in field k of word w; 128 dims per block
 *            at 4 bits, 64 dims at 8 bits; zero padded)
 *  align     row stride alignment in bytes: 32 (the paper's padding, App. D),
 *            64 or 128
 *  capacity  number of slots of the store (may be 0 for encode-only use)
 *  mem_budget_bytes  cap on device memory owned by the index (0 = none)   */
typedef struct {
    int32_t dim, bits1, bits2;
    int32_t metric, layout, align;
    int64_t capacity;
    int64_t mem_budget_bytes;
} lvq_config;

/* Row format.  Each slot holds one row of row_bytes: a 32-byte header
 *   [0]  float l        per-vector lower bound (Eq. 1)
 *   [4]  float delta    first-level step (Eq. 2); 0 when u == l
 *   [8]  float delta2   residual step delta / (2^B2 - 1); 0 without residual
 *   [12] uint8 mean id  index of the mean the vector was encoded against (Def. 1)
 *   [13] uint8 flags    bit 0: slot holds a stored vector
 *   [16] uint32 insert epoch, [20] uint32 delete epoch (0xFFFFFFFF = live)
 *   [24] uint64 external id
 * then the first-level codes (little-endian fields of B1 bits by code
 * position), zero padded to a multiple of align.  The residual codes of the
 * same slot occupy resid_bytes in a separate array, by the same code
 * positions.  lvq_encode writes zero store fields.  A vector rejected as
 * non-finite is written as all-zero except l = NaN.                        */
int lvq_row_format(const lvq_config *cfg, int32_t *row_bytes, int32_t *resid_bytes,
                   int32_t *code_positions);

/* Create an index on the current device.  means_host: n_means x dim float32,
 * the centres of Def. 1 (n_means = 1 is plain LVQ with the global mean);
 * 1 <= n_means <= 256, values finite.                                      */
int lvq_create(const lvq_config *cfg, const float *means_host, int32_t n_means,
               lvq_index **out);
int lvq_destroy(lvq_index *index);

/* Append means (M-LVQ re-estimation, Sec. 3.2): the new centres get ids
 * n_old .. n_old + n_means - 1 (*first_id_out, may be NULL, receives n_old);
 * existing rows keep their mean ids and the table never drops an entry, so
 * at most 256 means exist over the index's life.  The copies are enqueued
 * on `stream` and later calls on any stream are ordered after them; work
 * already queued reads only the old ids.  Synchronises `stream`.          */
int lvq_set_means(lvq_index *index, const float *means_host, int32_t n_means,
                  int32_t *first_id_out, void *stream);

/* Encode n vectors (Eq. 1-3, residual level, Def. 1) into caller buffers:
 * rows_dev n x row_bytes, resid_dev n x resid_bytes (NULL when bits2 == 0).
 * Rows are bit-identical to a binary32 evaluation with one rounding per
 * operation.  Pure: the store is not touched.                              */
int lvq_encode(lvq_index *index, const float *x_dev, int64_t n, uint8_t *rows_dev,
               uint8_t *resid_dev, void *stream);

/* Encode n vectors into free slots (a new insert epoch).  Slots are taken
 * from the top of the free-slot stack: vector i receives the i-th slot
 * popped; slots_out_dev (n int32) receives them.  ext_ids_dev (n uint64) may
 * be NULL (external id = slot).  LVQ_ERR_CAPACITY if fewer than n slots are
 * free (checked synchronously; nothing is written).                        */
int lvq_insert(lvq_index *index, const float *x_dev, int64_t n, const uint64_t *ext_ids_dev,
               int32_t *slots_out_dev, void *stream);

/* Lazy delete (Sec. 2.2 / App. A, delete consolidation): tombstone n slots at
 * a new epoch.  A slot that is out of range or not live sets LVQ_ERR_BAD_SLOT
 * (sticky) and is skipped.                                                 */
int lvq_delete(lvq_index *index, const int32_t *slots_dev, int64_t n, void *stream);

/* Batched consolidation: every tombstoned slot whose delete epoch no
 * in-flight query (lvq_distances / lvq_topk not yet complete) can still see
 * is cleared and pushed on the free-slot stack, in descending slot order (so
 * later inserts pop them in ascending order).  Synchronises `stream`;
 * *n_freed_out (may be NULL) receives the number of slots freed.           */
int lvq_consolidate(lvq_index *index, void *stream, int64_t *n_freed_out);

/* Similarities of nq queries (q_dev nq x dim float32) to their candidate
 * lists: CSR offsets_dev (nq+1 int64, offsets[0] = 0, offsets[nq] = total)
 * and ids_dev (total int32 slots).  dist_dev (total float32, may be NULL when
 * k > 0) receives one value per listed entry, computed also for tombstoned
 * slots (lazy deletes are still traversed).  level LVQ_PRIMARY uses the first
 * level, LVQ_FULL both levels (Sec. 2.3: first level during traversal,
 * both to re-rank).  With k > 0 (k <= 1024) the best k entries of each list
 * that are live at the call are written to topk_ids_dev / topk_dist_dev
 * (nq x k), padded with slot -1 and the worst value (+inf for L2, -inf for
 * IP).  Duplicate ids are scored once per entry.                           */
int lvq_distances(lvq_index *index, const float *q_dev, int64_t nq, const int64_t *offsets_dev,
                  const int32_t *ids_dev, int64_t total, int32_t level, float *dist_dev,
                  int32_t k, int32_t *topk_ids_dev, float *topk_dist_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * allocation): lvq_distances with the same arguments, semantics, kernels and
 * results, except that its scratch -- the queries in kernel order
 * (nq x kpos floats, kpos = code positions rounded up to 16-byte chunks),
 * the sums of q (nq floats), the per-mean terms (nq x n_means floats), the
 * list order (nq int32) and a work counter, each rounded up to 256 bytes --
 * lives in one fixed array of LVQ_NOALLOC_SCRATCH_BYTES per device instead of
 * the stream's workspace.  The call allocates nothing and creates no event
 * (with no spare in-flight record it waits for the oldest query launch of
 * the index), and lvq_set_timing does not time it.  The array is set up by
 * lvq_create on each device an index is created on and is held until the
 * process ends.  Every call on a device shares that device's array, and it
 * keeps the last call's contents: calls that overlap on one device (on
 * different streams, or from different indices) race and must be ordered by
 * the caller.  A call needing more scratch than the array returns
 * LVQ_ERR_SCRATCH before enqueuing anything (at d = 768, 4-bit codes: up to
 * about 10,900 queries); LVQ_ERR_INVALID_ARG if the current device is not
 * the index's.                                                             */
#define LVQ_NOALLOC_SCRATCH_BYTES (32u << 20)
int lvq_distances_noalloc(lvq_index *index, const float *q_dev, int64_t nq, const int64_t *offsets_dev,
                          const int32_t *ids_dev, int64_t total, int32_t level, float *dist_dev,
                          int32_t k, int32_t *topk_ids_dev, float *topk_dist_dev, void *stream);

/* Tile shapes of the candidate-list kernel (lanes per candidate, bytes per
 * load, loads per lane, software pipelining; see the library source for the
 * table).  lvq_autotune runs lvq_distances on the caller's representative
 * batch with every shape the index's format admits (one warm-up, three timed
 * repetitions each, HIP events on `stream`), keeps the fastest for this
 * level and top-k mode (k > 0 or not), and returns its index and the
 * milliseconds of one call.  It allocates and frees its own output buffers
 * and synchronises `stream`.  lvq_set_tile selects a shape directly (-1
 * restores the built-in choice), e.g. from a saved tuning result.          */
int lvq_autotune(lvq_index *index, const float *q_dev, int64_t nq, const int64_t *offsets_dev,
                 const int32_t *ids_dev, int64_t total, int32_t level, int32_t k, int32_t *shape_out,
                 float *ms_out, void *stream);
int lvq_set_tile(lvq_index *index, int32_t level, int32_t topk, int32_t shape);
/* Number of tile shapes (valid shape indices are 0 .. count - 1) and the
 * parameters of one: lanes per candidate, bytes per load, loads per lane and
 * round, pipeline flags (bit 0 software-pipelined, bit 1 query in
 * registers, bit 2 two blocks ahead, bit 3 registers allotted for at least
 * six waves per SIMD).  Outputs may be NULL.                              */
int lvq_num_tile_shapes(void);
int lvq_tile_shape(int32_t shape, int32_t *lanes, int32_t *piece_bytes, int32_t *pieces, int32_t *pipe);

/* Exhaustive top-k over every slot live at the call (Sec. 2.1 k-NN problem),
 * for nq queries q_dev (nq x dim) of precision prec at `level`: LVQ_FP32
 * takes float queries and FP32 products -- on the FP32 matrix cores
 * (v_mfma_f32_32x32x2_f32, codes converted exactly) for the first-level inner
 * product of an index with one mean and k <= 512, else on the vector ALUs;
 * LVQ_BF16 / LVQ_FP16 take queries already in that type and run matrix-core
 * (MFMA) products of queries and exactly converted integer codes with FP32
 * accumulation (inner product; both levels need 8-bit residual codes).
 * 1 <= k <= 1024 (the per-query candidate buffers must fit the LDS:
 * LVQ_ERR_UNSUPPORTED otherwise).  Output ids_dev / dist_dev nq x k, padded
 * as for lvq_distances.  LVQ_FP32_VALU takes float queries on the vector
 * path whatever the format (the plain FP32 kernel, for comparisons).        */
int lvq_topk(lvq_index *index, const void *q_dev, int32_t prec, int64_t nq, int32_t k,
             int32_t level, int32_t *ids_dev, float *dist_dev, void *stream);

/* M-LVQ as a soft inverted index (the Sec. 3.2 remark that a query touches
 * only a few centres).  For each of nq float queries q_dev (nq x dim): the
 * nprobe means nearest the query by the Def. 1 distance (squared Euclidean,
 * binary32, summed in dimension order, ties to the lower mean id, NaN last:
 * the rule that assigns rows to means), and the best k rows at `level` among
 * the rows assigned to those means and live at the call (lvq_distances'
 * similarities and ranking).  1 <= nprobe <= number of means, 1 <= k <= 1024.
 * probe_out_dev (nq x nprobe int32, may be NULL) receives the probed mean
 * ids, nearest first; ids_dev / dist_dev (nq x k) are padded as for
 * lvq_distances.  The per-mean member lists are kept per stream and rebuilt
 * by the first call after a store update (one pass over the occupied slots);
 * the candidate kernel walks the probed means' member ranges in place.  The
 * call is asynchronous; captured into a HIP graph (after a first call on the
 * stream has sized its buffers) it replays at the epoch of capture.        */
int lvq_probe_topk(lvq_index *index, const float *q_dev, int64_t nq, int32_t nprobe, int32_t k,
                   int32_t level, int32_t *probe_out_dev, int32_t *ids_dev, float *dist_dev,
                   void *stream);

/* Greedy graph search (Alg. 1) with first-level similarities (Sec. 2.3: the
 * first level traverses; re-rank the result with lvq_distances at both
 * levels).  graph_dev: capacity x degree int32 out-neighbour slots of every
 * stored slot (-1: no edge; 1 <= degree <= 64); entries_dev: n_entries start
 * nodes shared by all queries (1 <= n_entries <= 64).  Per query the
 * candidate set starts at the entries; the closest unexplored node is
 * explored, its out-neighbours not proposed before join the set, and the set
 * is cut to the `window` closest (1 <= k <= window <= 256); ranks are
 * lvq_distances' similarities, ties to the lower slot.  Deleted rows are
 * traversed but left out of the result: ids_dev / dist_dev (nq x k) hold the
 * k best live nodes of the final set, padded as for lvq_distances;
 * explored_dev (nq x 2 int32, may be NULL) the nodes explored and the nodes
 * scored (distinct entries, then one per out-neighbour entry scored: a
 * neighbour rejected once is scored again when proposed again, and a node
 * listed twice in one row counts twice) per query.  The nodes that enter a
 * query's candidate set are kept in a table of 8 * (window + 64) entries
 * (at most 16384); a query in which more enter
 * stops there and sets the sticky error (lvq_sync reports
 * LVQ_ERR_INVALID_ARG).                                                    */
int lvq_graph_search(lvq_index *index, const float *q_dev, int64_t nq, const int32_t *graph_dev,
                     int32_t degree, const int32_t *entries_dev, int32_t n_entries, int32_t window,
                     int32_t k, int32_t *ids_dev, float *dist_dev, int32_t *explored_dev, void *stream);

/* Neighbourhood pruning (Alg. 2) over float vectors x_dev (n x dim, row i =
 * node i; 1 <= dim <= 4096).  For each of the m distinct nodes p =
 * nodes_dev[i] (device int32): the candidates cand_ids_dev[cand_offsets_dev[i]
 * .. cand_offsets_dev[i + 1]) (device int64 offsets, m + 1; -1 entries are
 * skipped) together with p's current out-neighbours graph_dev[p * degree ..]
 * (n x degree int32, -1 padded, 1 <= degree <= 64), without p and without
 * repeats, are ranked by similarity to p (L2: binary32 squared distance,
 * smaller first; IP: inner product, larger first; ties to the lower node);
 * the best remaining candidate x* becomes an out-neighbour and leaves the
 * candidates, and until `degree` are chosen every candidate x' is dropped for
 * which x* is at least alpha times as similar (L2: alpha * |x* - x'|^2 <=
 * |p - x'|^2; IP: alpha * <x*, x'> >= <p, x'>).  The row of p is rewritten
 * with the chosen nodes in selection order, -1 padded.  Long candidate
 * lists are taken in groups -- whole blocks of 256 entries, in order, as many
 * as fit in 256 + degree candidates beside the out-neighbours chosen so far
 * -- each group pruned together with them.  Synchronises `stream`; LVQ_ERR_BAD_SLOT for a node outside
 * [0, n).                                                                  */
int lvq_graph_prune(const float *x_dev, int64_t n, int32_t dim, int32_t metric, const int32_t *nodes_dev,
                    int64_t m, const int64_t *cand_offsets_dev, const int32_t *cand_ids_dev, int32_t degree,
                    float alpha, int32_t *graph_dev, void *stream);

/* Graph construction (App. A) over float vectors x_dev (n x dim, row i =
 * node i), into graph_dev (n x degree int32, -1 padded).  Nodes [0, first)
 * already form a graph whose rows are kept; nodes [first, n) are inserted
 * with the update routine: the `window` nodes nearest to x found by greedy
 * search (Alg. 1, float similarities as lvq_graph_prune) from `entry` are
 * pruned with x's out-neighbours into its new out-neighbours (lvq_graph_prune
 * with alpha), and x is added to the out-neighbours of each of them, which are
 * pruned when that exceeds `degree`.  first = 0 is the initial build: the
 * entry node goes first, then the others in node order, and with passes = 2
 * the routine runs over all of them twice, with alpha = 1 and then `alpha`
 * (1.2 for L2, 0.95 for IP in the paper); passes = 1 runs it once with
 * `alpha` (inserts).  Nodes are processed in batches of at most max_batch
 * (and at most the number of nodes already in the graph): the nodes of a
 * batch search the graph as it was before the batch, so the result depends
 * on max_batch.  Requires degree <= window <= 256, 0 <= entry < n (entry <
 * first when first > 0).  Synchronises `stream`.                           */
int lvq_graph_build(const float *x_dev, int64_t n, int32_t dim, int32_t metric, int64_t first, int32_t degree,
                    int32_t window, float alpha, int32_t passes, int32_t entry, int32_t max_batch,
                    int32_t *graph_dev, void *stream);

/* Insertions (App. A): the update routine of lvq_graph_build, once with
 * `alpha`, for the m distinct nodes nodes_host[0 .. m) (host int32, in that
 * order; their rows are cleared first; none of them the entry), into the
 * graph formed by the other nodes -- e.g. slots freed by a consolidation and
 * filled again.  Batches as lvq_graph_build.  Synchronises `stream`.        */
int lvq_graph_insert(const float *x_dev, int64_t n, int32_t dim, int32_t metric, const int32_t *nodes_host,
                     int64_t m, int32_t degree, int32_t window, float alpha, int32_t entry, int32_t max_batch,
                     int32_t *graph_dev, void *stream);

/* Delete consolidation (App. A) of the nodes flagged in deleted_dev (n bytes,
 * nonzero = deleted): every kept node x' with deleted out-neighbours takes as
 * candidates its kept out-neighbours and the kept out-neighbours of each
 * deleted one (x' -> x -> x'' becomes x' -> x''); more than `degree` distinct
 * candidates are pruned as in lvq_graph_prune (the degree x degree table of
 * neighbours' neighbours read in blocks of 256 positions, grouped as
 * lvq_graph_prune groups its candidates; a single group for degree <= 16).
 * Every row is read as it was before the call; rows of deleted nodes become
 * -1.  A deleted node must no longer serve as an entry.  Synchronises
 * `stream`.                                                                */
int lvq_graph_delete(const float *x_dev, int64_t n, int32_t dim, int32_t metric, const uint8_t *deleted_dev,
                     int32_t degree, float alpha, int32_t *graph_dev, void *stream);

/* Online re-estimation of M-LVQ means with selective re-encoding (Sec. 3.2;
 * updating means needs the rows of the moved centres re-encoded).
 *
 * lvq_retire_means: the listed ids are no longer chosen by the nearest-mean
 * search of later encodes and inserts; rows already assigned keep them, and
 * routing (lvq_probe_topk) still ranks every id.  At least one mean must stay
 * active (LVQ_ERR_INVALID_ARG otherwise).
 *
 * lvq_add_means: n new centres (n x dim, host memory).  Each takes the lowest
 * retired id that no occupied slot refers to any more (its rows deleted and
 * freed by lvq_consolidate, so no unfinished query can see them), else the
 * next unused id (at most 256 ids over the index's life); ids_out_host (n)
 * receives the ids.  LVQ_ERR_CAPACITY when fewer than n ids are free.
 *
 * lvq_mean_members: the slots of the rows live at the call whose mean is one
 * of mean_ids_host[0 .. n): offsets_host (n + 1, host) receives the ranges
 * and slots_dev[offsets_host[i] .. offsets_host[i + 1]) the slots of mean i,
 * in no particular order; LVQ_ERR_CAPACITY if more than cap rows.  Re-encoding
 * them is a delete plus an insert of their original vectors (with their
 * external ids).
 *
 * All three are ordered after earlier updates, synchronise `stream`, and
 * cannot be captured into a HIP graph (LVQ_ERR_UNSUPPORTED).              */
int lvq_retire_means(lvq_index *index, const int32_t *ids_host, int32_t n, void *stream);
int lvq_add_means(lvq_index *index, const float *means_host, int32_t n, int32_t *ids_out_host,
                  void *stream);
int lvq_mean_members(lvq_index *index, const int32_t *mean_ids_host, int32_t n, int64_t *offsets_host,
                     int32_t *slots_dev, int64_t cap, void *stream);

/* Copy stored rows of n slots (slots_dev int32) into rows_dev / resid_dev. */
int lvq_read_rows(lvq_index *index, const int32_t *slots_dev, int64_t n, uint8_t *rows_dev,
                  uint8_t *resid_dev, void *stream);

/* Bandwidth probes, for measurement: the loads of an access pattern without
 * the arithmetic, giving the ceiling a kernel with that pattern can reach.
 * Both write to *sink_dev (device uint32, zeroed first) the XOR of every
 * 32-bit word they read, so no load can be elided and the result can be
 * checked.  Asynchronous on `stream`.
 *
 * lvq_bw_stream: a coalesced streaming read of `bytes` (a multiple of 16) at
 * src_dev (16-byte aligned); LVQ_ERR_INVALID_ARG otherwise.
 * lvq_bw_gather: for each of the n slots ids_dev[i] (device int32; out of
 * range ones skipped), the bytes the similarity kernels fetch: the 32-byte
 * header and the first-level code chunks and, at LVQ_FULL, the residual row
 * (4, 8 or 16 lanes per slot, whichever covers a row in one round of
 * 16-byte loads), in list order.                                           */
int lvq_bw_stream(const void *src_dev, int64_t bytes, uint32_t *sink_dev, void *stream);
int lvq_bw_gather(lvq_index *index, const int32_t *ids_dev, int64_t n, int32_t level, uint32_t *sink_dev,
                  void *stream);

/* Store statistics (host values).  The last_* fields describe the most
 * recent lvq_distances, lvq_topk or lvq_probe_topk call on the index (zero
 * before the first): last_workgroups is the grid of its main similarity
 * launch, last_lists the lists it scored (lvq_distances, lvq_probe_topk:
 * the persistent workgroups pop lists from a device counter, so a grid
 * smaller than the list count makes workgroups take several lists), and
 * last_parts the row parts an exhaustive scan split the occupied slots
 * into (lvq_topk; each part keeps its own top-k, merged afterwards).      */
typedef struct {
    int64_t capacity, free_slots, live_estimate, device_bytes;
    int32_t n_means, row_bytes, resid_bytes, code_positions;
    uint32_t epoch;
    int64_t last_workgroups, last_lists;
    int32_t last_parts;
} lvq_stats;
int lvq_get_stats(lvq_index *index, lvq_stats *out);

/* Measurement support.  While enabled, each launch of the main similarity
 * kernel of lvq_distances / lvq_topk is bracketed by HIP events recorded on
 * the call's stream.  lvq_kernel_time waits for those events and returns the
 * summed kernel milliseconds and the number of launches since the previous
 * read (or since enabling), then starts a new count.                       */
int lvq_set_timing(lvq_index *index, int enable);
int lvq_kernel_time(lvq_index *index, double *ms_out, int64_t *launches_out);

/* Synchronise `stream` and return (then clear) the sticky kernel error. */
int lvq_sync(lvq_index *index, void *stream);

/* Column mean of n x dim float32 vectors (the global mean of Sec. 2.3),
 * accumulated in binary64, rounded to float32.                            */
int lvq_mean(const float *x_dev, int64_t n, int32_t dim, float *mean_out_dev, void *stream);

/* k-means (Lloyd) for the M-LVQ centres (Sec. 3.2): start from the vectors at
 * init_idx_host (k distinct indices, the seed's random draws), `iters`
 * iterations of nearest-centre assignment and centroid update (an empty
 * cluster keeps its centre).  means_out_dev k x dim float32.              */
int lvq_kmeans(const float *x_dev, int64_t n, int32_t dim, int32_t k, const int64_t *init_idx_host,
               int32_t iters, float *means_out_dev, void *stream);

/* ---- Request server -------------------------------------------------------
 * Continuous batching of k-NN query batches (the problem of Sec. 2.1) over an
 * index that changes meanwhile (inserts and deletes, Sec. 2.2).  A server
 * owns `slots` HIP streams and a device pool of pool_bytes (drawn from the
 * index's memory budget).  lvq_server_submit copies a batch of nq float32
 * queries (host memory, nq x dim) and queues it; batches are admitted in
 * arrival order as soon as a stream slot is free and the pool can hold the
 * batch's buffers (admission by memory: small batches take less), and
 * admitted batches run concurrently, one per stream.  Each batch is answered
 * at the store epoch current at its admission: an exhaustive top-k (as
 * lvq_topk, at `precision` and scan_level), or a first-level top-k_first
 * whose candidates are re-ranked with both levels (as lvq_distances with a
 * top-k, Sec. 2.3: the second level re-ranks).  The result of a batch
 * equals that of the same batch run alone at the same epoch.  Store updates
 * (lvq_insert, lvq_delete, lvq_consolidate, lvq_set_means) may be issued on
 * the index from other threads at any time; batches admitted after an update
 * see it, and consolidation keeps every slot an unfinished batch may see.
 * Sticky kernel errors are reported by lvq_sync as usual.  Destroy the
 * server before its index.                                                 */
typedef struct lvq_server lvq_server;

typedef struct {
    int32_t slots;         /* batches in flight at once (streams), 1..64 */
    int32_t max_batch;     /* largest nq of one batch, 1..65536 */
    int32_t k;             /* results per query, 1..1024 */
    int32_t k_first;       /* first-level candidates per query, k..1024 (LVQ_FULL) */
    int32_t precision;     /* exhaustive scan: LVQ_FP32, LVQ_BF16 or LVQ_FP16 (IP) */
    int32_t scan_level;    /* level of the exhaustive scan: LVQ_PRIMARY, or LVQ_FULL
                              (one stage: its top-k is the result) */
    int32_t rerank_level;  /* with scan_level LVQ_PRIMARY: LVQ_FULL re-ranks the
                              k_first candidates with both levels (needs bits2 > 0);
                              LVQ_PRIMARY takes the first-level top-k as the result */
    int64_t pool_bytes;    /* device memory of admitted batches together;
                              0 = room for `slots` batches of max_batch */
} lvq_server_config;

/* Per-batch record: status (LVQ_OK or the error the batch met), its size,
 * the epoch it was answered at, the slot that ran it, and times in seconds
 * since the server's creation (steady clock) of submission, admission and
 * observed completion.                                                     */
typedef struct {
    int32_t status, nq;
    uint32_t epoch;
    int32_t slot;
    double t_submit, t_admit, t_done;
} lvq_request_info;

typedef struct {
    int64_t submitted, completed;
    int64_t pool_bytes, pool_peak, batch_bytes_max;
    int32_t slots, peak_in_flight, peak_queue, queued, in_flight;
} lvq_server_stats;

/* Create a server on the index's device: streams, the pool, pinned staging
 * buffers, and every stream's scan workspace for all batch sizes up to
 * max_batch, so that serving allocates no device memory.                  */
int lvq_server_create(lvq_index *index, const lvq_server_config *cfg, lvq_server **out);
/* Queue a batch (1 <= nq <= max_batch); q_host is copied before return.
 * *ticket_out identifies it to lvq_server_wait.                           */
int lvq_server_submit(lvq_server *server, const float *q_host, int32_t nq, int64_t *ticket_out);
/* Block until the batch is done; copy its nq x k results (ids_host int32,
 * dist_host float32, ordered best first, padded as for lvq_topk; either may
 * be NULL) and its record (may be NULL); forget the ticket.  Returns the
 * batch's status; LVQ_ERR_INVALID_ARG for an unknown ticket.              */
int lvq_server_wait(lvq_server *server, int64_t ticket, int32_t *ids_host, float *dist_host,
                    lvq_request_info *info);
/* Block until every submitted batch is done. */
int lvq_server_drain(lvq_server *server);
int lvq_server_get_stats(lvq_server *server, lvq_server_stats *out);
/* Finish every submitted batch, then release the server. */
int lvq_server_destroy(lvq_server *server);

const char *lvq_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
