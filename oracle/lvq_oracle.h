/*
 * lvq_oracle.h -- plain CPU statement of Locally-adaptive Vector Quantization
 * (LVQ) encoding and of the similarities computed on LVQ codes.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library; it
 * is called only by the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark.  The product path never links or calls it,
 * and it shares no code with the GPU library.
 *
 * Paper: "Locally-Adaptive Quantization for Streaming Vector Search"
 * (arXiv 2402.02044).  Every function names the passage it follows.
 *
 * Precision: encoding decides integer codes from floating point, so it is
 * carried out in IEEE binary32 with one rounding per operation, no fused
 * multiply-add (build with -ffp-contract=off), which is the precision of the
 * paper's own listing (App. C works on float32 arrays).  Reconstructions,
 * distances and everything downstream are binary64.
 */
#ifndef LVQ_ORACLE_H
#define LVQ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_NONFINITE = -6 };
enum { ORC_L2 = 0, ORC_IP = 1 };                 /* similarity */
enum { ORC_SEQUENTIAL = 0, ORC_TURBO = 1 };     /* code layout (Sec. 3.1) */
enum { ORC_PRIMARY = 1, ORC_FULL = 2 };          /* level (Sec. 2.3) */

/* Storage format of one encoded vector.  A row is a 32-byte header followed by
 * the first-level codes, zero padded to a multiple of `align` bytes (the paper
 * pads LVQ vectors to multiples of 32 bytes, Sec. 3.2 and App. D).  The
 * optional second-level (residual) codes live in a separate array, one row per
 * slot, in the same position order as the first level.                        */
typedef struct {
    int32_t dim, bits1, bits2, layout, align;
    int32_t npos;         /* number of code positions (dims padded to the block) */
    int32_t code_bytes;   /* bytes of first-level codes                          */
    int32_t row_bytes;    /* header + codes, padded to align                     */
    int32_t resid_bytes;  /* residual row stride (0 when bits2 == 0)             */
} orc_format;

#define ORC_HEADER_BYTES 32

int orc_format_init(orc_format *f, int dim, int bits1, int bits2, int layout, int align);
/* Logical dimension stored at code position p, or -1 for padding. */
int orc_pos_to_dim(const orc_format *f, int p);

/* Index of the nearest mean by squared Euclidean distance (Def. 1). */
int orc_assign(const float *x, int d, const float *means, int n_means);

/* Def. 1 distances of x to every mean (sequential binary32 sums in dimension
 * order), and the soft-inverted-index routing: the nprobe means nearest x,
 * nearest first, ties to the lower index, NaN distances last (Sec. 3.2). */
void orc_mean_dists(const float *x, int d, const float *means, int n_means, float *s_out);
int orc_probe(const float *x, int d, const float *means, int n_means, int nprobe, int32_t *out);

/* First and second level codes of one vector against one mean
 * (Eq. 1, Eq. 2, Eq. 3 and the residual level of Sec. 2.3 / Def. 1).
 * c2 may be NULL when bits2 == 0.  Returns ORC_OK or ORC_NONFINITE.           */
int orc_encode_codes(const float *x, int d, const float *mean, int bits1, int bits2,
                     float *l, float *delta, float *delta2, uint8_t *c1, uint8_t *c2);

/* Encode n vectors into rows (n x row_bytes) and residual rows
 * (n x resid_bytes, may be NULL when bits2 == 0).  Returns the number of
 * vectors that were rejected as non-finite.                                 */
int64_t orc_encode_rows(const orc_format *f, const float *X, int64_t n,
                        const float *means, int n_means, uint8_t *rows, uint8_t *resid);

/* Read one row back: header fields and codes in logical dimension order. */
void orc_unpack(const orc_format *f, const uint8_t *row, const uint8_t *resid,
                float *l, float *delta, float *delta2, int *mean_id,
                uint8_t *c1, uint8_t *c2);

/* Reconstruction x_hat (binary64) of one stored row at the given level. */
void orc_reconstruct(const orc_format *f, const uint8_t *row, const uint8_t *resid,
                     const float *means, int level, double *xhat);
/* orc_unpack / orc_reconstruct over n consecutive rows (and residual rows). */
void orc_unpack_rows(const orc_format *f, const uint8_t *rows, const uint8_t *resid, int64_t n,
                     float *l, float *delta, float *delta2, int32_t *mean_id, uint8_t *c1, uint8_t *c2);
void orc_reconstruct_rows(const orc_format *f, const uint8_t *rows, const uint8_t *resid, int64_t n,
                          const float *means, int level, double *xhat);

/* Similarity of queries to listed slots: L2 = squared Euclidean distance to
 * the reconstruction, IP = inner product with it (Sec. 3.2).  offsets has
 * nq+1 entries; ids[offsets[i] .. offsets[i+1]) are the slots of query i.   */
void orc_distances(const orc_format *f, int metric, int level, const float *Q, int64_t nq,
                   const uint8_t *rows, const uint8_t *resid, const float *means,
                   const int64_t *offsets, const int32_t *ids, double *out);

/* Best k entries of a scored list: L2 ascending, IP descending, ties to the
 * lower slot; entries with keep[i] == 0 are skipped; missing entries are
 * padded with slot -1 and the worst value.                                  */
void orc_select_topk(int metric, const double *score, const int32_t *slot, const uint8_t *keep,
                     int64_t n, int k, int32_t *top_slot, double *top_score);

/* First-level quantisation error of Eq. 4 as a sum over the given rows,
 * measured against the float vectors X.                                      */
double orc_eps1(const orc_format *f, const float *X, int64_t n, const uint8_t *rows,
                const float *means);

#ifdef __cplusplus
}
#endif
#endif
