/*
 * lvq_oracle.c -- plain CPU oracle for LVQ encoding and LVQ similarities.
 *
 * TEST INFRASTRUCTURE ONLY (see lvq_oracle.h).  Written for clarity, not
 * speed: scalar loops in the order of the paper's definitions.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -std=c11 -shared -fPIC.
 * -ffp-contract=off matters: every binary32 operation of the encoder must be
 * rounded on its own, as the definitions are written.
 *
 * Pinning of silent or ambiguous points of the paper (readings):
 *  - Eq. 1: u = max_j (x_j - mu_j), l = min_j (x_j - mu_j).
 *  - Eq. 2: the division by Delta is carried out as a multiplication by the
 *    correctly rounded reciprocal 1/Delta, as the paper's App. C listing does;
 *    the rounding is floor(v + 1/2) and codes are clamped to [0, 2^B - 1].
 *  - u == l (Delta = 0), and a Delta below the smallest normal binary32:
 *    Delta is stored as 0 and every code is 0 (no division by zero).
 *  - Residual level: Def. 1 is followed literally: Q_{B2,-Delta/2,Delta/2}
 *    with step Delta2 = Delta / (2^B2 - 1), unsigned codes, floor(v + 1/2).
 *  - Def. 1 nearest mean: sequential binary32 sum of squared differences in
 *    dimension order, ties to the lowest mean index.
 *  - A vector with a non-finite component (or a non-finite x - mu or u - l) is
 *    rejected: its row is all zero except l = NaN.
 *  - L2 is returned as the squared distance (same ranking as the norm).
 */
#include "lvq_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

/* Positions per layout block: Turbo 4-bit packs 128 dims into 64 bytes as
 * sixteen 32-bit words of eight nibbles (Sec. 3.1, App. B); Turbo 8-bit packs
 * 64 dims as sixteen words of four bytes (App. B, B1 = 8 remark); sequential
 * layouts store dimension j at position j, in 32-bit words.                */
static int block_positions(int bits, int layout)
{
    if (layout == ORC_TURBO) return bits == 4 ? 128 : 64;
    return bits == 4 ? 8 : 4;
}

int orc_format_init(orc_format *f, int dim, int bits1, int bits2, int layout, int align)
{
    if (!f || dim < 1 || dim > 65536) return ORC_EINVAL;
    if (bits1 != 4 && bits1 != 8) return ORC_EINVAL;
    if (bits2 != 0 && bits2 != 4 && bits2 != 8) return ORC_EINVAL;
    if (layout != ORC_SEQUENTIAL && layout != ORC_TURBO) return ORC_EINVAL;
    if (align != 32 && align != 64 && align != 128) return ORC_EINVAL;
    f->dim = dim;
    f->bits1 = bits1;
    f->bits2 = bits2;
    f->layout = layout;
    f->align = align;
    f->npos = round_up(dim, block_positions(bits1, layout));
    f->code_bytes = f->npos * bits1 / 8;
    f->row_bytes = round_up(ORC_HEADER_BYTES + f->code_bytes, align);
    f->resid_bytes = bits2 ? round_up(f->npos * bits2 / 8, align) : 0;
    return ORC_OK;
}

int orc_pos_to_dim(const orc_format *f, int p)
{
    int dim;
    if (p < 0 || p >= f->npos) return -1;
    if (f->layout == ORC_SEQUENTIAL) {
        dim = p;
    } else {
        /* Turbo: within a block, 32-bit word w holds, in its k-th field, the
         * dimension 16*k + w ("dimension 0 in nibble 0 of word 0, dimension 1
         * in nibble 0 of word 1, ... dimension 16 in nibble 1 of word 0"). */
        int per_word = 32 / f->bits1;           /* fields per 32-bit word */
        int blk = block_positions(f->bits1, f->layout);
        int b = p / blk, r = p % blk;
        int w = r / per_word, k = r % per_word;
        dim = b * blk + 16 * k + w;
    }
    return dim < f->dim ? dim : -1;
}

/* Field at position p of a packed little-endian code array of `bits` bits. */
static unsigned get_field(const uint8_t *codes, int bits, int p)
{
    if (bits == 8) return codes[p];
    return (codes[p / 2] >> (4 * (p % 2))) & 0xFu;
}

static void put_field(uint8_t *codes, int bits, int p, unsigned v)
{
    if (bits == 8) {
        codes[p] = (uint8_t)v;
    } else {
        int sh = 4 * (p % 2);
        codes[p / 2] = (uint8_t)((codes[p / 2] & ~(0xFu << sh)) | ((v & 0xFu) << sh));
    }
}

/* Def. 1: mu_* = argmin_m ||x - mu_m||^2. */
int orc_assign(const float *x, int d, const float *means, int n_means)
{
    int best = 0;
    float best_s = 0.0f;
    for (int m = 0; m < n_means; ++m) {
        float s = 0.0f;
        for (int j = 0; j < d; ++j) {
            float e = x[j] - means[(int64_t)m * d + j];
            float e2 = e * e;
            s = s + e2;
        }
        if (m == 0 || s < best_s) {
            best = m;
            best_s = s;
        }
    }
    return best;
}

/* Def. 1 distance of x to every mean, s_m = sum_j (x_j - mu_mj)^2, each a
 * sequential binary32 sum in dimension order (the values orc_assign ranks). */
void orc_mean_dists(const float *x, int d, const float *means, int n_means, float *s_out)
{
    for (int m = 0; m < n_means; ++m) {
        float s = 0.0f;
        for (int j = 0; j < d; ++j) {
            float e = x[j] - means[(int64_t)m * d + j];
            float sq = e * e;
            s = s + sq;
        }
        s_out[m] = s;
    }
}

/* Probe order of the soft inverted index: mean a comes before mean b when its
 * distance is smaller, or equal with the lower index; NaN distances last. */
static int probe_before(float sa, int ma, float sb, int mb)
{
    if (isnan(sa) != isnan(sb)) return isnan(sb);
    if (!isnan(sa) && sa != sb) return sa < sb;
    return ma < mb;
}

/* M-LVQ as a soft inverted index (the Sec. 3.2 remark that a query touches
 * only a few centres): the nprobe means nearest x by the Def. 1 distance,
 * nearest first.  Plain selection: nprobe passes, each taking the first
 * remaining mean in probe order.                                            */
int orc_probe(const float *x, int d, const float *means, int n_means, int nprobe, int32_t *out)
{
    if (nprobe < 1 || nprobe > n_means) return ORC_EINVAL;
    float *s = (float *)malloc(sizeof(float) * (size_t)n_means);
    char *taken = (char *)calloc((size_t)n_means, 1);
    if (!s || !taken) {
        free(s);
        free(taken);
        return ORC_EINVAL;
    }
    orc_mean_dists(x, d, means, n_means, s);
    for (int r = 0; r < nprobe; ++r) {
        int best = -1;
        for (int m = 0; m < n_means; ++m) {
            if (taken[m]) continue;
            if (best < 0 || probe_before(s[m], m, s[best], best)) best = m;
        }
        taken[best] = 1;
        out[r] = best;
    }
    free(s);
    free(taken);
    return ORC_OK;
}

/* Eq. 2 applied at one component: floor((t - lo) * inv + 1/2), clamped. */
static unsigned quantize_one(float t, float lo, float inv, unsigned top)
{
    float a = t - lo;
    float b = a * inv;
    float c = b + 0.5f;
    float v = floorf(c);
    if (!(v > 0.0f)) return 0;            /* also maps NaN to 0 */
    if (v > (float)top) return top;
    return (unsigned)v;
}

int orc_encode_codes(const float *x, int d, const float *mean, int bits1, int bits2,
                     float *l_out, float *delta_out, float *delta2_out, uint8_t *c1, uint8_t *c2)
{
    const unsigned top1 = (1u << bits1) - 1u;
    const unsigned top2 = bits2 ? (1u << bits2) - 1u : 0u;
    float *t = (float *)malloc(sizeof(float) * (size_t)d);
    float u = 0.0f, l = 0.0f, delta, delta2 = 0.0f;
    int finite = 1;

    /* Eq. 1: t = x - mu, u = max_j t_j, l = min_j t_j. */
    for (int j = 0; j < d; ++j) {
        t[j] = x[j] - mean[j];
        if (!isfinite(x[j]) || !isfinite(t[j])) finite = 0;
        if (j == 0 || t[j] > u) u = t[j];
        if (j == 0 || t[j] < l) l = t[j];
    }
    if (finite && !isfinite(u - l)) finite = 0;
    memset(c1, 0, (size_t)d);
    if (c2) memset(c2, 0, (size_t)d);
    if (!finite) {
        *l_out = NAN;
        *delta_out = 0.0f;
        *delta2_out = 0.0f;
        free(t);
        return ORC_NONFINITE;
    }

    /* Eq. 2 and Eq. 3: Delta = (u - l) / (2^B1 - 1), codes of t. */
    delta = (u - l) / (float)top1;
    if (!(delta >= FLT_MIN)) {
        delta = 0.0f;                      /* u == l: every code is 0 */
    } else {
        float inv = 1.0f / delta;
        for (int j = 0; j < d; ++j) c1[j] = (uint8_t)quantize_one(t[j], l, inv, top1);

        /* Residual level: r = t - (l + Delta c1) quantised by
         * Q_{B2, -Delta/2, Delta/2}, step Delta2 = Delta / (2^B2 - 1). */
        if (bits2) {
            delta2 = delta / (float)top2;
            if (!(delta2 >= FLT_MIN)) {
                delta2 = 0.0f;
            } else {
                float inv2 = 1.0f / delta2;
                float half = 0.5f * delta;
                for (int j = 0; j < d; ++j) {
                    float y = delta * (float)c1[j];
                    y = y + l;
                    float r = t[j] - y;
                    c2[j] = (uint8_t)quantize_one(r, -half, inv2, top2);
                }
            }
        }
    }
    *l_out = l;
    *delta_out = delta;
    *delta2_out = delta2;
    free(t);
    return ORC_OK;
}

static void put_f32(uint8_t *p, float v) { memcpy(p, &v, 4); }
static float get_f32(const uint8_t *p) { float v; memcpy(&v, p, 4); return v; }

int64_t orc_encode_rows(const orc_format *f, const float *X, int64_t n,
                        const float *means, int n_means, uint8_t *rows, uint8_t *resid)
{
    const int d = f->dim;
    uint8_t *c1 = (uint8_t *)malloc((size_t)d);
    uint8_t *c2 = (uint8_t *)malloc((size_t)d);
    int64_t rejected = 0;
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + i * d;
        uint8_t *row = rows + i * f->row_bytes;
        uint8_t *res = (resid && f->bits2) ? resid + i * f->resid_bytes : NULL;
        float l, delta, delta2;
        int finite = 1;
        for (int j = 0; j < d; ++j)
            if (!isfinite(x[j])) finite = 0;
        int m = (finite && n_means > 1) ? orc_assign(x, d, means, n_means) : 0;
        int rc = orc_encode_codes(x, d, means + (int64_t)m * d, f->bits1, f->bits2,
                                  &l, &delta, &delta2, c1, f->bits2 ? c2 : NULL);
        memset(row, 0, (size_t)f->row_bytes);
        if (res) memset(res, 0, (size_t)f->resid_bytes);
        if (rc != ORC_OK) {
            put_f32(row + 0, NAN);
            ++rejected;
            continue;
        }
        /* header: l, Delta, Delta2, mean id (store fields stay zero) */
        put_f32(row + 0, l);
        put_f32(row + 4, delta);
        put_f32(row + 8, delta2);
        row[12] = (uint8_t)m;
        for (int p = 0; p < f->npos; ++p) {
            int j = orc_pos_to_dim(f, p);
            if (j < 0) continue;
            put_field(row + ORC_HEADER_BYTES, f->bits1, p, c1[j]);
            if (res) put_field(res, f->bits2, p, c2[j]);
        }
    }
    free(c1);
    free(c2);
    return rejected;
}

void orc_unpack(const orc_format *f, const uint8_t *row, const uint8_t *resid,
                float *l, float *delta, float *delta2, int *mean_id, uint8_t *c1, uint8_t *c2)
{
    *l = get_f32(row + 0);
    *delta = get_f32(row + 4);
    *delta2 = get_f32(row + 8);
    *mean_id = row[12];
    for (int p = 0; p < f->npos; ++p) {
        int j = orc_pos_to_dim(f, p);
        if (j < 0) continue;
        c1[j] = (uint8_t)get_field(row + ORC_HEADER_BYTES, f->bits1, p);
        if (c2) c2[j] = (uint8_t)(resid && f->bits2 ? get_field(resid, f->bits2, p) : 0);
    }
}

/* x_hat = mu_* + l + Delta c1 (+ (-Delta/2 + Delta2 c2) at the full level). */
void orc_reconstruct(const orc_format *f, const uint8_t *row, const uint8_t *resid,
                     const float *means, int level, double *xhat)
{
    const int d = f->dim;
    uint8_t *c1 = (uint8_t *)malloc((size_t)d);
    uint8_t *c2 = (uint8_t *)malloc((size_t)d);
    float l, delta, delta2;
    int m;
    orc_unpack(f, row, resid, &l, &delta, &delta2, &m, c1, c2);
    const float *mu = means + (int64_t)m * d;
    int full = (level == ORC_FULL && f->bits2 && resid);
    for (int j = 0; j < d; ++j) {
        double v = (double)mu[j] + (double)l + (double)delta * (double)c1[j];
        if (full) v += -0.5 * (double)delta + (double)delta2 * (double)c2[j];
        xhat[j] = v;
    }
    free(c1);
    free(c2);
}

/* The two routines above over n consecutive rows (test bookkeeping). */
void orc_unpack_rows(const orc_format *f, const uint8_t *rows, const uint8_t *resid, int64_t n,
                     float *l, float *delta, float *delta2, int32_t *mean_id, uint8_t *c1, uint8_t *c2)
{
    for (int64_t i = 0; i < n; ++i) {
        int m;
        orc_unpack(f, rows + i * f->row_bytes, resid ? resid + i * f->resid_bytes : NULL, l + i, delta + i,
                   delta2 + i, &m, c1 + i * f->dim, c2 ? c2 + i * f->dim : NULL);
        mean_id[i] = m;
    }
}

void orc_reconstruct_rows(const orc_format *f, const uint8_t *rows, const uint8_t *resid, int64_t n,
                          const float *means, int level, double *xhat)
{
    for (int64_t i = 0; i < n; ++i)
        orc_reconstruct(f, rows + i * f->row_bytes, resid ? resid + i * f->resid_bytes : NULL, means, level,
                        xhat + i * f->dim);
}

void orc_distances(const orc_format *f, int metric, int level, const float *Q, int64_t nq,
                   const uint8_t *rows, const uint8_t *resid, const float *means,
                   const int64_t *offsets, const int32_t *ids, double *out)
{
    const int d = f->dim;
    double *xhat = (double *)malloc(sizeof(double) * (size_t)d);
    for (int64_t i = 0; i < nq; ++i) {
        const float *q = Q + i * d;
        for (int64_t e = offsets[i]; e < offsets[i + 1]; ++e) {
            int64_t s = ids[e];
            orc_reconstruct(f, rows + s * f->row_bytes,
                            resid ? resid + s * f->resid_bytes : NULL, means, level, xhat);
            double acc = 0.0;
            for (int j = 0; j < d; ++j) {
                if (metric == ORC_L2) {
                    double diff = (double)q[j] - xhat[j];
                    acc += diff * diff;
                } else {
                    acc += (double)q[j] * xhat[j];
                }
            }
            out[e] = acc;
        }
    }
    free(xhat);
}

/* Ranking (Sec. 2.1: higher similarity is better; L2 is a dissimilarity).
 * Returns nonzero when (sa, ia) ranks strictly before (sb, ib).           */
static int g_metric;
static int ranks_before(double sa, int32_t ia, double sb, int32_t ib)
{
    int na = isnan(sa), nb = isnan(sb);
    if (na != nb) return nb;               /* NaN ranks last */
    if (!na && sa != sb) return g_metric == ORC_L2 ? sa < sb : sa > sb;
    return ia < ib;
}

typedef struct { double s; int32_t id; } orc_pair;

static int cmp_pair(const void *a, const void *b)
{
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (ranks_before(x->s, x->id, y->s, y->id)) return -1;
    if (ranks_before(y->s, y->id, x->s, x->id)) return 1;
    return 0;
}

void orc_select_topk(int metric, const double *score, const int32_t *slot, const uint8_t *keep,
                     int64_t n, int k, int32_t *top_slot, double *top_score)
{
    orc_pair *v = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (keep && !keep[i]) continue;
        v[m].s = score[i];
        v[m].id = slot[i];
        ++m;
    }
    g_metric = metric;
    qsort(v, (size_t)m, sizeof(orc_pair), cmp_pair);
    for (int r = 0; r < k; ++r) {
        if (r < m) {
            top_slot[r] = v[r].id;
            top_score[r] = v[r].s;
        } else {
            top_slot[r] = -1;
            top_score[r] = metric == ORC_L2 ? INFINITY : -INFINITY;
        }
    }
    free(v);
}

/* Eq. 4: sum over vectors of || x - mu_* - Q(x) ||^2, first level only. */
double orc_eps1(const orc_format *f, const float *X, int64_t n, const uint8_t *rows,
                const float *means)
{
    const int d = f->dim;
    double *xhat = (double *)malloc(sizeof(double) * (size_t)d);
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        orc_reconstruct(f, rows + i * f->row_bytes, NULL, means, ORC_PRIMARY, xhat);
        for (int j = 0; j < d; ++j) {
            double e = (double)X[i * d + j] - xhat[j];
            total += e * e;
        }
    }
    free(xhat);
    return total;
}
